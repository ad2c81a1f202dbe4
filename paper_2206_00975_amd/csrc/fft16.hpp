// Complex arithmetic and a 16-point DFT held in registers, for the DCT-II sketch.  Every
// twiddle used here is a power of w = e^{-2 pi i / 32}; after unrolling, the exponents are
// compile-time constants and the multiplications by 1 and -i disappear.
#pragma once

namespace nsk {

template <typename T> struct alignas(2 * sizeof(T)) cx { T r, i; };

template <typename T> __host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T> __host__ __device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}

// cos(pi a / 16) for 0 <= a <= 16 (decimal expansions of the exact values).
__host__ __device__ constexpr double cos_pi16_first(int a) {
  return a == 0 ? 1.0
       : a == 1 ? 0.98078528040323044912618223613424
       : a == 2 ? 0.92387953251128675612818318939679
       : a == 3 ? 0.83146961230254523707878837761791
       : a == 4 ? 0.70710678118654752440084436210485
       : a == 5 ? 0.55557023301960222474283081394853
       : a == 6 ? 0.38268343236508977172845998403040
       : a == 7 ? 0.19509032201612826784828486847702
       : 0.0;
}
__host__ __device__ constexpr double cos_pi16(int a) { return a <= 8 ? cos_pi16_first(a) : -cos_pi16_first(16 - a); }

// x * e^{-2 pi i a / 32} for 0 <= a <= 16.
template <typename T> __host__ __device__ inline cx<T> mul_w32(cx<T> x, int a) {
  if (a == 0) return x;
  if (a == 8) return {x.i, -x.r};
  if (a == 16) return {-x.r, -x.i};
  const T c = (T)cos_pi16(a);
  const T s = (T)cos_pi16(a < 8 ? 8 - a : a - 8);  // sin(pi a / 16)
  return {x.r * c + x.i * s, x.i * c - x.r * s};
}

// In-place 16-point DFT X[k] = sum_n x[n] e^{-2 pi i n k / 16}: radix-2 decimation in time
// on the bit-reversed input, natural-order output.
template <typename T> __host__ __device__ inline void dft16(cx<T> (&x)[16]) {
  cx<T> y[16];
#pragma unroll
  for (int n = 0; n < 16; ++n) y[n] = x[((n & 1) << 3) | ((n & 2) << 1) | ((n & 4) >> 1) | ((n & 8) >> 3)];
#pragma unroll
  for (int h = 1; h < 16; h <<= 1) {
#pragma unroll
    for (int g = 0; g < 16; g += 2 * h) {
#pragma unroll
      for (int j = 0; j < h; ++j) {
        const cx<T> a = y[g + j];
        const cx<T> b = mul_w32(y[g + j + h], j * (16 / h));  // e^{-2 pi i j / (2h)}
        y[g + j] = a + b;
        y[g + j + h] = a - b;
      }
    }
  }
#pragma unroll
  for (int n = 0; n < 16; ++n) x[n] = y[n];
}

}  // namespace nsk
