// Row updates and downdates of a sketch (Section 5, Algorithms 2 and 3):
//     SA += sum_t op_t S_r(:, j_t) a_t,
// op_t = +1 for a row added at index j_t, -1 for the row at j_t removed.  S_r is the updated
// sketching matrix: column j of the call's S for a row j < m of the sketched matrix; for a row
// appended at j >= m, a Gaussian column g_j / sqrt(s) (Algorithm 2; Section 5.3 takes the same
// column for the non-Gaussian kinds).  For the Gaussian kind every column is G_hat(:, j) / sqrt(s),
// so updates agree with sketching the changed matrix from scratch.  Columns are regenerated
// from the draws' counters; nothing of S is stored.
//
// One thread per element (i, c) of SA adds its r terms in order (deterministic, no atomics);
// the work is s N r entries of S_r, each a few integer operations (Hadamard), one sincospi
// (DCT), one Floyd column (sparse sign) or one Box-Muller pair (Gaussian).
#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "sketch_device.hpp"

namespace nsk {

// OCP E4M3 (no infinities): sign, 4 exponent bits (bias 7), 3 mantissa bits.
__device__ inline float e4m3_value(uint8_t b) {
  const uint32_t e = (b >> 3) & 15u, mnt = b & 7u;
  float v;
  if ((b & 0x7Fu) == 0x7Fu) v = __builtin_nanf("");
  else if (e == 0) v = (float)mnt * 0x1p-9f;
  else v = ldexpf(1.0f + (float)mnt * 0.125f, (int)e - 7);
  return (b & 0x80u) ? -v : v;
}

template <typename T> __device__ inline double row_value(const T* p) { return (double)*p; }
template <> __device__ inline double row_value<uint16_t>(const uint16_t* p) {
  return (double)__uint_as_float((uint32_t)*p << 16);
}
template <> __device__ inline double row_value<uint8_t>(const uint8_t* p) { return (double)e4m3_value(*p); }

struct RowUpdate {
  int kind;
  int64_t m;      // rows of the sketched matrix
  int64_t M;      // Hadamard: next power of two of m; DCT-II: its padded length
  int N, s, zeta, r, gdtype;
  uint64_t seed;
  const int* srows;       // Hadamard / DCT-II: sorted sampled rows
  const int64_t* idx;     // r row indices j_t
  const int8_t* ops;      // r signs op_t
};

// Entry (i, j) of G (stream 5): block (j, i / 4); words 0, 1 give rows 4q, 4q + 1 and words 2, 3
// rows 4q + 2, 4q + 3 by Box-Muller with u = (a + 1) 2^-32, v = b 2^-32.
__device__ inline double gauss_fp64(uint64_t seed, int i, int64_t j) {
  const Words w = philox(seed, (uint64_t)j, (uint32_t)(i >> 2), kGauss);
  const int h = (i >> 1) & 1;
  const uint32_t a = h ? w.w[2] : w.w[0], b = h ? w.w[3] : w.w[1];
  const double u = ((double)a + 1.0) * 0x1p-32, v = (double)b * 0x1p-32;
  const double rad = sqrt(-2.0 * log(u));
  double sn, cs;
  sincospi(2.0 * v, &sn, &cs);
  return (i & 1) ? rad * sn : rad * cs;
}

__device__ inline double gauss_hat(uint64_t seed, int i, int64_t j, int gdtype) {
  const Words w = philox(seed, (uint64_t)j, (uint32_t)(i >> 2), kGauss);
  float g[4];
  if (gdtype == NSK_BF16) gauss_hat4<NSK_BF16>(w, g); else gauss_hat4<NSK_F8E4M3>(w, g);
  return (double)g[i & 3];
}

// S_r(i, j)
__device__ inline double sr_entry(const RowUpdate& u, int i, int64_t j) {
  const double rs = 1.0 / sqrt((double)u.s);
  if (u.kind == NSK_GAUSSIAN) return gauss_hat(u.seed, i, j, u.gdtype) * rs;
  if (j >= u.m) return gauss_fp64(u.seed, i, j) * rs;
  if (u.kind == NSK_SPARSE_SIGN) {
    int rw[32];
    uint32_t neg;
    sparse_column<32>(u.seed, (uint64_t)j, u.s, u.zeta, rw, neg);
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < 32; ++t)
      if (t < u.zeta && rw[t] == i) v = ((neg >> t) & 1u) ? -1.0 : 1.0;
    return v / sqrt((double)u.zeta);
  }
  const uint32_t dw = word(philox(u.seed, (uint64_t)(j >> 7), 0, kSigns), (uint32_t)((j >> 5) & 3));
  const double d = ((dw >> (j & 31)) & 1u) ? -1.0 : 1.0;
  const int64_t k = u.srows[i];
  if (u.kind == NSK_SRHT) return (__popcll((uint64_t)(k & j)) & 1) ? -d * rs : d * rs;
  // DCT-II: d_j w_k cos(pi k (2j + 1) / (2M)), the angle reduced modulo one period
  const uint64_t n = ((uint64_t)k * (uint64_t)(2 * j + 1)) & (4 * (uint64_t)u.M - 1);
  const double w = k == 0 ? rs : sqrt(2.0 / (double)u.s);
  return d * w * cospi((double)n / (2.0 * (double)u.M));
}

template <typename T>
__global__ __launch_bounds__(256) void row_update_kernel(Operand op, RowUpdate u, double* __restrict__ SA,
                                                         int64_t ldsa) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)u.s * u.N) return;
  const int i = (int)(e / u.N), c = (int)(e % u.N);
  const T* base;
  int64_t ld;
  column_ref<T>(op, c, base, ld);
  const double scale = ldexp(1.0, column_exp(op, c));  // FP8 operands: per-column exponent
  double acc = 0.0;
  for (int t = 0; t < u.r; ++t) {
    const double a = row_value<T>(base + (int64_t)t * ld) * scale;
    acc += (double)u.ops[t] * sr_entry(u, i, u.idx[t]) * a;
  }
  SA[(int64_t)i * ldsa + c] += acc;
}

hipError_t launch_row_update(const Operand& op, const SketchPlan& p, const int64_t* idx, const int8_t* ops, int r,
                             double* SA, int64_t ldsa, hipStream_t st) {
  RowUpdate u;
  u.kind = p.kind;
  u.m = p.m;
  u.M = p.kind == NSK_SRDCT ? srdct_pool(p.m) : next_pow2(p.m);
  u.N = p.N;
  u.s = p.s;
  u.zeta = p.zeta;
  u.r = r;
  u.gdtype = op.dtype;
  u.seed = p.seed;
  u.srows = p.rows;
  u.idx = idx;
  u.ops = ops;
  const unsigned blocks = (unsigned)(((int64_t)p.s * p.N + 255) / 256);
  switch (op.dtype) {
    case NSK_F64: row_update_kernel<double><<<blocks, 256, 0, st>>>(op, u, SA, ldsa); break;
    case NSK_F32: row_update_kernel<float><<<blocks, 256, 0, st>>>(op, u, SA, ldsa); break;
    case NSK_BF16: row_update_kernel<uint16_t><<<blocks, 256, 0, st>>>(op, u, SA, ldsa); break;
    default: row_update_kernel<uint8_t><<<blocks, 256, 0, st>>>(op, u, SA, ldsa); break;
  }
  return hipGetLastError();
}

}  // namespace nsk
