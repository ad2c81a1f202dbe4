// Stages after the SVD: the residual |A V_k|_F with FP64 accumulation (Problem 2.1), the
// TLS solution x = -v(1:n)/v(N) (Section 4), and the backward pass of a loss L(x) through the
// sketched TLS solution (S^T applied by regenerating S from its seed).
#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "svd_device.hpp"
#include "svd_pipeline.hpp"

namespace nsk {

// ============================================================================ residual
constexpr int kResThreads = 256;

template <typename T>
__global__ __launch_bounds__(kResThreads) void residual_kernel(Operand op, int64_t m, int N,
                                                               const double* __restrict__ Vk, int k,
                                                               double* __restrict__ partial) {
  extern __shared__ double vsh[];  // N x k row-major
  __shared__ double wsum[kResThreads / 64];
  for (int e = threadIdx.x; e < N * k; e += blockDim.x) vsh[e] = Vk[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  double local = 0;
  for (int64_t row = (int64_t)blockIdx.x * wpb + wave; row < m; row += (int64_t)gridDim.x * wpb) {
    for (int q0 = 0; q0 < k; q0 += 4) {
      double d[4] = {0, 0, 0, 0};
      for (int c = lane; c < N; c += 64) {
        const T* b;
        int64_t ld;
        column_ref<T>(op, c, b, ld);
        const double a = (double)b[row * ld];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q0 + q < k) d[q] += a * vsh[c * k + q0 + q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q0 + q < k) {
          const double t = wave_sum(d[q]);
          local += t * t;
        }
    }
  }
  if (lane == 0) wsum[wave] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < wpb; ++w) t += wsum[w];
    partial[blockIdx.x] = t;
  }
}

__global__ void residual_finish(const double* __restrict__ partial, int parts, double* out, nsk_info* info) {
  if (threadIdx.x != 0) return;
  double t = 0;
  for (int i = 0; i < parts; ++i) t += partial[i];
  const double r = sqrt(t);
  if (out) *out = r;
  if (info) info->residual = r;
}

hipError_t launch_residual(const Operand& op, int64_t m, const double* Vk, int k, double* partial, int parts,
                           double* out, nsk_info* info, hipStream_t st) {
  const int N = op.col0[op.nb];
  const size_t lds = (size_t)N * k * sizeof(double);
  if (op.dtype == NSK_F64)
    residual_kernel<double><<<parts, kResThreads, lds, st>>>(op, m, N, Vk, k, partial);
  else
    residual_kernel<float><<<parts, kResThreads, lds, st>>>(op, m, N, Vk, k, partial);
  residual_finish<<<1, 64, 0, st>>>(partial, parts, out, info);
  return hipGetLastError();
}

// ========================================================================= TLS forward
// x = -v(1:n) / v(N) with v the trailing right singular vector of the sketched [A | b].
__global__ void tls_extract_kernel(int N, const double* __restrict__ v, double* __restrict__ x) {
  const double last = v[N - 1];
  for (int e = threadIdx.x; e < N - 1; e += blockDim.x) x[e] = -v[e] / last;
}

hipError_t launch_tls_extract(int N, const double* v, double* x, hipStream_t st) {
  tls_extract_kernel<<<1, 256, 0, st>>>(N, v, x);
  return hipGetLastError();
}

// ======================================================================== TLS backward
// g_bar = dL/dv = -(1/v_N) [g; g.x];  w = V D V^T g_bar with D_c = 1 / (sigma_N^2 - sigma_c^2)
// for every column c except the trailing one (D = 0 there): the first-order change of the
// trailing right singular vector of SA.  V^T g_bar and V z are applied by replaying the
// Jacobi rotation log forward (transposed) and backward.  work = [SA v (s), SA w (s), v, w].
__global__ __launch_bounds__(512) void tls_adjoint_kernel(int s, int N, TlsBack tb, const double* __restrict__ gx,
                                                           double* __restrict__ work) {
  extern __shared__ double sm[];
  const JacobiShape js = jacobi_shape(N);
  const int ncols = js.nb * js.B;
  double* xb = sm;             // ncols
  double* wl = xb + ncols;     // N: w
  __shared__ double red[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int n = N - 1;
  double gxdot = 0;
  for (int e = tid; e < n; e += blockDim.x) gxdot += gx[e] * tb.x[e];
  gxdot = wave_sum(gxdot);
  if (lane == 0) red[wave] = gxdot;
  __syncthreads();
  if (tid == 0) {
    double t = 0;
    for (int w = 0; w < nw; ++w) t += red[w];
    red[0] = t;
  }
  __syncthreads();
  const double gx_x = red[0];
  const double inv = -1.0 / tb.v[N - 1];
  for (int e = tid; e < ncols; e += blockDim.x) xb[e] = e < N ? inv * (e < n ? gx[e] : gx_x) : 0.0;
  __syncthreads();
  const int sweeps = tb.jres->sweeps;
  if (wave == 0) replay_dispatch(xb, tb.log, js, sweeps, true, lane);
  __syncthreads();
  const int cN = tb.order[N - 1];
  const double lamN = tb.colnorm[cN] * tb.colnorm[cN];
  for (int c = tid; c < ncols; c += blockDim.x) {
    const double sc = tb.colnorm[c < N ? c : 0];
    xb[c] = (c < N && c != cN) ? xb[c] / (lamN - sc * sc) : 0.0;
  }
  __syncthreads();
  if (wave == 0) replay_dispatch(xb, tb.log, js, sweeps, false, lane);
  __syncthreads();
  for (int e = tid; e < N; e += blockDim.x) wl[e] = xb[e];
  __syncthreads();
  for (int i = tid; i < s; i += blockDim.x) {
    double a = 0, b = 0;
    for (int c = 0; c < N; ++c) {
      const double m = tb.sa_rm[(size_t)i * N + c];
      a += m * tb.v[c];
      b += m * wl[c];
    }
    work[i] = a;
    work[s + i] = b;
  }
  for (int e = tid; e < N; e += blockDim.x) {
    work[2 * s + e] = tb.v[e];
    work[2 * s + N + e] = wl[e];
  }
}

template <typename TOut, int ZMAX>
__global__ __launch_bounds__(256) void tls_grad_sparse_kernel(int64_t m, int N, int s, int zeta, uint64_t seed,
                                                              const double* __restrict__ work, TOut* __restrict__ dA,
                                                              int64_t ldda, TOut* __restrict__ db) {
  extern __shared__ double sm[];
  double* yv = sm;
  double* yw = yv + s;
  double* vv = yw + s;
  double* ww = vv + N;
  for (int e = threadIdx.x; e < 2 * s + 2 * N; e += blockDim.x) sm[e] = work[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double scale = 1.0 / sqrt((double)zeta);
  const int n = N - 1;
  const int64_t rows_per_wave = 64;
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6) * rows_per_wave;
  for (int64_t r0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * rows_per_wave; r0 < m; r0 += stride) {
    const int64_t j = r0 + lane;
    double p = 0, q = 0;
    if (j < m) {
      int rw[ZMAX];
      uint32_t nb;
      sparse_column<ZMAX>(seed, (uint64_t)j, s, zeta, rw, nb);
#pragma unroll
      for (int z = 0; z < ZMAX; ++z)
        if (z < zeta) {
          const double sg = ((nb >> z) & 1u) ? -scale : scale;
          p += sg * yv[rw[z]];
          q += sg * yw[rw[z]];
        }
    }
    const int nrow = (int)(m - r0 < 64 ? m - r0 : 64);
    for (int rr = 0; rr < nrow; ++rr) {
      const double pj = __shfl(p, rr, 64), qj = __shfl(q, rr, 64);
      const int64_t row = r0 + rr;
      for (int c = lane; c < n; c += 64) dA[row * ldda + c] = (TOut)(pj * ww[c] + qj * vv[c]);
      if (lane == 0) db[row] = (TOut)(pj * ww[n] + qj * vv[n]);
    }
  }
}

template <typename TOut>
__global__ __launch_bounds__(256) void tls_grad_srht_kernel(int64_t m, int N, int s, uint64_t seed,
                                                            const int* __restrict__ rows,
                                                            const double* __restrict__ work, TOut* __restrict__ dA,
                                                            int64_t ldda, TOut* __restrict__ db) {
  extern __shared__ double sm[];
  double* yv = sm;
  double* yw = yv + s;
  double* vv = yw + s;
  double* ww = vv + N;
  int* sr = reinterpret_cast<int*>(ww + N);
  for (int e = threadIdx.x; e < 2 * s + 2 * N; e += blockDim.x) sm[e] = work[e];
  for (int e = threadIdx.x; e < s; e += blockDim.x) sr[e] = rows[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double scale = 1.0 / sqrt((double)s);
  const int n = N - 1;
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6) * 64;
  for (int64_t r0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * 64; r0 < m; r0 += stride) {
    const int64_t j = r0 + lane;
    double p = 0, q = 0;
    if (j < m) {
      for (int i = 0; i < s; ++i) {
        const bool neg = __popcll((uint64_t)((int64_t)sr[i] & j)) & 1;
        p += neg ? -yv[i] : yv[i];
        q += neg ? -yw[i] : yw[i];
      }
      const uint32_t bits = word(philox(seed, (uint64_t)(j >> 7), 0, kSigns), (uint32_t)((j >> 5) & 3));
      const double d = ((bits >> (j & 31)) & 1u) ? -scale : scale;
      p *= d;
      q *= d;
    }
    const int nrow = (int)(m - r0 < 64 ? m - r0 : 64);
    for (int rr = 0; rr < nrow; ++rr) {
      const double pj = __shfl(p, rr, 64), qj = __shfl(q, rr, 64);
      const int64_t row = r0 + rr;
      for (int c = lane; c < n; c += 64) dA[row * ldda + c] = (TOut)(pj * ww[c] + qj * vv[c]);
      if (lane == 0) db[row] = (TOut)(pj * ww[n] + qj * vv[n]);
    }
  }
}

hipError_t launch_tls_backward(const SketchPlan& p, int64_t m, const TlsBack& tb, const double* gx, double* work,
                               void* dA, int64_t ldda, void* db, int out_dtype, hipStream_t st) {
  const int N = p.N, s = p.s;
  const JacobiShape js = jacobi_shape(N);
  const size_t alds = (size_t)(js.nb * js.B + N) * sizeof(double);
  tls_adjoint_kernel<<<1, 512, alds, st>>>(s, N, tb, gx, work);
  const size_t lds = (size_t)(2 * s + 2 * N) * sizeof(double) + (size_t)s * 4;
  const unsigned blocks = (unsigned)((m + 4 * 64 - 1) / (4 * 64)) < 4096u ? (unsigned)((m + 255) / 256) : 4096u;
  if (p.kind == NSK_SPARSE_SIGN) {
    if (out_dtype == NSK_F64) {
      if (p.zeta <= 8)
        tls_grad_sparse_kernel<double, 8><<<blocks, 256, lds, st>>>(m, N, s, p.zeta, p.seed, work, (double*)dA, ldda, (double*)db);
      else
        tls_grad_sparse_kernel<double, 32><<<blocks, 256, lds, st>>>(m, N, s, p.zeta, p.seed, work, (double*)dA, ldda, (double*)db);
    } else {
      if (p.zeta <= 8)
        tls_grad_sparse_kernel<float, 8><<<blocks, 256, lds, st>>>(m, N, s, p.zeta, p.seed, work, (float*)dA, ldda, (float*)db);
      else
        tls_grad_sparse_kernel<float, 32><<<blocks, 256, lds, st>>>(m, N, s, p.zeta, p.seed, work, (float*)dA, ldda, (float*)db);
    }
  } else {
    if (out_dtype == NSK_F64)
      tls_grad_srht_kernel<double><<<blocks, 256, lds, st>>>(m, N, s, p.seed, p.rows, work, (double*)dA, ldda, (double*)db);
    else
      tls_grad_srht_kernel<float><<<blocks, 256, lds, st>>>(m, N, s, p.seed, p.rows, work, (float*)dA, ldda, (float*)db);
  }
  return hipGetLastError();
}

}  // namespace nsk
