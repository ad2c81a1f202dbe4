// Stages after the SVD: the residual |A V_k|_F with FP64 accumulation (Problem 2.1), the
// TLS solution x = -v(1:n)/v(N) (Section 4), and the backward pass of a loss L(x) through the
// sketched TLS solution (S^T applied by regenerating S from its seed).
#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "svd_device.hpp"
#include "svd_pipeline.hpp"

namespace nsk {

// ============================================================================ residual
// |A V_k|_F^2 = sum over rows r and vectors q of (a_r . v_q)^2.  A wave takes RT rows at a
// time: lane l loads columns l + 64 i of all RT rows (every load of the tile in flight at
// once, each row read as contiguous 256-byte segments), accumulates the RT partial dots
// per vector in FP64, and one transposed reduction leaves row (l >> (6 - log2 RT))'s dot in
// lane l.  Per-workgroup partial sums are combined in a fixed order by residual_finish, so
// the result is bitwise reproducible.
constexpr int kResThreads = 256;

// Column group i of this lane for the pass starting at column cb: pointers resolved once;
// invalid columns read column 0 and are masked after the load.
template <typename T, int CI>
__device__ inline void residual_columns(const Operand& op, int N, int cb, int lane, const T* (&base)[CI],
                                        int64_t (&ld)[CI], bool (&live)[CI]) {
#pragma unroll
  for (int i = 0; i < CI; ++i) {
    const int c = cb + lane + 64 * i;
    live[i] = c < N;
    column_ref<T>(op, live[i] ? c : 0, base[i], ld[i]);
  }
}

// Adds this lane's contribution of columns cb + lane + 64 i to the RT row dots d[q][r].
// Every load of the tile is issued before the first use (rows past the end re-read row r0).
template <typename T, int KQ, int RT, int CI>
__device__ inline void residual_tile(const T* (&base)[CI], const int64_t (&ld)[CI], const bool (&live)[CI],
                                     const double* vsh, int cb, int k, int q0, int64_t r0, int nrow, int lane,
                                     double (&d)[KQ][16]) {
  T a[CI][RT];
#pragma unroll
  for (int i = 0; i < CI; ++i)
#pragma unroll
    for (int r = 0; r < RT; ++r) a[i][r] = base[i][(r0 + (r < nrow ? r : 0)) * ld[i]];
#pragma unroll
  for (int i = 0; i < CI; ++i) {
    double v[KQ];
    const int c = cb + lane + 64 * i;
#pragma unroll
    for (int q = 0; q < KQ; ++q) v[q] = live[i] && q0 + q < k ? vsh[c * k + q0 + q] : 0.0;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const double x = r < nrow ? (double)a[i][r] : 0.0;
#pragma unroll
      for (int q = 0; q < KQ; ++q) d[q][r] += x * v[q];
    }
  }
}

template <typename T, int KQ, int RT, int CI>
__global__ __launch_bounds__(kResThreads) void residual_kernel(Operand op, int64_t m, int N,
                                                               const double* __restrict__ Vk, int k,
                                                               double* __restrict__ partial) {
  extern __shared__ __align__(16) double vsh[];  // N x k row-major
  __shared__ double wsum[kResThreads / 64];
  for (int e = threadIdx.x; e < N * k; e += blockDim.x) vsh[e] = Vk[e];
  __syncthreads();
  constexpr int SH = 6 - ceil_log2(RT);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int my_row = lane >> SH;
  const bool lead = (lane & ((1 << SH) - 1)) == 0;
  const bool one_pass = N <= 64 * CI;
  const T* base[CI];
  int64_t ld[CI];
  bool live[CI];
  residual_columns<T, CI>(op, N, 0, lane, base, ld, live);
  double local = 0;
  for (int64_t r0 = ((int64_t)blockIdx.x * wpb + wave) * RT; r0 < m; r0 += (int64_t)gridDim.x * wpb * RT) {
    const int nrow = m - r0 < RT ? (int)(m - r0) : RT;
    for (int q0 = 0; q0 < k; q0 += KQ) {
      double d[KQ][16];
#pragma unroll
      for (int q = 0; q < KQ; ++q)
#pragma unroll
        for (int r = 0; r < RT; ++r) d[q][r] = 0;
      if (one_pass) {
        residual_tile<T, KQ, RT, CI>(base, ld, live, vsh, 0, k, q0, r0, nrow, lane, d);
      } else {
        for (int cb = 0; cb < N; cb += 64 * CI) {
          const T* pb[CI];
          int64_t pl[CI];
          bool pv[CI];
          residual_columns<T, CI>(op, N, cb, lane, pb, pl, pv);
          residual_tile<T, KQ, RT, CI>(pb, pl, pv, vsh, cb, k, q0, r0, nrow, lane, d);
        }
      }
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        const double t = reduce_t<RT>(d[q], lane);
        if (lead && my_row < nrow && q0 + q < k) local += t * t;
      }
    }
  }
  local = wave_sum64(local);
  if (lane == 0) wsum[wave] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < wpb; ++w) t += wsum[w];
    partial[blockIdx.x] = t;
  }
}

// FP32 rows stored contiguously (one row-major block, or adjacent blocks of one buffer), k = 1,
// 4 <= N <= 256: lane l reads columns 4l .. 4l + 3 of a row with one 16-byte load (4-byte
// alignment suffices for it), so a row is one wave load instead of one per 64 columns.  The
// lane holding column N - 1 reads the window N - 4 .. N - 1 with zero weight on the columns
// below its own (no load passes the row's end); lanes past N read that window with zero
// weights.  Row sums as in residual_kernel.
template <int RT>
__global__ __launch_bounds__(kResThreads) void residual_rows_kernel(const float* __restrict__ A, int64_t ld,
                                                                    int64_t m, int N, const double* __restrict__ v,
                                                                    double* __restrict__ partial) {
  __shared__ double wsum[kResThreads / 64];
  constexpr int SH = 6 - ceil_log2(RT);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int my_row = lane >> SH;
  const bool lead = (lane & ((1 << SH) - 1)) == 0;
  const int c0 = 4 * lane;
  const int cs = c0 + 4 <= N ? c0 : N - 4;  // window start
  double w[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) w[j] = (cs + j >= c0 && cs + j < N) ? v[cs + j] : 0.0;
  double local = 0;
  for (int64_t r0 = ((int64_t)blockIdx.x * wpb + wave) * RT; r0 < m; r0 += (int64_t)gridDim.x * wpb * RT) {
    const int nrow = m - r0 < RT ? (int)(m - r0) : RT;
    float4 a[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) __builtin_memcpy(&a[r], A + (r0 + (r < nrow ? r : 0)) * ld + cs, sizeof(float4));
    double d[16];
#pragma unroll
    for (int r = 0; r < RT; ++r)
      d[r] = (double)a[r].x * w[0] + (double)a[r].y * w[1] + (double)a[r].z * w[2] + (double)a[r].w * w[3];
    const double t = reduce_t<RT>(d, lane);
    if (lead && my_row < nrow) local += t * t;
  }
  local = wave_sum64(local);
  if (lane == 0) wsum[wave] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int q = 0; q < wpb; ++q) t += wsum[q];
    partial[blockIdx.x] = t;
  }
}

// The blocks of op are one row-major FP32 buffer: each starts where the previous one's columns
// end, with the same row stride.
static bool contiguous_rows(const Operand& op) {
  if (op.dtype != NSK_F32) return false;
  const float* p0 = static_cast<const float*>(op.ptr[0]);
  for (int b = 1; b < op.nb; ++b)
    if (op.ld[b] != op.ld[0] || static_cast<const float*>(op.ptr[b]) != p0 + op.col0[b]) return false;
  return true;
}

// Fixed-order sum of the partials: lane l adds parts l, l + 64, ...; then a fixed butterfly.
__global__ void residual_finish(const double* __restrict__ partial, int parts, double* out, nsk_info* info) {
  double t = 0;
  for (int i = threadIdx.x; i < parts; i += 64) t += partial[i];
  t = wave_sum64(t);
  if (threadIdx.x != 0) return;
  const double r = sqrt(t);
  if (out) *out = r;
  if (info) info->residual = r;
}

hipError_t launch_residual(const Operand& op, int64_t m, const double* Vk, int k, double* partial, int parts,
                           double* out, nsk_info* info, hipStream_t st) {
  const int N = op.col0[op.nb];
  const size_t lds = (size_t)N * k * sizeof(double);
#define NSK_RES(T, KQ, RT, CI) \
  residual_kernel<T, KQ, RT, CI><<<parts, kResThreads, lds, st>>>(op, m, N, Vk, k, partial)
  const bool wide = N > 128;
  if (k == 1 && N >= 4 && N <= 256 && contiguous_rows(op)) {
    residual_rows_kernel<16><<<parts, kResThreads, 0, st>>>(static_cast<const float*>(op.ptr[0]), op.ld[0], m, N, Vk,
                                                            partial);
  } else if (op.dtype == NSK_F64) {
    if (k == 1) { if (wide) NSK_RES(double, 1, 8, 4); else NSK_RES(double, 1, 16, 2); }
    else if (k == 2) { if (wide) NSK_RES(double, 2, 8, 4); else NSK_RES(double, 2, 16, 2); }
    else { if (wide) NSK_RES(double, 4, 4, 4); else NSK_RES(double, 4, 8, 2); }
  } else {
    if (k == 1) { if (wide) NSK_RES(float, 1, 16, 4); else NSK_RES(float, 1, 16, 2); }
    else if (k == 2) { if (wide) NSK_RES(float, 2, 16, 4); else NSK_RES(float, 2, 16, 2); }
    else { if (wide) NSK_RES(float, 4, 8, 4); else NSK_RES(float, 4, 8, 2); }
  }
#undef NSK_RES
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

// ============================================================ multi-RHS TLS extraction
// Section 4 with k right-hand sides: X = -V12 V22^{-1} from the trailing k right singular
// vectors Vk (N x k row-major, N = n + k) of [A | B], V12 = Vk(0:n, :), V22 = Vk(n:N, :).
// Row i of X solves x V22 = -V12(i, :), i.e. V22^T x^T = -V12(i, :)^T: one workgroup factors
// M = V22^T = P^T L U with partial pivoting in LDS (k <= kTlsMaxRhs), then each thread solves
// its rows.  A singular V22 (no TLS solution, Section 4) gives non-finite entries.
constexpr int kTlsMaxRhs = 64;

__global__ __launch_bounds__(256) void tls_extract_multi_kernel(const double* __restrict__ Vk, int n, int k,
                                                                double* __restrict__ X) {
  __shared__ double M[kTlsMaxRhs * kTlsMaxRhs];  // row-major k x k: M[r][c] = V22[c][r]
  __shared__ int piv[kTlsMaxRhs];
  for (int e = threadIdx.x; e < k * k; e += 256) {
    const int r = e / k, c = e % k;
    M[r * k + c] = Vk[(size_t)(n + c) * k + r];
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {  // elimination step j, pivot chosen by one thread
    if (threadIdx.x == 0) {
      int pr = j;
      double best = fabs(M[j * k + j]);
      for (int r = j + 1; r < k; ++r)
        if (fabs(M[r * k + j]) > best) { best = fabs(M[r * k + j]); pr = r; }
      piv[j] = pr;
      if (pr != j)
        for (int c = 0; c < k; ++c) { const double t = M[j * k + c]; M[j * k + c] = M[pr * k + c]; M[pr * k + c] = t; }
    }
    __syncthreads();
    for (int r = j + 1 + (int)threadIdx.x; r < k; r += 256) {
      const double l = M[r * k + j] / M[j * k + j];
      M[r * k + j] = l;
      for (int c = j + 1; c < k; ++c) M[r * k + c] -= l * M[j * k + c];
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += 256) {
    double y[kTlsMaxRhs];
    for (int c = 0; c < k; ++c) y[c] = -Vk[(size_t)i * k + c];
    for (int j = 0; j < k; ++j) {  // the row swaps, then L (unit diagonal), then U
      const int pr = piv[j];
      if (pr != j) { const double t = y[j]; y[j] = y[pr]; y[pr] = t; }
    }
    for (int r = 1; r < k; ++r)
      for (int c = 0; c < r; ++c) y[r] -= M[r * k + c] * y[c];
    for (int r = k - 1; r >= 0; --r) {
      for (int c = r + 1; c < k; ++c) y[r] -= M[r * k + c] * y[c];
      y[r] /= M[r * k + r];
    }
    for (int c = 0; c < k; ++c) X[(size_t)i * k + c] = y[c];
  }
}

hipError_t launch_tls_extract_multi(const double* Vk, int n, int k, double* X, hipStream_t st) {
  tls_extract_multi_kernel<<<1, 256, 0, st>>>(Vk, n, k, X);
  return hipGetLastError();
}

// ================================================================ epsilon null space
// Section 2's epsilon version of Algorithm 1: the number of singular values (non-increasing,
// sigma[0] the largest) below eps, or below eps * sigma[0] when `relative`.
__global__ __launch_bounds__(256) void count_below_kernel(const double* __restrict__ sigma, int N, double eps,
                                                          int relative, int32_t* __restrict__ count) {
  __shared__ int part[4];
  const double thr = relative ? eps * sigma[0] : eps;
  int c = 0;
  for (int b = 0; b < N; b += 256) {  // uniform trip count: every lane takes part in the ballot
    const int i = b + (int)threadIdx.x;
    c += __popcll(__ballot(i < N && sigma[i] < thr));
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) *count = part[0] + part[1] + part[2] + part[3];
}

hipError_t launch_count_below(const double* sigma, int N, double eps, int relative, int32_t* count,
                              hipStream_t st) {
  count_below_kernel<<<1, 256, 0, st>>>(sigma, N, eps, relative, count);
  return hipGetLastError();
}

// ======================================================================== TLS backward
// g_bar = dL/dv = -(1/v_N) [g; g.x];  w = V D V^T g_bar with D_c = 1 / (sigma_N^2 - sigma_c^2)
// for every column c except the trailing one (D = 0 there): the first-order change of the
// trailing right singular vector of SA.  V^T g_bar and V z are applied by replaying the
// Jacobi rotation log forward (transposed) and backward.  work = [SA v (s), SA w (s), v, w].
__global__ __launch_bounds__(512) void tls_adjoint_kernel(int s, int N, TlsBack tb, const double* __restrict__ gx,
                                                           double* __restrict__ work) {
  extern __shared__ __align__(16) double sm[];
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
  const int vw = replay_waves(js);
  replay_any(xb, tb.log, js, sweeps, true, tid, wave < vw);
  __syncthreads();
  const int cN = tb.order[N - 1];
  const double lamN = tb.colnorm[cN] * tb.colnorm[cN];
  for (int c = tid; c < ncols; c += blockDim.x) {
    const double sc = tb.colnorm[c < N ? c : 0];
    xb[c] = (c < N && c != cN) ? xb[c] / (lamN - sc * sc) : 0.0;
  }
  __syncthreads();
  replay_any(xb, tb.log, js, sweeps, false, tid, wave < vw);
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

// Rows r0 .. r0 + 63 of dM = p w^T + q v^T (lane l holds p, q of row r0 + l): the row's
// scalars are broadcast with readlane, the lane's entries of w and v stay in registers for
// a pass over 256 columns, and every row is written as contiguous 256-byte (FP32) segments.
template <typename TOut>
__device__ inline void grad_write_rows(double p, double q, int64_t r0, int64_t m, int n, const double* ww,
                                       const double* vv, TOut* __restrict__ dA, int64_t ldda, TOut* __restrict__ db,
                                       int lane) {
  const int nrow = (int)(m - r0 < 64 ? m - r0 : 64);
  for (int cb = 0; cb < n; cb += 256) {
    double wr[4], vr[4];
    bool live[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = cb + lane + 64 * i;
      live[i] = c < n;
      wr[i] = live[i] ? ww[c] : 0.0;
      vr[i] = live[i] ? vv[c] : 0.0;
    }
    for (int rr = 0; rr < nrow; ++rr) {
      const double pj = bcast_d(p, rr), qj = bcast_d(q, rr);
      TOut* rowp = uniform_ptr(dA + (r0 + rr) * ldda + cb);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (live[i]) rowp[lane + 64 * i] = (TOut)(pj * wr[i] + qj * vr[i]);
    }
  }
  if (lane < nrow) db[r0 + lane] = (TOut)(p * ww[n] + q * vv[n]);
}

template <typename TOut, int ZMAX>
__global__ __launch_bounds__(256) void tls_grad_sparse_kernel(int64_t m, int N, int s, int zeta, uint64_t seed,
                                                              const double* __restrict__ work, TOut* __restrict__ dA,
                                                              int64_t ldda, TOut* __restrict__ db) {
  extern __shared__ __align__(16) double sm[];
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
    grad_write_rows<TOut>(p, q, r0, m, n, ww, vv, dA, ldda, db, lane);
  }
}

template <typename TOut>
__global__ __launch_bounds__(256) void tls_grad_srht_kernel(int64_t m, int N, int s, uint64_t seed,
                                                            const int* __restrict__ rows,
                                                            const double* __restrict__ work, TOut* __restrict__ dA,
                                                            int64_t ldda, TOut* __restrict__ db) {
  extern __shared__ __align__(16) double sm[];
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
    grad_write_rows<TOut>(p, q, r0, m, n, ww, vv, dA, ldda, db, lane);
  }
}

// Dynamic LDS above the 64 KB default must be requested per kernel (160 KB per CU).
static hipError_t lds_limit(const void* fn, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_tls_backward(const SketchPlan& p, int64_t m, const TlsBack& tb, const double* gx, double* work,
                               void* dA, int64_t ldda, void* db, int out_dtype, hipStream_t st) {
  const int N = p.N, s = p.s;
  const JacobiShape js = jacobi_shape(N);
  const size_t alds = (size_t)((js.nb * js.B + N + 1) & ~1) * sizeof(double);
  if (hipError_t e = lds_limit((const void*)tls_adjoint_kernel, alds)) return e;
  tls_adjoint_kernel<<<1, 512, alds, st>>>(s, N, tb, gx, work);
  const size_t lds = (size_t)(2 * s + 2 * N) * sizeof(double) + (size_t)s * 4;
  const unsigned blocks = (unsigned)((m + 4 * 64 - 1) / (4 * 64)) < 4096u ? (unsigned)((m + 255) / 256) : 4096u;
#define NSK_GRAD(KERNEL, ...)                                                 \
  {                                                                           \
    if (hipError_t e = lds_limit((const void*)KERNEL, lds)) return e;         \
    KERNEL<<<blocks, 256, lds, st>>>(__VA_ARGS__);                            \
  }
  if (p.kind == NSK_SPARSE_SIGN) {
    if (out_dtype == NSK_F64) {
      if (p.zeta <= 8)
        NSK_GRAD((tls_grad_sparse_kernel<double, 8>), m, N, s, p.zeta, p.seed, work, (double*)dA, ldda, (double*)db)
      else
        NSK_GRAD((tls_grad_sparse_kernel<double, 32>), m, N, s, p.zeta, p.seed, work, (double*)dA, ldda, (double*)db)
    } else {
      if (p.zeta <= 8)
        NSK_GRAD((tls_grad_sparse_kernel<float, 8>), m, N, s, p.zeta, p.seed, work, (float*)dA, ldda, (float*)db)
      else
        NSK_GRAD((tls_grad_sparse_kernel<float, 32>), m, N, s, p.zeta, p.seed, work, (float*)dA, ldda, (float*)db)
    }
  } else {
    if (out_dtype == NSK_F64)
      NSK_GRAD(tls_grad_srht_kernel<double>, m, N, s, p.seed, p.rows, work, (double*)dA, ldda, (double*)db)
    else
      NSK_GRAD(tls_grad_srht_kernel<float>, m, N, s, p.seed, p.rows, work, (float*)dA, ldda, (float*)db)
  }
#undef NSK_GRAD
  return hipGetLastError();
}

}  // namespace nsk
