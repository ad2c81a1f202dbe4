// AAA rational approximation with a reused sketch (Section 6), real sample points: the
// device side of the loop that nsk_aaa drives.
//
// Each step evaluates the barycentric approximant r = n / d at every sample point (the mean of
// f before the first support point), takes the point of largest |f - r| (the lowest index on
// ties; support points are excluded), and, when the loop goes on, writes the new support
// point's Loewner row L(j, c) = (f_j - f_c) / (z_j - z_c) over the current support points (for
// the row downdate of the sketch), marks it, and writes the new Loewner column
// (f_i - f_j) / (z_i - z_j), zero at every support point (for the column update).  All
// reductions use a fixed partition and a fixed tree, so the loop is deterministic.
#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"

namespace nsk {

constexpr int kAaaThreads = 256;

static unsigned aaa_blocks(int64_t m) {
  const int64_t b = (m + kAaaThreads - 1) / kAaaThreads;
  return (unsigned)(b < kAaaParts ? b : kAaaParts);
}

// sum of f and max |f| per block, then over blocks: stats[0] = mean(f), stats[1] = max |f|
__global__ __launch_bounds__(kAaaThreads) void aaa_stats_kernel(const double* __restrict__ f, int64_t m,
                                                                double* __restrict__ part) {
  __shared__ double ss[kAaaThreads], sm[kAaaThreads];
  double sum = 0.0, mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kAaaThreads + threadIdx.x; i < m; i += (int64_t)gridDim.x * kAaaThreads) {
    sum += f[i];
    mx = fmax(mx, fabs(f[i]));
  }
  ss[threadIdx.x] = sum;
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int h = kAaaThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      ss[threadIdx.x] += ss[threadIdx.x + h];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ss[0];
    part[2 * blockIdx.x + 1] = sm[0];
  }
}

__global__ __launch_bounds__(kAaaThreads) void aaa_stats_finish(const double* __restrict__ part, int nparts,
                                                                int64_t m, double* __restrict__ stats) {
  __shared__ double ss[kAaaThreads], sm[kAaaThreads];
  double sum = 0.0, mx = 0.0;
  for (int p = threadIdx.x; p < nparts; p += kAaaThreads) {
    sum += part[2 * p];
    mx = fmax(mx, part[2 * p + 1]);
  }
  ss[threadIdx.x] = sum;
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int h = kAaaThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      ss[threadIdx.x] += ss[threadIdx.x + h];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[0] = ss[0] / (double)m;
    stats[1] = sm[0];
  }
}

// the larger error wins, the lower index on ties
__device__ inline void argmax_merge(double& v, int64_t& i, double v2, int64_t i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

// |f - r| at every non-support point; per block the largest and its index
__global__ __launch_bounds__(kAaaThreads) void aaa_error_kernel(const double* __restrict__ z,
                                                                const double* __restrict__ f,
                                                                const uint8_t* __restrict__ mask, int64_t m,
                                                                const double* __restrict__ sz,
                                                                const double* __restrict__ sf,
                                                                const double* __restrict__ w, int k,
                                                                const double* __restrict__ stats,
                                                                double* __restrict__ pval,
                                                                int64_t* __restrict__ pidx) {
  __shared__ double lz[kAaaMaxSupport], lwf[kAaaMaxSupport], lw[kAaaMaxSupport];
  __shared__ double rv[kAaaThreads];
  __shared__ int64_t ri[kAaaThreads];
  for (int c = threadIdx.x; c < k; c += kAaaThreads) {
    lz[c] = sz[c];
    lw[c] = w[c];
    lwf[c] = w[c] * sf[c];
  }
  __syncthreads();
  const double mean = stats[0];
  double best = -2.0;
  int64_t bi = m;
  for (int64_t i = (int64_t)blockIdx.x * kAaaThreads + threadIdx.x; i < m; i += (int64_t)gridDim.x * kAaaThreads) {
    double e = -1.0;
    if (!mask[i]) {
      double r = mean;
      if (k > 0) {
        const double zi = z[i];
        double num = 0.0, den = 0.0;
        for (int c = 0; c < k; ++c) {
          const double q = 1.0 / (zi - lz[c]);
          num = fma(lwf[c], q, num);
          den = fma(lw[c], q, den);
        }
        r = num / den;
      }
      e = fabs(f[i] - r);
    }
    argmax_merge(best, bi, e, i);
  }
  rv[threadIdx.x] = best;
  ri[threadIdx.x] = bi;
  __syncthreads();
  for (int h = kAaaThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      double v = rv[threadIdx.x];
      int64_t ix = ri[threadIdx.x];
      argmax_merge(v, ix, rv[threadIdx.x + h], ri[threadIdx.x + h]);
      rv[threadIdx.x] = v;
      ri[threadIdx.x] = ix;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pval[blockIdx.x] = rv[0];
    pidx[blockIdx.x] = ri[0];
  }
}

__global__ __launch_bounds__(kAaaThreads) void aaa_pick_kernel(const double* __restrict__ pval,
                                                               const int64_t* __restrict__ pidx, int nparts,
                                                               AaaPick* __restrict__ out) {
  __shared__ double rv[kAaaThreads];
  __shared__ int64_t ri[kAaaThreads];
  double v = -3.0;
  int64_t ix = INT64_MAX;
  for (int p = threadIdx.x; p < nparts; p += kAaaThreads) argmax_merge(v, ix, pval[p], pidx[p]);
  rv[threadIdx.x] = v;
  ri[threadIdx.x] = ix;
  __syncthreads();
  for (int h = kAaaThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      double a = rv[threadIdx.x];
      int64_t b = ri[threadIdx.x];
      argmax_merge(a, b, rv[threadIdx.x + h], ri[threadIdx.x + h]);
      rv[threadIdx.x] = a;
      ri[threadIdx.x] = b;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out->err = rv[0];
    out->idx = ri[0];
  }
}

// support point j joins: its Loewner row over the k current support points, the row-update
// arguments (index j, sign -1), its coordinates appended to the support arrays, its mark
__global__ __launch_bounds__(kAaaThreads) void aaa_join_kernel(const double* __restrict__ z,
                                                               const double* __restrict__ f, int64_t j, int k,
                                                               double* __restrict__ sz, double* __restrict__ sf,
                                                               uint8_t* __restrict__ mask,
                                                               double* __restrict__ row, int64_t* __restrict__ idx,
                                                               int8_t* __restrict__ ops) {
  const double zj = z[j], fj = f[j];
  for (int c = threadIdx.x; c < k; c += kAaaThreads) row[c] = (fj - sf[c]) / (zj - sz[c]);
  if (threadIdx.x == 0) {
    idx[0] = j;
    ops[0] = -1;
    sz[k] = zj;
    sf[k] = fj;
    mask[j] = 1;
  }
}

// the new Loewner column, zero at the support points (j included)
__global__ __launch_bounds__(kAaaThreads) void aaa_column_kernel(const double* __restrict__ z,
                                                                 const double* __restrict__ f,
                                                                 const uint8_t* __restrict__ mask, int64_t m,
                                                                 int64_t j, double* __restrict__ col) {
  const int64_t i = (int64_t)blockIdx.x * kAaaThreads + threadIdx.x;
  if (i >= m) return;
  col[i] = mask[i] ? 0.0 : (f[i] - f[j]) / (z[i] - z[j]);
}

// columns 0..N-1 of a row-major s x ld matrix into a column-major s x N one
__global__ __launch_bounds__(kAaaThreads) void aaa_transpose_kernel(const double* __restrict__ a, int64_t ld,
                                                                    int s, int N, double* __restrict__ cm) {
  const int64_t e = (int64_t)blockIdx.x * kAaaThreads + threadIdx.x;
  if (e >= (int64_t)s * N) return;
  const int c = (int)(e / s), i = (int)(e % s);
  cm[e] = a[(int64_t)i * ld + c];
}

hipError_t launch_aaa_stats(const double* f, int64_t m, double* part, double* stats, hipStream_t st) {
  const unsigned nb = aaa_blocks(m);
  aaa_stats_kernel<<<nb, kAaaThreads, 0, st>>>(f, m, part);
  aaa_stats_finish<<<1, kAaaThreads, 0, st>>>(part, (int)nb, m, stats);
  return hipGetLastError();
}

hipError_t launch_aaa_error(const double* z, const double* f, const uint8_t* mask, int64_t m, const double* sz,
                            const double* sf, const double* w, int k, const double* stats, double* pval,
                            int64_t* pidx, AaaPick* out, hipStream_t st) {
  const unsigned nb = aaa_blocks(m);
  aaa_error_kernel<<<nb, kAaaThreads, 0, st>>>(z, f, mask, m, sz, sf, w, k, stats, pval, pidx);
  aaa_pick_kernel<<<1, kAaaThreads, 0, st>>>(pval, pidx, (int)nb, out);
  return hipGetLastError();
}

hipError_t launch_aaa_join(const double* z, const double* f, int64_t m, int64_t j, int k, double* sz, double* sf,
                           uint8_t* mask, double* row, int64_t* idx, int8_t* ops, double* col, hipStream_t st) {
  aaa_join_kernel<<<1, kAaaThreads, 0, st>>>(z, f, j, k, sz, sf, mask, row, idx, ops);
  aaa_column_kernel<<<(unsigned)((m + kAaaThreads - 1) / kAaaThreads), kAaaThreads, 0, st>>>(z, f, mask, m, j, col);
  return hipGetLastError();
}

hipError_t launch_aaa_transpose(const double* a, int64_t ld, int s, int N, double* cm, hipStream_t st) {
  aaa_transpose_kernel<<<(unsigned)(((int64_t)s * N + kAaaThreads - 1) / kAaaThreads), kAaaThreads, 0, st>>>(
      a, ld, s, N, cm);
  return hipGetLastError();
}

}  // namespace nsk
