// SVD of SA for the sizes past the register-blocked fast path (N > 320 or s > 4096):
// one-sided Jacobi on SA itself (its columns, s long, are rotated in HBM) across the whole GPU.
//
// A cooperative grid of workgroups of four waves takes the N/2 disjoint column pairs of each
// round of the cyclic round-robin (circle) ordering, one pair per wave, and every round ends in
// a grid barrier, whose device-scope fences publish the rotated columns to the next round's
// readers on other CUs.  A pair (p, q) rotates when |x_p . x_q| > N u |x_p| |x_q| (the
// single-workgroup path's rule and rotation formulas), V (N x N, from the identity) is rotated
// alongside, and a sweep with no rotation ends the loop for every workgroup at once (the
// rotation count is read after the barrier).  No QR first: Jacobi on SA sees the same column
// inner products as Jacobi on its R factor.  The finish (one workgroup) takes the column norms
// as singular values, ranks them and writes the trailing k columns of V, sign-normalised.
#pragma once

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "svd_device.hpp"

namespace nsk {

constexpr int kBigThreads = 256;  // four waves, one column pair each per round

// counters: [0, max_sweeps) rotations per sweep, [max_sweeps, 2 max_sweeps) largest relative
// cosine bits per sweep, then sweeps performed and the converged flag
__host__ __device__ inline size_t svd_big_counter_bytes(int max_sweeps) { return (size_t)(2 * max_sweeps + 2) * 8; }

// x <- c x - sn y, y <- sn x + c y over n entries of two columns, lane-strided; CH > 0: the
// pair is held in registers (n <= 64 CH), all loads issued before the first use
template <int CH>
__device__ inline void big_pair(double* __restrict__ xp, double* __restrict__ xq, int n, int lane, bool dots,
                                double& a, double& b, double& g, bool rotate, double c, double sn) {
  if constexpr (CH > 0) {
    double x[CH], y[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int e = lane + 64 * u;
      x[u] = e < n ? xp[e] : 0.0;
      y[u] = e < n ? xq[e] : 0.0;
    }
    if (dots) {
      a = b = g = 0.0;
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        a = fma(x[u], x[u], a);
        b = fma(y[u], y[u], b);
        g = fma(x[u], y[u], g);
      }
    }
    if (rotate) {
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int e = lane + 64 * u;
        if (e < n) {
          xp[e] = c * x[u] - sn * y[u];
          xq[e] = sn * x[u] + c * y[u];
        }
      }
    }
  } else {
    if (dots) {
      a = b = g = 0.0;
      for (int e0 = lane; e0 < n; e0 += 64 * 8) {
        double x[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + 64 * u;
          x[u] = e < n ? xp[e] : 0.0;
          y[u] = e < n ? xq[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          a = fma(x[u], x[u], a);
          b = fma(y[u], y[u], b);
          g = fma(x[u], y[u], g);
        }
      }
    }
    if (rotate) {
      for (int e0 = lane; e0 < n; e0 += 64 * 8) {
        double x[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + 64 * u;
          x[u] = e < n ? xp[e] : 0.0;
          y[u] = e < n ? xq[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + 64 * u;
          if (e < n) {
            xp[e] = c * x[u] - sn * y[u];
            xq[e] = sn * x[u] + c * y[u];
          }
        }
      }
    }
  }
}

// SCH: register chunks of 64 for a column of SA (s <= 64 SCH; 0 = any s, streamed)
template <int SCH>
__global__ __launch_bounds__(kBigThreads) void svd_big_jacobi_kernel(double* __restrict__ sa, int s, int N,
                                                                     double* __restrict__ V, int max_sweeps,
                                                                     unsigned long long* __restrict__ counters) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (kBigThreads / 64) + (threadIdx.x >> 6);
  const int W = gridDim.x * (kBigThreads / 64);
  const int64_t gt = (int64_t)blockIdx.x * kBigThreads + threadIdx.x, GT = (int64_t)gridDim.x * kBigThreads;
  for (int64_t e = gt; e < (int64_t)N * N; e += GT) V[e] = (e / N == e % N) ? 1.0 : 0.0;
  for (int64_t i = gt; i < 2 * max_sweeps + 2; i += GT) counters[i] = 0;
  grid.sync();
  const int n_even = N + (N & 1);
  const int P = n_even / 2;
  const double tol = (double)N * 0x1p-53;
  int sweeps = 0, conv = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    int nrot = 0;
    for (int r = 0; r < n_even - 1; ++r) {
      for (int i = gw; i < P; i += W) {
        int p = circle_col(i, r, n_even), q = circle_col(n_even - 1 - i, r, n_even);
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        if (q >= N) continue;
        double* xp = sa + (size_t)p * s;
        double* xq = sa + (size_t)q * s;
        // the sums are wave-uniform after the reduction, so the whole wave takes one branch;
        // with SCH > 0 the pair stays in registers from the sums to the rotation
        double a, b, g;
        double x[SCH > 0 ? SCH : 1], y[SCH > 0 ? SCH : 1];
        if constexpr (SCH > 0) {
#pragma unroll
          for (int u = 0; u < SCH; ++u) {
            const int e = lane + 64 * u;
            x[u] = e < s ? xp[e] : 0.0;
            y[u] = e < s ? xq[e] : 0.0;
          }
          a = b = g = 0.0;
#pragma unroll
          for (int u = 0; u < SCH; ++u) {
            a = fma(x[u], x[u], a);
            b = fma(y[u], y[u], b);
            g = fma(x[u], y[u], g);
          }
        } else {
          big_pair<0>(xp, xq, s, lane, true, a, b, g, false, 0.0, 0.0);
        }
        a = wave_sum(a);
        b = wave_sum(b);
        g = wave_sum(g);
        const double nab = sqrt(a * b);
        if (nab > 0 && lane == 0)
          atomicMax(&counters[max_sweeps + sw], (unsigned long long)__double_as_longlong(fabs(g) / nab));
        if (!(fabs(g) > tol * nab)) continue;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double sn = c * t;
        if constexpr (SCH > 0) {
#pragma unroll
          for (int u = 0; u < SCH; ++u) {
            const int e = lane + 64 * u;
            if (e < s) {
              xp[e] = c * x[u] - sn * y[u];
              xq[e] = sn * x[u] + c * y[u];
            }
          }
        } else {
          big_pair<0>(xp, xq, s, lane, false, a, b, g, true, c, sn);
        }
        double da, db, dg;
        big_pair<16>(V + (size_t)p * N, V + (size_t)q * N, N, lane, false, da, db, dg, true, c, sn);  // N <= 1024
        ++nrot;
      }
      grid.sync();
    }
    if (lane == 0 && nrot) atomicAdd(&counters[sw], (unsigned long long)nrot);
    grid.sync();
    sweeps = sw + 1;
    if (__hip_atomic_load(&counters[sw], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      conv = 1;
      break;
    }
  }
  if (gt == 0) {
    counters[2 * max_sweeps] = (unsigned long long)sweeps;
    counters[2 * max_sweeps + 1] = (unsigned long long)conv;
  }
}

// One workgroup: singular values (column norms of the rotated SA), their non-increasing order
// (index ascending on ties, NaN last), and the trailing k columns of V, sign-normalised.
// smem: N doubles + N ints.
__global__ __launch_bounds__(1024) void svd_big_finish_kernel(const double* __restrict__ sa, int s, int N, int k,
                                                              const double* __restrict__ V, int max_sweeps,
                                                              const unsigned long long* __restrict__ counters,
                                                              double* __restrict__ sigma, int* __restrict__ order,
                                                              double* __restrict__ Vk, double* __restrict__ sigma_k,
                                                              nsk_info* info) {
  extern __shared__ unsigned char smem[];
  double* nrm = reinterpret_cast<double*>(smem);
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  for (int c = wave; c < N; c += nw) {
    double a = 0;
    for (int e = lane; e < s; e += 64) a = fma(sa[(size_t)c * s + e], sa[(size_t)c * s + e], a);
    a = wave_sum(a);
    if (lane == 0) nrm[c] = sqrt(a);
  }
  __syncthreads();
  for (int c = tid; c < N; c += nt) {
    const double xv = nrm[c];
    const double x = xv != xv ? -1.0 : xv;
    int r = 0;
    for (int d = 0; d < N; ++d) {
      const double yv = nrm[d];
      const double y = yv != yv ? -1.0 : yv;
      r += (y > x) || (y == x && d < c);
    }
    order[r] = c;
    sigma[r] = xv;
  }
  __syncthreads();
  for (int q = wave; q < k; q += nw) {
    const int c = order[N - k + q];
    const double* v = V + (size_t)c * N;
    double best = -1;
    int bi = 0;
    for (int e = lane; e < N; e += 64) {
      const double a = fabs(v[e]);
      if (a > best) { best = a; bi = e; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const double sgn = v[bi] < 0 ? -1.0 : 1.0;
    if (Vk)
      for (int e = lane; e < N; e += 64) Vk[(size_t)e * k + q] = sgn * v[e];
    if (sigma_k && lane == 0) sigma_k[q] = sigma[N - k + q];
  }
  if (info && tid == 0) {
    const int sweeps = (int)counters[2 * max_sweeps];
    info->sweeps = sweeps;
    info->converged = (int)counters[2 * max_sweeps + 1];
    info->off = sweeps > 0 ? __longlong_as_double((long long)counters[max_sweeps + sweeps - 1]) : 0.0;
    info->sigma_max = sigma[0];
  }
}

}  // namespace nsk
