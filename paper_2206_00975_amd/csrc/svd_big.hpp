// SVD of SA for the sizes past the register-blocked fast path (N > 320 or s > 4096):
// one-sided Jacobi on SA itself (its columns, s long, are rotated in HBM) across the whole GPU.
//
// Block round-robin: the columns form blocks of kBigW; in each round of the circle ordering of
// the blocks, a workgroup of kBigW waves takes one pair of blocks and runs a full one-sided
// Jacobi sweep over their 2 kBigW columns (the circle ordering again, one column pair per wave,
// workgroup barriers between its rounds), so the block pair's columns stay in the XCD's L2
// while it works on them and the whole matrix crosses HBM once per block round instead of once
// per column round.  Block rounds end in a grid barrier (one cache write-back per workgroup),
// which publishes the rotated columns to the next round's readers on other CUs.  A pair (p, q) rotates when
// |x_p . x_q| > N u |x_p| |x_q| (rule and formulas as in the register-blocked Jacobi), V (N x N,
// from the identity) is rotated alongside, and a sweep with no rotation -- every column pair
// within tolerance -- ends the loop for every workgroup at once (the count is read after the
// barrier).  No QR first: Jacobi on SA sees the same column inner products as Jacobi on its R
// factor.  The finish (one workgroup) takes the column norms as singular values, ranks them and
// writes the trailing k columns of V, sign-normalised.
#pragma once

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "svd_device.hpp"

namespace nsk {

constexpr int kBigW = 4;                // columns per block (256 threads: room for both pairs)
constexpr int kBigThreads = 64 * kBigW;  // one wave per column pair of a block pair's round

// counters: [0, max_sweeps) rotations per sweep, [max_sweeps, 2 max_sweeps) largest relative
// cosine bits per sweep, then sweeps performed and the converged flag; then, 64-byte aligned,
// the grid barrier's words
__host__ __device__ inline size_t svd_big_bar_offset(int max_sweeps) {
  return ((size_t)(2 * max_sweeps + 2) * 8 + 63) & ~(size_t)63;
}
__host__ __device__ inline size_t svd_big_counter_bytes(int max_sweeps) {
  return svd_big_bar_offset(max_sweeps) + (size_t)kAgentBarWords * 4;
}

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

// One column pair (p < q) by one wave: the sums, and the rotation of SA's columns and V's when
// they are not orthogonal to tolerance.  The sums are wave-uniform after the reduction, so the
// whole wave takes one branch.  SCH > 0: the pair stays in registers (s <= 64 SCH) from the sums
// to the rotation, and V's pair (N <= 1024) is loaded with it, so a round costs one load latency.
// off: the wave's largest relative cosine so far.  Returns 1 if it rotated.
template <int SCH>
__device__ inline int big_pair_step(double* __restrict__ sa, int s, int N, double* __restrict__ V, int p, int q,
                                    int lane, double tol, double& off) {
  double* xp = sa + (size_t)p * s;
  double* xq = sa + (size_t)q * s;
  double* vp = V + (size_t)p * N;
  double* vq = V + (size_t)q * N;
  double a, b, g;
  double x[SCH > 0 ? SCH : 1], y[SCH > 0 ? SCH : 1];
  constexpr int VCH = SCH > 0 ? 16 : 1;  // N <= 1024
  double vx[VCH], vy[VCH];
  if constexpr (SCH > 0) {
#pragma unroll
    for (int u = 0; u < SCH; ++u) {
      const int e = lane + 64 * u;
      x[u] = e < s ? xp[e] : 0.0;
      y[u] = e < s ? xq[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < VCH; ++u) {
      const int e = lane + 64 * u;
      vx[u] = e < N ? vp[e] : 0.0;
      vy[u] = e < N ? vq[e] : 0.0;
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
  if (nab > 0) off = fmax(off, fabs(g) / nab);
  if (!(fabs(g) > tol * nab)) return 0;
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
#pragma unroll
    for (int u = 0; u < VCH; ++u) {
      const int e = lane + 64 * u;
      if (e < N) {
        vp[e] = c * vx[u] - sn * vy[u];
        vq[e] = sn * vx[u] + c * vy[u];
      }
    }
  } else {
    big_pair<0>(xp, xq, s, lane, false, a, b, g, true, c, sn);
    double da, db, dg;
    big_pair<16>(vp, vq, N, lane, false, da, db, dg, true, c, sn);  // N <= 1024
  }
  return 1;
}

// SCH: register chunks of 64 for a column of SA (s <= 64 SCH; 0 = any s, streamed)
template <int SCH>
__global__ __launch_bounds__(kBigThreads) void svd_big_jacobi_kernel(double* __restrict__ sa, int s, int N,
                                                                     double* __restrict__ V, int max_sweeps,
                                                                     unsigned long long* __restrict__ counters) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t gt = (int64_t)blockIdx.x * kBigThreads + threadIdx.x, GT = (int64_t)gridDim.x * kBigThreads;
  for (int64_t e = gt; e < (int64_t)N * N; e += GT) V[e] = (e / N == e % N) ? 1.0 : 0.0;
  for (int64_t i = gt; i < (int64_t)(svd_big_counter_bytes(max_sweeps) / 8); i += GT) counters[i] = 0;
  unsigned* bar = reinterpret_cast<unsigned*>(reinterpret_cast<unsigned char*>(counters) + svd_big_bar_offset(max_sweeps));
  unsigned epoch = 0;
  grid.sync();
  const int nb = (N + kBigW - 1) / kBigW;
  const int nb_even = nb + (nb & 1);
  const int P = nb_even / 2;  // block pairs per block round
  const double tol = (double)N * 0x1p-53;
  int sweeps = 0, conv = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    int nrot = 0;
    double off = 0.0;  // one atomic per wave and sweep: the counters are not contended per pair
    for (int r = 0; r < nb_even - 1; ++r) {
      for (int bp = blockIdx.x; bp < P; bp += gridDim.x) {  // uniform over the workgroup
        const int bI = circle_col(bp, r, nb_even), bJ = circle_col(nb_even - 1 - bp, r, nb_even);
        for (int ir = 0; ir < 2 * kBigW - 1; ++ir) {
          // positions 0..kBigW-1 are block bI's columns, kBigW..2 kBigW-1 block bJ's
          const int pa = circle_col(wave, ir, 2 * kBigW), pb = circle_col(2 * kBigW - 1 - wave, ir, 2 * kBigW);
          int p = pa < kBigW ? bI * kBigW + pa : bJ * kBigW + pa - kBigW;
          int q = pb < kBigW ? bI * kBigW + pb : bJ * kBigW + pb - kBigW;
          if (p > q) { const int tmp = p; p = q; q = tmp; }
          if (q < N) nrot += big_pair_step<SCH>(sa, s, N, V, p, q, lane, tol, off);
          __syncthreads();  // the next inner round's pairs read this one's columns
        }
      }
      agent_barrier(bar, gridDim.x, epoch);
    }
    if (lane == 0 && nrot) atomicAdd(&counters[sw], (unsigned long long)nrot);
    if (lane == 0 && off > 0) atomicMax(&counters[max_sweeps + sw], (unsigned long long)__double_as_longlong(off));
    agent_barrier(bar, gridDim.x, epoch);
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
  extern __shared__ __align__(16) unsigned char smem[];
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
