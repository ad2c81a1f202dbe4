// Householder QR of the sketch SA spread over workgroups (cooperative launch).
//
// The columns are dealt out in panels of NB: panel p belongs to workgroup p mod G, which
// keeps every column of its panels up to date.  For panel p its owner factorises the panel
// exactly as the single-workgroup QR does (wave w holds panel column w in registers; the
// reflector of column jj is formed by its wave and applied by the later ones), stores each
// Householder vector below the diagonal of its column of SA (the unit leading entry is
// implicit) and tau in a scratch array, and writes the panel's entries of R.  After a grid
// barrier every workgroup copies the panel's vectors into LDS and applies the NB reflectors,
// in order, to its own columns to the right of the panel, CPW columns per wave; the rows of
// the panel become final entries of R.  One grid barrier per panel; the owner of panel p + 1
// factorises it as soon as its own columns have received panel p.
#pragma once

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "qr_panel.hpp"
#include "wave_ops.hpp"

namespace nsk {

// A (s x N column-major, ld s) is overwritten; R (ldr rows, zeroed here) receives the N x N
// upper triangle; tau (N doubles of global scratch).  NB <= waves per workgroup.
template <int RPL, int NB, int CPW>
__device__ inline void qr_coop(double* __restrict__ A, int s, int N, double* __restrict__ R, int ldr, size_t r_elems,
                               double* __restrict__ tau_g, unsigned char* smem) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  double* vbuf = reinterpret_cast<double*>(smem);  // NB x s (rows relative to the panel)
  double* tau = vbuf + (size_t)NB * s;             // NB
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int G = gridDim.x, me = blockIdx.x;
  for (size_t e = (size_t)me * blockDim.x + threadIdx.x; e < r_elems; e += (size_t)G * blockDim.x) R[e] = 0.0;
  grid.sync();
  const int npanels = (N + NB - 1) / NB;
  for (int p = 0; p < npanels; ++p) {
    const int j0 = p * NB;
    const int nbc = N - j0 < NB ? N - j0 : NB;
    const int rows = s - j0;
    double cl[CPW][RPL];
    if (p % G == me) {
      // ---- factorise panel p (its columns already hold every earlier reflection)
      double (&col)[RPL] = cl[0];
      const bool owner = wave < nbc;
      if (owner) {
        const double* a = uniform_ptr(A + (size_t)(j0 + wave) * s + j0);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          col[i] = rr < rows ? a[rr] : 0.0;
        }
      }
      for (int jj = 0; jj < nbc; ++jj) {
        if (wave == jj) {
          double ss = 0, alpha_part = 0;
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            const int rr = lane + 64 * i;
            if (rr > jj) ss += col[i] * col[i];
            if (rr == jj) alpha_part = col[i];
          }
          ss = wave_sum64(ss);
          const double alpha = wave_sum64(alpha_part);
          double t = 0, beta = alpha, scal = 0;
          if (ss > 0) {
            const double nrm = sqrt(alpha * alpha + ss);
            beta = alpha >= 0 ? -nrm : nrm;
            t = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
          }
          double* v = vbuf + (size_t)jj * s;
          double* acol = A + (size_t)(j0 + jj) * s + j0;
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            const int rr = lane + 64 * i;
            if (rr < rows) {
              const double vv = rr < jj ? 0.0 : rr == jj ? 1.0 : col[i] * scal;
              v[rr] = vv;
              if (rr > jj) acol[rr] = vv;  // the reflector, below the diagonal
            }
            if (rr < jj) R[(size_t)(j0 + jj) * ldr + j0 + rr] = col[i];
          }
          if (lane == 0) {
            tau[jj] = t;
            tau_g[j0 + jj] = t;
            R[(size_t)(j0 + jj) * ldr + j0 + jj] = beta;
          }
        }
        lds_barrier();
        if (owner && wave > jj) {
          const double* v = vbuf + (size_t)jj * s;
          const double t = tau[jj];
          double d = 0;
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            const int rr = lane + 64 * i;
            if (rr < rows) d += v[rr] * col[i];
          }
          d = wave_sum64(d) * t;
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            const int rr = lane + 64 * i;
            if (rr < rows) col[i] -= d * v[rr];
          }
        }
      }
    }
    grid.sync();
    if (p % G != me) {
      // ---- the panel's reflectors into LDS (unit leading entries and zeros implicit)
      for (int jj = 0; jj < nbc; ++jj) {
        const double* acol = A + (size_t)(j0 + jj) * s + j0;
        for (int rr = threadIdx.x; rr < rows; rr += blockDim.x)
          vbuf[(size_t)jj * s + rr] = rr < jj ? 0.0 : rr == jj ? 1.0 : acol[rr];
      }
      if (threadIdx.x < nbc) tau[threadIdx.x] = tau_g[j0 + threadIdx.x];
    }
    __syncthreads();
    // ---- apply panel p to this workgroup's columns right of it
    // owned columns: panels q > p with q mod G == me; CPW consecutive columns per wave task
    const int first_q = p + 1 + ((me - (p + 1) % G) % G + G) % G;
    const int per_panel_tasks = (NB + CPW - 1) / CPW;
    int ntasks = 0;
    for (int q = first_q; q < npanels; q += G) ++ntasks;
    ntasks *= per_panel_tasks;
    for (int task = wave; task < ntasks; task += nw) {
      const int q = first_q + (task / per_panel_tasks) * G;
      const int c0 = q * NB + (task % per_panel_tasks) * CPW;
      const int cend = (q + 1) * NB < N ? (q + 1) * NB : N;
#pragma unroll
      for (int u = 0; u < CPW; ++u) {
        const bool cu = c0 + u < cend;
        const double* a = uniform_ptr(A + (size_t)(cu ? c0 + u : c0) * s + j0);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          cl[u][i] = cu && rr < rows ? a[rr] : 0.0;
        }
      }
      for (int jj = 0; jj < nbc; ++jj) {
        const double* v = vbuf + (size_t)jj * s;
        double d[CPW];
#pragma unroll
        for (int u = 0; u < CPW; ++u) d[u] = 0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          const double vv = rr < rows ? v[rr] : 0.0;
#pragma unroll
          for (int u = 0; u < CPW; ++u) d[u] += vv * cl[u][i];
        }
        const double tj = tau[jj];
        {
          constexpr int SH = 6 - ceil_log2(CPW);
          double v16[16];
#pragma unroll
          for (int u = 0; u < CPW; ++u) v16[u] = d[u];
          const double tot = reduce_t<CPW>(v16, lane);
#pragma unroll
          for (int u = 0; u < CPW; ++u) d[u] = bcast_d(tot, u << SH) * tj;
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          const double vv = rr < rows ? v[rr] : 0.0;
#pragma unroll
          for (int u = 0; u < CPW; ++u) cl[u][i] -= d[u] * vv;
        }
      }
#pragma unroll
      for (int u = 0; u < CPW; ++u) {
        if (c0 + u >= cend) continue;
        double* a = opaque_uniform(A + (size_t)(c0 + u) * s + j0);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          if (rr < nbc) R[(size_t)(c0 + u) * ldr + j0 + rr] = cl[u][i];
          else if (rr < rows) a[rr] = cl[u][i];
        }
      }
    }
    __syncthreads();
  }
}

// The same factorisation with a one-panel lookahead.  After panel p is published, the owner
// of panel p + 1 applies p's reflectors to panel p + 1 only and factorises it at once; its
// other columns receive panel p afterwards, together with panel p + 1.  Reflectors of two
// panels live in LDS at a time (double buffer).  Within a factorisation the pivot entry is read
// from its lane, and the later columns keep the reflector in registers between the dot product
// and the update.  Needs at least two workgroups (the lookahead owner differs from the panel's).
//
// No grid barrier per panel: the only dependency between workgroups is that panel p's
// reflectors are complete before anyone reads them, so its owner raises a flag (flags[p]) after
// writing them and every other workgroup waits for that flag alone before copying them; each
// workgroup applies the panels to its own columns in order.  The wait is bounded: past
// kQrSpinLimit polls a workgroup raises flags[npanels] (abort), every later wait returns at
// once, and the factor is marked invalid (R[0] = NaN), so a fault in the protocol cannot hang
// the GPU.  flags: npanels + 1 words of global scratch.  LDS: qr_coop_la_lds_bytes(s, NB).
__host__ __device__ inline size_t qr_coop_la_lds_bytes(int s, int NB) {
  return 2 * ((size_t)NB * s * 8 + (size_t)NB * 8) + 64;
}

constexpr unsigned kQrSpinLimit = 1u << 20;

// Every wave's stores have reached the L2 (each waits for its own), then one thread raises the
// flag; with workers on several XCDs it first releases the stores at agent scope (the L2's
// dirty lines are written back for the other XCDs).
__device__ inline void qr_publish(unsigned* flag, bool local) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (local) __hip_atomic_store(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else __hip_atomic_store(flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One thread polls the flag; with workers on several XCDs it then takes an agent-scope acquire
// (stale cached lines dropped for the whole workgroup, whose waves share the CU's caches) before
// the workgroup reads; on one XCD the reads themselves are agent-scope (load_handed).
__device__ inline void qr_wait(unsigned* flag, unsigned* abort_word, bool local) {
  if (threadIdx.x == 0) {
    unsigned spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
      if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
      __builtin_amdgcn_s_sleep(2);
      if (++spins == kQrSpinLimit) {
        __hip_atomic_store(abort_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    if (!local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Launched with `stride` workgroups per worker (see coop_worker); flags: npanels + 1 words, then
// one XCC id word per worker.  allow_local: take the one-XCD hand-over when the placement allows.
template <int RPL, int NB, int CPW>
__device__ inline void qr_coop_la(double* __restrict__ A, int s, int N, double* __restrict__ R, int ldr,
                                  size_t r_elems, double* __restrict__ tau_g, unsigned* flags, int stride,
                                  bool allow_local, unsigned char* smem) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  double* vbase = reinterpret_cast<double*>(smem);
  // buffer b: vbase + b * (NB * s + NB): NB x s reflector rows (relative to the panel), then NB taus
  auto vbuf = [&](int p) { return vbase + (size_t)(p & 1) * ((size_t)NB * s + NB); };
  auto taus = [&](int p) { return vbuf(p) + (size_t)NB * s; };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int G = coop_workers(stride), me = coop_worker_index(stride);
  const bool worker = coop_worker(stride);
  if (worker)
    for (size_t e = (size_t)me * blockDim.x + threadIdx.x; e < r_elems; e += (size_t)G * blockDim.x) R[e] = 0.0;
  const int npanels = (N + NB - 1) / NB;

  auto factorise = [&](int p) {
    const int j0 = p * NB;
    const int nbc = N - j0 < NB ? N - j0 : NB;
    const int rows = s - j0;
    double* vb = vbuf(p);
    double* tau = taus(p);
    double col[RPL];
    const bool holds = wave < nbc;
    {
      const double* a = uniform_ptr(A + (size_t)(j0 + (holds ? wave : 0)) * s + j0);
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int rr = lane + 64 * i;
        const double x = a[rr < rows ? rr : 0];
        col[i] = holds && rr < rows ? x : 0.0;
      }
    }
    for (int jj = 0; jj < nbc; ++jj) {
      if (wave == jj) {
        double ss = 0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          ss += rr > jj ? col[i] * col[i] : 0.0;
        }
        ss = wave_sum64(ss);
        const double alpha = bcast_d(col[0], jj);  // row jj sits in lane jj, register 0
        double t = 0, beta = alpha, scal = 0;
        if (ss > 0) {
          const double nrm = sqrt(alpha * alpha + ss);
          beta = alpha >= 0 ? -nrm : nrm;
          t = (beta - alpha) / beta;
          scal = 1.0 / (alpha - beta);
        }
        double* v = vb + (size_t)jj * s;
        double* acol = A + (size_t)(j0 + jj) * s + j0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          if (rr < rows) {
            const double vv = rr < jj ? 0.0 : rr == jj ? 1.0 : col[i] * scal;
            v[rr] = vv;
            if (rr > jj) acol[rr] = vv;  // the reflector, below the diagonal
          }
          if (rr < jj) R[(size_t)(j0 + jj) * ldr + j0 + rr] = col[i];
        }
        if (lane == 0) {
          tau[jj] = t;
          tau_g[j0 + jj] = t;
          R[(size_t)(j0 + jj) * ldr + j0 + jj] = beta;
        }
      }
      lds_barrier();
      if (holds && wave > jj) {
        const double* v = vb + (size_t)jj * s;
        double vv[RPL];
        double d = 0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          vv[i] = rr < rows ? v[rr] : 0.0;
          d += vv[i] * col[i];
        }
        d = wave_sum64(d) * tau[jj];
#pragma unroll
        for (int i = 0; i < RPL; ++i) col[i] -= d * vv[i];
      }
    }
  };

  // panel p's reflectors, as its owner stored them in A and tau_g, into this workgroup's LDS;
  // every load is issued before the first store (agent-scope loads in the one-XCD hand-over)
  auto copy = [&](int p, bool local) {
    const int j0 = p * NB;
    const int nbc = N - j0 < NB ? N - j0 : NB;
    const int rows = s - j0;
    double* vb = vbuf(p);
    // rows per thread: s <= 64 RPL rows over the 512 (RPL < 64) or 256 (RPL = 64) threads
    constexpr int RR = RPL >= 64 ? RPL / 4 : RPL / 8;
    double val[NB][RR];
    auto fetch = [&](auto handed) {
#pragma unroll
      for (int jj = 0; jj < NB; ++jj)
#pragma unroll
        for (int k = 0; k < RR; ++k) {
          const int rr = threadIdx.x + k * (int)blockDim.x;
          const bool ok = jj < nbc && rr < rows;
          const double* xp = &A[(size_t)(j0 + (ok ? jj : 0)) * s + j0 + (ok ? rr : 0)];
          const double x = decltype(handed)::value ? load_handed(xp) : *xp;
          val[jj][k] = rr < jj ? 0.0 : rr == jj ? 1.0 : x;
        }
    };
    if (local) fetch(std::true_type{});
    else fetch(std::false_type{});
#pragma unroll
    for (int jj = 0; jj < NB; ++jj)
#pragma unroll
      for (int k = 0; k < RR; ++k) {
        const int rr = threadIdx.x + k * (int)blockDim.x;
        if (jj < nbc && rr < rows) vb[(size_t)jj * s + rr] = val[jj][k];
      }
    if (threadIdx.x < nbc) taus(p)[threadIdx.x] = local ? load_handed(&tau_g[j0 + threadIdx.x]) : tau_g[j0 + threadIdx.x];
  };

  // panel pv's reflectors (in LDS) applied, in order, to this workgroup's columns in panels
  // qa..qb (those with q mod G == me), CW consecutive columns per wave task (CW = CPW for the
  // bulk of the trailing matrix; one column per wave for the single lookahead panel, so that
  // all waves take part in the step on the critical path)
  auto apply = [&](auto cw_tag, int pv, int qa, int qb) {
    constexpr int CW = decltype(cw_tag)::value;
    const int j0 = pv * NB;
    const int nbc = N - j0 < NB ? N - j0 : NB;
    const int rows = s - j0;
    const double* vb = vbuf(pv);
    const double* tau = taus(pv);
    const int first_q = qa + ((me - qa % G) % G + G) % G;
    const int per_panel_tasks = (NB + CW - 1) / CW;
    int ntasks = 0;
    for (int q = first_q; q <= qb; q += G) ++ntasks;
    ntasks *= per_panel_tasks;
    for (int task = wave; task < ntasks; task += nw) {
      const int q = first_q + (task / per_panel_tasks) * G;
      const int c0 = q * NB + (task % per_panel_tasks) * CW;
      const int cend = (q + 1) * NB < N ? (q + 1) * NB : N;
      double cl[CW][RPL];
#pragma unroll
      for (int u = 0; u < CW; ++u) {
        const bool cu = c0 + u < cend;
        const double* a = uniform_ptr(A + (size_t)(cu ? c0 + u : c0) * s + j0);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          const double x = a[rr < rows ? rr : 0];
          cl[u][i] = cu && rr < rows ? x : 0.0;
        }
      }
      for (int jj = 0; jj < nbc; ++jj) {
        const double* v = vb + (size_t)jj * s;
        double vv[RPL];
        double d[CW];
#pragma unroll
        for (int u = 0; u < CW; ++u) d[u] = 0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          vv[i] = rr < rows ? v[rr] : 0.0;
#pragma unroll
          for (int u = 0; u < CW; ++u) d[u] += vv[i] * cl[u][i];
        }
        const double tj = tau[jj];
        {
          constexpr int SH = 6 - ceil_log2(CW);
          double v16[16];
#pragma unroll
          for (int u = 0; u < CW; ++u) v16[u] = d[u];
          const double tot = reduce_t<CW>(v16, lane);
#pragma unroll
          for (int u = 0; u < CW; ++u) d[u] = bcast_d(tot, u << SH) * tj;
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i)
#pragma unroll
          for (int u = 0; u < CW; ++u) cl[u][i] -= d[u] * vv[i];
      }
#pragma unroll
      for (int u = 0; u < CW; ++u) {
        if (c0 + u >= cend) continue;
        double* a = opaque_uniform(A + (size_t)(c0 + u) * s + j0);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          if (rr < nbc) R[(size_t)(c0 + u) * ldr + j0 + rr] = cl[u][i];
          else if (rr < rows) a[rr] = cl[u][i];
        }
      }
    }
  };

  unsigned* xcc_ids = flags + npanels + 1;
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i <= npanels; i += blockDim.x) flags[i] = 0u;
  xcd_record(xcc_ids, stride);
  grid.sync();  // R and the flags zeroed everywhere before any panel writes or polls them
  if (!worker) return;
  const bool local = xcd_all_local(xcc_ids, stride, allow_local);
  unsigned* abort_word = flags + npanels;
  if (me == 0 % G) {
    factorise(0);
    qr_publish(flags, local);
  }
  for (int p = 0; p < npanels; ++p) {
    const int owner = p % G;
    const int nx = p + 1;
    if (me != owner) {
      qr_wait(flags + p, abort_word, local);  // panel p's reflectors are in A and tau_g
      copy(p, local);
    }
    __syncthreads();
    using One = std::integral_constant<int, 1>;
    using Bulk = std::integral_constant<int, CPW>;
    if (nx < npanels && me == nx % G) {
      apply(One{}, p, nx, nx);  // the next panel first, then factorise it
      __syncthreads();
      factorise(nx);
      qr_publish(flags + nx, local);
    } else if (me == owner && p > 0) {
      apply(Bulk{}, p - 1, p + 1, npanels - 1);  // deferred while this workgroup factorised panel p
      __syncthreads();
      apply(Bulk{}, p, p + 1, npanels - 1);
    } else {
      apply(Bulk{}, p, p + 1, npanels - 1);
    }
    __syncthreads();
  }
  // a wait that gave up leaves a wrong factor: mark it (no later write in this launch touches R[0])
  if (threadIdx.x == 0 && __hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
    R[0] = __builtin_nan("");
}

}  // namespace nsk
