// SVD of the sketch SA for N <= 320 and s <= 4096: panel Householder QR -> block
// one-sided Jacobi with a rotation log -> singular values, ordering and the requested
// right singular vectors rebuilt from the log.  Every stage runs inside one workgroup and
// synchronises with barriers only (the batched persistent kernel calls it directly, with the
// one-workgroup block shape jacobi_shape_wg); the single-instance path launches the stages as
// kernels (one-workgroup QR and Jacobi for N <= 64, where the two shapes agree; the
// multi-workgroup kernels and the finish stage with jacobi_shape above).
#pragma once

#include <hip/hip_runtime.h>

#include "jacobi_block.hpp"
#include "jacobi_coop.hpp"
#include "nsk_internal.hpp"
#include "qr_panel.hpp"

namespace nsk {

constexpr int kFastMaxN = 320;
constexpr int kFastMaxS = 4096;

struct SvdWork {
  double* sa;          // s x N column-major, overwritten by the QR
  double* R;           // (64 NR) x (nb B) column-major, ld = 64 NR
  double2* log;        // max_sweeps * jacobi_log_entries_per_sweep
  double* sigma;       // N, sorted non-increasing
  int* order;          // N, column of R holding sigma[i]
  double* colnorm;     // N, |R_c| for every column c
  JacobiResult* jres;  // sweeps / convergence of the Jacobi stage
  double* Vk;          // N x k row-major (nullable)
  double* sigma_k;     // k (nullable)
  nsk_info* info;      // nullable
  int s, N, k, max_sweeps;
  int coop_local;      // multi-workgroup QR and Jacobi may take the one-XCD hand-over
  int coop_stride;     // workgroups launched per worker of the multi-workgroup QR and Jacobi
};

// rotation log, followed by the per-sweep counters of the multi-workgroup Jacobi; large enough
// for the log of either shape (the one-workgroup Jacobi keeps no counters)
__host__ __device__ inline size_t svd_fast_log_bytes(int N, int max_sweeps) {
  const size_t coop = (size_t)max_sweeps * jacobi_log_entries_per_sweep(jacobi_shape(N)) * sizeof(double2) +
                      jacobi_coop_counter_bytes(max_sweeps);
  const size_t wg = (size_t)max_sweeps * jacobi_log_entries_per_sweep(jacobi_shape_wg(N)) * sizeof(double2);
  return coop > wg ? coop : wg;
}

__host__ __device__ inline unsigned long long* jacobi_counters(double2* log, int N, int max_sweeps) {
  const JacobiShape js = jacobi_shape(N);
  return reinterpret_cast<unsigned long long*>(log + (size_t)max_sweeps * jacobi_log_entries_per_sweep(js));
}

__host__ __device__ inline size_t svd_fast_R_bytes(int N) {
  const JacobiShape a = jacobi_shape(N), b = jacobi_shape_wg(N);
  const int cols = a.nb * a.B > b.nb * b.B ? a.nb * a.B : b.nb * b.B;
  return (size_t)64 * a.NR * cols * sizeof(double);
}

__host__ __device__ inline int qr_panel_width(int s, int nwaves) {
  int nb = nwaves < 16 ? nwaves : 16;
  while (nb > 1 && qr_panel_lds_bytes(s, nb) > 120 * 1024) nb >>= 1;
  return nb;
}

// vector groups of the finish stage that replay concurrently (js: the Jacobi's shape)
__host__ __device__ inline int finish_groups(const JacobiShape& js, int nwaves) {
  const int g = nwaves / replay_waves(js);
  return g > 0 ? g : 1;
}

__host__ __device__ inline size_t finish_head_bytes(int N) { return ((size_t)N * 12 + 255) & ~(size_t)255; }

__host__ __device__ inline size_t finish_vec_bytes(const JacobiShape& js) {
  return ((size_t)js.nb * js.B * 8 + 255) & ~(size_t)255;
}

__host__ __device__ inline size_t finish_lds_bytes(const JacobiShape& js, int nwaves) {
  return finish_head_bytes(js.N) + (size_t)finish_groups(js, nwaves) * finish_vec_bytes(js);
}

// LDS of the one-workgroup pipeline (QR, then the finish stage in the one-workgroup shape)
__host__ __device__ inline size_t svd_fast_lds_bytes(int s, int N, int nwaves) {
  const size_t qr = qr_panel_lds_bytes(s, qr_panel_width(s, nwaves));
  const size_t fin = finish_lds_bytes(jacobi_shape_wg(N), nwaves);
  return qr > fin ? qr : fin;
}

// ---------------------------------------------------------------- stage 1: QR
// rows per lane of a panel column: s <= 64 RPL
__host__ __device__ inline int qr_rpl(int s) { return s <= 1024 ? 16 : s <= 2048 ? 32 : 64; }

// trailing-update columns per wave: CPW x RPL doubles stay in registers
template <int RPL>
struct QrCpw {
  static constexpr int value = RPL <= 16 ? 4 : RPL <= 32 ? 2 : 1;
};

// R goes into the one-workgroup Jacobi's layout
template <int RPL>
__device__ inline void svd_stage_qr_rpl(const SvdWork& w, unsigned char* smem) {
  constexpr int C = QrCpw<RPL>::value;
  const JacobiShape js = jacobi_shape_wg(w.N);
  const int ldr = 64 * js.NR;
  const size_t total = (size_t)ldr * js.nb * js.B;
  for (size_t e = threadIdx.x; e < total; e += blockDim.x) w.R[e] = 0.0;
  __syncthreads();
  switch (qr_panel_width(w.s, blockDim.x >> 6)) {
    case 16: qr_panel<RPL, 16, C>(w.sa, w.s, w.N, w.R, ldr, smem); break;
    case 8: qr_panel<RPL, 8, C>(w.sa, w.s, w.N, w.R, ldr, smem); break;
    case 4: qr_panel<RPL, 4, C>(w.sa, w.s, w.N, w.R, ldr, smem); break;
    case 2: qr_panel<RPL, 2, C>(w.sa, w.s, w.N, w.R, ldr, smem); break;
    default: qr_panel<RPL, 1, C>(w.sa, w.s, w.N, w.R, ldr, smem); break;
  }
  __syncthreads();
}

__device__ inline void svd_stage_qr(const SvdWork& w, unsigned char* smem) {
  switch (qr_rpl(w.s)) {
    case 16: svd_stage_qr_rpl<16>(w, smem); break;
    case 32: svd_stage_qr_rpl<32>(w, smem); break;
    default: svd_stage_qr_rpl<64>(w, smem); break;
  }
}

// ---------------------------------------------------------------- stage 2: Jacobi
// the one-workgroup Jacobi, in the shape jacobi_shape_wg(w.N) (B must be its block size)
template <int NR, int B>
__device__ inline void svd_stage_jacobi_nr(const SvdWork& w, unsigned char* smem) {
  const JacobiShape js = jacobi_shape_wg(w.N);
  int* sh_rot = reinterpret_cast<int*>(smem);
  double* sh_off = reinterpret_cast<double*>(smem + 8);
  int conv = 0;
  double off = 0;
  const int sweeps = jacobi_block_sweeps<NR, B>(w.R, js, w.max_sweeps, w.log, sh_rot, sh_off, &conv, &off);
  if (threadIdx.x == 0) {
    w.jres->sweeps = sweeps;
    w.jres->converged = conv;
    w.jres->off = off;
  }
  __syncthreads();
}

template <int NR>
struct JacobiB {
  static constexpr int value = jacobi_block_size(NR);
};


__device__ inline void svd_stage_jacobi(const SvdWork& w, unsigned char* smem) {
  switch (jacobi_shape(w.N).NR) {
    case 1: svd_stage_jacobi_nr<1, JacobiB<1>::value>(w, smem); break;
    case 2: svd_stage_jacobi_nr<2, JacobiB<2>::value>(w, smem); break;
    case 3: svd_stage_jacobi_nr<3, JacobiB<3>::value>(w, smem); break;
    case 4:
      if (jacobi_shape_wg(w.N).B == 8) svd_stage_jacobi_nr<4, 8>(w, smem);
      else svd_stage_jacobi_nr<4, JacobiB<4>::value>(w, smem);
      break;
    default: svd_stage_jacobi_nr<5, JacobiB<5>::value>(w, smem); break;
  }
}

// ---------------------------------------------------------------- stage 3: finish
// x <- V x (fwd = false) or V^T x (fwd = true), any block size; called by every thread of
// the workgroup (see jacobi_replay)
__device__ inline void replay_any(double* x, const double2* log, const JacobiShape& js, int sweeps, bool fwd,
                                  int vl, bool member) {
  switch (js.NR) {
    case 1: jacobi_replay<jacobi_block_size(1)>(x, log, js, sweeps, fwd, vl, member); break;
    case 2: jacobi_replay<jacobi_block_size(2)>(x, log, js, sweeps, fwd, vl, member); break;
    case 3: jacobi_replay<jacobi_block_size(3)>(x, log, js, sweeps, fwd, vl, member); break;
    case 4: jacobi_replay<jacobi_block_size(4)>(x, log, js, sweeps, fwd, vl, member); break;
    default: jacobi_replay<jacobi_block_size(5)>(x, log, js, sweeps, fwd, vl, member); break;
  }
}

// The log was written in the shape js with blocks of B (the one-workgroup shape in the batched
// pipeline, the multi-workgroup one after the single-instance kernels).
template <int NR, int B>
__device__ inline void svd_stage_finish_nr(const SvdWork& w, const JacobiShape& js, unsigned char* smem) {
  const int N = w.N, k = w.k;
  const int ldr = 64 * js.NR;
  const int ncols = js.nb * js.B;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  double* nrm = reinterpret_cast<double*>(smem);
  int* rk = reinterpret_cast<int*>(nrm + N);
  const int vw = replay_waves(js), ngroups = finish_groups(js, nw);
  const int grp = wave / vw;
  const bool member = grp < ngroups;
  const int vl = (wave - grp * vw) * 64 + lane;
  double* x = reinterpret_cast<double*>(smem + finish_head_bytes(N) + (size_t)(member ? grp : 0) * finish_vec_bytes(js));
  // singular values: column norms of the rotated R
  for (int c = wave; c < N; c += nw) {
    double a = 0;
    for (int e = lane; e < ldr; e += 64) a += w.R[(size_t)c * ldr + e] * w.R[(size_t)c * ldr + e];
    a = wave_sum64(a);
    if (lane == 0) {
      nrm[c] = sqrt(a);
      if (w.colnorm) w.colnorm[c] = sqrt(a);
    }
  }
  __syncthreads();
  // rank by (norm descending, index ascending); NaN ranks last so ranks are a permutation
  for (int c = tid; c < N; c += blockDim.x) {
    const double xv = nrm[c];
    const double kx = xv != xv ? -1.0 : xv;
    int r = 0;
    for (int d = 0; d < N; ++d) {
      const double yv = nrm[d];
      const double ky = yv != yv ? -1.0 : yv;
      r += (ky > kx) || (ky == kx && d < c);
    }
    rk[c] = r;
    w.order[r] = c;
    w.sigma[r] = xv;
  }
  __syncthreads();
  const int sweeps = w.jres->sweeps;
  // trailing vectors: vector group q rebuilds V e_{order[N-k+q]} from the log
  for (int q0 = 0; q0 < k; q0 += ngroups) {
    const int q = q0 + grp;
    const bool mine = member && q < k;
    if (mine) {
      const int c = w.order[N - k + q];
      for (int e = vl; e < ncols; e += vw * 64) x[e] = e == c ? 1.0 : 0.0;
    }
    lds_barrier();
    jacobi_replay<B>(x, w.log, js, sweeps, false, vl, mine);
    // sign: largest-magnitude entry positive, lowest index on ties (first wave of the group)
    if (mine && vl < 64) {
      double best = -1;
      int bi = 0;
      for (int e = lane; e < N; e += 64) {
        const double a = fabs(x[e]);
        if (a > best) {
          best = a;
          bi = e;
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      const double sgn = x[bi] < 0 ? -1.0 : 1.0;
      if (w.Vk)
        for (int e = lane; e < N; e += 64) w.Vk[(size_t)e * k + q] = sgn * x[e];
      if (w.sigma_k && lane == 0) w.sigma_k[q] = w.sigma[N - k + q];
    }
    __syncthreads();
  }
  if (w.info && tid == 0) {
    w.info->sweeps = sweeps;
    w.info->converged = w.jres->converged;
    w.info->off = w.jres->off;
    w.info->sigma_max = w.sigma[0];
  }
  __syncthreads();
}

__device__ inline void svd_stage_finish(const SvdWork& w, unsigned char* smem) {
  const JacobiShape js = jacobi_shape_wg(w.N);
  switch (js.NR) {
    case 1: svd_stage_finish_nr<1, JacobiB<1>::value>(w, js, smem); break;
    case 2: svd_stage_finish_nr<2, JacobiB<2>::value>(w, js, smem); break;
    case 3: svd_stage_finish_nr<3, JacobiB<3>::value>(w, js, smem); break;
    case 4:
      if (js.B == 8) svd_stage_finish_nr<4, 8>(w, js, smem);
      else svd_stage_finish_nr<4, JacobiB<4>::value>(w, js, smem);
      break;
    default: svd_stage_finish_nr<5, JacobiB<5>::value>(w, js, smem); break;
  }
}

// the single-workgroup SVD
__device__ inline void svd_pipeline(const SvdWork& w, unsigned char* smem) {
  svd_stage_qr(w, smem);
  svd_stage_jacobi(w, smem);
  svd_stage_finish(w, smem);
}

}  // namespace nsk
