// Single-instance SVD launches.
//
// N <= 320 and s <= 4096: three kernels, one workgroup each -- panel Householder QR (1024
// threads), block one-sided Jacobi with the blocks in registers, and the finish stage (1024
// threads) that ranks the singular values and rebuilds the requested vectors from the
// rotation log.  The Jacobi kernel is specialised on the rows per lane NR: NR <= 3 runs 8
// waves (2 per SIMD, 256 VGPRs each); NR >= 4 holds two blocks of 4 x 13 or 5 x 10 doubles per
// lane and runs 4 waves (1 per SIMD), whose accumulation registers absorb the overflow.
// Larger problems run one-sided Jacobi on SA itself across the whole GPU (svd_big.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>

#include "nsk_internal.hpp"
#include "svd_device.hpp"
#include "qr_coop.hpp"
#include "svd_pipeline.hpp"
#include "svd_big.hpp"

namespace nsk {

__host__ __device__ constexpr int jacobi_threads(int NR) { return NR <= 3 ? 512 : 256; }

static SvdWork to_work(const SvdPlan& p) {
  SvdWork w;
  w.sa = p.sa;
  w.R = p.R;
  w.log = p.log;
  w.sigma = p.sigma;
  w.order = p.order;
  w.colnorm = p.colnorm;
  w.jres = p.jres;
  w.Vk = p.Vk;
  w.sigma_k = p.sigma_k;
  w.info = p.info;
  w.s = p.s;
  w.N = p.N;
  w.k = p.k;
  w.max_sweeps = p.max_sweeps;
  // NSK_COOP_LOCAL=0 keeps the agent-scope hand-over even where all workers share an XCD
  const char* env = std::getenv("NSK_COOP_LOCAL");
  w.coop_local = env != nullptr && env[0] == '0' ? 0 : 1;
  w.coop_stride = 1;
  return w;
}

// The QR (CPW x RPL = 64 trailing-column doubles per lane) and the log replay (prefetch
// registers plus a block pair per lane) need more than the 128 VGPRs a 1024-thread
// workgroup leaves each wave; they run 512 threads.
__host__ __device__ constexpr int qr_threads(int rpl) { return rpl >= 64 ? 256 : 512; }
constexpr int kFinishThreads = 512;
constexpr int kFinishGroups = 2;

template <int RPL>
__global__ __launch_bounds__(qr_threads(RPL)) void svd_qr_kernel(SvdWork w) {
  extern __shared__ __align__(16) unsigned char smem[];
  svd_stage_qr_rpl<RPL>(w, smem);
}

template <int NR>
__global__ __launch_bounds__(jacobi_threads(NR)) void svd_jacobi_kernel(SvdWork w) {
  __shared__ unsigned char smem[64];
  svd_stage_jacobi_nr<NR, JacobiB<NR>::value>(w, smem);
}

static hipError_t lds_attr(const void* fn, size_t lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// Multi-workgroup QR: panels of NB columns dealt round-robin over the workgroups; tau in
// the sigma array (overwritten by the finish stage).
template <int RPL>
__global__ __launch_bounds__(qr_threads(RPL)) void svd_qr_coop_kernel(SvdWork w) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int C = QrCpw<RPL>::value;
  const JacobiShape js = jacobi_shape(w.N);
  const int ldr = 64 * js.NR;
  const size_t relems = (size_t)ldr * js.nb * js.B;
  switch (qr_panel_width(w.s, blockDim.x >> 6)) {
    case 16: qr_coop<RPL, 16, C>(w.sa, w.s, w.N, w.R, ldr, relems, w.sigma, smem); break;
    case 8: qr_coop<RPL, 8, C>(w.sa, w.s, w.N, w.R, ldr, relems, w.sigma, smem); break;
    case 4: qr_coop<RPL, 4, C>(w.sa, w.s, w.N, w.R, ldr, relems, w.sigma, smem); break;
    case 2: qr_coop<RPL, 2, C>(w.sa, w.s, w.N, w.R, ldr, relems, w.sigma, smem); break;
    default: qr_coop<RPL, 1, C>(w.sa, w.s, w.N, w.R, ldr, relems, w.sigma, smem); break;
  }
}

// Lookahead variant (two panels of reflectors in LDS, at least two workgroups).
template <int RPL>
__global__ __launch_bounds__(qr_threads(RPL)) void svd_qr_coop_la_kernel(SvdWork w) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int C = QrCpw<RPL>::value;
  // the rotation log is free until the Jacobi stage: the panel flags live at its start
  unsigned* flags = reinterpret_cast<unsigned*>(w.log);
  const JacobiShape js = jacobi_shape(w.N);
  const int ldr = 64 * js.NR;
  const size_t relems = (size_t)ldr * js.nb * js.B;
  switch (qr_panel_width(w.s, blockDim.x >> 6)) {
    case 16: qr_coop_la<RPL, 16, C>(w.sa, w.s, w.N, w.R, ldr, relems, w.sigma, flags, w.coop_stride, w.coop_local != 0, smem); break;
    case 8: qr_coop_la<RPL, 8, C>(w.sa, w.s, w.N, w.R, ldr, relems, w.sigma, flags, w.coop_stride, w.coop_local != 0, smem); break;
    case 4: qr_coop_la<RPL, 4, C>(w.sa, w.s, w.N, w.R, ldr, relems, w.sigma, flags, w.coop_stride, w.coop_local != 0, smem); break;
    case 2: qr_coop_la<RPL, 2, C>(w.sa, w.s, w.N, w.R, ldr, relems, w.sigma, flags, w.coop_stride, w.coop_local != 0, smem); break;
    default: qr_coop_la<RPL, 1, C>(w.sa, w.s, w.N, w.R, ldr, relems, w.sigma, flags, w.coop_stride, w.coop_local != 0, smem); break;
  }
}

// Workgroups launched per worker of the multi-workgroup QR and Jacobi: kXcds (the workers on one
// XCD) when the device has a CU for each of the groups * kXcds workgroups, else 1.
// The CU count is queried once per device (the query is slow next to a solve).
static hipError_t set_coop_stride(SvdWork& w, int groups) {
  constexpr int kMaxDevices = 64;
  static std::atomic<int> cus_of[kMaxDevices];
  int dev = 0;
  if (hipError_t e = hipGetDevice(&dev)) return e;
  int cus = dev < kMaxDevices ? cus_of[dev].load(std::memory_order_relaxed) : 0;
  if (cus == 0) {
    if (hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) return e;
    if (dev < kMaxDevices) cus_of[dev].store(cus, std::memory_order_relaxed);
  }
  w.coop_stride = cus >= groups * kXcds ? kXcds : 1;
  return hipSuccess;
}

// workgroups of the multi-workgroup QR: one per panel, at most 16
static int qr_coop_groups(int s, int N, int threads) {
  const int nb = qr_panel_width(s, threads / 64);
  const int panels = (N + nb - 1) / nb;
  return panels < 16 ? panels : 16;
}

template <int RPL>
static hipError_t launch_qr_coop(SvdWork& w, hipStream_t st) {
  const int threads = qr_threads(RPL);
  const int nb = qr_panel_width(w.s, threads / 64);
  const int groups = qr_coop_groups(w.s, w.N, threads);
  void* args[] = {&w};
  const size_t lds_la = qr_coop_la_lds_bytes(w.s, nb);
  // up to 16 rows per lane (s <= 1024): the variant for more rows per lane spills registers
  if (RPL <= 16 && groups >= 2 && lds_la <= 160 * 1024) {
    if (hipError_t e = lds_attr((const void*)svd_qr_coop_la_kernel<RPL>, lds_la)) return e;
    // coop_stride workgroups per worker: the workers (b = kXcds w) share one XCD's L2
    if (hipError_t e = set_coop_stride(w, groups)) return e;
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(svd_qr_coop_la_kernel<RPL>),
                                      dim3(groups * w.coop_stride), dim3(threads), args, lds_la, st);
  }
  const size_t lds = qr_panel_lds_bytes(w.s, nb);
  if (hipError_t e = lds_attr((const void*)svd_qr_coop_kernel<RPL>, lds)) return e;
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(svd_qr_coop_kernel<RPL>), dim3(groups),
                                    dim3(threads), args, lds, st);
}

// Multi-workgroup Jacobi: nb / 2 workgroups of NR waves (one row per lane).
template <int NR>
__global__ __launch_bounds__(NR * 64) void svd_jacobi_coop_kernel(SvdWork w) {
  // colnorm is free until the finish stage recomputes it: scratch for the Gram check
  jacobi_coop_sweeps<NR, JacobiB<NR>::value>(w.R, w.N, w.max_sweeps, w.log,
                                             jacobi_counters(w.log, w.N, w.max_sweeps), w.jres, w.colnorm,
                                             w.coop_stride, w.coop_local != 0);
}

template <int NR>
static hipError_t launch_jacobi_coop(SvdWork& w, hipStream_t st) {
  void* args[] = {&w};
  const int groups = jacobi_shape(w.N).nb / 2;
  // coop_stride workgroups per worker: the workers (b = kXcds w) share one XCD's L2
  if (hipError_t e = set_coop_stride(w, groups)) return e;
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(svd_jacobi_coop_kernel<NR>),
                                    dim3(groups * w.coop_stride), dim3(NR * 64), args, 0, st);
}

template <int NR>
__global__ __launch_bounds__(kFinishThreads) void svd_finish_kernel(SvdWork w) {
  extern __shared__ __align__(16) unsigned char smem[];
  // launched as kFinishGroups workgroups of which only the last works: it runs on XCD 1, away
  // from XCD 0's L2, where the Jacobi's workers left the rotation log (replayed from XCD 0 the
  // stage measured 0.203 ms at config 2, from XCD 1 0.186 ms)
  if (blockIdx.x != gridDim.x - 1) return;
  svd_stage_finish_nr<NR, JacobiB<NR>::value>(w, jacobi_shape(w.N), smem);
}



bool svd_fast_path(int s, int N) { return N <= kFastMaxN && s <= kFastMaxS; }

// Past the fast path, a sketch of at most kFastMaxS rows (and more rows than columns) is first
// reduced to R by the multi-workgroup QR, and the large-N Jacobi runs on R's 64 NR rows
// (zero-padded, ld = 64 NR) instead of SA's s rows: R^T R = (SA)^T SA, so the rotations are the
// same and every column pair moves fewer rows.
static bool svd_big_qr_first(int s, int N) { return !svd_fast_path(s, N) && s <= kFastMaxS && s > N; }

size_t svd_work_R_bytes(int s, int N) {
  return svd_fast_path(s, N) || svd_big_qr_first(s, N) ? svd_fast_R_bytes(N) : 0;
}

// the fast path's rotation log; the large path's per-sweep counters (and, before them, the QR's
// panel flags and XCC ids: at most N + 1 + kCoopMaxBlocks / 2 words)
size_t svd_work_log_bytes(int s, int N, int max_sweeps) {
  if (svd_fast_path(s, N)) return svd_fast_log_bytes(N, max_sweeps);
  const size_t flags = (size_t)(N + 1 + kCoopMaxBlocks / 2) * sizeof(unsigned);
  return std::max(svd_big_counter_bytes(max_sweeps), flags);
}

hipError_t launch_svd(const SvdPlan& p, hipStream_t st) {
  if (svd_fast_path(p.s, p.N)) {
    SvdWork w = to_work(p);
    hipError_t e = hipSuccess;
    const int rpl = qr_rpl(p.s), tq = qr_threads(rpl);
    if (p.N > 64) {
      // the panels' trailing updates run on several CUs
      switch (rpl) {
        case 16: e = launch_qr_coop<16>(w, st); break;
        case 32: e = launch_qr_coop<32>(w, st); break;
        default: e = launch_qr_coop<64>(w, st); break;
      }
    } else {
      const size_t lq = svd_fast_lds_bytes(p.s, p.N, tq / 64);
      switch (rpl) {
        case 16:
          e = lds_attr((const void*)svd_qr_kernel<16>, lq);
          if (e == hipSuccess) svd_qr_kernel<16><<<1, tq, lq, st>>>(w);
          break;
        case 32:
          e = lds_attr((const void*)svd_qr_kernel<32>, lq);
          if (e == hipSuccess) svd_qr_kernel<32><<<1, tq, lq, st>>>(w);
          break;
        default:
          e = lds_attr((const void*)svd_qr_kernel<64>, lq);
          if (e == hipSuccess) svd_qr_kernel<64><<<1, tq, lq, st>>>(w);
          break;
      }
    }
    if (e != hipSuccess) return e;
    prof_mark(3, st);
    // the block pairs of a round run on separate CUs once there are rows enough (N > 64)
    switch (jacobi_shape(p.N).NR) {
      case 1: svd_jacobi_kernel<1><<<1, jacobi_threads(1), 0, st>>>(w); break;
      case 2: e = launch_jacobi_coop<2>(w, st); break;
      case 3: e = launch_jacobi_coop<3>(w, st); break;
      case 4: e = launch_jacobi_coop<4>(w, st); break;
      default: e = launch_jacobi_coop<5>(w, st); break;
    }
    if (e != hipSuccess) return e;
    prof_mark(4, st);
    const int tf = kFinishThreads;
    const size_t lf = finish_lds_bytes(jacobi_shape(p.N), tf / 64);  // the log's shape (see svd_stage_finish_nr)
    switch (jacobi_shape(p.N).NR) {
      case 1:
        e = lds_attr((const void*)svd_finish_kernel<1>, lf);
        if (e == hipSuccess) svd_finish_kernel<1><<<kFinishGroups, tf, lf, st>>>(w);
        break;
      case 2:
        e = lds_attr((const void*)svd_finish_kernel<2>, lf);
        if (e == hipSuccess) svd_finish_kernel<2><<<kFinishGroups, tf, lf, st>>>(w);
        break;
      case 3:
        e = lds_attr((const void*)svd_finish_kernel<3>, lf);
        if (e == hipSuccess) svd_finish_kernel<3><<<kFinishGroups, tf, lf, st>>>(w);
        break;
      case 4:
        e = lds_attr((const void*)svd_finish_kernel<4>, lf);
        if (e == hipSuccess) svd_finish_kernel<4><<<kFinishGroups, tf, lf, st>>>(w);
        break;
      default:
        e = lds_attr((const void*)svd_finish_kernel<5>, lf);
        if (e == hipSuccess) svd_finish_kernel<5><<<kFinishGroups, tf, lf, st>>>(w);
        break;
    }
    if (e != hipSuccess) return e;
    prof_mark(5, st);
    return hipGetLastError();
  }
  // large sizes: the QR when it applies, cooperative Jacobi on R (or SA), then the one-workgroup
  // finish
  double* sa = p.sa;
  int s = p.s, N = p.N, sweeps = p.max_sweeps;
  if (svd_big_qr_first(p.s, p.N)) {
    SvdWork w = to_work(p);
    hipError_t e = hipSuccess;
    switch (qr_rpl(p.s)) {
      case 16: e = launch_qr_coop<16>(w, st); break;
      case 32: e = launch_qr_coop<32>(w, st); break;
      default: e = launch_qr_coop<64>(w, st); break;
    }
    if (e != hipSuccess) return e;
    sa = p.R;
    s = 64 * jacobi_shape(p.N).NR;
  }
  int dev = 0, cus = 0;
  if (hipError_t e = hipGetDevice(&dev)) return e;
  if (hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) return e;
  const int nb = (p.N + kBigW - 1) / kBigW;
  const int groups = std::max(1, std::min(cus, (nb + (nb & 1)) / 2));
  double* V = p.V;
  unsigned long long* counters = reinterpret_cast<unsigned long long*>(p.log);
  void* args[] = {&sa, &s, &N, &V, &sweeps, &counters};
  prof_mark(3, st);
  const void* fn = s <= 1024   ? reinterpret_cast<const void*>(svd_big_jacobi_kernel<16>)
                   : s <= 2048 ? reinterpret_cast<const void*>(svd_big_jacobi_kernel<32>)
                               : reinterpret_cast<const void*>(svd_big_jacobi_kernel<0>);
  if (hipError_t e = hipLaunchCooperativeKernel(fn, dim3(groups), dim3(kBigThreads), args, 0, st)) return e;
  prof_mark(4, st);
  svd_big_finish_kernel<<<1, 1024, (size_t)p.N * 8, st>>>(sa, s, p.N, p.k, p.V, p.max_sweeps, counters, p.sigma,
                                                          p.order, p.Vk, p.sigma_k, p.info);
  prof_mark(5, st);
  return hipGetLastError();
}

}  // namespace nsk
