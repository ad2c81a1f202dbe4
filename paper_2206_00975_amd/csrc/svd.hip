// Single-instance SVD launches.
//
// N <= 320 and s <= 4096: three kernels, one workgroup each -- panel Householder QR (1024
// threads), block one-sided Jacobi with the blocks in registers (512 threads: 8 waves with up
// to 256 VGPRs each), and the finish stage (1024 threads) that ranks the singular values and
// rebuilds the requested vectors from the rotation log.
// Larger problems use svd_instance (scalar Jacobi on global-memory R with V accumulated).
#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "svd_device.hpp"
#include "svd_pipeline.hpp"

namespace nsk {

constexpr int kSvdThreads = 1024;
constexpr int kJacobiThreads = 512;

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
  return w;
}

__global__ __launch_bounds__(kSvdThreads) void svd_qr_kernel(SvdWork w) {
  extern __shared__ unsigned char smem[];
  svd_stage_qr(w, smem);
}

__global__ __launch_bounds__(kJacobiThreads) void svd_jacobi_kernel(SvdWork w) {
  __shared__ unsigned char smem[64];
  svd_stage_jacobi(w, smem);
}

__global__ __launch_bounds__(kSvdThreads) void svd_finish_kernel(SvdWork w) {
  extern __shared__ unsigned char smem[];
  svd_stage_finish(w, smem);
}

__global__ __launch_bounds__(kSvdThreads) void svd_kernel(SvdPlan p) {
  extern __shared__ unsigned char smem[];
  svd_instance(p.sa, p.s, p.N, p.k, p.max_sweeps, p.R, p.V, p.sigma, p.order, p.Vk, p.sigma_k, p.info, smem);
}

static hipError_t lds_attr(const void* fn, size_t lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

bool svd_fast_path(int s, int N) { return N <= kFastMaxN && s <= kFastMaxS; }

size_t svd_work_R_bytes(int s, int N) {
  return svd_fast_path(s, N) ? svd_fast_R_bytes(N) : (size_t)N * N * 8;
}

size_t svd_work_log_bytes(int s, int N, int max_sweeps) {
  return svd_fast_path(s, N) ? svd_fast_log_bytes(N, max_sweeps) : 0;
}

hipError_t launch_svd(const SvdPlan& p, hipStream_t st) {
  if (svd_fast_path(p.s, p.N)) {
    const SvdWork w = to_work(p);
    const size_t l1 = svd_fast_lds_bytes(p.s, p.N, kSvdThreads / 64);
    hipError_t e = lds_attr((const void*)svd_qr_kernel, l1);
    if (e == hipSuccess) e = lds_attr((const void*)svd_finish_kernel, l1);
    if (e != hipSuccess) return e;
    svd_qr_kernel<<<1, kSvdThreads, l1, st>>>(w);
    svd_jacobi_kernel<<<1, kJacobiThreads, 0, st>>>(w);
    svd_finish_kernel<<<1, kSvdThreads, l1, st>>>(w);
    return hipGetLastError();
  }
  const size_t lds = svd_lds_bytes(p.s, p.N);
  if (hipError_t e = lds_attr((const void*)svd_kernel, lds)) return e;
  svd_kernel<<<1, kSvdThreads, lds, st>>>(p);
  return hipGetLastError();
}

}  // namespace nsk
