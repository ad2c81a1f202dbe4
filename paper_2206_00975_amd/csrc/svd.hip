// Single-instance SVD launch: one workgroup runs svd_instance (QR + one-sided Jacobi).
#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "svd_device.hpp"

namespace nsk {

constexpr int kSvdThreads = 1024;

__global__ __launch_bounds__(kSvdThreads) void svd_kernel(SvdPlan p) {
  extern __shared__ unsigned char smem[];
  svd_instance(p.sa, p.s, p.N, p.k, p.max_sweeps, p.R, p.V, p.sigma, p.order, p.Vk, p.sigma_k, p.info, smem);
}

hipError_t launch_svd(const SvdPlan& p, hipStream_t st) {
  const size_t lds = svd_lds_bytes(p.s, p.N);
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute((const void*)svd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  svd_kernel<<<1, kSvdThreads, lds, st>>>(p);
  return hipGetLastError();
}

}  // namespace nsk
