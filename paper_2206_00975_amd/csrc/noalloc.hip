// Allocation-free variant of nsk_trailing_rsv for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops): the workspace is a fixed array in
// device memory that the library's code object carries, one copy per GPU, instead of a
// caller buffer.  Same kernels and launch sequence as nsk_trailing_rsv.
#include <hip/hip_runtime.h>

#include <mutex>

#include "nsk.h"

namespace {

constexpr size_t kScratchBytes = (size_t)96 << 20;
constexpr int kMaxDevices = 64;

// The workspace of nsk_trailing_rsv_noalloc on each GPU that runs it, held until the process
// ends.  Host code must never pass `scratch` itself to a kernel or a copy: its device address
// comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchAddr {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
ScratchAddr g_addr[kMaxDevices];

// Device address of the current GPU's copy of `scratch` (nullptr on failure), looked up once
// per device with that device current.
void* scratch_ptr() {
  int device = -1;
  if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= kMaxDevices) return nullptr;
  ScratchAddr& a = g_addr[device];
  std::call_once(a.once, [&a] {
    void* p = nullptr;
    a.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    a.ptr = a.err == hipSuccess ? p : nullptr;
  });
  return a.ptr;
}

}  // namespace

extern "C" {

size_t nsk_noalloc_scratch_bytes(void) { return kScratchBytes; }

int nsk_trailing_rsv_noalloc(const nsk_operand* blocks, int32_t nblocks, int64_t m, int64_t k, const nsk_desc* d,
                             double* Vk, double* sigma_k, nsk_info* info, void* stream) {
  if (!blocks || nblocks < 1 || !d) return NSK_EINVAL;
  int64_t N = 0;
  for (int b = 0; b < nblocks; ++b) N += blocks[b].cols;
  const size_t need = nsk_workspace_bytes(m, N, k, d);
  if (need == 0) return NSK_EINVAL;
  if (need > kScratchBytes) return NSK_EWORKSPACE;
  void* ws = scratch_ptr();
  if (!ws) return NSK_EDEVICE;
  return nsk_trailing_rsv(blocks, nblocks, m, k, d, Vk, sigma_k, info, ws, kScratchBytes, stream);
}

}  // extern "C"
