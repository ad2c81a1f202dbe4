// Batched Algorithm 1: many independent, unevenly sized instances in one persistent launch.
//
// The host lists every SRHT sketch tile (instance, column tile, row group) with the tiles
// of the instances with the most expensive SVD first.  Each workgroup repeatedly takes the
// next tile from a global counter, computes its partial sketch, and increments its
// instance's completion counter (release at device scope).  The workgroup that completes
// the last tile of an instance (acquire at device scope) sums that instance's partials in a
// fixed order and runs its QR + one-sided Jacobi in place, so SVDs of finished instances
// overlap with the sketches of the others and no device-wide barrier is needed.  The grid
// drains when the tile counter passes the end of the list.
#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "sketch_device.hpp"
#include "svd_device.hpp"
#include "svd_pipeline.hpp"

namespace nsk {

struct BatchInst {
  Operand op;
  int64_t m;
  int N, s, k, groups, ctiles, tiles, max_sweeps, pad;
  uint64_t seed;
  const int* rows;
  void* partial;      // groups x s x N (TAcc)
  double* sa_cm;      // s x N column-major
  double* R;          // fast-path R buffer
  double2* log;       // rotation log
  double* sigma;
  int* order;
  double* colnorm;
  JacobiResult* jres;
  double* Vk;
  double* sigma_k;
  nsk_info* info;
};

struct BatchTile {
  int inst, ctile, g, pad;
};

__global__ void batched_reset(int* counters, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) counters[i] = 0;
}

// Every instance's row sample, one workgroup per instance.
__global__ __launch_bounds__(kFloydThreads) void batched_rows_kernel(const BatchInst* __restrict__ insts) {
  __shared__ __align__(16) unsigned char smem[floyd_smem_bytes()];
  const BatchInst& I = insts[blockIdx.x];
  floyd_rows_block(I.seed, next_pow2(I.m), I.s, const_cast<int*>(I.rows), smem);
}

constexpr int kBatchThreads = SrhtTile<kBatchCols>::kThreads;

template <typename TIn, typename TAcc>
__global__ __launch_bounds__(kBatchThreads) void batched_kernel(const BatchInst* __restrict__ insts,
                                                               const BatchTile* __restrict__ tiles, int ntiles,
                                                               int* __restrict__ counters) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sh_task;
  __shared__ int sh_last;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) sh_task = atomicAdd(&counters[0], 1);
    __syncthreads();
    const int task = sh_task;
    __syncthreads();
    if (task >= ntiles) break;
    const BatchTile tile = tiles[task];
    const BatchInst& I = insts[tile.inst];
    TAcc* part = static_cast<TAcc*>(I.partial) + (size_t)tile.g * I.s * I.N;
    if (I.s <= 256)
      srht_tile<TIn, TAcc, 8, kBatchCols, true>(I.op, I.m, I.N, I.s, I.seed, I.rows, tile.ctile, tile.g, I.groups, part, smem);
    else if (I.s <= 512)
      srht_tile<TIn, TAcc, 16, kBatchCols, true>(I.op, I.m, I.N, I.s, I.seed, I.rows, tile.ctile, tile.g, I.groups, part, smem);
    else
      srht_tile<TIn, TAcc, 32, kBatchCols, false>(I.op, I.m, I.N, I.s, I.seed, I.rows, tile.ctile, tile.g, I.groups, part, smem);
    // every wave's partial stores complete before the barrier: thread 0's release below waits
    // only for its own wave's stores, and the workgroup barrier does not wait for stores
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      const int prev = __hip_atomic_fetch_add(&counters[1 + tile.inst], 1, __ATOMIC_ACQ_REL,
                                              __HIP_MEMORY_SCOPE_AGENT);
      sh_last = prev == I.tiles - 1;
    }
    __syncthreads();
    if (sh_last) {
      const double scale = 1.0 / sqrt((double)I.s);
      const TAcc* pp = static_cast<const TAcc*>(I.partial);
      const size_t sn = (size_t)I.s * I.N;
      for (size_t e = tid; e < sn; e += blockDim.x) {
        double a = 0;
        for (int g = 0; g < I.groups; ++g) a += (double)pp[(size_t)g * sn + e];
        const int i = (int)(e / I.N), c = (int)(e % I.N);
        I.sa_cm[(size_t)c * I.s + i] = a * scale;
      }
      __syncthreads();
      SvdWork w;
      w.sa = I.sa_cm;
      w.R = I.R;
      w.log = I.log;
      w.sigma = I.sigma;
      w.order = I.order;
      w.colnorm = I.colnorm;
      w.jres = I.jres;
      w.Vk = I.Vk;
      w.sigma_k = I.sigma_k;
      w.info = I.info;
      w.s = I.s;
      w.N = I.N;
      w.k = I.k;
      w.max_sweeps = I.max_sweeps;
      w.coop_local = 0;
      w.coop_stride = 1;
      svd_pipeline(w, smem);
    }
    __syncthreads();
  }
}

size_t batched_lds_bytes(int s_max, int n_max) {
  const size_t a = srht_smem_bytes(s_max, kBatchCols), b = svd_fast_lds_bytes(s_max, n_max, kBatchThreads / 64);
  return a > b ? a : b;
}

// counters: the tile counter followed by one completion counter per instance (count + 1).
hipError_t launch_batched(const void* insts, int count, const void* tiles, int ntiles, int* counters, int dtype,
                          int acc, int grid, size_t lds, hipStream_t st) {
  const int ncounters = count + 1;
  batched_reset<<<(ncounters + 255) / 256, 256, 0, st>>>(counters, ncounters);
  const BatchInst* I = static_cast<const BatchInst*>(insts);
  batched_rows_kernel<<<count, kFloydThreads, 0, st>>>(I);
  const BatchTile* T = static_cast<const BatchTile*>(tiles);
#define NSK_BATCH(TI, TA)                                                                           \
  {                                                                                                 \
    if (lds > 64 * 1024) {                                                                          \
      const hipError_t e = hipFuncSetAttribute((const void*)batched_kernel<TI, TA>,                 \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
      if (e != hipSuccess) return e;                                                                \
    }                                                                                               \
    batched_kernel<TI, TA><<<grid, kBatchThreads, lds, st>>>(I, T, ntiles, counters);                \
  }
  if (dtype == NSK_F64) {
    if (acc == NSK_F64) NSK_BATCH(double, double) else NSK_BATCH(double, float)
  } else {
    if (acc == NSK_F64) NSK_BATCH(float, double) else NSK_BATCH(float, float)
  }
#undef NSK_BATCH
  return hipGetLastError();
}

size_t batch_inst_bytes() { return sizeof(BatchInst); }
size_t batch_tile_bytes() { return sizeof(BatchTile); }

// Fill one instance record (host side); layout private to this file.
void batch_fill_inst(void* dst, const Operand& op, int64_t m, int N, int s, int k, int groups, int ctiles,
                     int max_sweeps, uint64_t seed, const int* rows, void* partial, double* sa_cm, double* R,
                     double2* log, double* sigma, int* order, double* colnorm, void* jres, double* Vk,
                     double* sigma_k, nsk_info* info) {
  BatchInst b;
  b.op = op;
  b.m = m;
  b.N = N;
  b.s = s;
  b.k = k;
  b.groups = groups;
  b.ctiles = ctiles;
  b.tiles = groups * ctiles;
  b.max_sweeps = max_sweeps;
  b.pad = 0;
  b.seed = seed;
  b.rows = rows;
  b.partial = partial;
  b.sa_cm = sa_cm;
  b.R = R;
  b.log = log;
  b.sigma = sigma;
  b.order = order;
  b.colnorm = colnorm;
  b.jres = static_cast<JacobiResult*>(jres);
  b.Vk = Vk;
  b.sigma_k = sigma_k;
  b.info = info;
  *static_cast<BatchInst*>(dst) = b;
}

void batch_fill_tile(void* dst, int inst, int ctile, int g) {
  BatchTile t{inst, ctile, g, 0};
  *static_cast<BatchTile*>(dst) = t;
}

}  // namespace nsk
