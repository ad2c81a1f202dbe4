// Hashed randomized Hadamard transform (the H-RHT of Section 2): S = Phi (H / sqrt(m_p)) D on
// A zero-padded to m_p rows, Phi a 1-hashing matrix (one +-1 per column).  Every row of the
// transform is hashed, so the whole m_p-point transform is formed (O(m log m) per column, the
// practical cost Section 2 mentions) in two passes over an m_p x N FP64 buffer Y:
//   pass 1 (rht_block_kernel): per 1024-row block j1, the signed rows and the 1024-point
//     transform along them (in-register butterflies, one LDS transpose, in-register
//     butterflies), written to Y in natural row order j1 * 1024 + i2;
//   pass 2 (rht_outer_kernel): per in-block index i2, the B = m_p / 1024 rows j1 * 1024 + i2
//     of a column tile, transformed across j1 in LDS (Sylvester: H_{m_p} = H_B (x) H_1024) and
//     written back in place, scaled by 1 / sqrt(m_p) -- every workgroup owns its rows;
// then the hashing is the sparse-sign sketch with zeta = 1 of Y (its draws over the m_p rows),
// run by the sparse-sign kernels.  For m_p < 1024 the single block's first m_p transformed rows
// are H_{m_p} x, since the higher index bits are zero.
#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "sketch_device.hpp"

namespace nsk {

constexpr int kRhtT = 1024;

static hipError_t rht_lds_limit(const void* fn, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static size_t rht_block_lds_bytes(int cols) { return (size_t)(kRhtT * cols + 64) * 8 + (kRhtT / 32) * 4; }

// Thread (rs, col) of 32 * COLS: rows rs + 32 k (k < 32) of block j1 for the first butterflies,
// rows 32 rs + k after the transpose (the layout of the Hadamard sketch's tile).
template <typename TIn, int COLS>
__global__ __launch_bounds__(32 * COLS) void rht_block_kernel(Operand op, int64_t m, int N, uint64_t seed,
                                                              int64_t B, double* __restrict__ Y) {
  extern __shared__ unsigned char smem[];
  constexpr int RS = 32 * COLS + 2;
  double* tile = reinterpret_cast<double*>(smem);
  uint32_t* signbits = reinterpret_cast<uint32_t*>(tile + kRhtT * COLS + 64);
  const int tiles = (N + COLS - 1) / COLS;
  const int64_t item = xcd_work_item(blockIdx.x, (int64_t)tiles * B);
  if (item < 0) return;
  const int ctile = (int)(item % tiles);
  const int64_t j1 = item / tiles;
  const int t = threadIdx.x, col = t % COLS, rs = t / COLS;
  const int c = ctile * COLS + col;
  const bool live = c < N;
  const TIn* base = nullptr;
  int64_t ld = 0;
  column_ref<TIn>(op, live ? c : 0, base, ld);

  if (t < kRhtT / 128) {
    const Words w = philox(seed, (uint64_t)(j1 * kRhtT >> 7) + t, 0, kSigns);
    *reinterpret_cast<uint4*>(signbits + 4 * t) = make_uint4(w.w[0], w.w[1], w.w[2], w.w[3]);
  }
  double x[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const int64_t r = j1 * kRhtT + rs + 32 * k;
    const TIn v = base[(r < m ? r : 0) * ld];
    x[k] = r < m ? (double)v : 0.0;
  }
  __syncthreads();
  // row rs + 32 k carries bit rs of sign word k
#pragma unroll
  for (int k = 0; k < 32; ++k) x[k] = ((signbits[k] >> rs) & 1u) ? -x[k] : x[k];
#pragma unroll
  for (int h = 1; h < 32; h <<= 1) {
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      if ((k & h) == 0) {
        const double a = x[k], b = x[k + h];
        x[k] = a + b;
        x[k + h] = a - b;
      }
    }
  }
  double* tw = tile + rs * COLS + col;  // row rs + 32 k at tw[k * RS]
#pragma unroll
  for (int k = 0; k < 32; ++k) tw[k * RS] = x[k];
  __syncthreads();
  const double* tr = tile + 32 * rs * COLS + col + rs * 2;  // row 32 rs + k at tr[k * COLS]
#pragma unroll
  for (int k = 0; k < 32; ++k) x[k] = tr[k * COLS];
#pragma unroll
  for (int h = 1; h < 32; h <<= 1) {
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      if ((k & h) == 0) {
        const double a = x[k], b = x[k + h];
        x[k] = a + b;
        x[k + h] = a - b;
      }
    }
  }
  if (live) {
    double* out = Y + (j1 * kRhtT + 32 * rs) * N + c;
#pragma unroll
    for (int k = 0; k < 32; ++k) out[(int64_t)k * N] = x[k];
  }
}

// Workgroup (column tile, i2): the B rows j1 * 1024 + i2 of the tile's columns, transformed
// across j1 by radix-2 butterflies in LDS, written back in place times `scale`.
template <int COLS>
__global__ __launch_bounds__(32 * COLS) void rht_outer_kernel(int N, int64_t B, double scale, double* __restrict__ Y) {
  extern __shared__ unsigned char smem[];
  double* buf = reinterpret_cast<double*>(smem);  // B x COLS
  const int tiles = (N + COLS - 1) / COLS;
  const int64_t item = xcd_work_item(blockIdx.x, (int64_t)tiles * kRhtT);
  if (item < 0) return;
  const int ctile = (int)(item % tiles);
  const int64_t i2 = item / tiles;
  const int t = threadIdx.x, col = t % COLS, rs = t / COLS;
  const int c = ctile * COLS + col;
  const bool live = c < N;
  double* base = Y + i2 * N + (live ? c : 0);
  const int64_t step = (int64_t)kRhtT * N;
  // the rows are 1024 N apart: issue them in groups of kBatch so that their latencies overlap
  constexpr int kBatch = 16;
  for (int64_t j0 = rs; j0 < B; j0 += 32 * kBatch) {
    double v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int64_t j = j0 + 32 * u;
      v[u] = base[(j < B ? j : 0) * step];
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int64_t j = j0 + 32 * u;
      if (j < B) buf[j * COLS + col] = live ? v[u] : 0.0;
    }
  }
  __syncthreads();
  const int half = (int)(B / 2);  // B <= 2048: 32-bit indices; h a power of two (shifts, no division)
  for (int lh = 0; (1 << lh) < B; ++lh) {
    const int h = 1 << lh;
    for (int p = rs; p < half; p += 32) {
      const int j = ((p >> lh) << (lh + 1)) | (p & (h - 1));
      const double a = buf[j * COLS + col], b = buf[(j + h) * COLS + col];
      buf[j * COLS + col] = a + b;
      buf[(j + h) * COLS + col] = a - b;
    }
    __syncthreads();
  }
  if (live)
    for (int64_t j = rs; j < B; j += 32) base[j * step] = buf[j * COLS + col] * scale;
}

// columns per tile of the outer pass: B x COLS doubles in LDS (64 KB at B = 1024: two
// workgroups per CU)
static int rht_outer_cols(int64_t) { return 8; }

hipError_t launch_rht_transform(const Operand& op, int64_t m, int N, uint64_t seed, double* Y, hipStream_t st) {
  const int64_t mp = next_pow2(m);
  const int64_t B = (mp < kRhtT ? kRhtT : mp) / kRhtT;
  constexpr int C1 = 16;
  const size_t l1 = rht_block_lds_bytes(C1);
  const int64_t tiles1 = (N + C1 - 1) / C1;
  const dim3 g1((unsigned)xcd_grid(tiles1 * B));
  if (op.dtype == NSK_F64) {
    if (hipError_t e = rht_lds_limit((const void*)rht_block_kernel<double, C1>, l1)) return e;
    rht_block_kernel<double, C1><<<g1, 32 * C1, l1, st>>>(op, m, N, seed, B, Y);
  } else {
    if (hipError_t e = rht_lds_limit((const void*)rht_block_kernel<float, C1>, l1)) return e;
    rht_block_kernel<float, C1><<<g1, 32 * C1, l1, st>>>(op, m, N, seed, B, Y);
  }
  const double scale = 1.0 / sqrt((double)mp);
  if (rht_outer_cols(B) == 16) {
    const size_t l2 = (size_t)B * 16 * 8;
    const dim3 g2((unsigned)xcd_grid((int64_t)((N + 15) / 16) * kRhtT));
    if (hipError_t e = rht_lds_limit((const void*)rht_outer_kernel<16>, l2)) return e;
    rht_outer_kernel<16><<<g2, 32 * 16, l2, st>>>(N, B, scale, Y);
  } else {
    const size_t l2 = (size_t)B * 8 * 8;
    const dim3 g2((unsigned)xcd_grid((int64_t)((N + 7) / 8) * kRhtT));
    if (hipError_t e = rht_lds_limit((const void*)rht_outer_kernel<8>, l2)) return e;
    rht_outer_kernel<8><<<g2, 32 * 8, l2, st>>>(N, B, scale, Y);
  }
  return hipGetLastError();
}

}  // namespace nsk
