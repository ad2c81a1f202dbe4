// Hashed randomized Hadamard transform (the H-RHT of Section 2): S = Phi (H / sqrt(m_p)) D on
// A zero-padded to m_p rows, Phi a 1-hashing matrix (one +-1 per column).  Every row of the
// transform is hashed, so the whole m_p-point transform is formed (O(m log m) per column, the
// practical cost Section 2 mentions):
//   rht_hash_table_kernel: per transformed row r, its hashed row and sign in one word (the
//     sparse-sign draw with zeta = 1 at index r);
//   rht_block_kernel: per 1024-row block j1, the signed rows and the 1024-point transform along
//     them (in-register butterflies, one LDS transpose, in-register butterflies), written to an
//     FP64 buffer Y in natural row order j1 * 1024 + i2;
//   rht_hash_kernel: a workgroup owns a column tile and a range of in-block indices i2; for each
//     it reads the B = m_p / 1024 rows j1 * 1024 + i2 of its columns, transforms them across j1
//     in LDS (Sylvester: H_{m_p} = H_B (x) H_1024), scales by 1 / sqrt(m_p) and adds every row
//     r = j1 * 1024 + i2 with its sign into row h(r) of an s x COLS accumulator in LDS; the
//     accumulator is its partial sketch, summed in a fixed order by the reduce.
// The transformed rows never return to HBM.  For m_p < 1024 the single block's first m_p
// transformed rows are H_{m_p} x (the higher index bits are zero); the rest are not hashed.
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
  extern __shared__ __align__(16) unsigned char smem[];
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

// one word per transformed row r < m_p: the hashed row in bits 0..30, the sign in bit 31
__global__ __launch_bounds__(256) void rht_hash_table_kernel(uint64_t seed, int64_t mp, int s,
                                                             uint32_t* __restrict__ hash) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= mp) return;
  int h[1];
  uint32_t neg;
  sparse_column<1>(seed, (uint64_t)r, s, 1, h, neg);
  hash[r] = (uint32_t)h[0] | ((neg & 1u) << 31);
}

// Thread (rs, col) of 32 * COLS.  LDS: the B x COLS block of the current i2, then the s x COLS
// accumulator.
template <int COLS>
__global__ __launch_bounds__(32 * COLS) void rht_hash_kernel(int N, int64_t B, int64_t mp, int s, double scale,
                                                             const double* __restrict__ Y,
                                                             const uint32_t* __restrict__ hash, int groups,
                                                             double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* buf = reinterpret_cast<double*>(smem);  // B x COLS
  double* acc = buf + B * COLS;                   // s x COLS
  const int tiles = (N + COLS - 1) / COLS;
  const int64_t item = xcd_work_item(blockIdx.x, (int64_t)tiles * groups);
  if (item < 0) return;
  const int ctile = (int)(item % tiles), g = (int)(item / tiles);
  const int t = threadIdx.x, col = t % COLS, rs = t / COLS;
  const int c = ctile * COLS + col;
  const bool live = c < N;
  for (int e = t; e < s * COLS; e += 32 * COLS) acc[e] = 0.0;
  const int per = (kRhtT + groups - 1) / groups;
  const int i2b = g * per < kRhtT ? g * per : kRhtT;
  const int i2e = i2b + per < kRhtT ? i2b + per : kRhtT;
  const int64_t step = (int64_t)kRhtT * N;
  const int half = (int)(B / 2);  // B <= 2048: 32-bit indices; h a power of two (shifts, no division)
  constexpr int kBatch = 16;      // rows 1024 N apart: issue them in groups so their latencies overlap
  for (int i2 = i2b; i2 < i2e; ++i2) {
    const double* base = Y + (int64_t)i2 * N + (live ? c : 0);
    __syncthreads();  // the accumulator is cleared / the previous i2's block is hashed
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
    if (live) {
      for (int64_t j = rs; j < B; j += 32) {
        const int64_t r = j * kRhtT + i2;
        if (r < mp) {
          const uint32_t hw = hash[r];
          const double y = buf[j * COLS + col] * scale;
          atomicAdd(&acc[(int)(hw & 0x7FFFFFFFu) * COLS + col], (hw >> 31) ? -y : y);
        }
      }
    }
  }
  __syncthreads();
  if (live) {
    double* out = partial + (size_t)g * s * N + c;
    for (int i = rs; i < s; i += 32) out[(size_t)i * N] = acc[i * COLS + col];
  }
}

// B = 1024 (m_p = 2^20): the block pass's layout across blocks -- thread (rs, col) holds rows
// j1 = rs + 32 k of the current i2 in registers, butterflies over k, one LDS transpose, then
// butterflies over the low bits of j1 = 32 rs + k and the hashing straight from registers; the
// next i2's 32 values are in flight meanwhile.  Two barriers per i2.  LDS: the transposed block
// (1024 x 8 + 64 doubles), then the s x 8 accumulator.
constexpr int kRhtRegCols = 8;
static size_t rht_reg_lds_bytes(int s) { return (size_t)(kRhtT * kRhtRegCols + 64 + s * kRhtRegCols) * 8; }

__global__ __launch_bounds__(32 * kRhtRegCols) void rht_hash_reg_kernel(int N, int64_t mp, int s, double scale,
                                                                        const double* __restrict__ Y,
                                                                        const uint32_t* __restrict__ hash,
                                                                        int groups, double* __restrict__ partial) {
  constexpr int COLS = kRhtRegCols, RS = 32 * COLS + 2;
  extern __shared__ __align__(16) unsigned char smem[];
  double* tile = reinterpret_cast<double*>(smem);
  double* acc = tile + kRhtT * COLS + 64;
  const int tiles = (N + COLS - 1) / COLS;
  const int64_t item = xcd_work_item(blockIdx.x, (int64_t)tiles * groups);
  if (item < 0) return;
  const int ctile = (int)(item % tiles), g = (int)(item / tiles);
  const int t = threadIdx.x, col = t % COLS, rs = t / COLS;
  const int c = ctile * COLS + col;
  const bool live = c < N;
  for (int e = t; e < s * COLS; e += 32 * COLS) acc[e] = 0.0;
  const int per = (kRhtT + groups - 1) / groups;
  const int i2b = g * per < kRhtT ? g * per : kRhtT;
  const int i2e = i2b + per < kRhtT ? i2b + per : kRhtT;
  const int64_t step = (int64_t)kRhtT * N;
  const double* lane0 = Y + (int64_t)rs * step + (live ? c : 0);  // row (rs + 32 k) * 1024 + i2
  double* tw = tile + rs * COLS + col;
  const double* tr = tile + 32 * rs * COLS + col + rs * 2;
  auto fetch = [&](int i2, double (&v)[32]) {
#pragma unroll
    for (int k = 0; k < 32; ++k) v[k] = lane0[(int64_t)(32 * k) * step + i2 * N];
  };
  double cur[32];
  if (i2b < i2e) fetch(i2b, cur);
  for (int i2 = i2b; i2 < i2e; ++i2) {
    double nxt[32];
    fetch(i2 + 1 < i2e ? i2 + 1 : i2, nxt);
#pragma unroll
    for (int h = 1; h < 32; h <<= 1) {
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        if ((k & h) == 0) {
          const double a = cur[k], b = cur[k + h];
          cur[k] = a + b;
          cur[k + h] = a - b;
        }
      }
    }
    __syncthreads();  // the previous i2's transposed block has been read
#pragma unroll
    for (int k = 0; k < 32; ++k) tw[k * RS] = cur[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 32; ++k) cur[k] = tr[k * COLS];
#pragma unroll
    for (int h = 1; h < 32; h <<= 1) {
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        if ((k & h) == 0) {
          const double a = cur[k], b = cur[k + h];
          cur[k] = a + b;
          cur[k + h] = a - b;
        }
      }
    }
    if (live) {
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        const int64_t r = (int64_t)(32 * rs + k) * kRhtT + i2;  // j1 = 32 rs + k < 1024 = B: r < m_p
        const uint32_t hw = hash[r];
        const double y = cur[k] * scale;
        atomicAdd(&acc[(int)(hw & 0x7FFFFFFFu) * COLS + col], (hw >> 31) ? -y : y);
      }
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) cur[k] = nxt[k];
  }
  __syncthreads();
  if (live) {
    double* out = partial + (size_t)g * s * N + c;
    for (int i = rs; i < s; i += 32) out[(size_t)i * N] = acc[i * COLS + col];
  }
}

static size_t rht_hash_lds_bytes(int64_t B, int s, int cols) { return (size_t)(B + s) * cols * 8; }

hipError_t launch_rht(const Operand& op, const SketchPlan& p, uint32_t* hash, double* Y, hipStream_t st) {
  const int64_t mp = next_pow2(p.m);
  const int64_t B = (mp < kRhtT ? kRhtT : mp) / kRhtT;
  rht_hash_table_kernel<<<(unsigned)((mp + 255) / 256), 256, 0, st>>>(p.seed, mp, p.s, hash);
  prof_mark(0, st);
  constexpr int C1 = 16;
  const size_t l1 = rht_block_lds_bytes(C1);
  const dim3 g1((unsigned)xcd_grid((int64_t)((p.N + C1 - 1) / C1) * B));
  if (op.dtype == NSK_F64) {
    if (hipError_t e = rht_lds_limit((const void*)rht_block_kernel<double, C1>, l1)) return e;
    rht_block_kernel<double, C1><<<g1, 32 * C1, l1, st>>>(op, p.m, p.N, p.seed, B, Y);
  } else {
    if (hipError_t e = rht_lds_limit((const void*)rht_block_kernel<float, C1>, l1)) return e;
    rht_block_kernel<float, C1><<<g1, 32 * C1, l1, st>>>(op, p.m, p.N, p.seed, B, Y);
  }
  const double scale = 1.0 / sqrt((double)mp);
  double* part = static_cast<double*>(p.partial);
  const int cols = rht_hash_cols(p.m, p.s);
  if (cols == kRhtRegCols && B == kRhtT) {
    const size_t l2 = rht_reg_lds_bytes(p.s);
    const dim3 g2((unsigned)xcd_grid((int64_t)((p.N + kRhtRegCols - 1) / kRhtRegCols) * p.groups));
    if (hipError_t e = rht_lds_limit((const void*)rht_hash_reg_kernel, l2)) return e;
    rht_hash_reg_kernel<<<g2, 32 * kRhtRegCols, l2, st>>>(p.N, mp, p.s, scale, Y, hash, p.groups, part);
    return hipGetLastError();
  }
  const size_t l2 = rht_hash_lds_bytes(B, p.s, cols);
  const dim3 g2((unsigned)xcd_grid((int64_t)((p.N + cols - 1) / cols) * p.groups));
#define NSK_RHT_CASE(C)                                                                                   \
  {                                                                                                       \
    if (hipError_t e = rht_lds_limit((const void*)rht_hash_kernel<C>, l2)) return e;                      \
    rht_hash_kernel<C><<<g2, 32 * C, l2, st>>>(p.N, B, mp, p.s, scale, Y, hash, p.groups, part);          \
  }
  if (cols == 8) NSK_RHT_CASE(8)
  else if (cols == 4) NSK_RHT_CASE(4)
  else NSK_RHT_CASE(2)
#undef NSK_RHT_CASE
  return hipGetLastError();
}

}  // namespace nsk
