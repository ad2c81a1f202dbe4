// Device-side building blocks of the sketches, shared by the single-instance kernels and
// the batched persistent kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"

namespace nsk {

// ------------------------------------------------------------------------------ helpers
template <typename T> __device__ inline double to_f64(T x) { return (double)x; }

__device__ inline float bf16_round(float x) {
  uint32_t b = __float_as_uint(x);
  b = (b + 0x7FFFu + ((b >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(b);
}

// Round to FP8 E4M3 (OCP, no infinities, max 448) to nearest even, saturating.
__device__ inline float e4m3_round(float x) {
  const float ax = fabsf(x);
  if (ax < 0.015625f) return rintf(x * 512.0f) * (1.0f / 512.0f);
  uint32_t b = __float_as_uint(x);
  b = (b + 0x7FFFFu + ((b >> 20) & 1u)) & 0xFFF00000u;
  const float r = __uint_as_float(b);
  return fminf(fmaxf(r, -448.0f), 448.0f);
}

__device__ inline uint32_t e4m3_bits(float r) {  // r already rounded
  const uint32_t sign = (__float_as_uint(r) >> 24) & 0x80u;
  const float a = fabsf(r);
  if (a < 0.015625f) return sign | (uint32_t)(a * 512.0f);
  const uint32_t b = __float_as_uint(a);
  const uint32_t e = ((b >> 23) & 0xFFu) - 127u + 7u;
  const uint32_t mant = (b >> 20) & 7u;
  return sign | (e << 3) | mant;
}

// Box-Muller on FP32 hardware transcendentals: v_log_f32 is log2, v_sin/cos_f32 take
// their argument in revolutions.  Two words (a, b) give r cos(2 pi v), r sin(2 pi v) with
// u = (a + 1) 2^-32, v = b 2^-32, r = sqrt(-2 ln u).
__device__ inline void box_muller(uint32_t a, uint32_t b, float& g0, float& g1) {
  const float u = fmaf((float)a, 0x1p-32f, 0x1p-32f);
  const float v = (float)b * 0x1p-32f;
  const float r = __builtin_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u));
  g0 = r * __builtin_amdgcn_cosf(v);
  g1 = r * __builtin_amdgcn_sinf(v);
}

// =================================================================================== SRHT
constexpr int kT = 1024;  // rows per transform block

// A workgroup of 32 * COLS threads sketches a tile of COLS columns: thread (rs, col) holds
// rows rs + 32 k (k = 0..31) of its column for phase 1.  A wave covers 64 / COLS rows of COLS
// adjacent columns per load, so wider tiles read longer contiguous pieces of each row.
template <int COLS> struct SrhtTile {
  static_assert(COLS == 8 || COLS == 16, "column tiles of 8 or 16");
  static constexpr int kThreads = 32 * COLS;
};

// SRHT partial sketch of column tile `ctile` (COLS columns) over the row blocks
// j1 = g0, g0 + gstride, ...; the result for the s sampled rows is written to
// out[i * N + c].  Must be called by all 32 * COLS threads of the workgroup.
// smem: at least srht_smem_bytes(s, COLS) bytes.  PF: prefetch the next block's values while
// the current one is transformed (32 more registers a thread).
__host__ __device__ inline size_t srht_smem_bytes(int s, int cols) {
  return (size_t)(kT * cols + 64) * 8 + (kT / 32) * 4 + (size_t)s * 8;
}

template <typename TIn, typename TAcc, int UMAX, int COLS, bool PF = true>
__device__ inline void srht_tile(const Operand& op, int64_t m, int N, int s, uint64_t seed,
                                 const int* __restrict__ rows, int ctile, int64_t g0, int64_t gstride,
                                 TAcc* __restrict__ out, unsigned char* smem) {
  constexpr int NT = SrhtTile<COLS>::kThreads;
  constexpr int RS = 32 * COLS + 2;            // doubles between rows rl and rl + 32 of the tile
  double* tile = reinterpret_cast<double*>(smem);
  uint32_t* signbits = reinterpret_cast<uint32_t*>(tile + kT * COLS + 64);
  int2* srec = reinterpret_cast<int2*>(signbits + kT / 32);  // per sample: tile offset of i2, i1

  const int t = threadIdx.x;
  const int col = t % COLS;
  const int rs = t / COLS;                    // 0..31
  const int c = ctile * COLS + col;
  const bool live = c < N;

  // columns past N read column 0; their sums are never written out
  const TIn* base = nullptr;
  int64_t ld = 0;
  column_ref<TIn>(op, live ? c : 0, base, ld);

  __syncthreads();
  for (int i = t; i < s; i += NT) {
    const int r = rows[i];
    const int i2 = r & (kT - 1);
    srec[i] = make_int2(i2 * COLS + (i2 >> 5) * 2, r >> 10);
  }

  TAcc acc[UMAX];
#pragma unroll
  for (int u = 0; u < UMAX; ++u) acc[u] = 0;

  const int64_t nfull = m / kT;                 // blocks with all kT rows present
  const int64_t nblocks = (m + kT - 1) / kT;
  const TIn* lane0 = base + (int64_t)rs * ld;   // row rs of block 0
  const int64_t kstep = 32 * ld;                // rows rs + 32 k
  auto fetch_full = [&](int64_t j1, TIn (&raw)[32]) {
    const TIn* p = lane0 + j1 * kT * ld;
#pragma unroll
    for (int k = 0; k < 32; ++k) raw[k] = p[k * kstep];
  };

  // One block: signs, the kT-point transform (bits 5..9 in registers, LDS transpose, bits
  // 0..4 in registers) and the sampled outer stage.  raw holds rows rs + 32 k of block j1
  // (zero past m).
  auto block = [&](int64_t j1, const TIn (&raw)[32]) {
    __syncthreads();
    if (t < kT / 128) {
      const Words w = philox(seed, (uint64_t)(j1 * kT >> 7) + t, 0, kSigns);
      *reinterpret_cast<uint4*>(signbits + 4 * t) = make_uint4(w.w[0], w.w[1], w.w[2], w.w[3]);
    }
    __syncthreads();
    // phase 1: row rs + 32 k carries bit rs of sign word k (the same word across the wave)
    TAcc x[32];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint4 w4 = reinterpret_cast<const uint4*>(signbits)[q];
      const uint32_t ws[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 4 * q + e;
        const TAcc v = (TAcc)to_f64(raw[k]);
        x[k] = ((ws[e] >> rs) & 1u) ? -v : v;
      }
    }
#pragma unroll
    for (int h = 1; h < 32; h <<= 1) {
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        if ((k & h) == 0) {
          const TAcc a = x[k], b = x[k + h];
          x[k] = a + b;
          x[k + h] = a - b;
        }
      }
    }
    double* tw = tile + rs * COLS + col;      // row rs + 32 k at tw[k * RS]
#pragma unroll
    for (int k = 0; k < 32; ++k) tw[k * RS] = (double)x[k];
    __syncthreads();
    // phase 2: rows 32 rs + k, butterflies over row bits 0..4; each thread writes back only
    // the cells it read, so no barrier is needed between the read and the write
    double* tr = tile + 32 * rs * COLS + col + rs * 2;  // row 32 rs + k at tr[k * COLS]
#pragma unroll
    for (int k = 0; k < 32; ++k) x[k] = (TAcc)tr[k * COLS];
#pragma unroll
    for (int h = 1; h < 32; h <<= 1) {
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        if ((k & h) == 0) {
          const TAcc a = x[k], b = x[k + h];
          x[k] = a + b;
          x[k + h] = a - b;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) tr[k * COLS] = (double)x[k];
    __syncthreads();
    // sampled outer stage: sample i = rs + 32 u takes row i2 of the block with the sign
    // (-1)^popcount(i1 & j1)
    const uint32_t jlo = (uint32_t)j1;
#pragma unroll
    for (int u = 0; u < UMAX; ++u) {
      const int i = rs + 32 * u;
      if (i < s) {
        const int2 rec = srec[i];
        const TAcc y = (TAcc)tile[rec.x + col];
        acc[u] += (__popc((uint32_t)rec.y & jlo) & 1) ? -y : y;
      }
    }
  };

  // full blocks: the next block's values are in flight while this one is transformed; the
  // prefetch issued with the last full block re-reads that block and is discarded
  if (g0 < nfull) {
    TIn cur[32];
    fetch_full(g0, cur);
    for (int64_t j1 = g0; j1 < nfull; j1 += gstride) {
      if (PF) {
        TIn nxt[32];
        const int64_t jn = j1 + gstride < nfull ? j1 + gstride : j1;
        fetch_full(jn, nxt);
        block(j1, cur);
#pragma unroll
        for (int k = 0; k < 32; ++k) cur[k] = nxt[k];
      } else {
        block(j1, cur);
        if (j1 + gstride < nfull) fetch_full(j1 + gstride, cur);
      }
    }
  }
  // the partial last block, if this tile's blocks include it: rows past m read as zero
  if (nblocks > nfull && (nfull - g0) % gstride == 0 && nfull >= g0) {
    TIn raw[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int64_t row = nfull * kT + rs + 32 * k;
      const TIn v = base[(row < m ? row : m - 1) * ld];
      raw[k] = row < m ? v : (TIn)0;
    }
    block(nfull, raw);
  }
  if (live) {
#pragma unroll
    for (int u = 0; u < UMAX; ++u) {
      const int i = rs + 32 * u;
      if (i < s) out[(size_t)i * N + c] = acc[u];
    }
  }
}

template <typename TIn, typename TAcc, int UMAX, int COLS>
__global__ __launch_bounds__(SrhtTile<COLS>::kThreads) void srht_kernel(Operand op, int64_t m, int N, int s,
                                                                         uint64_t seed, const int* __restrict__ rows,
                                                                         int groups, TAcc* __restrict__ partial) {
  extern __shared__ unsigned char smem[];
  const int tiles = (N + COLS - 1) / COLS;
  const int64_t item = xcd_work_item(blockIdx.x, (int64_t)tiles * groups);
  if (item < 0) return;
  const int tile = (int)(item % tiles), g = (int)(item / tiles);
  srht_tile<TIn, TAcc, UMAX, COLS>(op, m, N, s, seed, rows, tile, g, groups, partial + (size_t)g * s * N, smem);
}

}  // namespace nsk
