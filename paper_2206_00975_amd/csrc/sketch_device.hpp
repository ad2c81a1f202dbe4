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
constexpr int kT = 1024;       // rows per transform block
constexpr int kSrhtCols = 8;   // columns per workgroup
constexpr int kSrhtThreads = 256;

// SRHT partial sketch of column tile `ctile` (kSrhtCols columns) over the row blocks
// j1 = g0, g0 + gstride, ...; the result for the s sampled rows is written to
// out[i * N + c].  Must be called by all kSrhtThreads threads of the workgroup.
// smem: at least srht_smem_bytes(s) bytes.
__host__ __device__ inline size_t srht_smem_bytes(int s) {
  return (size_t)(kT * kSrhtCols + 64) * 8 + (kT / 32) * 4 + (size_t)((s + 1) & ~1) * 4;
}

template <typename TIn, typename TAcc, int UMAX>
__device__ inline void srht_tile(const Operand& op, int64_t m, int N, int s, uint64_t seed,
                                 const int* __restrict__ rows, int ctile, int64_t g0, int64_t gstride,
                                 TAcc* __restrict__ out, unsigned char* smem) {
  double* tile = reinterpret_cast<double*>(smem);
  uint32_t* signbits = reinterpret_cast<uint32_t*>(tile + kT * kSrhtCols + 64);
  int* srow = reinterpret_cast<int*>(signbits + kT / 32);

  const int t = threadIdx.x;
  const int col = t & (kSrhtCols - 1);
  const int rs = t >> 3;                      // 0..31
  const int c = ctile * kSrhtCols + col;
  const bool live = c < N;

  // dead columns read column 0 and are masked after the load (no branch around the loads)
  const TIn* base = nullptr;
  int64_t ld = 0;
  column_ref<TIn>(op, live ? c : 0, base, ld);

  __syncthreads();
  for (int i = t; i < s; i += kSrhtThreads) srow[i] = rows[i];

  TAcc acc[UMAX];
#pragma unroll
  for (int u = 0; u < UMAX; ++u) acc[u] = 0;

  const int64_t nblocks = (m + kT - 1) / kT;
  for (int64_t j1 = g0; j1 < nblocks; j1 += gstride) {
    const int64_t r0 = j1 * kT;
    __syncthreads();
    if (t < kT / 128) {
      const Words w = philox(seed, (uint64_t)(r0 >> 7) + t, 0, kSigns);
#pragma unroll
      for (int q = 0; q < 4; ++q) signbits[t * 4 + q] = w.w[q];
    }
    __syncthreads();
    // phase 1: rows rs + 32k, butterflies over row bits 5..9 (bits of k)
    TAcc x[32];
    TIn raw[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int64_t row = r0 + rs + 32 * k;
      raw[k] = base[(row < m ? row : r0) * ld];
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int rl = rs + 32 * k;
      const TAcc v = live && r0 + rl < m ? (TAcc)to_f64(raw[k]) : (TAcc)0;
      const bool neg = (signbits[rl >> 5] >> (rl & 31)) & 1u;
      x[k] = neg ? -v : v;
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
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int rl = rs + 32 * k;
      tile[rl * kSrhtCols + col + (rl >> 5) * 2] = (double)x[k];
    }
    __syncthreads();
    // phase 2: rows 32 rs + k, butterflies over row bits 0..4
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int rl = 32 * rs + k;
      x[k] = (TAcc)tile[rl * kSrhtCols + col + rs * 2];
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
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int rl = 32 * rs + k;
      tile[rl * kSrhtCols + col + rs * 2] = (double)x[k];
    }
    __syncthreads();
    // sampled outer stage: sample i = rs + 32u takes signed row i2 of the block
#pragma unroll
    for (int u = 0; u < UMAX; ++u) {
      const int i = rs + 32 * u;
      if (i < s) {
        const int r = srow[i];
        const int i2 = r & (kT - 1);
        const int64_t i1 = (int64_t)r >> 10;
        const TAcc y = (TAcc)tile[i2 * kSrhtCols + col + (i2 >> 5) * 2];
        const bool neg = __popcll((uint64_t)(i1 & j1)) & 1;
        acc[u] += neg ? -y : y;
      }
    }
  }
  if (live) {
#pragma unroll
    for (int u = 0; u < UMAX; ++u) {
      const int i = rs + 32 * u;
      if (i < s) out[(size_t)i * N + c] = acc[u];
    }
  }
}

template <typename TIn, typename TAcc, int UMAX>
__global__ __launch_bounds__(kSrhtThreads) void srht_kernel(Operand op, int64_t m, int N, int s,
                                                            uint64_t seed, const int* __restrict__ rows,
                                                            int groups, TAcc* __restrict__ partial) {
  extern __shared__ unsigned char smem[];
  const int tiles = (N + kSrhtCols - 1) / kSrhtCols;
  const int64_t item = xcd_work_item(blockIdx.x, (int64_t)tiles * groups);
  if (item < 0) return;
  const int tile = (int)(item % tiles), g = (int)(item / tiles);
  srht_tile<TIn, TAcc, UMAX>(op, m, N, s, seed, rows, tile, g, groups, partial + (size_t)g * s * N, smem);
}

}  // namespace nsk
