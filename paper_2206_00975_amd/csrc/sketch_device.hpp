// Device-side building blocks of the sketches, shared by the single-instance kernels and
// the batched persistent kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "wave_ops.hpp"

namespace nsk {

// ------------------------------------------------------------------------------ helpers
template <typename T> __device__ inline double to_f64(T x) { return (double)x; }

// x with its sign bit flipped by bit 31 of `sign` (the other bits of `sign` are ignored).
__device__ inline double flip_sign(double x, uint32_t sign) {
  return __hiloint2double(__double2hiint(x) ^ (int)(sign & 0x80000000u), __double2loint(x));
}
__device__ inline float flip_sign(float x, uint32_t sign) {
  return __uint_as_float(__float_as_uint(x) ^ (sign & 0x80000000u));
}

__device__ inline float bf16_round(float x) {
  uint32_t b = __float_as_uint(x);
  b = (b + 0x7FFFu + ((b >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(b);
}

// Round to FP8 E4M3 (OCP, no infinities, max 448) to nearest even, saturating.
// Both forms are evaluated and selected, here and in e4m3_bits: an early return becomes a
// divergent branch.
__device__ inline float e4m3_round(float x) {
  const float ax = fabsf(x);
  const float sub = rintf(x * 512.0f) * (1.0f / 512.0f);
  uint32_t b = __float_as_uint(x);
  b = (b + 0x7FFFFu + ((b >> 20) & 1u)) & 0xFFF00000u;
  const float r = fminf(fmaxf(__uint_as_float(b), -448.0f), 448.0f);
  return ax < 0.015625f ? sub : r;
}

__device__ inline uint32_t e4m3_bits(float r) {  // r already rounded
  const uint32_t sign = (__float_as_uint(r) >> 24) & 0x80u;
  const float a = fabsf(r);
  const uint32_t sub = sign | (uint32_t)(a * 512.0f);
  const uint32_t b = __float_as_uint(a);
  const uint32_t e = ((b >> 23) & 0xFFu) - 127u + 7u;  // wraps below 2^-6, where sub is taken
  const uint32_t mant = (b >> 20) & 7u;
  const uint32_t normal = sign | (e << 3) | mant;
  return a < 0.015625f ? sub : normal;
}

// Round an FP64 value to bfloat16 (8 significant bits) and to E4M3 (4 significant bits, quantum
// 2^-9 below 2^-6, saturating at 448), to nearest even, directly from FP64.
__device__ inline float bf16_round_f64(double x) {
  uint64_t b = (uint64_t)__double_as_longlong(x);
  b = (b + 0x00000FFFFFFFFFFFull + ((b >> 45) & 1u)) & 0xFFFFE00000000000ull;
  return (float)__longlong_as_double((long long)b);
}
__device__ inline float e4m3_round_f64(double x) {
  if (fabs(x) < 0x1p-6) return (float)(rint(x * 512.0) * (1.0 / 512.0));
  uint64_t b = (uint64_t)__double_as_longlong(x);
  b = (b + 0x0000FFFFFFFFFFFFull + ((b >> 49) & 1u)) & 0xFFFE000000000000ull;
  return fminf(fmaxf((float)__longlong_as_double((long long)b), -448.0f), 448.0f);
}

// Box-Muller from two 32-bit words (a, b): u = (a + 1) 2^-32, v = b 2^-32, r = sqrt(-2 ln u),
// (g0, g1) = (r cos 2 pi v, r sin 2 pi v).  FP32 evaluation on the hardware transcendentals
// (v_log_f32 is log2, v_sin/cos_f32 take revolutions):
//  * for u <= 1/2, log2 of u itself; for u > 1/2, 1 - u = (~a) 2^-32 exactly and
//    ln(1 - x) = ln(w) x / (w - 1) with w = fl(1 - x) (the log1p identity), so that radii of
//    u near 1 keep their relative accuracy;
//  * the angle as the signed revolution (int32) b 2^-32 in [-1/2, 1/2), the same point of the
//    circle, where the hardware sine and cosine are most accurate.
// Measured over all 2^32 values of each word on gfx950: radius relative error <= 1.9e-7,
// sine and cosine absolute error <= 1.9e-7.
struct GaussPair { float g0, g1, r; };
__device__ inline GaussPair box_muller32(uint32_t a, uint32_t b) {
  // both branches evaluated and selected (one logarithm a pair); the identity's ratio
  // x / (1 - w) takes the reciprocal estimate and one Newton step
  const bool low = a < 0x80000000u;
  const float u = fmaf((float)a, 0x1p-32f, 0x1p-32f);
  const float x = (float)(~a) * 0x1p-32f;
  const float w = 1.0f - x;
  const float dw = 1.0f - w;
  float rc = __builtin_amdgcn_rcpf(dw);
  rc = fmaf(rc, fmaf(-dw, rc, 1.0f), rc);
  const float lg = __builtin_amdgcn_logf(low ? u : w);
  const float tiny = -x * 1.4426950408889634f;
  const float ident = lg * (x * rc);
  const float upper = w == 1.0f ? tiny : ident;
  const float l2 = low ? lg : upper;
  const float r = __builtin_sqrtf(-1.3862943611198906f * l2);
  const float v = (float)(int32_t)b * 0x1p-32f;
  return GaussPair{r * __builtin_amdgcn_cosf(v), r * __builtin_amdgcn_sinf(v), r};
}

__device__ inline void box_muller(uint32_t a, uint32_t b, float& g0, float& g1) {
  const GaussPair p = box_muller32(a, b);
  g0 = p.g0;
  g1 = p.g1;
}

// Entry h (0 or 1) of the pair in FP64, the formulas of the definition evaluated in FP64
// (u and v exact).
__device__ inline double box_muller64(uint32_t a, uint32_t b, int h) {
  const double u = ((double)a + 1.0) * 0x1p-32, v = (double)b * 0x1p-32;
  const double r = sqrt(-2.0 * log(u));
  const double ang = 6.283185307179586 * v;
  return h ? r * sin(ang) : r * cos(ang);
}

// Rounded Gaussian entries G_hat (FMT: NSK_BF16 or NSK_F8E4M3) of one Philox block: words
// (0, 1) give entries 0, 1 and words (2, 3) entries 2, 3.  The FP32 value g is within
// E = 2^-21 (|g| + r) of the exact Gaussian (about twice the measured bounds); when g - E and
// g + E round to the same narrow value, rounding is monotone, so the exact value rounds to it
// as well.  Otherwise (a rounding tie within E, rare) the entry is recomputed in FP64 and
// rounded from FP64: the rounding decision is then the one taken on the FP64 value.
template <int FMT> __device__ inline float round_fmt(float x) {
  if constexpr (FMT == NSK_BF16) return bf16_round(x); else return e4m3_round(x);
}
template <int FMT> __device__ inline float round_fmt64(double x) {
  if constexpr (FMT == NSK_BF16) return bf16_round_f64(x); else return e4m3_round_f64(x);
}
// The FP32 part alone: out[h] rounded from the FP32 value, and bit h of the returned mask set
// when that rounding is not certified (the entry must then be taken from gauss_hat64).
template <int FMT> __device__ inline unsigned gauss_hat4_fast(const Words& w, float (&out)[4]) {
  unsigned doubt = 0;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const GaussPair g = box_muller32(w.w[2 * p], w.w[2 * p + 1]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float x = h ? g.g1 : g.g0;
      const float e = 0x1p-21f * (fabsf(x) + g.r);
      doubt |= (round_fmt<FMT>(x - e) != round_fmt<FMT>(x + e) ? 1u : 0u) << (2 * p + h);
      out[2 * p + h] = round_fmt<FMT>(x);
    }
  }
  return doubt;
}
// Entry h (0..3) of a block, rounded from its FP64 Box-Muller value.
template <int FMT> __device__ inline float gauss_hat64(const Words& w, int h) {
  const uint32_t a = h < 2 ? w.w[0] : w.w[2], b = h < 2 ? w.w[1] : w.w[3];
  return round_fmt64<FMT>(box_muller64(a, b, h & 1));
}

template <int FMT> __device__ inline void gauss_hat4(const Words& w, float (&out)[4]) {
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const uint32_t a = w.w[2 * p], b = w.w[2 * p + 1];
    const GaussPair g = box_muller32(a, b);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float x = h ? g.g1 : g.g0;
      const float e = 0x1p-21f * (fabsf(x) + g.r);
      const float lo = round_fmt<FMT>(x - e), hi = round_fmt<FMT>(x + e);
      float q = round_fmt<FMT>(x);
      if (lo != hi) q = round_fmt64<FMT>(box_muller64(a, b, h));
      out[2 * p + h] = q;
    }
  }
}

// ========================================================================= sampled rows
// The SRFT's row sample R (s distinct rows of [0, pool), sorted), drawn on the device.
// Floyd's rule takes the draws in sequence: draw t (i_t = pool - s + t) takes
// x_t = floor(u_t (i_t + 1) / 2^64), u_t from words 0 and 1 of Philox block (t, 0, stream 2),
// unless an earlier draw already holds x_t, in which case it takes i_t.  The sequence is
// resolved here in parallel.  An earlier draw t' holds x_t' or i_t', and i_t' exceeds every
// x of an earlier draw, so x_t is already held exactly when
//   (a) x_t = x_t' for some t' < t (draw t' kept x_t', or x_t' was held before t'), or
//   (b) t' = x_t - (pool - s) satisfies 0 <= t' < t and draw t' took its i_t'.
// (b) links draw t to one earlier draw, so "t takes i_t" is the OR of (a) along a chain of
// decreasing indices, evaluated by pointer jumping in ceil(log2 s) rounds.  The s values
// taken are distinct; each is stored at its rank.  One workgroup of kFloydThreads threads.
constexpr int kFloydThreads = 1024;
constexpr int kFloydMax = 2 * kFloydThreads;  // draws per workgroup (two per thread)
__host__ __device__ constexpr size_t floyd_smem_bytes() { return (size_t)kFloydMax * 12; }

__device__ inline void floyd_rows_block(uint64_t seed, int64_t pool, int s, int* __restrict__ out,
                                        unsigned char* smem) {
  int* xs = reinterpret_cast<int*>(smem);     // x_t, later the value taken
  int* link = xs + kFloydMax;                  // pointer-jumping link (-1: end of chain)
  int* flag = link + kFloydMax;                // "t takes i_t" along the chain so far
  const int tid = threadIdx.x;
  const int64_t base = pool - s;
  int x[2], f[2], l[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = tid + h * kFloydThreads;
    x[h] = 0;
    if (t < s) {
      const Words w = philox(seed, (uint64_t)t, 0, kRows);
      const uint64_t u = (uint64_t)w.w[0] | ((uint64_t)w.w[1] << 32);
      x[h] = (int)__umul64hi(u, (uint64_t)(base + t + 1));
      xs[t] = x[h];
    }
  }
  __syncthreads();
  // (a): an equal value among the earlier draws
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = tid + h * kFloydThreads;
    bool dup = false;
    if (t < s) {
      int q = 0;
      for (; q + 4 <= t; q += 4) {
        const int4 v = *reinterpret_cast<const int4*>(xs + q);
        dup |= (v.x == x[h]) | (v.y == x[h]) | (v.z == x[h]) | (v.w == x[h]);
      }
      for (; q < t; ++q) dup |= xs[q] == x[h];
      const int64_t tp = (int64_t)x[h] - base;
      l[h] = (tp >= 0 && tp < t) ? (int)tp : -1;
    } else {
      l[h] = -1;
    }
    f[h] = dup;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = tid + h * kFloydThreads;
    link[t] = l[h];
    flag[t] = f[h];
  }
  __syncthreads();
  // (b): OR of (a) along the chain, by pointer jumping
  for (int span = 1; span < s; span <<= 1) {
    int nf[2], nl[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      nf[h] = f[h];
      nl[h] = l[h];
      if (l[h] >= 0) {
        nf[h] |= flag[l[h]];
        nl[h] = link[l[h]];
      }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = tid + h * kFloydThreads;
      f[h] = nf[h];
      l[h] = nl[h];
      flag[t] = f[h];
      link[t] = l[h];
    }
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = tid + h * kFloydThreads;
    if (t < s) {
      x[h] = f[h] ? (int)(base + t) : x[h];
      xs[t] = x[h];
    }
  }
  __syncthreads();
  // sort: each taken value goes to its rank
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = tid + h * kFloydThreads;
    if (t < s) {
      int rank = 0, q = 0;
      for (; q + 4 <= s; q += 4) {
        const int4 v = *reinterpret_cast<const int4*>(xs + q);
        rank += (v.x < x[h]) + (v.y < x[h]) + (v.z < x[h]) + (v.w < x[h]);
      }
      for (; q < s; ++q) rank += xs[q] < x[h];
      out[rank] = x[h];
    }
  }
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
// LDS: the block tile, a zero row, one set of sign words per wave (cols / 2 waves), the sample
// records padded to 32 UMAX (the padding points at the zero row).
__host__ __device__ constexpr int srht_umax(int s) { return s <= 256 ? 8 : s <= 512 ? 16 : s <= 1024 ? 32 : 64; }
__host__ __device__ inline size_t srht_smem_bytes(int s, int cols) {
  return (size_t)(kT * cols + 64 + cols) * 8 + (size_t)(kT / 32) * 4 * (cols / 2) + (size_t)32 * srht_umax(s) * 8;
}

template <typename TIn, typename TAcc, int UMAX, int COLS, bool PF = true>
__device__ inline void srht_tile(const Operand& op, int64_t m, int N, int s, uint64_t seed,
                                 const int* __restrict__ rows, int ctile, int64_t g0, int64_t gstride,
                                 TAcc* __restrict__ out, unsigned char* smem) {
  constexpr int NT = SrhtTile<COLS>::kThreads;
  constexpr int RS = 32 * COLS + 2;            // doubles between rows rl and rl + 32 of the tile
  constexpr int kZero = kT * COLS + 64;        // the zero row, after the tile
  double* tile = reinterpret_cast<double*>(smem);
  uint32_t* signbits = reinterpret_cast<uint32_t*>(tile + kZero + COLS) + (threadIdx.x >> 6) * (kT / 32);
  int2* srec = reinterpret_cast<int2*>(reinterpret_cast<uint32_t*>(tile + kZero + COLS) + (NT / 64) * (kT / 32));

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
  // records past s read the zero row with sign +, so the sampled stage needs no branch
  for (int i = t; i < 32 * UMAX; i += NT) {
    if (i < s) {
      const int r = rows[i];
      const int i2 = r & (kT - 1);
      srec[i] = make_int2(i2 * COLS + (i2 >> 5) * 2, r >> 10);
    } else {
      srec[i] = make_int2(kZero, 0);
    }
  }
  if (t < COLS) tile[kZero + t] = 0.0;

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
    // every wave draws the block's sign words into its own slot (lanes 0..7, one Philox block
    // each), so only the tile needs the workgroup barrier: the previous block's sampled reads
    // are done before this block's rows are written
    const int lane = t & 63;
    if (lane < kT / 128) {
      const Words w = philox(seed, (uint64_t)(j1 * kT >> 7) + lane, 0, kSigns);
      *reinterpret_cast<uint4*>(signbits + 4 * lane) = make_uint4(w.w[0], w.w[1], w.w[2], w.w[3]);
    }
    wave_lds_sync();
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
        x[k] = flip_sign((TAcc)to_f64(raw[k]), (ws[e] >> rs) << 31);
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
    // (-1)^popcount(i1 & j1); groups of 8 samples, each group's reads issued together, groups
    // wholly past s skipped (a wave-uniform test)
    const uint32_t jlo = (uint32_t)j1;
#pragma unroll
    for (int u0 = 0; u0 < UMAX; u0 += 8) {
      if (32 * u0 < s) {
        int2 rec[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) rec[u] = srec[rs + 32 * (u0 + u)];
        double y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) y[u] = tile[rec[u].x + col];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          acc[u0 + u] += flip_sign((TAcc)y[u], (uint32_t)__popc((uint32_t)rec[u].y & jlo) << 31);
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
  extern __shared__ __align__(16) unsigned char smem[];
  const int tiles = (N + COLS - 1) / COLS;
  const int64_t item = xcd_work_item(blockIdx.x, (int64_t)tiles * groups);
  if (item < 0) return;
  const int tile = (int)(item % tiles), g = (int)(item / tiles);
  srht_tile<TIn, TAcc, UMAX, COLS>(op, m, N, s, seed, rows, tile, g, groups, partial + (size_t)g * s * N, smem);
}

}  // namespace nsk
