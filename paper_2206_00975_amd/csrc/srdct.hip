// Subsampled randomized DCT-II sketch: the SRFT of Section 2 with the orthonormal DCT-II as
// the trig transform, the real transform Section 4 uses for real data.
//
// S = sqrt(M/s) R C D on A zero-padded to M = max(1024, 2^ceil(log2 m)) rows, where
// C[k, j] = c_k cos(pi k (2j+1) / (2M)) with c_0 = sqrt(1/M) and c_k = sqrt(2/M) otherwise, and
// D, R are the sign diagonal and sorted row sample of the Hadamard kind (rows drawn from
// [0, M)).  For a sampled row k the sketch row is w_k X_k with X_k = sum_j x_j cos(pi k (2j+1)
// / (2M)), x = D A, w_0 = sqrt(1/s) and w_k = sqrt(2/s): the partials hold X_k times 1 or
// sqrt(2) and the reduce applies 1/sqrt(s).
//
// Fast form.  With v_p = x_{2p} and v_{M-1-p} = x_{2p+1} for p < M/2 (Makhoul's reordering),
// X_k = Re[e^{-i pi k / (2M)} V_k] where V is the M-point DFT of v.  Splitting p = j1 + B j2
// (T = 1024, B = M / T, j1 < B, j2 < T) gives V_k = sum_j1 e^{-2 pi i j1 k / M} Y_j1[k mod T],
// with Y_j1 the T-point DFT of the strided block v_{j1 + B j2}, so
//     X_k = sum_j1 Re[e^{-i theta} Y_j1[k mod T]],   theta = pi k (4 j1 + 1) / (2M).
// A workgroup owns a column tile and a contiguous range of blocks j1.  Per block it loads the
// block's T rows of A (even rows 2 j1 + 2B j2 for j2 < T/2, odd rows M - 1 - 2 j1 - 2B (j2 -
// T/2) for the rest; rows past m are zero), applies D, and takes the T-point real DFT as the
// 512-point complex DFT Z of z_t = v_{2t} + i v_{2t+1}: a 16-point DFT in registers, a
// twiddle, an LDS transpose, one radix-2 step and a second 16-point DFT.  With q' = k mod 512,
// Y[k mod T] = E + e^{-2 pi i k / T} O where E = (Z[q'] + conj Z[-q']) / 2 and
// O = (Z[q'] - conj Z[-q']) / (2i), so every sampled row adds
//     Re[e^{-i theta} E] + Re[e^{-i (theta + 2 pi k / T)} O]
//   = alpha Re Z[q'] + beta Re Z[-q'] + gamma Im Z[q'] + delta Im Z[-q']
// (four multiply-adds per column).  Per block and sample the coefficients need e^{-i theta}
// and e^{-i theta} e^{-2 pi i k / T}.  Consecutive blocks differ by the rotation
// e^{-2 pi i k / M}, so the workgroup advances each sample's e^{-i theta} by one complex
// multiply, and takes it exactly (sincospi of the integer angle k (4 j1 + 1) reduced modulo 4M,
// one period) at its first block and every kDctAnchor blocks after, which bounds the rounding
// the recurrence gathers.  The two per-sample rotations are computed once per call.  A is read
// once; the per-element work is the FFT (about 5 log2 T flops) plus 8 s / T flops for the
// sampled rows.
#include <hip/hip_runtime.h>

#include "fft16.hpp"
#include "nsk_internal.hpp"

namespace nsk {

constexpr int kDctT = 1024;      // rows per transform block
constexpr int kDctAnchor = 32;  // blocks between exact evaluations of a sample's angle

// LDS: the 512-point transform of each column, the quarter-period twiddle table, two
// coefficient pairs and one index word per sampled row.
__host__ __device__ inline size_t srdct_lds_bytes_cols(int s, int cols, int acc) {
  const size_t el = acc == NSK_F64 ? 8 : 4;
  return (size_t)512 * cols * 2 * el + 128 * 2 * el + (size_t)s * 4 * el + (size_t)s * 4;
}

// 16-column tiles (512 threads, at most 256 registers a thread) only for FP32 loads with FP32
// arithmetic; an FP64 transform takes 8-column tiles, whose 256 threads have twice the
// registers (and the FP64 rate per column is the same).
int srdct_cols(int N, int s, int acc, int dtype) {
  return N > 8 && s <= 1024 && acc == NSK_F32 && dtype == NSK_F32 ? 16 : 8;
}

size_t srdct_lds_bytes(int N, int s, int acc, int dtype) {
  return srdct_lds_bytes_cols(s, srdct_cols(N, s, acc, dtype), acc);
}

// Sign table (m_p / 8 bytes), then two FP64 complex rotations per sampled row.
size_t srdct_table_bytes(int64_t m, int s) { return (size_t)(srdct_pool(m) / 8) + (size_t)s * 32; }

// Sign table: word j1 * 32 + rs holds, at bit 2b + e, the sign of D for the row that thread rs
// of the transform takes as value (b, e) of block j1 (zero for padding rows), so the transform
// reads one word per block.  One thread per bit; the wave's ballot forms two words.
__global__ __launch_bounds__(256) void srdct_sign_kernel(uint64_t seed, int64_t m, int64_t M,
                                                         uint32_t* __restrict__ tab) {
  const int64_t B = M / kDctT;
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;  // M bits in all
  const int64_t w = gid >> 5;
  const int bit = (int)(gid & 31), b = bit >> 1, e = bit & 1;
  const int64_t j1 = w >> 5;
  const int rs = (int)(w & 31);
  const int64_t off = (int64_t)(128 * (b & 7) + 2 * e) * B;
  const int64_t r = b < 8 ? 2 * j1 + 4 * B * rs + off : M - 1 - 2 * j1 - 4 * B * rs - off;
  bool neg = false;
  if (r < m) {
    const uint32_t wd = word(philox(seed, (uint64_t)(r >> 7), 0, kSigns), (uint32_t)((r >> 5) & 3));
    neg = (wd >> (r & 31)) & 1u;
  }
  const uint64_t mask = __ballot(neg);
  const int lane = threadIdx.x & 63;
  if ((lane & 31) == 0) tab[w] = (uint32_t)(mask >> lane);
}

// Per sampled row k: e^{-2 pi i k / M} (one block further) and e^{-2 pi i (k mod T) / T}.
__global__ __launch_bounds__(256) void srdct_rotation_kernel(const int* __restrict__ rows, int s, int64_t M,
                                                             cx<double>* __restrict__ rot) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= s) return;
  const int64_t k = rows[i];
  double sn, cs;
  sincospi(2.0 * (double)k / (double)M, &sn, &cs);  // 2k / M < 2, exact
  rot[2 * i] = cx<double>{cs, -sn};
  sincospi((double)(k & (kDctT - 1)) / (kDctT / 2), &sn, &cs);
  rot[2 * i + 1] = cx<double>{cs, -sn};
}

// Thread (rs, col) of a 32 * COLS workgroup: column col of the tile; in the first DFT stage it
// holds z_{rs + 32 b} (b < 16) of its column, in the second the outputs Z[cc + 32 d + 16 h]
// (cc = rs >> 1, h = rs & 1, d < 16); for the sampled rows it accumulates rows rs + 32 u.
template <typename TIn, typename TAcc, int UMAX, int COLS>
__global__ __launch_bounds__(32 * COLS) void srdct_kernel(Operand op, int64_t m, int N, int s, int64_t M,
                                                          const int* __restrict__ rows,
                                                          const uint32_t* __restrict__ signtab,
                                                          const cx<double>* __restrict__ rot, int groups,
                                                          TAcc* __restrict__ partial) {
  constexpr int NT = 32 * COLS;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<TAcc>* zb = reinterpret_cast<cx<TAcc>*>(smem);          // 512 x COLS: element q at q * COLS + col
  cx<TAcc>* wq = zb + 512 * COLS;                             // e^{-2 pi i r / 512}, r < 128
  cx<TAcc>* cf = wq + 128;                                    // per sample: (alpha, beta), (gamma, delta)
  uint32_t* sq = reinterpret_cast<uint32_t*>(cf + 2 * s);     // per sample: q' | (-q' mod 512) << 16

  const int tiles = (N + COLS - 1) / COLS;
  const int64_t item = xcd_work_item(blockIdx.x, (int64_t)tiles * groups);
  if (item < 0) return;
  const int ctile = (int)(item % tiles), g = (int)(item / tiles);

  const int t = threadIdx.x;
  const int col = t % COLS;
  const int rs = t / COLS;
  const int c = ctile * COLS + col;
  const bool live = c < N;
  const TIn* base = nullptr;
  int64_t ld = 0;
  column_ref<TIn>(op, live ? c : 0, base, ld);  // columns past N read column 0, never written

  const int64_t B = M / kDctT;
  const int64_t per = (B + groups - 1) / groups;
  const int64_t jb = (int64_t)g * per < B ? (int64_t)g * per : B;
  const int64_t je = jb + per < B ? jb + per : B;
  const double inv2M = 0.5 / (double)M;  // exact: M is a power of two
  const uint64_t pmask = 4 * (uint64_t)M - 1;

  for (int r = t; r < 128; r += NT) {
    double sn, cs;
    sincospi((double)r / 256.0, &sn, &cs);
    wq[r] = cx<TAcc>{(TAcc)cs, (TAcc)-sn};
  }
  for (int i = t; i < s; i += NT) {
    const uint32_t q1 = (uint32_t)rows[i] & 511u;
    sq[i] = q1 | (((512u - q1) & 511u) << 16);
  }

  TAcc acc[UMAX];
#pragma unroll
  for (int u = 0; u < UMAX; ++u) acc[u] = 0;

  // The 32 rows of block j1 that this thread takes, value (b, e) at raw[2b + e]; rows past m
  // read row 0 and are replaced by zero.
  auto fetch = [&](int64_t j1, TIn (&raw)[32], uint32_t& sw) {
    const int64_t re = 2 * j1 + 4 * B * rs;
    const int64_t ro = M - 1 - 2 * j1 - 4 * B * rs;
#pragma unroll
    for (int b = 0; b < 16; ++b) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int64_t off = (int64_t)(128 * (b & 7) + 2 * e) * B;
        const int64_t r = b < 8 ? re + off : ro - off;
        const bool in = r < m;
        const TIn v = base[(in ? r : 0) * ld];
        raw[2 * b + e] = in ? v : (TIn)0;
      }
    }
    sw = signtab[j1 * 32 + rs];
  };

  auto block = [&](int64_t j1, const TIn (&raw)[32], uint32_t sw) {
    __syncthreads();  // the previous block's transform and coefficients have been read
    // e^{-i theta} = c1 - i s1 and e^{-i theta} e^{-2 pi i k / T} = c2 - i s2; a sample's
    // coefficients are rewritten by the thread that wrote them for the previous block, which
    // recovers c1 = alpha + beta and s1 = gamma - delta from them
    const bool anchor = ((j1 - jb) & (kDctAnchor - 1)) == 0;
    for (int i = t; i < s; i += NT) {
      double c1, s1;
      if (anchor) {
        const uint64_t n1 = ((uint64_t)rows[i] * (uint64_t)(4 * j1 + 1)) & pmask;
        sincospi((double)n1 * inv2M, &s1, &c1);
      } else {
        const cx<TAcc> ab = cf[2 * i], gd = cf[2 * i + 1];
        const double pc = (double)ab.r + (double)ab.i, ps = (double)gd.r - (double)gd.i;
        const cx<double> w = rot[2 * i];
        c1 = pc * w.r + ps * w.i;
        s1 = ps * w.r - pc * w.i;
      }
      const cx<double> tq = rot[2 * i + 1];
      const double c2 = c1 * tq.r + s1 * tq.i, s2 = s1 * tq.r - c1 * tq.i;
      cf[2 * i] = cx<TAcc>{(TAcc)(0.5 * (c1 - s2)), (TAcc)(0.5 * (c1 + s2))};
      cf[2 * i + 1] = cx<TAcc>{(TAcc)(0.5 * (s1 + c2)), (TAcc)(0.5 * (c2 - s1))};
    }
    // stage 1: signs, 16-point DFT over b, twiddle e^{-2 pi i rs cc / 512}, transpose
    cx<TAcc> z[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      TAcc v0 = (TAcc)raw[2 * b], v1 = (TAcc)raw[2 * b + 1];
      v0 = ((sw >> (2 * b)) & 1u) ? -v0 : v0;
      v1 = ((sw >> (2 * b + 1)) & 1u) ? -v1 : v1;
      z[b] = cx<TAcc>{v0, v1};
    }
    dft16(z);
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      cx<TAcc> x = z[cc];
      if (cc > 0) {
        const int n = rs * cc;  // < 512: the table's quarter period times (-i)^(n >> 7)
        const cx<TAcc> w = wq[n & 127];
        const cx<TAcc> w1 = (n & 128) ? cx<TAcc>{w.i, -w.r} : w;
        const cx<TAcc> w2 = (n & 256) ? cx<TAcc>{-w1.r, -w1.i} : w1;
        x = cmul(x, w2);
      }
      zb[(cc * 32 + rs) * COLS + col] = x;
    }
    __syncthreads();
    // stage 2: radix-2 step on a, a + 16 (output parity h), then a 16-point DFT over a
    {
      const int cc = rs >> 1, h = rs & 1;
      cx<TAcc> y[16];
#pragma unroll
      for (int a = 0; a < 16; ++a) {
        const cx<TAcc> p0 = zb[(cc * 32 + a) * COLS + col];
        const cx<TAcc> p1 = zb[(cc * 32 + a + 16) * COLS + col];
        y[a] = h ? mul_w32(p0 - p1, a) : p0 + p1;
      }
      dft16(y);
      __syncthreads();  // every stage-1 value has been read
#pragma unroll
      for (int d = 0; d < 16; ++d) zb[(cc + 32 * d + 16 * h) * COLS + col] = y[d];
    }
    __syncthreads();
    // sampled rows
#pragma unroll
    for (int u = 0; u < UMAX; ++u) {
      const int i = rs + 32 * u;
      if (i < s) {
        const uint32_t q = sq[i];
        const cx<TAcc> za = zb[(q & 0xFFFFu) * COLS + col];
        const cx<TAcc> zc = zb[(q >> 16) * COLS + col];
        const cx<TAcc> ab = cf[2 * i], gd = cf[2 * i + 1];
        acc[u] += ab.r * za.r + ab.i * zc.r + gd.r * za.i + gd.i * zc.i;
      }
    }
  };

  // the next block's values are in flight while this one is transformed; the prefetch issued
  // with the last block re-reads it and is discarded
  if (jb < je) {
    TIn cur[32];
    uint32_t sw;
    fetch(jb, cur, sw);
    for (int64_t j1 = jb; j1 < je; ++j1) {
      TIn nxt[32];
      uint32_t swn;
      fetch(j1 + 1 < je ? j1 + 1 : j1, nxt, swn);
      block(j1, cur, sw);
#pragma unroll
      for (int k = 0; k < 32; ++k) cur[k] = nxt[k];
      sw = swn;
    }
  }
  if (live) {
    TAcc* out = partial + (size_t)g * s * N;
#pragma unroll
    for (int u = 0; u < UMAX; ++u) {
      const int i = rs + 32 * u;
      if (i < s) out[(size_t)i * N + c] = rows[i] == 0 ? acc[u] : acc[u] * (TAcc)1.41421356237309504880;
    }
  }
}

static hipError_t set_lds_limit_dct(const void* fn, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename TIn, typename TAcc, int COLS>
static hipError_t srdct_dispatch_cols(const Operand& op, const SketchPlan& p, hipStream_t st) {
  const int tiles = (p.N + COLS - 1) / COLS;
  const dim3 grid((unsigned)xcd_grid((int64_t)tiles * p.groups));
  const size_t lds = srdct_lds_bytes_cols(p.s, COLS, p.acc);
  const int64_t M = srdct_pool(p.m);
  const uint32_t* tab = static_cast<const uint32_t*>(p.draws);
  const cx<double>* rot = reinterpret_cast<const cx<double>*>(static_cast<const unsigned char*>(p.draws) + M / 8);
  TAcc* part = static_cast<TAcc*>(p.partial);
#define NSK_DCT_CASE(U)                                                                                    \
  {                                                                                                        \
    if (hipError_t e = set_lds_limit_dct((const void*)srdct_kernel<TIn, TAcc, U, COLS>, lds)) return e;    \
    srdct_kernel<TIn, TAcc, U, COLS><<<grid, 32 * COLS, lds, st>>>(op, p.m, p.N, p.s, M, p.rows, tab, rot,      \
                                                                   p.groups, part);                        \
  }
  if (p.s <= 512) NSK_DCT_CASE(16)
  else if (p.s <= 1024) NSK_DCT_CASE(32)
  else if constexpr (COLS == 8) NSK_DCT_CASE(64)
  else return hipErrorInvalidValue;
#undef NSK_DCT_CASE
  return hipGetLastError();
}

template <typename TIn, typename TAcc>
static hipError_t srdct_dispatch(const Operand& op, const SketchPlan& p, hipStream_t st) {
  if constexpr (sizeof(TIn) == 4 && sizeof(TAcc) == 4)
    if (srdct_cols(p.N, p.s, p.acc, op.dtype) == 16) return srdct_dispatch_cols<TIn, TAcc, 16>(op, p, st);
  return srdct_dispatch_cols<TIn, TAcc, 8>(op, p, st);
}

hipError_t launch_srdct_signs(const SketchPlan& p, hipStream_t st) {
  const int64_t M = srdct_pool(p.m);
  srdct_sign_kernel<<<(unsigned)(M / 256), 256, 0, st>>>(p.seed, p.m, M, static_cast<uint32_t*>(p.draws));
  cx<double>* rot = reinterpret_cast<cx<double>*>(static_cast<unsigned char*>(p.draws) + M / 8);
  srdct_rotation_kernel<<<(unsigned)((p.s + 255) / 256), 256, 0, st>>>(p.rows, p.s, M, rot);
  return hipGetLastError();
}

hipError_t launch_srdct(const Operand& op, const SketchPlan& p, hipStream_t st) {
  if (op.dtype == NSK_F64)
    return p.acc == NSK_F64 ? srdct_dispatch<double, double>(op, p, st) : srdct_dispatch<double, float>(op, p, st);
  return p.acc == NSK_F64 ? srdct_dispatch<float, double>(op, p, st) : srdct_dispatch<float, float>(op, p, st);
}

}  // namespace nsk
