// Internal declarations of the nsk library: counter-based draws, operand descriptors,
// kernel launchers.  Device and host code both include this header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nsk.h"

namespace nsk {

// ---------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 multiplies whose halves
// are xor-mixed with the other counter words and the key; the key advances by the two Weyl
// increments between rounds.  Counter (lo32(idx), hi32(idx), sub, stream), key = seed.
// ---------------------------------------------------------------------------------------
enum : uint32_t { kSigns = 1, kRows = 2, kSparseRows = 3, kSparseSigns = 4, kGauss = 5 };

struct Words { uint32_t w[4]; };

__host__ __device__ inline Words philox(uint64_t seed, uint64_t idx, uint32_t sub, uint32_t stream) {
  uint32_t x0 = (uint32_t)idx, x1 = (uint32_t)(idx >> 32), x2 = sub, x3 = stream;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p = (uint64_t)0xD2511F53u * x0;
    const uint64_t q = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t y0 = (uint32_t)(q >> 32) ^ x1 ^ k0;
    const uint32_t y2 = (uint32_t)(p >> 32) ^ x3 ^ k1;
    x1 = (uint32_t)q;
    x3 = (uint32_t)p;
    x0 = y0;
    x2 = y2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Words o;
  o.w[0] = x0; o.w[1] = x1; o.w[2] = x2; o.w[3] = x3;
  return o;
}

// Word i (0..3) of a block, selected without a dynamically indexed array.
__host__ __device__ inline uint32_t word(const Words& w, uint32_t i) {
  return i == 0 ? w.w[0] : i == 1 ? w.w[1] : i == 2 ? w.w[2] : w.w[3];
}

// Sparse-sign column j of S: zeta distinct rows in [0, s) by Floyd sampling (draw t uses
// word t&3 of block (j, t>>2, stream 3): x = floor(u (i+1) / 2^32), i = s - zeta + t, and
// i replaces x when x was taken), signs from bit t of word j&3 of block (j>>2, 0, stream 4).
template <int ZMAX>
__host__ __device__ inline void sparse_column(uint64_t seed, uint64_t j, int s, int zeta,
                                              int (&rows)[ZMAX], uint32_t& negbits) {
  Words w = philox(seed, j, 0, kSparseRows);
#pragma unroll
  for (int t = 0; t < ZMAX; ++t) {
    if (t < zeta) {
      if (t > 0 && (t & 3) == 0) w = philox(seed, j, (uint32_t)(t >> 2), kSparseRows);
      const uint32_t i = (uint32_t)(s - zeta + t);
      int x = (int)(((uint64_t)w.w[t & 3] * (uint64_t)(i + 1u)) >> 32);
      bool dup = false;
#pragma unroll
      for (int u = 0; u < t; ++u) dup |= (rows[u] == x);
      rows[t] = dup ? (int)i : x;
    }
  }
  negbits = word(philox(seed, j >> 2, 0, kSparseSigns), (uint32_t)(j & 3));
}

// Columns per workgroup of the sparse-sign sketch: the widest of 16, 8, 4 whose (s + 1) x cols
// accumulator plus the double-buffered draw table (1024 rows x zeta) fits in 160 KB of LDS.
// The sparse-sign kernel's column tile and draw staging: cols columns of (s + 1) accumulator
// rows in LDS beside the staged draws of `bufs` 1024-row chunks (two: the next chunk is staged
// while the current one is accumulated; one: a barrier more per chunk).  16 columns whenever
// they fit, single-buffered if need be: with 8 FP64 columns two target rows share each 16-lane
// group of a 64-bit LDS atomic, and random rows collide on the same half of the banks about half
// the time (39 % of the LDS cycles were bank conflicts at s = 1024), while 16 columns give each
// group one row.  Otherwise the widest tile that fits double-buffered.
struct SparseTile {
  int cols, bufs;
};
__host__ __device__ inline size_t sparse_lds_need(int s, int zeta, int acc, int cols, int bufs) {
  const size_t zmax = zeta <= 8 ? 8 : 32;
  const size_t el = acc == NSK_F64 ? 8 : 4;
  return (size_t)(s + 1) * cols * el + (size_t)bufs * 1024 * (zmax * 2 + 4);
}
__host__ __device__ inline SparseTile sparse_tile(int s, int zeta, int acc) {
  constexpr size_t kLds = 160 * 1024;
  if (sparse_lds_need(s, zeta, acc, 16, 2) <= kLds) return SparseTile{16, 2};
  if (sparse_lds_need(s, zeta, acc, 16, 1) <= kLds) return SparseTile{16, 1};
  if (sparse_lds_need(s, zeta, acc, 8, 2) <= kLds) return SparseTile{8, 2};
  return SparseTile{4, 2};
}
__host__ __device__ inline int sparse_cols(int s, int zeta, int acc) { return sparse_tile(s, zeta, acc).cols; }

// Columns per SRHT tile for an N-column operand sketched to s rows (host plans and kernels
// share it): 16-column tiles (512 threads, 256 registers a thread) hold up to 32 sampled rows
// per thread (s <= 1024); more samples per thread take 8-column tiles, which have twice the
// registers.  And the column tile of the batched kernel.
__host__ __device__ inline int srht_cols(int N, int s) { return N > 8 && s <= 1024 ? 16 : 8; }
constexpr int kBatchCols = 16;

// XCD-aware placement.  MI355X hands the workgroups of a grid to its 8 XCDs round-robin
// (workgroup b to XCD b mod 8), and every XCD has its own L2.  A 1-D grid of xcd_grid(n)
// workgroups is remapped so that XCD x runs work items x*per .. x*per + per - 1 in order:
// consecutive work items (the column tiles of one row range, which read the same cache
// lines) share an L2.  xcd_work_item returns -1 for the padding workgroups.
constexpr int kXcds = 8;
__host__ __device__ inline int64_t xcd_grid(int64_t n) { return (n + kXcds - 1) / kXcds * kXcds; }
__host__ __device__ inline int64_t xcd_work_item(int64_t b, int64_t n) {
  const int64_t per = xcd_grid(n) / kXcds;
  const int64_t w = (b % kXcds) * per + b / kXcds;
  return w < n ? w : -1;
}

// Cooperative kernels whose workgroups hand data to each other (the multi-workgroup QR and
// Jacobi) launch `stride` workgroups per worker and keep only b = stride w as worker w; with
// stride = kXcds and the dealing above all workers run on one XCD and share its L2 (stride 1
// where the device has too few CUs for that launch).  Each worker records the
// hardware XCC id it runs on (hwreg XCC_ID) before the launch's first grid barrier; after it,
// xcd_all_local tells every worker whether all W ids agree.  When they do, a hand-over needs
// neither the writer's L2 write-back (agent-scope release) nor the reader's L2 invalidation
// (agent-scope acquire): the writer waits for its stores, which the vector L1 writes through to
// the shared L2, and raises its flag; the reader fetches the handed-over data with agent-scope
// relaxed atomic loads (load_handed), which the CU's L1 does not serve, so they read the L2.
// Measured on gfx950: after another workgroup's stores and flag, plain loads and loads after a
// workgroup-scope invalidate (buffer_inv sc0) or with the sc0 bit return the CU's stale L1
// lines; agent-scope loads and loads after an agent-scope acquire return the new values.
// With workers on several XCDs the kernels keep agent-scope release and acquire.
__device__ inline unsigned xcc_id() { return __builtin_amdgcn_s_getreg(20 | (0 << 6) | (15 << 11)); }
__device__ inline bool coop_worker(int stride) { return blockIdx.x % stride == 0; }
__device__ inline int coop_worker_index(int stride) { return (int)(blockIdx.x / stride); }
__device__ inline int coop_workers(int stride) { return (int)(gridDim.x / stride); }
__device__ inline void xcd_record(unsigned* ids, int stride) {
  if (coop_worker(stride) && threadIdx.x == 0) ids[coop_worker_index(stride)] = xcc_id();
}
// Load of data another workgroup handed over: agent-scope (past the CU's L1) in the one-XCD
// hand-over, plain after an agent-scope acquire.
template <typename T> __device__ inline T load_handed(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// After a grid barrier that follows every worker's xcd_record (at most 64 workers); the same in
// every wave.  Lane w of each wave compares worker w's id with worker 0's (vector loads, no
// LDS: static LDS here would shift the callers' dynamic LDS off its 8-byte alignment).
__device__ inline bool xcd_all_local(const unsigned* ids, int stride, bool allowed) {
  const int lane = (int)(threadIdx.x & 63);
  const int W = coop_workers(stride);
  const unsigned mine = lane < W ? __hip_atomic_load(&ids[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
  const unsigned first = __shfl(mine, 0, 64);
  return allowed && W <= 64 && __all(lane >= W || mine == first);
}

__host__ __device__ inline int64_t next_pow2(int64_t m) {
  int64_t p = 1;
  while (p < m) p <<= 1;
  return p;
}

// Padded length of the DCT-II kind: a power of two holding at least one 1024-row block.
__host__ __device__ inline int64_t srdct_pool(int64_t m) { return m <= 1024 ? 1024 : next_pow2(m); }

// ---------------------------------------------------------------------------------------
// Operand: up to four row-major column blocks of one element type.
// ---------------------------------------------------------------------------------------
constexpr int kMaxBlocks = 4;
struct Operand {
  const void* ptr[kMaxBlocks];
  int64_t ld[kMaxBlocks];
  const int8_t* exp[kMaxBlocks];
  int32_t col0[kMaxBlocks + 1];  // first column of each block; col0[nb] = N
  int32_t nb;
  int32_t dtype;
};

// Block holding column `col`, selected with constant indices only (a dynamically indexed
// kernel-argument array would be copied to scratch memory).
__device__ inline int column_block(const Operand& op, int col) {
  int b = 0;
  if (op.nb > 1 && col >= op.col0[1]) b = 1;
  if (op.nb > 2 && col >= op.col0[2]) b = 2;
  if (op.nb > 3 && col >= op.col0[3]) b = 3;
  return b;
}

// Element (row, col) pointer parts for a column: base pointer and row stride.
template <typename T>
__device__ inline void column_ref(const Operand& op, int col, const T*& base, int64_t& ld) {
  const int b = column_block(op, col);
  const void* p = op.ptr[0];
  int64_t l = op.ld[0];
  int c0 = 0;
  if (b == 1) { p = op.ptr[1]; l = op.ld[1]; c0 = op.col0[1]; }
  if (b == 2) { p = op.ptr[2]; l = op.ld[2]; c0 = op.col0[2]; }
  if (b == 3) { p = op.ptr[3]; l = op.ld[3]; c0 = op.col0[3]; }
  base = static_cast<const T*>(p) + (col - c0);
  ld = l;
}

__device__ inline int column_exp(const Operand& op, int col) {
  const int b = column_block(op, col);
  const int8_t* e = op.exp[0];
  int c0 = 0;
  if (b == 1) { e = op.exp[1]; c0 = op.col0[1]; }
  if (b == 2) { e = op.exp[2]; c0 = op.col0[2]; }
  if (b == 3) { e = op.exp[3]; c0 = op.col0[3]; }
  return e ? (int)e[col - c0] : 0;
}

// ---------------------------------------------------------------------------------------
// Launch plans and launchers (defined in the .hip files).
// ---------------------------------------------------------------------------------------
struct SketchPlan {
  int kind;           // nsk_kind
  int64_t m;
  int N;
  int s;
  int zeta;
  uint64_t seed;
  int acc;            // NSK_F64 or NSK_F32
  int groups;         // row groups = number of partial sketches
  int col_tile;       // columns per workgroup
  const int* rows;    // SRHT, DCT-II: sorted sampled rows (device)
  void* draws;        // sparse sign: per-row draw table (sparse_table_bytes); DCT-II: sign
                      // table (srdct_table_bytes); device
  void* partial;      // groups x s x N (acc type)
};

// sparse sign: the per-call table of every row's packed draws, and the pass that writes it
size_t sparse_table_bytes(int64_t m, int zeta);
hipError_t launch_sparse_table(const SketchPlan& p, hipStream_t st);

// DCT-II: columns per tile (16 or 8), LDS bytes, the sign table and its pass, the sketch
int srdct_cols(int N, int s, int acc, int dtype);
size_t srdct_lds_bytes(int N, int s, int acc, int dtype);
size_t srdct_table_bytes(int64_t m, int s);
hipError_t launch_srdct_signs(const SketchPlan& p, hipStream_t st);
hipError_t launch_srdct(const Operand& op, const SketchPlan& p, hipStream_t st);

// H-RHT: columns per tile of the transform-and-hash pass, the widest of 8, 4, 2 whose LDS (the
// B x cols block of one in-block index, B = max(m_p, 1024) / 1024, and the s x cols accumulator)
// fits in 160 KB; 0 if none does.
inline int rht_hash_cols(int64_t m, int s) {
  const int64_t mp = next_pow2(m);
  const int64_t B = (mp < 1024 ? 1024 : mp) / 1024;
  if (B == 1024 && (1024 * 8 + 64 + (int64_t)s * 8) * 8 <= 160 * 1024) return 8;  // register kernel
  for (int c = 8; c >= 2; c >>= 1)
    if ((B + s) * c * 8 <= 160 * 1024) return c;
  return 0;
}
// the hash table (m_p words), the transform (Y: max(m_p, 1024) x N FP64) and the partial sketches
// (p.groups x s x N FP64) of the H-RHT sketch
hipError_t launch_rht(const Operand& op, const SketchPlan& p, uint32_t* hash, double* Y, hipStream_t st);

hipError_t launch_sketch(const Operand& op, const SketchPlan& p, hipStream_t st);
// SA (FP64, s x N) = scale * sum_g partial_g; row-major (ld_rm) and/or column-major (ld_cm)
hipError_t launch_reduce(const Operand& op, const SketchPlan& p, double* sa_rm, int64_t ld_rm,
                         double* sa_cm, int64_t ld_cm, hipStream_t st);

struct JacobiResult;  // svd_pipeline.hpp
struct SvdPlan {
  int s, N, k;
  int max_sweeps;
  double* sa;          // s x N column-major (ld = s), overwritten by the QR
  double* R;           // work: (64 NR) x (nb B) on the fast path, N x N otherwise
  double* V;           // work: N x N (only without the fast path)
  double2* log;        // work: rotation log (fast path)
  double* sigma;       // N: singular values in sorted order
  int* order;          // N: column index of each sorted singular value
  double* colnorm;     // N: singular value of each column (fast path; nullable)
  JacobiResult* jres;  // fast path: sweeps / convergence
  double* Vk;          // N x k row-major out (nullable)
  double* sigma_k;     // k out (nullable)
  nsk_info* info;      // nullable
};
bool svd_fast_path(int s, int N);
size_t svd_work_R_bytes(int s, int N);
size_t svd_work_log_bytes(int s, int N, int max_sweeps);
// Records the end of profiler stage `stage` on st when the stage profiler is on (api.cpp);
// launch_svd marks stages 3 (QR), 4 (Jacobi) and 5 (finish).
void prof_mark(int stage, hipStream_t st);
hipError_t launch_svd(const SvdPlan& p, hipStream_t st);

hipError_t launch_residual(const Operand& op, int64_t m, const double* Vk, int k, double* partial,
                           int parts, double* out, nsk_info* info, hipStream_t st);

hipError_t launch_tls_extract(int N, const double* v, double* x, hipStream_t st);
// TLS adjoint + gradient.  st: TLS state arrays (see api.cpp); the trailing vector v,
// singular values per column and the rotation log give w = V D V^T g_bar by two replays.
struct TlsBack {
  const double* sa_rm;     // s x N row-major
  const double* colnorm;   // N
  const int* order;        // N
  const double* v;         // N
  const double* x;         // n
  const JacobiResult* jres;
  const double2* log;
};
hipError_t launch_tls_backward(const SketchPlan& p, int64_t m, const TlsBack& tb, const double* gx, double* work,
                               void* dA, int64_t ldda, void* db, int out_dtype, hipStream_t st);

// AAA with a reused sketch (aaa.hip): reductions over at most kAaaParts blocks; at most
// kAaaMaxSupport support points (the single-instance SVD's fast path)
constexpr int kAaaParts = 1024;
constexpr int kAaaMaxSupport = 320;
struct AaaPick {
  double err;    // largest |f - r| over the non-support points
  int64_t idx;   // its sample index (the lowest on ties)
};
hipError_t launch_aaa_stats(const double* f, int64_t m, double* part, double* stats, hipStream_t st);
hipError_t launch_aaa_error(const double* z, const double* f, const uint8_t* mask, int64_t m, const double* sz,
                            const double* sf, const double* w, int k, const double* stats, double* pval,
                            int64_t* pidx, AaaPick* out, hipStream_t st);
hipError_t launch_aaa_join(const double* z, const double* f, int64_t m, int64_t j, int k, double* sz, double* sf,
                           uint8_t* mask, double* row, int64_t* idx, int8_t* ops, double* col, hipStream_t st);
hipError_t launch_aaa_transpose(const double* a, int64_t ld, int s, int N, double* cm, hipStream_t st);

// The SRFT row sample (s <= 2048 sorted distinct rows of [0, pool), pool <= 2^31) drawn on
// the device into rows[0..s).
hipError_t launch_srht_rows(uint64_t seed, int64_t pool, int s, int* rows, hipStream_t st);
hipError_t launch_draw_signs(uint64_t seed, int64_t m, int8_t* d, hipStream_t st);
hipError_t launch_draw_sparse(uint64_t seed, int64_t m, int s, int zeta, int32_t* rows,
                              int8_t* signs, hipStream_t st);
hipError_t launch_draw_gauss(uint64_t seed, int s, int64_t j0, int64_t j1, int dtype, float* G,
                             hipStream_t st);

}  // namespace nsk
