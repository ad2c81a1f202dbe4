// C ABI of the nsk library: argument checks, workspace layout, host-side draws and the
// launch sequence of Algorithm 1 (sketch -> reduce -> QR + Jacobi -> extraction).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "nsk.h"
#include "nsk_internal.hpp"

namespace nsk {
// defined in the .hip translation units
size_t sparse_lds_bytes(int s, int zeta, int acc);
int gauss_groups(int64_t m, int s, int N);
size_t batched_lds_bytes(int s_max, int n_max);
hipError_t launch_batched(const void* insts, int count, const void* tiles, int ntiles, int* counters, int dtype,
                          int acc, int grid, size_t lds, hipStream_t st);
size_t batch_inst_bytes();
size_t batch_tile_bytes();
void batch_fill_inst(void* dst, const Operand& op, int64_t m, int N, int s, int k, int groups, int ctiles,
                     int max_sweeps, uint64_t seed, const int* rows, void* partial, double* sa_cm, double* R,
                     double2* log, double* sigma, int* order, double* colnorm, void* jres, double* Vk,
                     double* sigma_k, nsk_info* info);
void batch_fill_tile(void* dst, int inst, int ctile, int g);
int tuned_rows_per_tile(int n, int64_t m, int dtype, int acc);
hipError_t launch_row_update(const Operand& op, const SketchPlan& p, const int64_t* idx, const int8_t* ops, int r,
                             double* SA, int64_t ldsa, hipStream_t st);
hipError_t launch_count_below(const double* sigma, int N, double eps, int relative, int32_t* count,
                              hipStream_t st);
hipError_t launch_tls_extract_multi(const double* Vk, int n, int k, double* X, hipStream_t st);
}  // namespace nsk

using namespace nsk;

namespace {

constexpr size_t kAlign = 256;
constexpr int kResParts = 1024;
constexpr int kMaxN = 1024;
constexpr int64_t kMaxResidualVec = 16384;  // N * k doubles of V_k held in LDS

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int dflt_zeta(const nsk_desc* d) { return d->zeta ? d->zeta : 8; }
int dflt_sweeps(const nsk_desc* d) { return d->max_sweeps ? d->max_sweeps : 30; }
int dflt_acc(const nsk_desc* d) { return d->acc == NSK_F32 ? NSK_F32 : NSK_F64; }

// H-RHT workspace: the hash word of each of the m_p transformed rows, then the transform
// (max(m_p, 1024) x N FP64)
size_t hrht_table_bytes(int64_t m) { return align_up((size_t)next_pow2(m) * 4); }
size_t hrht_draws_bytes(int64_t m, int64_t N) {
  return hrht_table_bytes(m) + (size_t)std::max<int64_t>(next_pow2(m), 1024) * N * 8;
}

// Row groups (number of partial sketches) for a single-instance sketch.
int plan_groups(const nsk_desc* d, int64_t m, int64_t N, int dtype) {
  if (d->row_groups > 0) return d->row_groups;
  if (d->kind == NSK_SRHT) {
    // about two workgroups per CU in total (a 16-column tile fills most of a CU's LDS)
    if (next_pow2(m) <= 64) return 1;
    const int cols = srht_cols((int)N, (int)d->s);
    const int64_t ct = (N + cols - 1) / cols, nb = (m + 1023) / 1024;
    const int64_t target = cols == 16 ? 512 : 1024;
    return (int)std::max<int64_t>(1, std::min<int64_t>(nb, target / ct));
  }
  if (d->kind == NSK_SRDCT) {
    // one or two workgroups per CU, as the LDS allows
    const int cols = srdct_cols((int)N, (int)d->s, dflt_acc(d), dtype);
    const int64_t ct = (N + cols - 1) / cols, nb = srdct_pool(m) / 1024;
    const int64_t per_cu = srdct_lds_bytes((int)N, (int)d->s, dflt_acc(d), dtype) <= 80 * 1024 ? 2 : 1;
    return (int)std::max<int64_t>(1, std::min<int64_t>(nb, 256 * per_cu / ct));
  }
  if (d->kind == NSK_HRHT) {
    // the transform-and-hash pass: one workgroup per CU (its LDS holds a block and the
    // accumulator), each over a range of the 1024 in-block indices
    const int cols = std::max(1, rht_hash_cols(m, (int)d->s));
    const int64_t ct = (N + cols - 1) / cols;
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, 256 / ct));
  }
  if (d->kind == NSK_SPARSE_SIGN) {
    // one workgroup per CU (the accumulator fills most of the LDS): about 256 workgroups
    const int cols = sparse_cols((int)d->s, dflt_zeta(d), dflt_acc(d));
    const int64_t ct = (N + cols - 1) / cols, nb = (m + 1023) / 1024;
    return (int)std::max<int64_t>(1, std::min<int64_t>(nb, 256 / ct));
  }
  return gauss_groups(m, (int)d->s, (int)N);
}

struct Layout {
  size_t rows, draws, partial, sa, R, V, log, sigma, order, colnorm, jres, res, work, total;
};

Layout layout(int64_t m, int64_t N, const nsk_desc* d) {
  Layout L{};
  const int64_t s = d->s;
  // the workspace query knows no operand dtype: room for the larger partial count
  const int groups = std::max(plan_groups(d, m, N, NSK_F32), plan_groups(d, m, N, NSK_F64));
  const bool fast = svd_fast_path((int)s, (int)N);
  size_t off = 0;
  L.rows = off;    off = align_up(off + (size_t)s * 4);
  const size_t draws = d->kind == NSK_SPARSE_SIGN ? sparse_table_bytes(m, dflt_zeta(d))
                     : d->kind == NSK_SRDCT     ? srdct_table_bytes(m, (int)d->s)
                     : d->kind == NSK_HRHT      ? hrht_draws_bytes(m, N)
                                                : 0;
  L.draws = off;   off = align_up(off + draws);
  L.partial = off; off = align_up(off + (size_t)groups * s * N * 8);
  L.sa = off;      off = align_up(off + (size_t)s * N * 8);
  L.R = off;       off = align_up(off + svd_work_R_bytes((int)s, (int)N));
  L.V = off;       off = align_up(off + (fast ? 0 : (size_t)N * N * 8));
  L.log = off;     off = align_up(off + svd_work_log_bytes((int)s, (int)N, dflt_sweeps(d)));
  L.sigma = off;   off = align_up(off + (size_t)N * 8);
  L.order = off;   off = align_up(off + (size_t)N * 4);
  L.colnorm = off; off = align_up(off + (size_t)N * 8);
  L.jres = off;    off = align_up(off + 64);
  L.res = off;     off = align_up(off + (size_t)kResParts * 8);
  L.work = off;    off = align_up(off + (size_t)(2 * s + 2 * N) * 8);
  L.total = off;
  return L;
}

SvdPlan svd_plan(const nsk_desc* d, int64_t N, unsigned char* w, const Layout& L) {
  SvdPlan sp{};
  sp.s = (int)d->s;
  sp.N = (int)N;
  sp.k = 1;
  sp.max_sweeps = dflt_sweeps(d);
  sp.sa = reinterpret_cast<double*>(w + L.sa);
  sp.R = reinterpret_cast<double*>(w + L.R);
  sp.V = reinterpret_cast<double*>(w + L.V);
  sp.log = reinterpret_cast<double2*>(w + L.log);
  sp.sigma = reinterpret_cast<double*>(w + L.sigma);
  sp.order = reinterpret_cast<int*>(w + L.order);
  sp.colnorm = reinterpret_cast<double*>(w + L.colnorm);
  sp.jres = reinterpret_cast<JacobiResult*>(w + L.jres);
  return sp;
}

int check_desc(const nsk_desc* d, int64_t m, int64_t N) {
  if (!d) return NSK_EINVAL;
  if (d->kind < NSK_SRHT || d->kind > NSK_HRHT) return NSK_EINVAL;
  if (m < N || N < 1 || d->s <= N || d->s > m) return NSK_EINVAL;
  if (d->kind == NSK_SPARSE_SIGN) {
    const int z = dflt_zeta(d);
    if (z < 1 || z > 32 || z > d->s || d->s > 65535) return NSK_EINVAL;
  }
  if ((d->kind == NSK_SRHT || d->kind == NSK_SRDCT) && (d->s > 2048 || next_pow2(m) > ((int64_t)1 << 31)))
    return NSK_EUNSUPPORTED;
  if (d->kind == NSK_HRHT && (d->acc == NSK_F32 || next_pow2(m) > ((int64_t)1 << 21) || rht_hash_cols(m, (int)d->s) == 0))
    return NSK_EUNSUPPORTED;
  if (d->kind == NSK_SPARSE_SIGN && sparse_lds_bytes((int)d->s, dflt_zeta(d), dflt_acc(d)) > 160 * 1024)
    return NSK_EUNSUPPORTED;
  if (d->acc != 0 && d->acc != NSK_F64 && d->acc != NSK_F32) return NSK_EINVAL;
  if (d->max_sweeps < 0 || d->row_groups < 0) return NSK_EINVAL;
  return NSK_OK;
}

int build_operand(const nsk_operand* blocks, int nblocks, const nsk_desc* d, Operand& op, int64_t& N) {
  if (!blocks || nblocks < 1 || nblocks > kMaxBlocks) return NSK_EINVAL;
  std::memset(&op, 0, sizeof(op));
  op.nb = nblocks;
  op.dtype = blocks[0].dtype;
  N = 0;
  for (int b = 0; b < nblocks; ++b) {
    const nsk_operand& o = blocks[b];
    if (!o.ptr || o.cols < 1 || o.ld < o.cols || o.reserved != 0) return NSK_EINVAL;
    if (o.dtype != op.dtype) return NSK_EINVAL;
    op.ptr[b] = o.ptr;
    op.ld[b] = o.ld;
    op.exp[b] = o.col_exp;
    op.col0[b] = (int32_t)N;
    N += o.cols;
  }
  op.col0[nblocks] = (int32_t)N;
  if (N > kMaxN) return NSK_EINVAL;
  if (!d) return NSK_EINVAL;
  const int dt = op.dtype;
  if (d->kind == NSK_GAUSSIAN) {
    if (dt != NSK_BF16 && dt != NSK_F8E4M3) return NSK_EUNSUPPORTED;
  } else if (dt != NSK_F32 && dt != NSK_F64) {
    return NSK_EUNSUPPORTED;
  }
  return NSK_OK;
}

// Host Floyd sampling of s distinct rows of [0, pool), sorted (same rule as the device
// hooks document: 64-bit uniform from words 0,1 of block (t, 0, stream 2)).
void srht_rows_host(uint64_t seed, int64_t pool, int64_t s, std::vector<int64_t>& out) {
  out.clear();
  out.reserve((size_t)s);
  // membership of the rows taken so far: open addressing, at most half full
  size_t cap = 16;
  while (cap < 2 * (size_t)s) cap <<= 1;
  std::vector<int64_t> table(cap, -1);
  auto slot = [&](int64_t x) {
    size_t h = (size_t)(((uint64_t)x * 0x9E3779B97F4A7C15ull) >> 17) & (cap - 1);
    while (table[h] != -1 && table[h] != x) h = (h + 1) & (cap - 1);
    return h;
  };
  for (int64_t t = 0; t < s; ++t) {
    const Words w = philox(seed, (uint64_t)t, 0, kRows);
    const unsigned __int128 u = (unsigned __int128)((uint64_t)w.w[0] | ((uint64_t)w.w[1] << 32));
    const int64_t i = pool - s + t;
    int64_t x = (int64_t)((u * (unsigned __int128)(uint64_t)(i + 1)) >> 64);
    size_t h = slot(x);
    if (table[h] == x) h = slot(x = i);  // i is new: every row taken so far is below it
    table[h] = x;
    out.push_back(x);
  }
  std::sort(out.begin(), out.end());
}

// The SRFT row sample drawn on the device into the workspace (stream-ordered, no host copy).
int draw_rows(uint64_t seed, int64_t pool, int64_t s, int* dst, hipStream_t st) {
  return launch_srht_rows(seed, pool, (int)s, dst, st) == hipSuccess ? NSK_OK : NSK_EDEVICE;
}

// ------------------------------------------------------------------ pinned staging
// Host-built records that a call copies to the device (the batched call's instance and tile
// lists, the row indices and signs of a row update) pass through library-owned pinned host
// buffers, so the copies are asynchronous and the call returns without waiting for the stream.
// A slot stays owned by its copy until the event recorded after that copy has completed; a
// later call that reuses the slot waits for that copy only (normally long finished).  Slots
// grow on demand (hipHostMalloc) and are kept for the life of the process.
struct StageSlot {
  void* ptr = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  int device = -1;
  bool inflight = false;
};
constexpr int kStageSlots = 4;
std::mutex g_stage_mu;
StageSlot g_stage[kStageSlots];
int g_stage_next = 0;

// Takes a slot of at least `bytes` and locks the staging until stage_release.  Returns the slot
// index, or -1 (lock released) on a runtime error.
int stage_acquire(size_t bytes) {
  g_stage_mu.lock();
  const int i = g_stage_next;
  g_stage_next = (g_stage_next + 1) % kStageSlots;
  StageSlot& sl = g_stage[i];
  int device = 0;
  bool ok = hipGetDevice(&device) == hipSuccess;
  if (ok && sl.inflight) ok = hipEventSynchronize(sl.ev) == hipSuccess;
  sl.inflight = false;
  if (ok && sl.cap < bytes) {
    if (sl.ptr) (void)hipHostFree(sl.ptr);
    sl.ptr = nullptr;
    sl.cap = 0;
    ok = hipHostMalloc(&sl.ptr, bytes, hipHostMallocDefault) == hipSuccess;
    if (ok) sl.cap = bytes;
  }
  if (ok && (sl.ev == nullptr || sl.device != device)) {
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    sl.ev = nullptr;
    ok = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) == hipSuccess;
    sl.device = device;
  }
  if (!ok) {
    g_stage_mu.unlock();
    return -1;
  }
  return i;
}

// Marks the copies enqueued from slot i on st and unlocks the staging.
int stage_release(int i, hipStream_t st) {
  const bool ok = hipEventRecord(g_stage[i].ev, st) == hipSuccess;
  g_stage[i].inflight = ok;
  g_stage_mu.unlock();
  return ok ? NSK_OK : NSK_EDEVICE;
}

SketchPlan make_plan(const nsk_desc* d, int64_t m, int64_t N, int dtype, unsigned char* ws, const Layout& L) {
  SketchPlan p{};
  p.kind = d->kind;
  p.m = m;
  p.N = (int)N;
  p.s = (int)d->s;
  p.zeta = dflt_zeta(d);
  p.seed = d->seed;
  p.acc = dflt_acc(d);
  p.groups = plan_groups(d, m, N, dtype);
  p.col_tile = 0;
  p.rows = reinterpret_cast<const int*>(ws + L.rows);
  p.draws = ws + L.draws;
  p.partial = ws + L.partial;
  return p;
}

int dev(hipError_t e) { return e == hipSuccess ? NSK_OK : NSK_EDEVICE; }

// ------------------------------------------------------------------ stage profiler
struct Profiler {
  std::vector<hipEvent_t> ev;  // (NSK_PROF_STAGES + 1) per call
  int max_calls = 0;
  int calls = 0;
  int cur = -1;                // call being recorded, -1 if none
};
Profiler g_prof;

void prof_begin(hipStream_t st) {
  g_prof.cur = -1;
  if (g_prof.max_calls == 0 || g_prof.calls >= g_prof.max_calls) return;
  g_prof.cur = g_prof.calls++;
  (void)hipEventRecord(g_prof.ev[(size_t)g_prof.cur * (NSK_PROF_STAGES + 1)], st);
}

}  // namespace

void nsk::prof_mark(int stage, hipStream_t st) {  // end of stage `stage`
  if (g_prof.cur < 0) return;
  (void)hipEventRecord(g_prof.ev[(size_t)g_prof.cur * (NSK_PROF_STAGES + 1) + stage + 1], st);
}

namespace {

// Sketch + reduce; SA written column-major into the workspace and optionally row-major out.
int run_sketch(const Operand& op, const nsk_desc* d, int64_t m, int64_t N, unsigned char* ws, const Layout& L,
               double* sa_rm, int64_t ld_rm, hipStream_t st, SketchPlan& p) {
  p = make_plan(d, m, N, op.dtype, ws, L);
  prof_begin(st);
  if (d->kind == NSK_SRHT || d->kind == NSK_SRDCT) {
    const int64_t pool = d->kind == NSK_SRHT ? next_pow2(m) : srdct_pool(m);
    const int rc = draw_rows(d->seed, pool, d->s, reinterpret_cast<int*>(ws + L.rows), st);
    if (rc) return rc;
  }
  if (d->kind == NSK_SRDCT) {
    const int rc = dev(launch_srdct_signs(p, st));
    if (rc) return rc;
  }
  if (d->kind == NSK_HRHT) {
    // transform every row, hash it into the partial sketches, reduce them (scale 1: the
    // hashing matrix has entries +-1)
    uint32_t* hash = reinterpret_cast<uint32_t*>(ws + L.draws);
    double* Y = reinterpret_cast<double*>(ws + L.draws + hrht_table_bytes(m));
    int rc = dev(launch_rht(op, p, hash, Y, st));  // marks the end of stage 0 after the table
    if (rc) return rc;
    prof_mark(1, st);
    SketchPlan hp = p;
    hp.kind = NSK_SPARSE_SIGN;
    hp.zeta = 1;
    hp.acc = NSK_F64;
    rc = dev(launch_reduce(op, hp, sa_rm, ld_rm, reinterpret_cast<double*>(ws + L.sa), d->s, st));
    prof_mark(2, st);
    return rc;
  }
  if (d->kind == NSK_SPARSE_SIGN) {
    const int rc = dev(launch_sparse_table(p, st));
    if (rc) return rc;
  }
  prof_mark(0, st);
  int rc = dev(launch_sketch(op, p, st));
  if (rc) return rc;
  prof_mark(1, st);
  rc = dev(launch_reduce(op, p, sa_rm, ld_rm, reinterpret_cast<double*>(ws + L.sa), d->s, st));
  prof_mark(2, st);
  return rc;
}

}  // namespace

extern "C" {

const char* nsk_status_str(int status) {
  switch (status) {
    case NSK_OK: return "ok";
    case NSK_EINVAL: return "invalid argument";
    case NSK_EWORKSPACE: return "workspace too small";
    case NSK_ENOCONV: return "Jacobi did not converge";
    case NSK_EDEVICE: return "HIP runtime error";
    case NSK_EUNSUPPORTED: return "unsupported kind/dtype combination";
    default: return "unknown status";
  }
}

int nsk_version(void) { return 10000; }

size_t nsk_workspace_bytes(int64_t m, int64_t N, int64_t k, const nsk_desc* d) {
  if (check_desc(d, m, N) != NSK_OK || k < 1 || k > N || N > kMaxN) return 0;
  return layout(m, N, d).total;
}

int nsk_sketch(const nsk_operand* blocks, int32_t nblocks, int64_t m, const nsk_desc* d, double* SA, int64_t ldsa,
               void* ws, size_t ws_bytes, void* stream) {
  Operand op;
  int64_t N;
  int rc = build_operand(blocks, nblocks, d, op, N);
  if (rc) return rc;
  if ((rc = check_desc(d, m, N))) return rc;
  if (!SA || ldsa < N || !ws) return NSK_EINVAL;
  const Layout L = layout(m, N, d);
  if (ws_bytes < L.total) return NSK_EWORKSPACE;
  SketchPlan p;
  rc = run_sketch(op, d, m, N, static_cast<unsigned char*>(ws), L, SA, ldsa, (hipStream_t)stream, p);
  for (int stage = 3; stage < NSK_PROF_STAGES; ++stage) prof_mark(stage, (hipStream_t)stream);
  return rc;
}

int nsk_trailing_rsv(const nsk_operand* blocks, int32_t nblocks, int64_t m, int64_t k, const nsk_desc* d,
                     double* Vk, double* sigma_k, nsk_info* info, void* ws, size_t ws_bytes, void* stream) {
  Operand op;
  int64_t N;
  int rc = build_operand(blocks, nblocks, d, op, N);
  if (rc) return rc;
  if ((rc = check_desc(d, m, N))) return rc;
  if (k < 1 || k > N || !Vk || !sigma_k || !ws) return NSK_EINVAL;
  const Layout L = layout(m, N, d);
  if (ws_bytes < L.total) return NSK_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  unsigned char* w = static_cast<unsigned char*>(ws);
  SketchPlan p;
  if ((rc = run_sketch(op, d, m, N, w, L, nullptr, 0, st, p))) return rc;
  SvdPlan sp = svd_plan(d, N, w, L);
  sp.k = (int)k;
  sp.Vk = Vk;
  sp.sigma_k = sigma_k;
  sp.info = info;
  if ((rc = dev(launch_svd(sp, st)))) return rc;
  if ((d->flags & NSK_FLAG_RESIDUAL) && info) {
    if (N * k > kMaxResidualVec) return NSK_EUNSUPPORTED;
    const int64_t parts = std::min<int64_t>(kResParts, std::max<int64_t>(1, m / 256));
    rc = dev(launch_residual(op, m, Vk, (int)k, reinterpret_cast<double*>(w + L.res), (int)parts, nullptr, info, st));
  }
  prof_mark(6, st);
  return rc;
}

int nsk_tls_solve_multi(const nsk_operand* blocks, int32_t nblocks, int64_t m, int64_t nrhs, const nsk_desc* d,
                        double* X, double* Vk, double* sigma_k, nsk_info* info, void* ws, size_t ws_bytes,
                        void* stream) {
  Operand op;
  int64_t N;
  int rc = build_operand(blocks, nblocks, d, op, N);
  if (rc) return rc;
  if (nrhs < 1 || nrhs > 64 || nrhs >= N || !X || !Vk) return NSK_EINVAL;
  if ((rc = nsk_trailing_rsv(blocks, nblocks, m, nrhs, d, Vk, sigma_k, info, ws, ws_bytes, stream))) return rc;
  return dev(launch_tls_extract_multi(Vk, (int)(N - nrhs), (int)nrhs, X, (hipStream_t)stream));
}

int nsk_null_space(const nsk_operand* blocks, int32_t nblocks, int64_t m, double eps, int32_t relative,
                   const nsk_desc* d, double* V, double* sigma, int32_t* count, nsk_info* info, void* ws,
                   size_t ws_bytes, void* stream) {
  if (!(eps >= 0.0) || !std::isfinite(eps) || !count || (relative != 0 && relative != 1)) return NSK_EINVAL;
  Operand op;
  int64_t N;
  int rc = build_operand(blocks, nblocks, d, op, N);
  if (rc) return rc;
  // all N vectors, non-increasing singular values: the trailing `count` columns are the answer
  if ((rc = nsk_trailing_rsv(blocks, nblocks, m, N, d, V, sigma, info, ws, ws_bytes, stream))) return rc;
  return dev(launch_count_below(sigma, (int)N, eps, relative, count, (hipStream_t)stream));
}

// ------------------------------------------------------------------------------ AAA
}  // extern "C"

namespace {

struct AaaLayout {
  Layout col;          // nsk workspace of an m x 1 sketch (the new Loewner column)
  size_t col_base;
  size_t sa_rm, sa_cm, R, log, sigma, order, colnorm, jres, sig1;
  size_t mask, colv, row, idx, ops, sz, sf, part, pval, pidx, stats, pick, total;
};

int aaa_check(int64_t m, int32_t n_max, const nsk_desc* d) {
  if (!d || n_max < 1 || n_max > kAaaMaxSupport) return NSK_EINVAL;
  if (d->kind == NSK_GAUSSIAN || d->kind == NSK_HRHT) return NSK_EUNSUPPORTED;
  int rc = check_desc(d, m, n_max);
  if (rc) return rc;
  if (!svd_fast_path((int)d->s, n_max)) return NSK_EUNSUPPORTED;
  return NSK_OK;
}

AaaLayout aaa_layout(int64_t m, int32_t n_max, const nsk_desc* d) {
  AaaLayout A{};
  A.col = layout(m, 1, d);
  size_t off = 0;
  A.col_base = off;  off = align_up(off + A.col.total);
  const size_t s = (size_t)d->s;
  size_t rb = 0, lb = 0;  // the SVD's work for any N <= n_max
  for (int N = 1; N <= n_max; ++N) {
    rb = std::max(rb, svd_work_R_bytes((int)s, N));
    lb = std::max(lb, svd_work_log_bytes((int)s, N, dflt_sweeps(d)));
  }
  A.sa_rm = off;   off = align_up(off + s * n_max * 8);
  A.sa_cm = off;   off = align_up(off + s * n_max * 8);
  A.R = off;       off = align_up(off + rb);
  A.log = off;     off = align_up(off + lb);
  A.sigma = off;   off = align_up(off + (size_t)n_max * 8);
  A.order = off;   off = align_up(off + (size_t)n_max * 4);
  A.colnorm = off; off = align_up(off + (size_t)n_max * 8);
  A.jres = off;    off = align_up(off + 64);
  A.sig1 = off;    off = align_up(off + 8);
  A.mask = off;    off = align_up(off + (size_t)m);
  A.colv = off;    off = align_up(off + (size_t)m * 8);
  A.row = off;     off = align_up(off + (size_t)n_max * 8);
  A.idx = off;     off = align_up(off + 8);
  A.ops = off;     off = align_up(off + 1);
  A.sz = off;      off = align_up(off + (size_t)n_max * 8);
  A.sf = off;      off = align_up(off + (size_t)n_max * 8);
  A.part = off;    off = align_up(off + (size_t)kAaaParts * 16);
  A.pval = off;    off = align_up(off + (size_t)kAaaParts * 8);
  A.pidx = off;    off = align_up(off + (size_t)kAaaParts * 8);
  A.stats = off;   off = align_up(off + 16);
  A.pick = off;    off = align_up(off + sizeof(AaaPick));
  A.total = off;
  return A;
}

}  // namespace

extern "C" {

size_t nsk_aaa_workspace_bytes(int64_t m, int32_t n_max, const nsk_desc* d) {
  if (aaa_check(m, n_max, d) != NSK_OK) return 0;
  return aaa_layout(m, n_max, d).total;
}

int nsk_aaa(const double* z, const double* f, int64_t m, int32_t n_max, double tol, const nsk_desc* d,
            int64_t* support, double* weights, int32_t* n_support, double* err_hist, void* ws, size_t ws_bytes,
            void* stream) {
  int rc = aaa_check(m, n_max, d);
  if (rc) return rc;
  if (!z || !f || !support || !weights || !n_support || !ws || !(tol >= 0.0)) return NSK_EINVAL;
  const AaaLayout A = aaa_layout(m, n_max, d);
  if (ws_bytes < A.total) return NSK_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  unsigned char* w = static_cast<unsigned char*>(ws);
  unsigned char* wcol = w + A.col_base;
  double* sa_rm = reinterpret_cast<double*>(w + A.sa_rm);
  uint8_t* mask = w + A.mask;
  double* colv = reinterpret_cast<double*>(w + A.colv);
  double* row = reinterpret_cast<double*>(w + A.row);
  int64_t* idx = reinterpret_cast<int64_t*>(w + A.idx);
  int8_t* ops = reinterpret_cast<int8_t*>(w + A.ops);
  double* sz = reinterpret_cast<double*>(w + A.sz);
  double* sf = reinterpret_cast<double*>(w + A.sf);
  double* stats = reinterpret_cast<double*>(w + A.stats);
  AaaPick* pick = reinterpret_cast<AaaPick*>(w + A.pick);
  if (hipMemsetAsync(mask, 0, (size_t)m, st) != hipSuccess) return NSK_EDEVICE;
  if ((rc = dev(launch_aaa_stats(f, m, reinterpret_cast<double*>(w + A.part), stats, st)))) return rc;
  double hstats[2];
  if (hipMemcpyAsync(hstats, stats, sizeof(hstats), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return NSK_EDEVICE;
  const double thr = tol * hstats[1];

  // the column sketch: an m x 1 FP64 operand in the workspace
  Operand cop{};
  cop.nb = 1;
  cop.dtype = NSK_F64;
  cop.ptr[0] = colv;
  cop.ld[0] = 1;
  cop.col0[0] = 0;
  cop.col0[1] = 1;
  Operand rop{};
  rop.nb = 1;
  rop.dtype = NSK_F64;
  rop.ptr[0] = row;
  rop.col0[0] = 0;

  int k = 0;
  for (;; ++k) {
    if ((rc = dev(launch_aaa_error(z, f, mask, m, sz, sf, weights, k, stats, reinterpret_cast<double*>(w + A.pval),
                                   reinterpret_cast<int64_t*>(w + A.pidx), pick, st))))
      return rc;
    AaaPick hp;
    if (hipMemcpyAsync(&hp, pick, sizeof(hp), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return NSK_EDEVICE;
    if (err_hist) err_hist[k] = hp.err;
    // no finite error at a non-support point (NaN in f or in r): nothing valid to join
    if (!(hp.err >= 0.0) || hp.idx < 0 || hp.idx >= m) break;
    if (hp.err <= thr || k == n_max) break;
    const int64_t j = hp.idx;
    if ((rc = dev(launch_aaa_join(z, f, m, j, k, sz, sf, mask, row, idx, ops, colv, st)))) return rc;
    if (k > 0) {  // Algorithm 3: the new support point's row leaves the Loewner matrix
      rop.ld[0] = k;
      rop.col0[1] = k;
      SketchPlan pr{};
      pr.kind = d->kind;
      pr.m = m;
      pr.N = k;
      pr.s = (int)d->s;
      pr.zeta = dflt_zeta(d);
      pr.seed = d->seed;
      pr.rows = reinterpret_cast<const int*>(wcol + A.col.rows);  // uploaded by the previous column sketch
      if ((rc = dev(launch_row_update(rop, pr, idx, ops, 1, sa_rm, n_max, st)))) return rc;
    }
    // column update: the sketch of the new Loewner column becomes column k of SA
    SketchPlan pc;
    if ((rc = run_sketch(cop, d, m, 1, wcol, A.col, sa_rm + k, n_max, st, pc))) return rc;
    // weights: the trailing right singular vector of the s x (k + 1) sketch
    const int N = k + 1;
    if ((rc = dev(launch_aaa_transpose(sa_rm, n_max, (int)d->s, N, reinterpret_cast<double*>(w + A.sa_cm), st))))
      return rc;
    SvdPlan sp{};
    sp.s = (int)d->s;
    sp.N = N;
    sp.k = 1;
    sp.max_sweeps = dflt_sweeps(d);
    sp.sa = reinterpret_cast<double*>(w + A.sa_cm);
    sp.R = reinterpret_cast<double*>(w + A.R);
    sp.V = nullptr;
    sp.log = reinterpret_cast<double2*>(w + A.log);
    sp.sigma = reinterpret_cast<double*>(w + A.sigma);
    sp.order = reinterpret_cast<int*>(w + A.order);
    sp.colnorm = reinterpret_cast<double*>(w + A.colnorm);
    sp.jres = reinterpret_cast<JacobiResult*>(w + A.jres);
    sp.Vk = weights;
    sp.sigma_k = reinterpret_cast<double*>(w + A.sig1);
    sp.info = nullptr;
    if ((rc = dev(launch_svd(sp, st)))) return rc;
    support[k] = j;
  }
  *n_support = k;
  return NSK_OK;
}

size_t nsk_update_workspace_bytes(int64_t r, const nsk_desc* d) {
  if (!d || r < 0 || d->s < 1) return 0;
  const size_t rr = (size_t)std::max<int64_t>(r, 1);
  return align_up((size_t)d->s * 4) + align_up(rr * 8) + align_up(rr);
}

int nsk_sketch_rows(const nsk_operand* blocks, int32_t nblocks, int64_t r, const int64_t* rows, const int8_t* ops,
                    int64_t m, const nsk_desc* d, double* SA, int64_t ldsa, void* ws, size_t ws_bytes, void* stream) {
  Operand op;
  int64_t N;
  int rc = build_operand(blocks, nblocks, d, op, N);
  if (rc) return rc;
  if ((rc = check_desc(d, m, N))) return rc;
  if (d->kind == NSK_HRHT) return NSK_EUNSUPPORTED;
  if (r < 0 || r > (int64_t)1 << 30 || (r > 0 && (!rows || !ops)) || !SA || ldsa < N || !ws) return NSK_EINVAL;
  for (int64_t t = 0; t < r; ++t)
    if (rows[t] < 0 || (ops[t] != 1 && ops[t] != -1)) return NSK_EINVAL;
  if (ws_bytes < nsk_update_workspace_bytes(r, d)) return NSK_EWORKSPACE;
  if (r == 0) return NSK_OK;
  hipStream_t st = (hipStream_t)stream;
  unsigned char* w = static_cast<unsigned char*>(ws);
  int* srows = reinterpret_cast<int*>(w);
  int64_t* idx = reinterpret_cast<int64_t*>(w + align_up((size_t)d->s * 4));
  int8_t* sg = reinterpret_cast<int8_t*>(w + align_up((size_t)d->s * 4) + align_up((size_t)r * 8));
  const size_t rb = align_up((size_t)r * 8);
  const int slot = stage_acquire(rb + (size_t)r);
  if (slot < 0) return NSK_EDEVICE;
  unsigned char* hs = static_cast<unsigned char*>(g_stage[slot].ptr);
  std::memcpy(hs, rows, (size_t)r * 8);
  std::memcpy(hs + rb, ops, (size_t)r);
  const bool copied = hipMemcpyAsync(idx, hs, (size_t)r * 8, hipMemcpyHostToDevice, st) == hipSuccess &&
                      hipMemcpyAsync(sg, hs + rb, (size_t)r, hipMemcpyHostToDevice, st) == hipSuccess;
  if ((rc = stage_release(slot, st)) || !copied) return NSK_EDEVICE;
  if (d->kind == NSK_SRHT || d->kind == NSK_SRDCT) {
    const int64_t pool = d->kind == NSK_SRHT ? next_pow2(m) : srdct_pool(m);
    if ((rc = draw_rows(d->seed, pool, d->s, srows, st))) return rc;
  }
  SketchPlan p{};
  p.kind = d->kind;
  p.m = m;
  p.N = (int)N;
  p.s = (int)d->s;
  p.zeta = dflt_zeta(d);
  p.seed = d->seed;
  p.rows = srows;
  return dev(launch_row_update(op, p, idx, sg, (int)r, SA, ldsa, st));
}

int nsk_residual(const nsk_operand* blocks, int32_t nblocks, int64_t m, const double* Vk, int64_t k, double* out,
                 void* ws, size_t ws_bytes, void* stream) {
  nsk_desc d{};
  d.kind = NSK_SRHT;
  Operand op;
  int64_t N;
  // residual accepts FP32 / FP64 operands: validate with a SRHT-shaped descriptor
  int rc = build_operand(blocks, nblocks, &d, op, N);
  if (rc) return rc;
  if (m < 1 || k < 1 || k > N || !Vk || !out || !ws) return NSK_EINVAL;
  if (N * k > kMaxResidualVec) return NSK_EUNSUPPORTED;
  if (ws_bytes < (size_t)kResParts * 8) return NSK_EWORKSPACE;
  const int64_t parts = std::min<int64_t>(kResParts, std::max<int64_t>(1, m / 256));
  return dev(launch_residual(op, m, Vk, (int)k, static_cast<double*>(ws), (int)parts, out, nullptr,
                             (hipStream_t)stream));
}

// TLS state layout (N = n + 1 <= 320): SA row-major (s x N), per-column singular values,
// order, sorted singular values, trailing vector v, x, Jacobi result, rotation log.
static void tls_state_layout(int64_t n, int64_t s, int max_sweeps, size_t* o) {
  const int64_t N = n + 1;
  size_t off = 0;
  o[0] = off; off = align_up(off + (size_t)s * N * 8);
  o[1] = off; off = align_up(off + (size_t)N * 8);
  o[2] = off; off = align_up(off + (size_t)N * 4);
  o[3] = off; off = align_up(off + (size_t)N * 8);
  o[4] = off; off = align_up(off + (size_t)N * 8);
  o[5] = off; off = align_up(off + (size_t)n * 8);
  o[6] = off; off = align_up(off + 64);
  o[7] = off; off = align_up(off + svd_work_log_bytes((int)s, (int)N, max_sweeps));
  o[8] = off;
}

size_t nsk_tls_state_bytes(int64_t n, int64_t s, int32_t max_sweeps) {
  if (n < 1 || s <= n + 1 || !svd_fast_path((int)s, (int)(n + 1)) || max_sweeps < 0) return 0;
  size_t o[9];
  tls_state_layout(n, s, max_sweeps ? max_sweeps : 30, o);
  return o[8];
}

int nsk_tls_solve(const nsk_operand* blocks, int32_t nblocks, int64_t m, const nsk_desc* d, double* x, void* state,
                  size_t state_bytes, nsk_info* info, void* ws, size_t ws_bytes, void* stream) {
  Operand op;
  int64_t N;
  int rc = build_operand(blocks, nblocks, d, op, N);
  if (rc) return rc;
  if ((rc = check_desc(d, m, N))) return rc;
  if (N < 2 || !x || !state || !ws) return NSK_EINVAL;
  if (!svd_fast_path((int)d->s, (int)N)) return NSK_EUNSUPPORTED;
  const int64_t n = N - 1;
  if (state_bytes < nsk_tls_state_bytes(n, d->s, d->max_sweeps)) return NSK_EWORKSPACE;
  const Layout L = layout(m, N, d);
  if (ws_bytes < L.total) return NSK_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  unsigned char* w = static_cast<unsigned char*>(ws);
  unsigned char* S = static_cast<unsigned char*>(state);
  size_t o[9];
  tls_state_layout(n, d->s, dflt_sweeps(d), o);
  SketchPlan p;
  if ((rc = run_sketch(op, d, m, N, w, L, reinterpret_cast<double*>(S + o[0]), N, st, p))) return rc;
  SvdPlan sp = svd_plan(d, N, w, L);
  sp.k = 1;
  sp.colnorm = reinterpret_cast<double*>(S + o[1]);
  sp.order = reinterpret_cast<int*>(S + o[2]);
  sp.sigma = reinterpret_cast<double*>(S + o[3]);
  sp.Vk = reinterpret_cast<double*>(S + o[4]);
  sp.jres = reinterpret_cast<JacobiResult*>(S + o[6]);
  sp.log = reinterpret_cast<double2*>(S + o[7]);
  sp.sigma_k = nullptr;
  sp.info = info;
  if ((rc = dev(launch_svd(sp, st)))) return rc;
  double* xs = reinterpret_cast<double*>(S + o[5]);
  if ((rc = dev(launch_tls_extract((int)N, sp.Vk, xs, st)))) return rc;
  if ((rc = dev(hipMemcpyAsync(x, xs, (size_t)n * 8, hipMemcpyDeviceToDevice, st)))) return rc;
  if ((d->flags & NSK_FLAG_RESIDUAL) && info) {
    const int64_t parts = std::min<int64_t>(kResParts, std::max<int64_t>(1, m / 256));
    rc = dev(launch_residual(op, m, sp.Vk, 1, reinterpret_cast<double*>(w + L.res), (int)parts, nullptr, info, st));
  }
  prof_mark(6, st);
  return rc;
}

int nsk_tls_backward(const nsk_desc* d, int64_t m, int64_t n, const void* state, const double* gx, void* dA,
                     int64_t ldda, void* db, int32_t out_dtype, void* ws, size_t ws_bytes, void* stream) {
  const int64_t N = n + 1;
  int rc = check_desc(d, m, N);
  if (rc) return rc;
  if (d->kind == NSK_GAUSSIAN || d->kind == NSK_SRDCT || d->kind == NSK_HRHT || !svd_fast_path((int)d->s, (int)N))
    return NSK_EUNSUPPORTED;
  if (!state || !gx || !dA || !db || !ws || ldda < n) return NSK_EINVAL;
  if (out_dtype != NSK_F32 && out_dtype != NSK_F64) return NSK_EINVAL;
  const Layout L = layout(m, N, d);
  if (ws_bytes < L.total) return NSK_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  unsigned char* w = static_cast<unsigned char*>(ws);
  const unsigned char* S = static_cast<const unsigned char*>(state);
  size_t o[9];
  tls_state_layout(n, d->s, dflt_sweeps(d), o);
  SketchPlan p = make_plan(d, m, N, NSK_F64, w, L);
  if (d->kind == NSK_SRHT && (rc = draw_rows(d->seed, next_pow2(m), d->s, reinterpret_cast<int*>(w + L.rows), st)))
    return rc;
  TlsBack tb;
  tb.sa_rm = reinterpret_cast<const double*>(S + o[0]);
  tb.colnorm = reinterpret_cast<const double*>(S + o[1]);
  tb.order = reinterpret_cast<const int*>(S + o[2]);
  tb.v = reinterpret_cast<const double*>(S + o[4]);
  tb.x = reinterpret_cast<const double*>(S + o[5]);
  tb.jres = reinterpret_cast<const JacobiResult*>(S + o[6]);
  tb.log = reinterpret_cast<const double2*>(S + o[7]);
  return dev(launch_tls_backward(p, m, tb, gx, reinterpret_cast<double*>(w + L.work), dA, ldda, db, out_dtype, st));
}

// ------------------------------------------------------------------------------ batched
struct BatchLayout {
  size_t insts, tiles, counters, rows, per_inst, total;
  std::vector<size_t> inst_off;
  std::vector<int> groups;
  int ntiles;
};

static int batch_plan(const nsk_problem* probs, int32_t count, const nsk_desc* base, BatchLayout& B) {
  if (!probs || count < 1 || !base) return NSK_EINVAL;
  if (base->kind != NSK_SRHT) return NSK_EUNSUPPORTED;
  B.inst_off.assign(count, 0);
  B.groups.assign(count, 0);
  B.ntiles = 0;
  size_t rows_total = 0;
  for (int i = 0; i < count; ++i) {
    const nsk_problem& q = probs[i];
    if (q.n < 1 || q.n > 256 || q.m < q.n || q.s <= q.n || q.s > q.m || q.s > 1024 || q.k < 1 || q.k > q.n ||
        q.ld < q.n || !q.A || !q.Vk || !q.sigma_k)
      return NSK_EINVAL;
    if (q.m > ((int64_t)1 << 31)) return NSK_EUNSUPPORTED;
    if (q.dtype != NSK_F32 && q.dtype != NSK_F64) return NSK_EUNSUPPORTED;
    const int rpt = tuned_rows_per_tile((int)q.n, q.m, q.dtype, dflt_acc(base));
    const int64_t nb = (q.m + 1023) / 1024;
    const int g = (int)std::max<int64_t>(1, (nb + rpt - 1) / rpt);
    B.groups[i] = g;
    B.ntiles += g * (int)((q.n + kBatchCols - 1) / kBatchCols);
    rows_total += align_up((size_t)q.s * 4);
  }
  size_t off = 0;
  B.insts = off;    off = align_up(off + (size_t)count * batch_inst_bytes());
  B.tiles = off;    off = align_up(off + (size_t)B.ntiles * batch_tile_bytes());
  B.counters = off; off = align_up(off + (size_t)(count + 1) * 4);
  B.rows = off;     off = align_up(off + rows_total);
  B.per_inst = off;
  for (int i = 0; i < count; ++i) {
    const nsk_problem& q = probs[i];
    B.inst_off[i] = off;
    const size_t s = (size_t)q.s, n = (size_t)q.n;
    off = align_up(off + (size_t)B.groups[i] * s * n * 8);                      // partial
    off = align_up(off + s * n * 8);                                            // sa
    off = align_up(off + svd_work_R_bytes((int)s, (int)n));                     // R
    off = align_up(off + svd_work_log_bytes((int)s, (int)n, dflt_sweeps(base)));  // log
    off = align_up(off + n * 8);                                                // sigma
    off = align_up(off + n * 4);                                                // order
    off = align_up(off + n * 8);                                                // colnorm
    off = align_up(off + 64);                                                   // jres
  }
  B.total = off;
  return NSK_OK;
}

size_t nsk_batched_workspace_bytes(const nsk_problem* probs, int32_t count, const nsk_desc* base) {
  BatchLayout B;
  if (batch_plan(probs, count, base, B) != NSK_OK) return 0;
  return B.total;
}

int nsk_trailing_rsv_batched(const nsk_problem* probs, int32_t count, const nsk_desc* base, void* ws,
                             size_t ws_bytes, void* stream) {
  BatchLayout B;
  int rc = batch_plan(probs, count, base, B);
  if (rc) return rc;
  if (!ws) return NSK_EINVAL;
  if (ws_bytes < B.total) return NSK_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  unsigned char* w = static_cast<unsigned char*>(ws);
  // instances in decreasing SVD cost (n^3), their tiles in that order
  std::vector<int> ord(count);
  for (int i = 0; i < count; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (probs[a].n != probs[b].n) return probs[a].n > probs[b].n;
    return probs[a].m > probs[b].m;
  });
  int dtype = probs[0].dtype;
  for (int i = 1; i < count; ++i)
    if (probs[i].dtype != dtype) return NSK_EINVAL;
  // instance and tile records, built in a pinned staging slot and copied asynchronously
  const size_t ib = align_up((size_t)count * batch_inst_bytes());
  const size_t tb = (size_t)B.ntiles * batch_tile_bytes();
  const int slot = stage_acquire(ib + tb);
  if (slot < 0) return NSK_EDEVICE;
  unsigned char* hinst = static_cast<unsigned char*>(g_stage[slot].ptr);
  unsigned char* htile = hinst + ib;
  std::vector<size_t> rows_off(count);
  size_t roff = 0;
  int s_max = 0, n_max = 0;
  const int acc = dflt_acc(base);
  for (int i = 0; i < count; ++i) {
    rows_off[i] = roff;
    roff += align_up((size_t)probs[i].s * 4);
  }
  for (int i = 0; i < count; ++i) {
    const nsk_problem& q = probs[i];
    s_max = std::max<int>(s_max, (int)q.s);
    n_max = std::max<int>(n_max, (int)q.n);
    Operand op;
    std::memset(&op, 0, sizeof(op));
    op.nb = 1;
    op.dtype = q.dtype;
    op.ptr[0] = q.A;
    op.ld[0] = q.ld;
    op.col0[0] = 0;
    op.col0[1] = (int)q.n;
    unsigned char* base_i = w + B.inst_off[i];
    const size_t s = (size_t)q.s, n = (size_t)q.n;
    size_t o = 0;
    void* partial = base_i + o; o = align_up(o + (size_t)B.groups[i] * s * n * 8);
    double* sa = reinterpret_cast<double*>(base_i + o); o = align_up(o + s * n * 8);
    double* R = reinterpret_cast<double*>(base_i + o); o = align_up(o + svd_work_R_bytes((int)s, (int)n));
    double2* lg = reinterpret_cast<double2*>(base_i + o); o = align_up(o + svd_work_log_bytes((int)s, (int)n, dflt_sweeps(base)));
    double* sig = reinterpret_cast<double*>(base_i + o); o = align_up(o + n * 8);
    int* order = reinterpret_cast<int*>(base_i + o); o = align_up(o + n * 4);
    double* cn = reinterpret_cast<double*>(base_i + o); o = align_up(o + n * 8);
    void* jr = base_i + o;
    batch_fill_inst(hinst + (size_t)i * batch_inst_bytes(), op, q.m, (int)q.n, (int)q.s, (int)q.k,
                    B.groups[i], (int)((q.n + kBatchCols - 1) / kBatchCols), dflt_sweeps(base), q.seed,
                    reinterpret_cast<const int*>(w + B.rows + rows_off[i]), partial, sa, R, lg, sig, order, cn, jr,
                    q.Vk, q.sigma_k, q.info);
  }
  int t = 0;
  for (int oi = 0; oi < count; ++oi) {
    const int i = ord[oi];
    const int ct = (int)((probs[i].n + kBatchCols - 1) / kBatchCols);
    for (int g = 0; g < B.groups[i]; ++g)
      for (int c = 0; c < ct; ++c) batch_fill_tile(htile + (size_t)(t++) * batch_tile_bytes(), i, c, g);
  }
  const bool copied = hipMemcpyAsync(w + B.insts, hinst, ib, hipMemcpyHostToDevice, st) == hipSuccess &&
                      hipMemcpyAsync(w + B.tiles, htile, tb, hipMemcpyHostToDevice, st) == hipSuccess;
  if ((rc = stage_release(slot, st)) || !copied) return NSK_EDEVICE;
  int devid = 0, cus = 256;
  if (hipGetDevice(&devid) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, devid) == hipSuccess && v > 0) cus = v;
  }
  const size_t lds = batched_lds_bytes(s_max, n_max);
  const int per_cu = lds <= 80 * 1024 ? 2 : 1;
  const int grid = std::min(B.ntiles, cus * per_cu);
  return dev(launch_batched(w + B.insts, count, w + B.tiles, B.ntiles, reinterpret_cast<int*>(w + B.counters), dtype,
                            acc, grid, lds, st));
}

// ------------------------------------------------------------------------------ profiler
int nsk_profile_enable(int32_t max_calls) {
  if (max_calls < 0 || max_calls > 100000) return NSK_EINVAL;
  for (hipEvent_t e : g_prof.ev) (void)hipEventDestroy(e);
  g_prof.ev.clear();
  g_prof.max_calls = 0;
  g_prof.calls = 0;
  g_prof.cur = -1;
  if (max_calls == 0) return NSK_OK;
  g_prof.ev.resize((size_t)max_calls * (NSK_PROF_STAGES + 1));
  for (auto& e : g_prof.ev)
    if (hipEventCreate(&e) != hipSuccess) return NSK_EDEVICE;
  g_prof.max_calls = max_calls;
  return NSK_OK;
}

int nsk_profile_read(double* ms, int32_t* calls) {
  if (!ms || !calls) return NSK_EINVAL;
  for (int st = 0; st < NSK_PROF_STAGES; ++st) ms[st] = 0;
  *calls = g_prof.calls;
  for (int c = 0; c < g_prof.calls; ++c) {
    hipEvent_t* e = &g_prof.ev[(size_t)c * (NSK_PROF_STAGES + 1)];
    if (hipEventSynchronize(e[NSK_PROF_STAGES]) != hipSuccess) return NSK_EDEVICE;
    for (int st = 0; st < NSK_PROF_STAGES; ++st) {
      float t = 0;
      if (hipEventElapsedTime(&t, e[st], e[st + 1]) != hipSuccess) return NSK_EDEVICE;
      ms[st] += t;
    }
  }
  return NSK_OK;
}

// ------------------------------------------------------------------------------ draws
int nsk_philox(uint64_t seed, uint64_t idx, uint32_t sub, uint32_t stream, uint32_t out[4]) {
  if (!out) return NSK_EINVAL;
  const Words w = philox(seed, idx, sub, stream);
  for (int i = 0; i < 4; ++i) out[i] = w.w[i];
  return NSK_OK;
}

int nsk_draw_signs(uint64_t seed, int64_t m, int8_t* d) {
  if (m < 1 || !d) return NSK_EINVAL;
  for (int64_t j = 0; j < m; ++j) {
    const uint32_t w = word(philox(seed, (uint64_t)(j >> 7), 0, kSigns), (uint32_t)((j >> 5) & 3));
    d[j] = ((w >> (j & 31)) & 1u) ? -1 : 1;
  }
  return NSK_OK;
}

int nsk_draw_srht_rows(uint64_t seed, int64_t m, int64_t s, int64_t* rows) {
  if (m < 1 || s < 1 || s > next_pow2(m) || !rows) return NSK_EINVAL;
  std::vector<int64_t> r;
  srht_rows_host(seed, next_pow2(m), s, r);
  std::copy(r.begin(), r.end(), rows);
  return NSK_OK;
}

int nsk_draw_sparse(uint64_t seed, int64_t m, int64_t s, int32_t zeta, int32_t* rows, int8_t* signs) {
  if (m < 1 || zeta < 1 || zeta > 32 || zeta > s || s > 65535 || !rows || !signs) return NSK_EINVAL;
  for (int64_t j = 0; j < m; ++j) {
    int rw[32];
    uint32_t nb;
    sparse_column<32>(seed, (uint64_t)j, (int)s, zeta, rw, nb);
    for (int t = 0; t < zeta; ++t) {
      rows[j * zeta + t] = rw[t];
      signs[j * zeta + t] = ((nb >> t) & 1u) ? -1 : 1;
    }
  }
  return NSK_OK;
}

int nsk_draw_signs_device(uint64_t seed, int64_t m, int8_t* d, void* stream) {
  if (m < 1 || !d) return NSK_EINVAL;
  return dev(launch_draw_signs(seed, m, d, (hipStream_t)stream));
}

int nsk_draw_srht_rows_device(uint64_t seed, int64_t m, int64_t s, int32_t* rows, void* stream) {
  if (m < 1 || m > ((int64_t)1 << 31) || s < 1 || s > 2048 || s > next_pow2(m) || !rows) return NSK_EINVAL;
  return dev(launch_srht_rows(seed, next_pow2(m), (int)s, rows, (hipStream_t)stream));
}

int nsk_draw_sparse_device(uint64_t seed, int64_t m, int64_t s, int32_t zeta, int32_t* rows, int8_t* signs,
                           void* stream) {
  if (m < 1 || zeta < 1 || zeta > 32 || zeta > s || s > 65535 || !rows || !signs) return NSK_EINVAL;
  return dev(launch_draw_sparse(seed, m, (int)s, zeta, rows, signs, (hipStream_t)stream));
}

int nsk_draw_gaussian_device(uint64_t seed, int64_t s, int64_t j0, int64_t j1, int32_t dtype, float* G,
                             void* stream) {
  if (s < 1 || j0 < 0 || j1 <= j0 || !G) return NSK_EINVAL;
  if (dtype != NSK_F32 && dtype != NSK_BF16 && dtype != NSK_F8E4M3) return NSK_EINVAL;
  return dev(launch_draw_gauss(seed, (int)s, j0, j1, dtype, G, (hipStream_t)stream));
}

}  // extern "C"
