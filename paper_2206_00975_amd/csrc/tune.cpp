// Autotuner for the batched persistent launch.
//
// The tunable is the number of 1024-row transform blocks in one sketch tile ("rows per
// tile"): small tiles balance uneven instances across the 256 CUs, large tiles write fewer
// partial sketches (each tile writes an s x 8 FP64 partial).  The tuner times candidate
// values per n-bucket (32 columns wide) on the caller's own instances with HIP events and
// keeps the fastest; results live in a process-wide table, optionally persisted as text in
// the file named by NSK_TUNE_CACHE ("n_bucket dtype acc rows_per_tile" per line).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "nsk.h"

namespace nsk {

namespace {
std::mutex g_mu;
std::map<std::tuple<int, int, int>, int> g_table;
thread_local int g_forced = 0;
bool g_loaded = false;

int bucket(int n) { return (n - 1) / 32; }

void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = std::getenv("NSK_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  int b, dt, acc, r;
  while (std::fscanf(f, "%d %d %d %d", &b, &dt, &acc, &r) == 4)
    if (r >= 1 && r <= 256) g_table[{b, dt, acc}] = r;
  std::fclose(f);
}

void save_locked() {
  const char* path = std::getenv("NSK_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  for (auto& kv : g_table)
    std::fprintf(f, "%d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), kv.second);
  std::fclose(f);
}
}  // namespace

// Default: each tile's FP64 partial (s x 16) stays near 1/16 of the FP32 data it covers
// (1024-row blocks x 16 columns), i.e. rows_per_tile ~ s / 32 blocks with s = 4n.
int heuristic_rows_per_tile(int n) {
  int r = 4;
  while (r < n / 8 && r < 64) r <<= 1;
  return r;
}

int tuned_rows_per_tile(int n, int64_t m, int dtype, int acc) {
  (void)m;
  if (g_forced > 0) return g_forced;
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  auto it = g_table.find({bucket(n), dtype, acc});
  return it == g_table.end() ? heuristic_rows_per_tile(n) : it->second;
}

}  // namespace nsk

using namespace nsk;

extern "C" {

int nsk_tune_lookup(int n, int dtype, int acc) { return tuned_rows_per_tile(n, 0, dtype, acc); }

int nsk_tune_set(int n, int dtype, int acc, int rows_per_tile) {
  if (n < 1 || rows_per_tile < 1 || rows_per_tile > 256) return NSK_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  g_table[{bucket(n), dtype, acc}] = rows_per_tile;
  return NSK_OK;
}

int nsk_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  g_loaded = true;
  return NSK_OK;
}

// Times the candidates on up to `per_bucket` instances of each n-bucket present in probs
// and records the fastest.  Host-blocking; uses the caller's workspace (candidates whose
// workspace would not fit are skipped) and overwrites the instances' outputs.
int nsk_autotune_batched(const nsk_problem* probs, int32_t count, const nsk_desc* base, void* ws, size_t ws_bytes,
                         void* stream, int32_t per_bucket) {
  if (!probs || count < 1 || !base || !ws) return NSK_EINVAL;
  if (per_bucket < 1) per_bucket = 8;
  hipStream_t st = (hipStream_t)stream;
  const int acc = base->acc == NSK_F32 ? NSK_F32 : NSK_F64;
  std::map<int, std::vector<nsk_problem>> groups;
  for (int i = 0; i < count; ++i) {
    auto& v = groups[bucket((int)probs[i].n)];
    if ((int)v.size() < per_bucket) v.push_back(probs[i]);
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return NSK_EDEVICE;
  const int cands[] = {2, 4, 8, 16, 32, 64};
  int rc = NSK_OK;
  for (auto& kv : groups) {
    const auto& sub = kv.second;
    float best = 1e30f;
    int best_r = heuristic_rows_per_tile((int)sub[0].n);
    for (int r : cands) {
      g_forced = r;
      const size_t need = nsk_batched_workspace_bytes(sub.data(), (int)sub.size(), base);
      if (need == 0 || need > ws_bytes) continue;
      float total = 0;
      bool ok = true;
      for (int rep = 0; rep < 3 && ok; ++rep) {
        ok = hipEventRecord(e0, st) == hipSuccess;
        ok = ok && nsk_trailing_rsv_batched(sub.data(), (int)sub.size(), base, ws, ws_bytes, stream) == NSK_OK;
        ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0;
        ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (rep > 0) total += ms;  // first run warms up
      }
      if (!ok) {
        rc = NSK_EDEVICE;
        continue;
      }
      if (total < best) {
        best = total;
        best_r = r;
      }
    }
    g_forced = 0;
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_table[{kv.first, (int)sub[0].dtype, acc}] = best_r;
  }
  g_forced = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    save_locked();
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
