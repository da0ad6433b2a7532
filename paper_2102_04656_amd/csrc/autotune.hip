// Autotuner of the launch schedules.
//
// The paper tunes only the number of centres and the candidate budget of the
// divide-and-conquer (Sec. 4.5); the schedule knobs here are the GPU's own:
// which distance tile runs (vector-ALU popcount or int8 matrix cores), the
// column-block width of the persistent build (the window of candidates all
// work-groups stream through L2 together), the tile schedule (the LDS split
// between the rows' pending-key buffers and the stage ring), and the work
// order of a batched launch. Every candidate computes the same graph (exact,
// (distance, index) order), so tuning never changes results; candidates are
// timed with HIP events on the caller's stream and the fastest is kept.
//
// Tuned single builds are remembered per (code length, K, size bucket) for
// the process, and appended as one JSON object per line to the file named by
// BDG_AUTOTUNE_CACHE (which is read back on first use), so that later builds
// with path AUTO and no explicit column block take the tuned schedule.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "bdg.h"
#include "kernels.h"

namespace bdg {
int api_error(int status, const char* fmt, ...);
int api_device_error(hipError_t e, const char* what);
void api_clear_error();

namespace {

struct Tuned {
  int path;
  uint32_t col_block;
  int schedule;
};

std::mutex g_mu;
bool g_loaded = false;
std::map<std::tuple<uint32_t, uint32_t, uint32_t>, Tuned> g_cache;

uint32_t size_bucket(uint32_t n) {
  uint32_t b = 0;
  while (b < 31 && (1u << (b + 1)) <= n) ++b;
  return b;  // floor(log2 n)
}

void load_cache_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = getenv("BDG_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    unsigned bits = 0, K = 0, bucket = 0, cb = 0;
    int p = 0, sc = 0;
    if (strstr(line, "\"kind\": \"build\"") &&
        sscanf(strstr(line, "\"bits\""), "\"bits\": %u, \"K\": %u, \"bucket\": %u, \"path\": %d, "
               "\"col_block\": %u, \"schedule\": %d", &bits, &K, &bucket, &p, &cb, &sc) == 6)
      g_cache[std::make_tuple(bits, K, bucket)] = Tuned{p, cb, sc};
  }
  fclose(f);
}

void append_cache_line(const char* json) {
  const char* path = getenv("BDG_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s\n", json);
  fclose(f);
}

void put_report(char* report, size_t len, const std::string& s) {
  if (!report || !len) return;
  const size_t m = s.size() < len - 1 ? s.size() : len - 1;
  memcpy(report, s.data(), m);
  report[m] = 0;
}

// Average milliseconds of `reps` runs of `fn` after one warm-up.
template <class F>
int time_ms(F&& fn, hipStream_t stream, int reps, float* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e != hipSuccess) return api_device_error(e, "event create");
  int st = fn();
  if (st == BDG_OK) {
    e = hipEventRecord(a, stream);
    for (int i = 0; i < reps && st == BDG_OK && e == hipSuccess; ++i) st = fn();
    if (e == hipSuccess) e = hipEventRecord(b, stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    if (e == hipSuccess) *ms /= (float)reps;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != BDG_OK) return st;
  if (e != hipSuccess) return api_device_error(e, "event timing");
  return BDG_OK;
}

}  // namespace

// The tuned schedule of a single build, if any (path AUTO, col_block 0).
bool tuned_schedule(uint32_t n, uint32_t bits, uint32_t K, int* path, uint32_t* col_block,
                    int* schedule) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_cache_locked();
  auto it = g_cache.find(std::make_tuple(bits, K, size_bucket(n)));
  if (it == g_cache.end()) return false;
  *path = it->second.path;
  *col_block = it->second.col_block;
  *schedule = it->second.schedule;
  return true;
}

}  // namespace bdg

extern "C" {

int bdg_autotune_build(const uint64_t* codes, uint32_t n, uint32_t bits, uint32_t K,
                       uint32_t* out_idx, uint16_t* out_dist, bdg_knn_opts* opts, void* stream_,
                       char* report, size_t report_len) {
  bdg::api_clear_error();
  if (!opts || opts->struct_size < sizeof(bdg_knn_opts))
    return bdg::api_error(BDG_EINVAL, "opts must be a full bdg_knn_opts");
  if (!codes || !out_idx || !out_dist) return bdg::api_error(BDG_EINVAL, "null device pointer");
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  struct Cand {
    int path;
    uint32_t col_block;
    int schedule;
    float ms;
  };
  std::vector<Cand> cands;
  for (int sc = 0; sc < bdg::kTileSchedules; ++sc)
    for (uint32_t cb : {131072u, 262144u, 524288u}) cands.push_back({BDG_PATH_MFMA, cb, sc, 0.f});
  cands.push_back({BDG_PATH_POPC, 131072u, 0, 0.f});
  // the candidates this build supports, and one workspace large enough for all
  size_t ws = 0;
  std::vector<Cand> ok;
  for (const Cand& c : cands) {
    bdg_knn_opts o = *opts;
    o.path = c.path;
    o.col_block = c.col_block;
    o.tile_schedule = (uint32_t)c.schedule;
    o.workspace = nullptr;
    o.workspace_bytes = 0;
    o.n_tile_events = 0;
    o.tile_events = nullptr;
    size_t b = 0;
    if (bdg_build_knn_workspace_size(n, bits, K, &o, &b) == BDG_OK) {
      // a column block wider than the input is the same schedule as the input's width
      bool dup = false;
      for (const Cand& d : ok)
        dup |= d.path == c.path && d.schedule == c.schedule && d.col_block >= n && c.col_block >= n;
      if (!dup) ok.push_back(c);
      if (b > ws) ws = b;
    }
  }
  bdg::api_clear_error();
  if (ok.empty()) return bdg::api_error(BDG_EUNSUPPORTED, "no schedule supports these arguments");
  void* buf = nullptr;
  if (ws) {
    hipError_t e = hipMalloc(&buf, ws);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return bdg::api_error(BDG_ENOMEM, "autotune workspace of %zu bytes failed", ws);
    }
  }
  int st = BDG_OK;
  size_t best = 0;
  for (size_t i = 0; i < ok.size() && st == BDG_OK; ++i) {
    bdg_knn_opts o = *opts;
    o.path = ok[i].path;
    o.col_block = ok[i].col_block;
    o.tile_schedule = (uint32_t)ok[i].schedule;
    o.workspace = buf;
    o.workspace_bytes = ws;
    o.n_tile_events = 0;
    o.tile_events = nullptr;
    st = bdg::time_ms([&] { return bdg_build_knn_ex(codes, n, bits, K, out_idx, out_dist, &o,
                                                    stream); },
                      stream, 2, &ok[i].ms);
    if (st == BDG_OK && ok[i].ms < ok[best].ms) best = i;
  }
  if (buf) (void)hipFree(buf);
  if (st != BDG_OK) return st;
  opts->path = ok[best].path;
  opts->col_block = ok[best].col_block;
  opts->tile_schedule = (uint32_t)ok[best].schedule;
  {
    std::lock_guard<std::mutex> lk(bdg::g_mu);
    bdg::load_cache_locked();
    bdg::g_cache[std::make_tuple(bits, K, bdg::size_bucket(n))] =
        bdg::Tuned{ok[best].path, ok[best].col_block, ok[best].schedule};
  }
  char line[512];
  snprintf(line, sizeof line,
           "{\"kind\": \"build\", \"bits\": %u, \"K\": %u, \"bucket\": %u, \"path\": %d, "
           "\"col_block\": %u, \"schedule\": %d, \"n\": %u, \"ms\": %.3f}",
           bits, K, bdg::size_bucket(n), ok[best].path, ok[best].col_block, ok[best].schedule, n,
           ok[best].ms);
  bdg::append_cache_line(line);
  std::string rep = "{\"chosen\": ";
  rep += line;
  rep += ", \"knobs\": [\"path\", \"col_block\", \"schedule\"], \"candidates\": [";
  for (size_t i = 0; i < ok.size(); ++i) {
    char c[160];
    snprintf(c, sizeof c, "%s{\"path\": %d, \"col_block\": %u, \"schedule\": %d, \"ms\": %.3f}",
             i ? ", " : "", ok[i].path, ok[i].col_block, ok[i].schedule, ok[i].ms);
    rep += c;
  }
  rep += "]}";
  bdg::put_report(report, report_len, rep);
  return BDG_OK;
}

int bdg_autotune_batched(bdg_batch_plan* plan, const uint64_t* codes, uint32_t* out_idx,
                         uint16_t* out_dist, void* stream_, char* report, size_t report_len) {
  bdg::api_clear_error();
  if (!plan) return bdg::api_error(BDG_EINVAL, "plan is NULL");
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  struct Cand {
    int order, schedule;
    float ms;
  };
  std::vector<Cand> cands;
  for (int sc = 0; sc < bdg::kTileSchedules; ++sc)
    for (int order : {BDG_ORDER_LONGEST_FIRST, BDG_ORDER_SHARD}) cands.push_back({order, sc, 0.f});
  int st = BDG_OK;
  size_t best = 0;
  std::vector<Cand> ok;
  for (Cand c : cands) {
    if (bdg_batch_plan_set_schedule(plan, c.schedule) != BDG_OK) continue;  // not built here
    st = bdg_batch_plan_set_order(plan, c.order);
    if (st == BDG_OK)
      st = bdg::time_ms([&] { return bdg_build_knn_batched_plan(plan, codes, out_idx, out_dist,
                                                                 stream); },
                        stream, 1, &c.ms);
    if (st != BDG_OK) return st;
    ok.push_back(c);
    if (c.ms < ok[best].ms) best = ok.size() - 1;
  }
  bdg::api_clear_error();
  if (ok.empty()) return bdg::api_error(BDG_EUNSUPPORTED, "no schedule supports this plan");
  st = bdg_batch_plan_set_schedule(plan, ok[best].schedule);
  if (st == BDG_OK) st = bdg_batch_plan_set_order(plan, ok[best].order);
  if (st != BDG_OK) return st;
  bdg_batch_info info;
  bdg_batch_plan_info(plan, &info);
  char line[256];
  snprintf(line, sizeof line,
           "{\"kind\": \"batched\", \"shards\": %u, \"rows\": %u, \"order\": %d, "
           "\"schedule\": %d, \"ms\": %.3f}",
           info.shards, info.rows, ok[best].order, ok[best].schedule, ok[best].ms);
  bdg::append_cache_line(line);
  std::string rep = "{\"chosen\": ";
  rep += line;
  rep += ", \"knobs\": [\"order\", \"schedule\"], \"candidates\": [";
  for (size_t i = 0; i < ok.size(); ++i) {
    char c[128];
    snprintf(c, sizeof c, "%s{\"order\": %d, \"schedule\": %d, \"ms\": %.3f}", i ? ", " : "",
             ok[i].order, ok[i].schedule, ok[i].ms);
    rep += c;
  }
  rep += "]}";
  bdg::put_report(report, report_len, rep);
  return BDG_OK;
}

}  // extern "C"
