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
// with path AUTO and no explicit column block take the tuned schedule. With
// BDG_AUTOTUNE_LOG set, every candidate's time goes to stderr as it is taken
// (a tuning run over large inputs takes minutes).
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
  uint32_t bound_group;  // 0: the library default
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
    unsigned bits = 0, K = 0, bucket = 0, cb = 0, bg = 0;
    int p = 0, sc = 0;
    const char* b = strstr(line, "\"bound_group\"");
    if (b) sscanf(b, "\"bound_group\": %u", &bg);
    if (strstr(line, "\"kind\": \"build\"") &&
        sscanf(strstr(line, "\"bits\""), "\"bits\": %u, \"K\": %u, \"bucket\": %u, \"path\": %d, "
               "\"col_block\": %u, \"schedule\": %d", &bits, &K, &bucket, &p, &cb, &sc) == 6)
      g_cache[std::make_tuple(bits, K, bucket)] = Tuned{p, cb, sc, bg};
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
                    int* schedule, uint32_t* bound_group) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_cache_locked();
  auto it = g_cache.find(std::make_tuple(bits, K, size_bucket(n)));
  if (it == g_cache.end()) return false;
  *path = it->second.path;
  *col_block = it->second.col_block;
  *schedule = it->second.schedule;
  *bound_group = it->second.bound_group;
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
  // Coordinate search from the library's defaults: each knob in turn (column
  // block, tile schedule, admission bounds) is swept with the others at their
  // best so far; then the vector-ALU path. Candidates a build does not support
  // are skipped.
  struct Cand {
    int path;
    uint32_t col_block;
    int schedule;
    uint32_t bound_group;
    float ms;
  };
  std::vector<Cand> ok;
  void* buf = nullptr;
  size_t buf_bytes = 0;
  auto same = [&](const Cand& a, const Cand& b) {
    return a.path == b.path && a.schedule == b.schedule && a.bound_group == b.bound_group &&
           (a.col_block == b.col_block || (a.col_block >= n && b.col_block >= n));
  };
  // time one candidate (or reuse its time); returns its index in ok, or -1 if
  // the build does not support it, or -2 - status on an error
  auto run = [&](Cand c) -> long {
    for (size_t i = 0; i < ok.size(); ++i)
      if (same(ok[i], c)) return (long)i;
    bdg_knn_opts o = *opts;
    o.path = c.path;
    o.col_block = c.col_block;
    o.tile_schedule = (uint32_t)c.schedule;
    o.bound_group = c.bound_group;
    o.workspace = nullptr;
    o.workspace_bytes = 0;
    o.n_tile_events = 0;
    o.tile_events = nullptr;
    size_t b = 0;
    if (bdg_build_knn_workspace_size(n, bits, K, &o, &b) != BDG_OK) {
      bdg::api_clear_error();
      return -1;
    }
    if (b > buf_bytes) {
      if (buf) (void)hipFree(buf);
      buf = nullptr;
      buf_bytes = 0;
      hipError_t e = hipMalloc(&buf, b);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return -2 - bdg::api_error(BDG_ENOMEM, "autotune workspace of %zu bytes failed", b);
      }
      buf_bytes = b;
    }
    o.workspace = buf;
    o.workspace_bytes = buf_bytes;
    const int st = bdg::time_ms([&] { return bdg_build_knn_ex(codes, n, bits, K, out_idx, out_dist,
                                                              &o, stream); },
                                stream, 2, &c.ms);
    if (st != BDG_OK) return -2 - st;
    ok.push_back(c);
    if (getenv("BDG_AUTOTUNE_LOG")) {
      fprintf(stderr, "[autotune] path %d col_block %u schedule %d bound_group %u: %.3f ms\n",
              c.path, c.col_block, c.schedule, c.bound_group, c.ms);
      fflush(stderr);
    }
    return (long)ok.size() - 1;
  };
  // the default schedule as the value it resolves to, so it is timed once
  Cand best{BDG_PATH_MFMA, 262144u, bdg::resolve_schedule(bits / 64, K, 0),
            BDG_BOUND_GROUP_DEFAULT, 0.f};
  long bi = -1;
  int st = BDG_OK;
  auto sweep = [&](std::vector<Cand> cs) {
    for (const Cand& c : cs) {
      if (st != BDG_OK) return;
      const long r = run(c);
      if (r <= -2) {
        st = (int)(-2 - r);
        return;
      }
      if (r >= 0 && (bi < 0 || ok[r].ms < ok[bi].ms)) bi = r;
    }
    if (bi >= 0) best = ok[bi];
  };
  {
    std::vector<Cand> cs;
    for (uint32_t cb : {262144u, 131072u, 524288u})
      cs.push_back({BDG_PATH_MFMA, cb, best.schedule, best.bound_group, 0.f});
    sweep(cs);
  }
  {
    std::vector<Cand> cs;
    for (int sc : bdg::kExplicitSchedules) {
      Cand c = best;
      c.schedule = sc;
      cs.push_back(c);
    }
    sweep(cs);
  }
  {
    std::vector<Cand> cs;
    for (uint32_t bg : {BDG_BOUND_GROUP_DEFAULT, BDG_BOUND_OFF, 128u, 512u, 64u}) {
      Cand c = best;
      c.bound_group = bg;
      cs.push_back(c);
    }
    sweep(cs);
  }
  sweep({{BDG_PATH_POPC, 131072u, 0, BDG_BOUND_GROUP_DEFAULT, 0.f}});
  if (buf) (void)hipFree(buf);
  if (st != BDG_OK) return st;
  bdg::api_clear_error();
  if (bi < 0) return bdg::api_error(BDG_EUNSUPPORTED, "no schedule supports these arguments");
  const Cand& w = ok[bi];
  opts->path = w.path;
  opts->col_block = w.col_block;
  opts->tile_schedule = (uint32_t)w.schedule;
  opts->bound_group = w.bound_group;
  {
    std::lock_guard<std::mutex> lk(bdg::g_mu);
    bdg::load_cache_locked();
    bdg::g_cache[std::make_tuple(bits, K, bdg::size_bucket(n))] =
        bdg::Tuned{w.path, w.col_block, w.schedule, w.bound_group};
  }
  char line[512];
  snprintf(line, sizeof line,
           "{\"kind\": \"build\", \"bits\": %u, \"K\": %u, \"bucket\": %u, \"path\": %d, "
           "\"col_block\": %u, \"schedule\": %d, \"bound_group\": %u, \"n\": %u, \"ms\": %.3f}",
           bits, K, bdg::size_bucket(n), w.path, w.col_block, w.schedule, w.bound_group, n, w.ms);
  bdg::append_cache_line(line);
  std::string rep = "{\"chosen\": ";
  rep += line;
  rep += ", \"knobs\": [\"path\", \"col_block\", \"schedule\", \"bound_group\"], \"candidates\": [";
  for (size_t i = 0; i < ok.size(); ++i) {
    char c[200];
    snprintf(c, sizeof c,
             "%s{\"path\": %d, \"col_block\": %u, \"schedule\": %d, \"bound_group\": %u, "
             "\"ms\": %.3f}",
             i ? ", " : "", ok[i].path, ok[i].col_block, ok[i].schedule, ok[i].bound_group, ok[i].ms);
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
  // Coordinate search from the plan's defaults: the work order, then the tile
  // schedule, then the admission bounds, each swept with the others at their
  // best so far. Settings a plan does not support are skipped.
  struct Cand {
    int order, schedule;
    uint32_t bound_group;
    float ms;
  };
  std::vector<Cand> ok;
  size_t best = 0;
  int st = BDG_OK;
  Cand cur{BDG_ORDER_LONGEST_FIRST, 0, BDG_BOUND_GROUP_DEFAULT, 0.f};
  auto sweep = [&](std::vector<Cand> cs) {
    for (Cand c : cs) {
      if (st != BDG_OK) return;
      bool seen = false;
      for (const Cand& o : ok)
        seen |= o.order == c.order && o.schedule == c.schedule && o.bound_group == c.bound_group;
      if (seen) continue;
      if (bdg_batch_plan_set_schedule(plan, c.schedule) != BDG_OK) continue;  // not built here
      st = bdg_batch_plan_set_bound(plan, c.bound_group);
      if (st != BDG_OK) return;
      bdg_batch_info in;
      bdg_batch_plan_info(plan, &in);
      if (in.bound_group != c.bound_group) continue;  // a plan without bounds: one setting
      st = bdg_batch_plan_set_order(plan, c.order);
      if (st == BDG_OK)
        st = bdg::time_ms([&] { return bdg_build_knn_batched_plan(plan, codes, out_idx, out_dist,
                                                                   stream); },
                          stream, 1, &c.ms);
      if (st != BDG_OK) return;
      ok.push_back(c);
      if (getenv("BDG_AUTOTUNE_LOG")) {
        fprintf(stderr, "[autotune] order %d schedule %d bound_group %u: %.3f ms\n", c.order,
                c.schedule, c.bound_group, c.ms);
        fflush(stderr);
      }
      if (c.ms < ok[best].ms) best = ok.size() - 1;
    }
    if (!ok.empty()) cur = ok[best];
  };
  {
    bdg_batch_info in;
    // the library's default schedule, as the value it resolves to for this
    // plan (so that it is timed once)
    st = bdg_batch_plan_set_schedule(plan, BDG_SCHEDULE_DEFAULT);
    if (st != BDG_OK) return st;
    bdg_batch_plan_info(plan, &in);
    cur.schedule = in.schedule;
    if (in.bound_group == BDG_BOUND_OFF) {
      // no bounds unless the plan can take them
      if (bdg_batch_plan_set_bound(plan, BDG_BOUND_GROUP_DEFAULT) == BDG_OK) {
        bdg_batch_plan_info(plan, &in);
        cur.bound_group = in.bound_group;
      }
    }
  }
  sweep({{BDG_ORDER_LONGEST_FIRST, cur.schedule, cur.bound_group, 0.f},
         {BDG_ORDER_SHARD, cur.schedule, cur.bound_group, 0.f}});
  {
    std::vector<Cand> cs;
    for (int sc : bdg::kExplicitSchedules) cs.push_back({cur.order, sc, cur.bound_group, 0.f});
    sweep(cs);
  }
  {
    std::vector<Cand> cs;
    for (uint32_t bg : {BDG_BOUND_GROUP_DEFAULT, BDG_BOUND_OFF, 128u, 512u, 64u})
      cs.push_back({cur.order, cur.schedule, bg, 0.f});
    sweep(cs);
  }
  if (st != BDG_OK) return st;
  bdg::api_clear_error();
  if (ok.empty()) return bdg::api_error(BDG_EUNSUPPORTED, "no schedule supports this plan");
  st = bdg_batch_plan_set_schedule(plan, ok[best].schedule);
  if (st == BDG_OK) st = bdg_batch_plan_set_bound(plan, ok[best].bound_group);
  if (st == BDG_OK) st = bdg_batch_plan_set_order(plan, ok[best].order);
  if (st != BDG_OK) return st;
  bdg_batch_info info;
  bdg_batch_plan_info(plan, &info);
  char line[256];
  snprintf(line, sizeof line,
           "{\"kind\": \"batched\", \"shards\": %u, \"rows\": %u, \"order\": %d, "
           "\"schedule\": %d, \"bound_group\": %u, \"ms\": %.3f}",
           info.shards, info.rows, ok[best].order, ok[best].schedule, ok[best].bound_group,
           ok[best].ms);
  bdg::append_cache_line(line);
  std::string rep = "{\"chosen\": ";
  rep += line;
  rep += ", \"knobs\": [\"order\", \"schedule\", \"bound_group\"], \"candidates\": [";
  for (size_t i = 0; i < ok.size(); ++i) {
    char c[160];
    snprintf(c, sizeof c,
             "%s{\"order\": %d, \"schedule\": %d, \"bound_group\": %u, \"ms\": %.3f}",
             i ? ", " : "", ok[i].order, ok[i].schedule, ok[i].bound_group, ok[i].ms);
    rep += c;
  }
  rep += "]}";
  bdg::put_report(report, report_len, rep);
  return BDG_OK;
}

}  // extern "C"
