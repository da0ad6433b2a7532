// Many independent partitions in one persistent launch (host side), and the
// autotuner of the launch schedules.
//
// The single-pass divide-and-conquer produces partitions of very uneven size
// (a record joins its t nearest centres until a candidate budget is reached,
// Sec. 3.2) and the paper balances them over the reduce nodes (Sec. 3.6 (1)).
// Here every partition (shard) is an independent exact kNN problem with
// shard-local indices, and all of them run in one persistent launch: work
// items of up to 256 rows of one shard against all of its columns are taken
// from a shared counter, longest first, by one work-group per CU. The plan
// (items, counter, operand workspace) is built once; the launch sequence
// (operand prep, counter reset, persistent kernel) allocates nothing and can
// be captured in a HIP graph and replayed.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "bdg.h"
#include "kernels.h"

namespace bdg {
int api_error(int status, const char* fmt, ...);
int api_device_error(hipError_t e, const char* what);
void api_clear_error();
}  // namespace bdg

struct bdg_batch_plan {
  uint32_t S = 0, bits = 0, words = 0, K = 0, idx_bits = 0;
  uint32_t n_total = 0, nitems = 0, grid = 0;
  uint32_t item_cap = 0;          // items the device item buffer holds
  int order = BDG_ORDER_LONGEST_FIRST;
  int schedule = 0;               // tile schedule (BDG_SCHEDULE_*)
  std::vector<uint64_t> offsets;  // host copy, S + 1 entries
  void* dev = nullptr;            // items | counter | operand fragments | bounds
  size_t dev_bytes = 0;
  bdg::BatchItem* items = nullptr;
  uint32_t* counter = nullptr;
  void* frags = nullptr;
  // admission bounds: rows per pivot group (0: none), pivots, and the device
  // segment tables (shard first rows, first pivots), bounds and scratch
  uint32_t bgroup = 0, npiv = 0, base = 0, total = 0;
  uint32_t* seg = nullptr;
  uint32_t* pseg = nullptr;
  uint16_t* bound = nullptr;
  void* bscr = nullptr;
  // optional events around the persistent kernel of eager enqueues
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  // captured launch sequence and the arguments it was captured with
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* g_codes = nullptr;
  void* g_idx = nullptr;
  void* g_dist = nullptr;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

std::vector<bdg::BatchItem> make_items(const std::vector<uint64_t>& off, uint32_t rows_per_item,
                                       int order) {
  std::vector<bdg::BatchItem> items;
  const size_t S = off.size() - 1;
  for (size_t s = 0; s < S; ++s) {
    const uint32_t lo = (uint32_t)off[s], hi = (uint32_t)off[s + 1];
    for (uint32_t r = lo; r < hi; r += rows_per_item) {
      bdg::BatchItem it;
      it.row0 = r;
      it.nrows = std::min(rows_per_item, hi - r);
      it.lo = lo;
      it.hi = hi;
      items.push_back(it);
    }
  }
  if (order == BDG_ORDER_LONGEST_FIRST) {
    // cost of an item ~ rows x columns; stable, so equal costs keep shard order
    std::stable_sort(items.begin(), items.end(), [](const bdg::BatchItem& a,
                                                    const bdg::BatchItem& b) {
      return (uint64_t)a.nrows * (a.hi - a.lo) > (uint64_t)b.nrows * (b.hi - b.lo);
    });
  }
  return items;
}

void drop_graph(bdg_batch_plan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

int upload_items(bdg_batch_plan* p) {
  std::vector<bdg::BatchItem> items =
      make_items(p->offsets, bdg::sched_rows_per_wg(p->K, p->schedule), p->order);
  // the item buffer holds the items of the smallest tile (every schedule's
  // tile has at least run_rows_per_wg(K) rows)
  if (items.size() > p->item_cap) return bdg::api_error(BDG_EDEVICE, "work item count changed");
  p->nitems = (uint32_t)items.size();
  if (p->nitems) {
    // A launch of this plan may still be in flight on any stream (a pool
    // stream does not wait for the null stream): let every queued launch
    // finish before its work list is rewritten. This is a set-up call, never
    // on the build path.
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
      e = hipMemcpy(p->items, items.data(), items.size() * sizeof(bdg::BatchItem),
                    hipMemcpyHostToDevice);
    if (e != hipSuccess) return bdg::api_device_error(e, "work item upload");
  }
  drop_graph(p);
  return BDG_OK;
}

// Pivots of every shard for a group size (the first pivot of shard s at
// pseg[s]); the scratch is sized for the smallest group size.
std::vector<uint32_t> pivot_offsets(const std::vector<uint64_t>& off, uint32_t group) {
  std::vector<uint32_t> ps(off.size(), 0);
  for (size_t s = 0; s + 1 < off.size(); ++s)
    ps[s + 1] = ps[s] + bdg::bound_pivots((uint32_t)(off[s + 1] - off[s]), group);
  return ps;
}

// Set the admission-bound group size (BDG_BOUND_OFF: none) and upload its
// pivot table. A set-up call: waits for queued work first.
int set_bound_group(bdg_batch_plan* p, uint32_t group) {
  if (group != BDG_BOUND_OFF && (group < BDG_BOUND_GROUP_MIN || group > BDG_BOUND_GROUP_MAX))
    return bdg::api_error(BDG_EUNSUPPORTED, "bound_group %u outside [%u, %u] (or BDG_BOUND_OFF)",
                          group, BDG_BOUND_GROUP_MIN, BDG_BOUND_GROUP_MAX);
  const uint32_t g = (group == BDG_BOUND_OFF || !p->seg) ? 0u : group;
  if (g == p->bgroup) return BDG_OK;
  hipError_t e = hipDeviceSynchronize();
  if (g) {
    const std::vector<uint32_t> ps = pivot_offsets(p->offsets, g);
    if (e == hipSuccess)
      e = hipMemcpy(p->pseg, ps.data(), ps.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    p->npiv = ps.back();
  }
  if (e != hipSuccess) return bdg::api_device_error(e, "bound table upload");
  p->bgroup = g;
  drop_graph(p);
  return BDG_OK;
}

int enqueue(const bdg_batch_plan* p, const uint64_t* codes, uint32_t* out_idx, uint16_t* out_dist,
            hipStream_t stream, bool timed) {
  if (p->nitems == 0) return BDG_OK;
  hipError_t e = bdg::launch_prep(codes, p->n_total, p->words, p->frags, stream);
  if (e == hipSuccess && p->bgroup) {
    bdg::BoundArgs b;
    b.codes = codes;
    b.words = p->words;
    b.bits = p->bits;
    b.K = p->K;
    b.group = p->bgroup;
    b.cap = 1023;
    b.nseg = p->S;
    b.seg = p->seg;
    b.pseg = p->pseg;
    b.base = p->base;
    b.total = p->total;
    b.npiv = p->npiv;
    b.scratch = p->bscr;
    b.bound = p->bound;
    e = bdg::launch_bounds_pass(b, stream);
  }
  if (e == hipSuccess) {
    bdg::BatchArgs a;
    a.codes = codes;
    a.frags = p->frags;
    a.words = p->words;
    a.bits = p->bits;
    a.K = p->K;
    a.idx_bits = p->idx_bits;
    a.items = p->items;
    a.nitems = p->nitems;
    a.counter = p->counter;
    a.grid = p->grid;
    a.out_idx = out_idx;
    a.out_dist = out_dist;
    a.schedule = p->schedule;
    a.bound = p->bgroup ? p->bound : nullptr;
    a.bound_base = p->base;
    timed = timed && p->ev_start && p->ev_stop;
    if (timed) e = hipEventRecord(p->ev_start, stream);
    if (e == hipSuccess) e = bdg::launch_mfma_batched(a, stream);
    if (e == hipSuccess && timed) e = hipEventRecord(p->ev_stop, stream);
  }
  if (e != hipSuccess) return bdg::api_device_error(e, "batched launch");
  return BDG_OK;
}

}  // namespace

extern "C" {

int bdg_batch_plan_create(const uint64_t* offsets, uint32_t S, uint32_t bits, uint32_t K,
                          const bdg_knn_opts* opts, bdg_batch_plan** plan) {
  bdg::api_clear_error();
  if (!plan) return bdg::api_error(BDG_EINVAL, "plan is NULL");
  *plan = nullptr;
  if (!offsets) return bdg::api_error(BDG_EINVAL, "offsets is NULL");
  if (opts && opts->struct_size < offsetof(bdg_knn_opts, workspace))
    return bdg::api_error(BDG_EINVAL, "opts->struct_size too small (%u)", opts->struct_size);
  if (bits == 0 || bits % 64 != 0)
    return bdg::api_error(BDG_EINVAL, "bits must be a positive multiple of 64 (got %u)", bits);
  if (bits > BDG_MAX_BITS) return bdg::api_error(BDG_EUNSUPPORTED, "bits > %u", BDG_MAX_BITS);
  if (K == 0) return bdg::api_error(BDG_EINVAL, "K must be >= 1");
  if (K > BDG_MAX_K_TILE) return bdg::api_error(BDG_EUNSUPPORTED, "K > %u", BDG_MAX_K_TILE);
  if (offsets[S] >= 0xFFFFFFFFull)
    return bdg::api_error(BDG_EUNSUPPORTED, "more than 2^32 - 2 rows in all shards");
  const uint32_t words = bits / 64;
  uint64_t largest = 0;
  for (uint32_t s = 0; s < S; ++s) {
    if (offsets[s + 1] < offsets[s])
      return bdg::api_error(BDG_EINVAL, "offsets must be non-decreasing (shard %u)", s);
    largest = std::max<uint64_t>(largest, offsets[s + 1] - offsets[s]);
  }
  if (!bdg::run_supported((uint32_t)largest, words, K))
    return bdg::api_error(BDG_EUNSUPPORTED,
                          "batched build does not support bits=%u K=%u with a %llu-row shard",
                          bits, K, (unsigned long long)largest);
  bdg_batch_plan* p = new (std::nothrow) bdg_batch_plan;
  if (!p) return bdg::api_error(BDG_ENOMEM, "plan allocation failed");
  p->S = S;
  p->bits = bits;
  p->words = words;
  p->K = K;
  p->idx_bits = bdg::run_idx_bits(bits);
  p->n_total = (uint32_t)offsets[S];
  p->offsets.assign(offsets, offsets + S + 1);
  p->order = (opts && opts->tile_variant == BDG_ORDER_SHARD) ? BDG_ORDER_SHARD
                                                             : BDG_ORDER_LONGEST_FIRST;
  const int sc = (opts && opts->struct_size >= sizeof(bdg_knn_opts)) ? (int)opts->tile_schedule : 0;
  if (!bdg::schedule_supported(words, K, sc)) {
    delete p;
    return bdg::api_error(BDG_EUNSUPPORTED, "tile schedule %d is not built for bits=%u", sc, bits);
  }
  p->schedule = bdg::resolve_schedule(words, K, sc);
  p->item_cap = (uint32_t)make_items(p->offsets, bdg::run_rows_per_wg(K), p->order).size();
  p->nitems = (uint32_t)make_items(p->offsets, bdg::sched_rows_per_wg(K, p->schedule),
                                   p->order).size();
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    delete p;
    return bdg::api_device_error(e, "device query");
  }
  p->grid = (uint32_t)(cus > 0 ? cus : 1);
  const size_t items_bytes = align256((size_t)std::max<uint32_t>(p->item_cap, 1) *
                                      sizeof(bdg::BatchItem));
  p->dev_bytes = items_bytes + 256 + align256(bdg::prep_bytes(p->n_total, words));
  // admission bounds: shards with more than K + 1 rows exist
  uint32_t bgroup = (opts && opts->struct_size >= sizeof(bdg_knn_opts)) ? opts->bound_group : 0;
  if (bgroup == 0) bgroup = BDG_BOUND_GROUP_DEFAULT;
  if (bgroup != BDG_BOUND_OFF && (bgroup < BDG_BOUND_GROUP_MIN || bgroup > BDG_BOUND_GROUP_MAX)) {
    delete p;
    return bdg::api_error(BDG_EUNSUPPORTED, "bound_group %u outside [%u, %u] (or BDG_BOUND_OFF)",
                          bgroup, BDG_BOUND_GROUP_MIN, BDG_BOUND_GROUP_MAX);
  }
  p->base = (uint32_t)offsets[0];
  p->total = (uint32_t)(offsets[S] - offsets[0]);
  size_t seg_off = 0, pseg_off = 0, bound_off = 0, bscr_off = 0;
  if (largest > K + 1) {
    const uint32_t npiv_max = pivot_offsets(p->offsets, BDG_BOUND_GROUP_MIN).back();
    seg_off = p->dev_bytes;
    pseg_off = seg_off + align256(((size_t)S + 1) * 4);
    bound_off = pseg_off + align256(((size_t)S + 1) * 4);
    bscr_off = bound_off + align256((size_t)p->total * 2);
    p->dev_bytes = bscr_off + bdg::bound_scratch_bytes(p->total, words, npiv_max);
  }
  const char* fail = getenv("BDG_TEST_FAIL_ALLOC");
  if (fail && fail[0] == '1') {
    delete p;
    return bdg::api_error(BDG_ENOMEM, "plan allocation failed (forced by test hook)");
  }
  e = hipMalloc(&p->dev, p->dev_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return bdg::api_error(BDG_ENOMEM, "plan device allocation of %zu bytes failed",
                          p->dev_bytes);
  }
  p->items = static_cast<bdg::BatchItem*>(p->dev);
  p->counter = reinterpret_cast<uint32_t*>(static_cast<char*>(p->dev) + items_bytes);
  p->frags = static_cast<char*>(p->dev) + items_bytes + 256;
  int st = BDG_OK;
  if (seg_off) {
    char* d = static_cast<char*>(p->dev);
    p->seg = reinterpret_cast<uint32_t*>(d + seg_off);
    p->pseg = reinterpret_cast<uint32_t*>(d + pseg_off);
    p->bound = reinterpret_cast<uint16_t*>(d + bound_off);
    p->bscr = d + bscr_off;
    std::vector<uint32_t> sg(p->offsets.begin(), p->offsets.end());
    e = hipMemcpy(p->seg, sg.data(), sg.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) st = bdg::api_device_error(e, "bound table upload");
    if (st == BDG_OK) st = set_bound_group(p, bgroup);
    if (st != BDG_OK) {
      bdg_batch_plan_destroy(p);
      return st;
    }
  }
  st = upload_items(p);
  if (st != BDG_OK) {
    bdg_batch_plan_destroy(p);
    return st;
  }
  *plan = p;
  return BDG_OK;
}

void bdg_batch_plan_destroy(bdg_batch_plan* plan) {
  if (!plan) return;
  drop_graph(plan);
  if (plan->dev) (void)hipFree(plan->dev);
  delete plan;
}

int bdg_batch_plan_info(const bdg_batch_plan* plan, bdg_batch_info* info) {
  if (!plan || !info) return bdg::api_error(BDG_EINVAL, "plan or info is NULL");
  info->shards = plan->S;
  info->rows = plan->n_total;
  info->work_items = plan->nitems;
  info->workgroups = plan->grid;
  info->order = plan->order;
  info->schedule = plan->schedule;
  info->bound_group = plan->bgroup ? plan->bgroup : BDG_BOUND_OFF;
  info->reserved = 0;
  uint64_t pairs = 0;
  for (uint32_t s = 0; s < plan->S; ++s) {
    const uint64_t ns = plan->offsets[s + 1] - plan->offsets[s];
    pairs += ns * (ns ? ns - 1 : 0);
  }
  info->pairs = pairs;
  info->device_bytes = plan->dev_bytes;
  return BDG_OK;
}

int bdg_batch_plan_set_order(bdg_batch_plan* plan, int order) {
  if (!plan) return bdg::api_error(BDG_EINVAL, "plan is NULL");
  if (order != BDG_ORDER_LONGEST_FIRST && order != BDG_ORDER_SHARD)
    return bdg::api_error(BDG_EINVAL, "unknown work order %d", order);
  if (order == plan->order) return BDG_OK;
  plan->order = order;
  return upload_items(plan);
}

int bdg_batch_plan_set_schedule(bdg_batch_plan* plan, int schedule) {
  if (!plan) return bdg::api_error(BDG_EINVAL, "plan is NULL");
  if (schedule < 0 || schedule >= bdg::kTileSchedules)
    return bdg::api_error(BDG_EINVAL, "unknown tile schedule %d", schedule);
  if (!bdg::schedule_supported(plan->words, plan->K, schedule))
    return bdg::api_error(BDG_EUNSUPPORTED, "tile schedule %d is not built for bits=%u", schedule,
                          plan->bits);
  schedule = bdg::resolve_schedule(plan->words, plan->K, schedule);
  if (schedule == plan->schedule) return BDG_OK;
  // a launch of the captured graph may still be queued: let it finish first
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return bdg::api_device_error(e, "synchronize");
  plan->schedule = schedule;
  // the tile's rows may differ: new work items (this drops the captured
  // launch, which holds the old kernel)
  return upload_items(plan);
}

int bdg_batch_plan_set_bound(bdg_batch_plan* plan, uint32_t bound_group) {
  if (!plan) return bdg::api_error(BDG_EINVAL, "plan is NULL");
  if (bound_group == 0) bound_group = BDG_BOUND_GROUP_DEFAULT;
  return set_bound_group(plan, bound_group);
}

int bdg_build_knn_batched_plan(const bdg_batch_plan* plan, const uint64_t* codes,
                               uint32_t* out_idx, uint16_t* out_dist, void* stream) {
  if (!plan) return bdg::api_error(BDG_EINVAL, "plan is NULL");
  if (plan->nitems && (!codes || !out_idx || !out_dist))
    return bdg::api_error(BDG_EINVAL, "null device pointer");
  (void)hipGetLastError();
  return enqueue(plan, codes, out_idx, out_dist, reinterpret_cast<hipStream_t>(stream), true);
}

int bdg_batch_plan_set_timing(bdg_batch_plan* plan, void* start_event, void* stop_event) {
  if (!plan) return bdg::api_error(BDG_EINVAL, "plan is NULL");
  if ((start_event == nullptr) != (stop_event == nullptr))
    return bdg::api_error(BDG_EINVAL, "give both events or neither");
  plan->ev_start = reinterpret_cast<hipEvent_t>(start_event);
  plan->ev_stop = reinterpret_cast<hipEvent_t>(stop_event);
  return BDG_OK;
}

int bdg_build_knn_batched_graph(bdg_batch_plan* plan, const uint64_t* codes, uint32_t* out_idx,
                                uint16_t* out_dist, void* stream_) {
  if (!plan) return bdg::api_error(BDG_EINVAL, "plan is NULL");
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  if (!stream) return bdg::api_error(BDG_EINVAL, "graph launches need a non-default stream");
  if (plan->nitems && (!codes || !out_idx || !out_dist))
    return bdg::api_error(BDG_EINVAL, "null device pointer");
  (void)hipGetLastError();
  if (plan->exec && (plan->g_codes != codes || plan->g_idx != out_idx ||
                     plan->g_dist != out_dist))
    drop_graph(plan);
  if (!plan->exec) {
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bdg::api_device_error(e, "begin capture");
    const int st = enqueue(plan, codes, out_idx, out_dist, stream, false);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(stream, &g);
    if (st != BDG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return bdg::api_device_error(e, "end capture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return bdg::api_device_error(e, "graph instantiate");
    }
    plan->graph = g;
    plan->exec = ex;
    plan->g_codes = codes;
    plan->g_idx = out_idx;
    plan->g_dist = out_dist;
  }
  hipError_t e = hipGraphLaunch(plan->exec, stream);
  if (e != hipSuccess) return bdg::api_device_error(e, "graph launch");
  return BDG_OK;
}

int bdg_build_knn_batched_ex(const uint64_t* codes, const uint64_t* offsets, uint32_t S,
                             uint32_t bits, uint32_t K, uint32_t* out_idx, uint16_t* out_dist,
                             const bdg_knn_opts* opts, void* stream) {
  bdg_batch_plan* plan = nullptr;
  int st = bdg_batch_plan_create(offsets, S, bits, K, opts, &plan);
  if (st != BDG_OK) return st;
  st = bdg_build_knn_batched_plan(plan, codes, out_idx, out_dist, stream);
  if (st == BDG_OK) {
    hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) st = bdg::api_device_error(e, "synchronize");
  }
  bdg_batch_plan_destroy(plan);
  return st;
}

}  // extern "C"
