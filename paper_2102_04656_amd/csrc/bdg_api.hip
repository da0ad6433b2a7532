// Host driver and C ABI of the Hamming kNN-graph builder.
//
// Blockwise schedule: rows are cut into row blocks, columns into column
// blocks. One tile launch per row block computes, for every (row, column
// block), the exact top-K of that block (the per-partition search of the
// first reduce, Sec. 3.2). With more than one column block the per-block
// lists land in a workspace and are merged into the output rows (the second
// reduce's merge, Sec. 3.2). Row blocks are independent units, so a run can
// stop after any row block and be resumed from the next one.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

#include "bdg.h"
#include "kernels.h"

namespace bdg {
bool tuned_schedule(uint32_t n, uint32_t bits, uint32_t K, int* path, uint32_t* col_block,
                    int* schedule, uint32_t* bound_group);
}  // namespace bdg

namespace {

thread_local std::string g_last_error;

int set_error(int status, const char* fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  g_last_error = msg;
  return status;
}

int device_error(hipError_t e, const char* what) {
  return set_error(BDG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr uint32_t kDefaultBlock = 131072;
// Matrix-core path: the column-block width is the width of one work item of
// the persistent launch; wider items spend less on list loads and stage-ring
// fills per pair, and the launch still ends on a short tail.
constexpr uint32_t kDefaultMfmaColBlock = 262144;
constexpr uint32_t kMaxColBlock = 1u << 21;  // column index field of a tile key

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Sentinel rows (no neighbour): index BDG_NO_IDX, distance BDG_NO_DIST.
__global__ void pad_rows_kernel(uint32_t* out_idx, uint16_t* out_dist, size_t cells) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= cells) return;
  out_idx[i] = BDG_NO_IDX;
  out_dist[i] = (uint16_t)BDG_NO_DIST;
}

// Test hook: BDG_TEST_FAIL_ALLOC=1 makes workspace allocations fail.
bool forced_alloc_failure() {
  const char* s = getenv("BDG_TEST_FAIL_ALLOC");
  return s && s[0] == '1';
}

struct Plan {
  uint32_t words, K, n;
  uint32_t row_block, col_block, nrb, ncb;
  int path;
  int schedule;     // matrix-core tile schedule
  bool running;     // lists carried across column blocks in the output rows
  uint32_t bgroup;  // admission bounds: rows per pivot group (0: none)
  uint32_t npiv;
  size_t ws_bytes;  // operand fragments + sweep control words (+ admission
                    // bounds and their scratch) (running), or partial lists
                    // of one row block
  size_t ws_idx_off, ws_dist_off, ws_ctl_off, ws_bound_off, ws_bscr_off, ws_brect_off;
};

// Members measured per row by the admission-bound pass, at most.
constexpr uint32_t kBoundCap = 1023;

int path_auto(uint32_t n, uint32_t words, uint32_t K) {
  if (bdg::run_supported(n, words, K)) return bdg::kPathMfma;
  return bdg::kPathPopc;
}

int make_plan(uint32_t n, uint32_t bits, uint32_t K, const bdg_knn_opts* opts, Plan* p) {
  if (opts && opts->struct_size < offsetof(bdg_knn_opts, workspace))
    return set_error(BDG_EINVAL, "opts->struct_size too small (%u)", opts->struct_size);
  if (bits == 0 || bits % 64 != 0)
    return set_error(BDG_EINVAL, "bits must be a positive multiple of 64 (got %u)", bits);
  if (bits > BDG_MAX_BITS) return set_error(BDG_EUNSUPPORTED, "bits > %u", BDG_MAX_BITS);
  if (K == 0) return set_error(BDG_EINVAL, "K must be >= 1");
  if (K > BDG_MAX_K) return set_error(BDG_EUNSUPPORTED, "K > %u", BDG_MAX_K);
  if (n == 0xFFFFFFFFu) return set_error(BDG_EUNSUPPORTED, "n must be < 2^32 - 1");
  p->words = bits / 64;
  p->K = K;
  p->n = n;
  int path = opts ? opts->path : BDG_PATH_AUTO;
  const bool full_opts = opts && opts->struct_size >= sizeof(bdg_knn_opts);
  int schedule = full_opts ? (int)opts->tile_schedule : 0;
  uint32_t bgroup = full_opts ? opts->bound_group : 0;
  uint32_t tuned_cb = 0;
  if (path == BDG_PATH_AUTO && !(opts && opts->col_block)) {
    int tp = 0, ts = 0;
    uint32_t tb = 0;
    if (bdg::tuned_schedule(n, bits, K, &tp, &tuned_cb, &ts, &tb)) {
      path = tp;
      if (!(full_opts && opts->tile_schedule)) schedule = ts;
      if (!(full_opts && opts->bound_group)) bgroup = tb;
    }
  }
  if (bgroup == 0) bgroup = BDG_BOUND_GROUP_DEFAULT;
  if (bgroup != BDG_BOUND_OFF && (bgroup < BDG_BOUND_GROUP_MIN || bgroup > BDG_BOUND_GROUP_MAX))
    return set_error(BDG_EUNSUPPORTED, "bound_group %u outside [%u, %u] (or BDG_BOUND_OFF)",
                     bgroup, BDG_BOUND_GROUP_MIN, BDG_BOUND_GROUP_MAX);
  if (path == BDG_PATH_AUTO) path = path_auto(n, p->words, K);
  if (path != BDG_PATH_POPC && path != BDG_PATH_MFMA)
    return set_error(BDG_EINVAL, "unknown path %d", path);
  const bool ok = path == BDG_PATH_MFMA ? bdg::run_supported(n, p->words, K)
                                        : bdg::tile_supported(path, p->words, K);
  if (!ok)
    return set_error(BDG_EUNSUPPORTED, "path %d does not support n=%u bits=%u K=%u", path, n,
                     bits, K);
  p->path = path;
  if (path == BDG_PATH_MFMA && !bdg::schedule_supported(p->words, K, schedule))
    return set_error(BDG_EUNSUPPORTED, "tile schedule %d is not built for bits=%u", schedule, bits);
  p->schedule = path == BDG_PATH_MFMA ? bdg::resolve_schedule(p->words, K, schedule) : 0;
  uint32_t cb = (opts && opts->col_block)
                    ? opts->col_block
                    : (tuned_cb ? tuned_cb
                                : (path == BDG_PATH_MFMA ? kDefaultMfmaColBlock : kDefaultBlock));
  uint32_t rb = (opts && opts->row_block) ? opts->row_block : kDefaultBlock;
  if (cb > kMaxColBlock)
    return set_error(BDG_EUNSUPPORTED, "col_block > %u", kMaxColBlock);
  if (n > 0) {
    if (cb > n) cb = n;
    if (rb > n) rb = n;
  }
  p->col_block = cb;
  p->row_block = rb;
  p->ncb = n ? (n + cb - 1) / cb : 0;
  p->nrb = n ? (n + rb - 1) / rb : 0;
  if (p->ncb > 65535)
    return set_error(BDG_EUNSUPPORTED, "more than 65535 column blocks (col_block %u)", cb);
  p->running = path == BDG_PATH_MFMA;
  p->ws_ctl_off = p->ws_bound_off = p->ws_bscr_off = p->ws_brect_off = 0;
  p->bgroup = p->npiv = 0;
  if (p->running) {
    p->ws_ctl_off = n ? align256(bdg::prep_bytes(n, p->words)) : 0;
    p->ws_bytes = n ? p->ws_ctl_off + align256(bdg::sweep_ctl_words(n, K) * 4) : 0;
    p->ws_idx_off = p->ws_dist_off = 0;
    // bounds only help where a row has more than K candidates
    if (bgroup != BDG_BOUND_OFF && n > K + 1) {
      p->bgroup = bgroup;
      p->npiv = bdg::bound_pivots(n, bgroup);
      p->ws_bound_off = p->ws_bytes;
      p->ws_bscr_off = p->ws_bound_off + align256((size_t)n * 2);
      p->ws_bytes = p->ws_bscr_off + bdg::bound_scratch_bytes(n, p->words, p->npiv);
      // nearest pivots on the matrix cores where the tile takes the shape
      const size_t rb = bdg::bound_rect_bytes(n, p->words, p->npiv);
      if (rb) {
        p->ws_brect_off = p->ws_bytes;
        p->ws_bytes += rb;
      }
    }
  } else if (p->ncb > 1) {
    const size_t entries = (size_t)p->ncb * rb * K;
    p->ws_idx_off = 0;
    p->ws_dist_off = align256(entries * 4);
    p->ws_bytes = p->ws_dist_off + align256(entries * 2);
  } else {
    p->ws_bytes = p->ws_idx_off = p->ws_dist_off = 0;
  }
  return BDG_OK;
}

}  // namespace

namespace bdg {
// Error reporting for the other host files of the library.
int api_error(int status, const char* fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  g_last_error = msg;
  return status;
}
int api_device_error(hipError_t e, const char* what) { return device_error(e, what); }
void api_clear_error() { g_last_error.clear(); }
}  // namespace bdg

extern "C" {

int bdg_version(void) { return BDG_VERSION; }

const char* bdg_status_string(int status) {
  switch (status) {
    case BDG_OK: return "ok";
    case BDG_EINVAL: return "invalid argument";
    case BDG_EUNSUPPORTED: return "unsupported argument";
    case BDG_ENOMEM: return "out of device memory";
    case BDG_EDEVICE: return "device error";
    default: return "unknown status";
  }
}

const char* bdg_last_error(void) { return g_last_error.c_str(); }

int bdg_build_knn_workspace_size(uint32_t n, uint32_t bits, uint32_t K, const bdg_knn_opts* opts,
                                 size_t* bytes) {
  if (!bytes) return set_error(BDG_EINVAL, "bytes is NULL");
  Plan p;
  int st = make_plan(n, bits, K, opts, &p);
  if (st != BDG_OK) return st;
  *bytes = p.ws_bytes;
  return BDG_OK;
}

int bdg_build_knn_ex(const uint64_t* codes, uint32_t n, uint32_t bits, uint32_t K,
                     uint32_t* out_idx, uint16_t* out_dist, const bdg_knn_opts* opts,
                     void* stream_) {
  g_last_error.clear();
  Plan p;
  int st = make_plan(n, bits, K, opts, &p);
  if (st != BDG_OK) return st;
  if (n == 0) return BDG_OK;
  if (!codes || !out_idx || !out_dist) return set_error(BDG_EINVAL, "null device pointer");
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);

  uint32_t first = opts ? opts->first_rowblock : 0;
  uint32_t stop = (opts && opts->stop_rowblock) ? opts->stop_rowblock : p.nrb;
  if (stop > p.nrb) stop = p.nrb;
  if (first >= stop) return BDG_OK;

  (void)hipGetLastError();  // start from a clean per-thread error state
  void* ws = nullptr;
  bool own_ws = false;
  if (p.ws_bytes) {
    if (opts && opts->workspace) {
      if (opts->workspace_bytes < p.ws_bytes)
        return set_error(BDG_ENOMEM, "workspace too small: %zu < %zu bytes",
                         opts->workspace_bytes, p.ws_bytes);
      ws = opts->workspace;
    } else {
      if (forced_alloc_failure())
        return set_error(BDG_ENOMEM, "workspace allocation failed (forced by test hook)");
      hipError_t e = hipMallocAsync(&ws, p.ws_bytes, stream);
      if (e != hipSuccess || !ws) {
        (void)hipGetLastError();
        return set_error(BDG_ENOMEM, "workspace allocation of %zu bytes failed", p.ws_bytes);
      }
      own_ws = true;
    }
  }

  int result = BDG_OK;
  if (p.running) {
    // Operand fragments of all codes, then the rows of the selected row blocks
    // against every column block in one persistent launch, each (row tile,
    // column block) item merging its columns into the rows' running lists.
    hipError_t e = bdg::launch_prep(codes, n, p.words, ws, stream);
    uint16_t* bound = nullptr;
    if (e == hipSuccess && p.bgroup) {
      bound = reinterpret_cast<uint16_t*>(static_cast<char*>(ws) + p.ws_bound_off);
      bdg::BoundArgs b;
      b.codes = codes;
      b.words = p.words;
      b.bits = bits;
      b.K = K;
      b.group = p.bgroup;
      b.cap = kBoundCap;
      b.nseg = 1;
      b.seg = b.pseg = nullptr;  // one segment: rows [0, n), pivots [0, npiv)
      b.base = 0;
      b.total = n;
      b.npiv = p.npiv;
      b.scratch = static_cast<char*>(ws) + p.ws_bscr_off;
      b.bound = bound;
      b.rect_scratch = p.ws_brect_off ? static_cast<char*>(ws) + p.ws_brect_off : nullptr;
      e = bdg::launch_bounds_pass(b, stream);
    }
    int dev = 0, cus = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) {
      const uint32_t r0 = first * p.row_block;
      const uint64_t r1 = (uint64_t)stop * p.row_block;
      bdg::SweepArgs a;
      a.codes = codes;
      a.frags = ws;
      a.words = p.words;
      a.bits = bits;
      a.K = K;
      a.idx_bits = bdg::run_idx_bits(bits);
      a.row0 = r0;
      a.nrows = (r1 < n ? (uint32_t)r1 : n) - r0;
      a.ncols = n;
      a.col_block = p.col_block;
      a.ctl = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + p.ws_ctl_off);
      a.grid = (uint32_t)(cus > 0 ? cus : 1);
      a.out_idx = out_idx + (size_t)r0 * K;
      a.out_dist = out_dist + (size_t)r0 * K;
      a.spin_limit = (opts && opts->struct_size >= sizeof(bdg_knn_opts)) ? opts->wait_limit : 0;
      a.schedule = p.schedule;
      a.bound = bound;
      const bool timed = opts && opts->tile_events && opts->n_tile_events >= 2;
      if (timed) e = hipEventRecord(reinterpret_cast<hipEvent_t>(opts->tile_events[0]), stream);
      if (e == hipSuccess) e = bdg::launch_mfma_sweep(a, stream);
      if (e == hipSuccess && timed)
        e = hipEventRecord(reinterpret_cast<hipEvent_t>(opts->tile_events[1]), stream);
    }
    if (e != hipSuccess) result = device_error(e, "tile launch");
  }
  for (uint32_t rb = first; rb < stop && !p.running; ++rb) {
    const uint32_t r0 = rb * p.row_block;
    const uint32_t nr = (n - r0 < p.row_block) ? n - r0 : p.row_block;
    bdg::TileArgs a;
    a.codes = codes;
    a.words = p.words;
    a.K = K;
    a.row0 = r0;
    a.nrows = nr;
    a.col0 = 0;
    a.col1 = n;
    a.col_block = p.col_block;
    if (p.ncb == 1) {
      a.out_idx = out_idx + (size_t)r0 * K;
      a.out_dist = out_dist + (size_t)r0 * K;
    } else {
      a.out_idx = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + p.ws_idx_off);
      a.out_dist = reinterpret_cast<uint16_t*>(static_cast<char*>(ws) + p.ws_dist_off);
    }
    const uint32_t ev = 2 * (rb - first);
    const bool timed = opts && opts->tile_events && ev + 1 < opts->n_tile_events;
    hipError_t e = hipSuccess;
    if (timed) e = hipEventRecord(reinterpret_cast<hipEvent_t>(opts->tile_events[ev]), stream);
    if (e == hipSuccess) e = bdg::launch_tile(p.path, a, stream);
    if (e == hipSuccess && timed)
      e = hipEventRecord(reinterpret_cast<hipEvent_t>(opts->tile_events[ev + 1]), stream);
    if (e != hipSuccess) {
      result = device_error(e, "tile launch");
      break;
    }
    if (p.ncb > 1) {
      e = bdg::launch_merge(a.out_idx, a.out_dist, nr, p.ncb, K, K, out_idx + (size_t)r0 * K,
                            out_dist + (size_t)r0 * K, /*dedup=*/0, stream);
      if (e != hipSuccess) {
        result = device_error(e, "merge launch");
        break;
      }
    }
  }
  if (own_ws) {
    hipError_t e = hipFreeAsync(ws, stream);
    if (e != hipSuccess && result == BDG_OK) result = device_error(e, "workspace free");
  }
  return result;
}

int bdg_build_knn_check(uint32_t n, uint32_t bits, uint32_t K, const bdg_knn_opts* opts,
                        void* stream) {
  g_last_error.clear();
  Plan p;
  int st = make_plan(n, bits, K, opts, &p);
  if (st != BDG_OK) return st;
  if (!p.running || n == 0) return BDG_OK;  // no persistent launch, no flag
  if (!opts || !opts->workspace) return set_error(BDG_EINVAL, "opts->workspace is NULL");
  if (opts->workspace_bytes < p.ws_bytes)
    return set_error(BDG_EINVAL, "workspace too small: %zu < %zu bytes", opts->workspace_bytes,
                     p.ws_bytes);
  (void)hipGetLastError();
  hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_error(e, "synchronize");
  uint32_t stall = 0;
  e = hipMemcpy(&stall,
                static_cast<const char*>(opts->workspace) + p.ws_ctl_off + 4 * bdg::kSweepStallWord,
                sizeof stall, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return device_error(e, "stall flag read");
  if (stall)
    return set_error(BDG_EDEVICE,
                     "a dependency wait of the persistent build ran out; lists unspecified");
  return BDG_OK;
}

int bdg_build_knn(const uint64_t* codes, uint32_t n, uint32_t bits, uint32_t K, uint32_t* out_idx,
                  uint16_t* out_dist) {
  g_last_error.clear();
  Plan p;
  int st = make_plan(n, bits, K, nullptr, &p);
  if (st != BDG_OK) return st;
  if (n == 0) return BDG_OK;
  if (!codes || !out_idx || !out_dist) return set_error(BDG_EINVAL, "null device pointer");
  // The call owns the workspace, so that after completion it can read the
  // persistent launch's stall flag.
  void* ws = nullptr;
  if (p.ws_bytes) {
    if (forced_alloc_failure())
      return set_error(BDG_ENOMEM, "workspace allocation failed (forced by test hook)");
    if (hipMalloc(&ws, p.ws_bytes) != hipSuccess || !ws) {
      (void)hipGetLastError();
      return set_error(BDG_ENOMEM, "workspace allocation of %zu bytes failed", p.ws_bytes);
    }
  }
  bdg_knn_opts o;
  memset(&o, 0, sizeof o);
  o.struct_size = sizeof o;
  o.workspace = ws;
  o.workspace_bytes = p.ws_bytes;
  st = bdg_build_knn_ex(codes, n, bits, K, out_idx, out_dist, &o, nullptr);
  if (st == BDG_OK) st = bdg_build_knn_check(n, bits, K, &o, nullptr);
  if (ws) (void)hipFree(ws);
  return st;
}

int bdg_merge_lists(const uint32_t* in_idx, const uint16_t* in_dist, uint32_t n, uint32_t L,
                    uint32_t K_in, uint32_t K, uint32_t* out_idx, uint16_t* out_dist,
                    void* stream) {
  g_last_error.clear();
  if (L == 0) return set_error(BDG_EINVAL, "L must be >= 1");
  if (K == 0 || K_in == 0) return set_error(BDG_EINVAL, "K and K_in must be >= 1");
  if (K > BDG_MAX_K || K_in > BDG_MAX_K)
    return set_error(BDG_EUNSUPPORTED, "K or K_in > %u", BDG_MAX_K);
  if (n == 0) return BDG_OK;
  if (!in_idx || !in_dist || !out_idx || !out_dist)
    return set_error(BDG_EINVAL, "null device pointer");
  (void)hipGetLastError();
  hipError_t e = bdg::launch_merge(in_idx, in_dist, n, L, K_in, K, out_idx, out_dist,
                                   /*dedup=*/1, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_error(e, "merge launch");
  return BDG_OK;
}

int bdg_propagate(const uint64_t* codes, uint32_t n, uint32_t bits, uint32_t K,
                  const uint32_t* in_idx, uint32_t* out_idx, uint16_t* out_dist, void* stream) {
  g_last_error.clear();
  if (bits == 0 || bits % 64 != 0)
    return set_error(BDG_EINVAL, "bits must be a positive multiple of 64 (got %u)", bits);
  if (bits > BDG_MAX_BITS) return set_error(BDG_EUNSUPPORTED, "bits > %u", BDG_MAX_BITS);
  if (K == 0) return set_error(BDG_EINVAL, "K must be >= 1");
  if (K > BDG_MAX_K_TILE) return set_error(BDG_EUNSUPPORTED, "K > %u", BDG_MAX_K_TILE);
  if (n == 0xFFFFFFFFu) return set_error(BDG_EUNSUPPORTED, "n must be < 2^32 - 1");
  if (n == 0) return BDG_OK;
  if (!codes || !in_idx || !out_idx || !out_dist)
    return set_error(BDG_EINVAL, "null device pointer");
  const uintptr_t ib = reinterpret_cast<uintptr_t>(in_idx);
  const uintptr_t ie = ib + (uintptr_t)n * K * sizeof(uint32_t);
  const uintptr_t ob = reinterpret_cast<uintptr_t>(out_idx);
  const uintptr_t oe = ob + (uintptr_t)n * K * sizeof(uint32_t);
  const uintptr_t db = reinterpret_cast<uintptr_t>(out_dist);
  const uintptr_t de = db + (uintptr_t)n * K * sizeof(uint16_t);
  if ((ob < ie && ib < oe) || (db < ie && ib < de))
    return set_error(BDG_EINVAL, "outputs overlap in_idx (rows read other rows' lists)");
  (void)hipGetLastError();
  hipError_t e = bdg::launch_propagate(codes, n, bits / 64, K, in_idx, out_idx, out_dist,
                                       reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_error(e, "propagate launch");
  return BDG_OK;
}

int bdg_bkmeans(const uint64_t* codes, uint32_t n, uint32_t bits, const uint32_t* sample,
                uint32_t ns, const uint32_t* init, uint32_t m, uint32_t iters,
                uint64_t* centres, void* stream) {
  g_last_error.clear();
  if (bits == 0 || bits % 64 != 0)
    return set_error(BDG_EINVAL, "bits must be a positive multiple of 64 (got %u)", bits);
  if (bits > BDG_MAX_BITS) return set_error(BDG_EUNSUPPORTED, "bits > %u", BDG_MAX_BITS);
  if (m == 0) return set_error(BDG_EINVAL, "m must be >= 1");
  if (m > (1u << 20)) return set_error(BDG_EUNSUPPORTED, "m > 2^20");
  if (!codes || !init || !centres || (ns > 0 && !sample))
    return set_error(BDG_EINVAL, "null pointer");
  for (uint32_t j = 0; j < m; ++j)
    if (init[j] >= n) return set_error(BDG_EINVAL, "init[%u] = %u is not a row (n = %u)", j, init[j], n);
  for (uint32_t i = 0; i < ns; ++i)
    if (sample[i] >= n)
      return set_error(BDG_EINVAL, "sample[%u] = %u is not a row (n = %u)", i, sample[i], n);
  const uint32_t words = bits / 64;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  const size_t b_s = (size_t)(ns ? ns : 1) * 4, b_i = (size_t)m * 4, b_h = b_s,
               b_c = (size_t)m * words * 64 * 4, b_z = (size_t)m * 4;
  const size_t b_main = (b_s + b_i + b_h + b_c + b_z + 255) & ~size_t(255);
  const size_t b_t = bdg::bkmeans_tile_scratch_bytes(ns, m, words);
  char* ws = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&ws), b_main + b_t, st);
  if (e != hipSuccess) return set_error(BDG_ENOMEM, "scratch: %s", hipGetErrorString(e));
  uint32_t* d_sample = reinterpret_cast<uint32_t*>(ws);
  uint32_t* d_init = reinterpret_cast<uint32_t*>(ws + b_s);
  uint32_t* d_home = reinterpret_cast<uint32_t*>(ws + b_s + b_i);
  uint32_t* d_cnt = reinterpret_cast<uint32_t*>(ws + b_s + b_i + b_h);
  uint32_t* d_size = reinterpret_cast<uint32_t*>(ws + b_s + b_i + b_h + b_c);
  if (ns) e = hipMemcpyAsync(d_sample, sample, (size_t)ns * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_init, init, b_i, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = bdg::launch_bkmeans(codes, words, d_sample, ns, d_init, m, iters, centres, d_home, d_cnt,
                            d_size, b_t ? ws + b_main : nullptr, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // host index arrays are read by the copies
  hipError_t f = hipFreeAsync(ws, st);
  if (e != hipSuccess) return device_error(e, "bkmeans");
  if (f != hipSuccess) return device_error(f, "bkmeans scratch");
  return BDG_OK;
}

int bdg_build_knn_dac(const uint64_t* codes, uint32_t n, uint32_t bits, const uint64_t* centres,
                      uint32_t m, uint32_t T, uint32_t coarse_num, uint32_t K, uint32_t* out_idx,
                      uint16_t* out_dist, void* stream) {
  g_last_error.clear();
  if (bits == 0 || bits % 64 != 0)
    return set_error(BDG_EINVAL, "bits must be a positive multiple of 64 (got %u)", bits);
  if (bits > BDG_MAX_BITS) return set_error(BDG_EUNSUPPORTED, "bits > %u", BDG_MAX_BITS);
  if (K == 0 || m == 0 || T == 0 || coarse_num == 0)
    return set_error(BDG_EINVAL, "K, m, T and coarse_num must be >= 1");
  if (K > BDG_MAX_K_TILE) return set_error(BDG_EUNSUPPORTED, "K > %u", BDG_MAX_K_TILE);
  if (T > 64) return set_error(BDG_EUNSUPPORTED, "T > 64");
  if (m > (1u << 20)) return set_error(BDG_EUNSUPPORTED, "m > 2^20");
  if (n == 0xFFFFFFFFu) return set_error(BDG_EUNSUPPORTED, "n must be < 2^32 - 1");
  if (n == 0) return BDG_OK;
  if (!codes || !centres || !out_idx || !out_dist) return set_error(BDG_EINVAL, "null pointer");
  const uint32_t words = bits / 64;
  const uint32_t Te = T < m ? T : m;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  const size_t b_top = (size_t)n * Te * 4, b_m = ((size_t)m + 1) * 4, b_n = (size_t)n * 4,
               b_hc = (size_t)n * words * 8;
  const size_t b_ts = bdg::dac_top_scratch_bytes(n, m, words, Te);
  const size_t b_main = (b_hc + b_top + 3 * b_m + b_n + 255) & ~size_t(255);
  char* ws = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&ws), b_main + b_ts, st);
  if (e != hipSuccess) return set_error(BDG_ENOMEM, "scratch: %s", hipGetErrorString(e));
  uint64_t* hcodes = reinterpret_cast<uint64_t*>(ws);
  uint32_t* top = reinterpret_cast<uint32_t*>(ws + b_hc);
  uint32_t* size = reinterpret_cast<uint32_t*>(ws + b_hc + b_top);
  uint32_t* off = reinterpret_cast<uint32_t*>(ws + b_hc + b_top + b_m);
  uint32_t* cursor = reinterpret_cast<uint32_t*>(ws + b_hc + b_top + 2 * b_m);
  uint32_t* member = reinterpret_cast<uint32_t*>(ws + b_hc + b_top + 3 * b_m);
  e = bdg::launch_dac(codes, n, words, centres, m, Te, coarse_num, K, top, size, off, cursor,
                      member, hcodes, out_idx, out_dist, b_ts ? ws + b_main : nullptr, st);
  hipError_t f = hipFreeAsync(ws, st);
  if (e != hipSuccess) return device_error(e, "dac launch");
  if (f != hipSuccess) return device_error(f, "dac scratch");
  return BDG_OK;
}

int bdg_hamming_knn(const uint64_t* queries, uint32_t nq, const uint64_t* base, uint32_t nb,
                    uint32_t bits, uint32_t K, uint32_t* out_idx, uint16_t* out_dist,
                    void* stream) {
  g_last_error.clear();
  if (bits == 0 || bits % 64 != 0)
    return set_error(BDG_EINVAL, "bits must be a positive multiple of 64 (got %u)", bits);
  if (bits > BDG_MAX_BITS) return set_error(BDG_EUNSUPPORTED, "bits > %u", BDG_MAX_BITS);
  if (K == 0) return set_error(BDG_EINVAL, "K must be >= 1");
  if (K > 64) return set_error(BDG_EUNSUPPORTED, "K > 64");
  const uint32_t words = bits / 64;
  if (nb > 0 && !bdg::run_supported(nb, words, K))
    return set_error(BDG_EUNSUPPORTED, "nb=%u too large for %u-bit keys", nb, bits);
  if (nq == 0) return BDG_OK;
  if (!queries || !out_idx || !out_dist || (nb > 0 && !base))
    return set_error(BDG_EINVAL, "null device pointer");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  if (nb == 0) {  // every row is padding
    const size_t cells = (size_t)nq * K;
    hipLaunchKernelGGL(pad_rows_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st,
                       out_idx, out_dist, cells);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? BDG_OK : device_error(e, "hamming knn padding");
  }
  // the base's operand fragments
  void* frags = nullptr;
  hipError_t e = hipMallocAsync(&frags, bdg::prep_bytes(nb, words), st);
  if (e != hipSuccess || !frags) {
    (void)hipGetLastError();
    return set_error(BDG_ENOMEM, "fragments of %u base rows", nb);
  }
  e = bdg::launch_prep(base, nb, words, frags, st);
  if (e == hipSuccess) {
    // rows = the queries, columns = the base: the rectangular tile, lists of
    // (distance, base index), no row left out
    bdg::RunArgs r;
    r.codes = queries;
    r.frags = frags;
    r.words = words;
    r.bits = bits;
    r.K = K;
    r.idx_bits = bdg::run_idx_bits(bits);
    r.row0 = 0;
    r.nrows = nq;
    r.cb = 0;
    r.ce = nb;
    r.fresh = 1;
    r.out_idx = out_idx;
    r.out_dist = out_dist;
    r.rect = 1;
    e = bdg::launch_mfma_run(r, st);
  }
  hipError_t f = hipFreeAsync(frags, st);
  if (e != hipSuccess) return device_error(e, "hamming knn launch");
  if (f != hipSuccess) return device_error(f, "hamming knn scratch");
  return BDG_OK;
}

int bdg_graph_search(const uint64_t* codes, uint32_t n, uint32_t bits, const uint32_t* graph,
                     uint32_t K, const float* feats, uint32_t d, const uint64_t* q_codes,
                     const float* q_feats, const uint32_t* q_exclude, uint32_t nq,
                     const uint32_t* entries, uint32_t S, uint32_t P, uint32_t N,
                     uint32_t* out_idx, float* out_dist, uint32_t* out_visited, void* stream) {
  g_last_error.clear();
  if (bits == 0 || bits % 64 != 0)
    return set_error(BDG_EINVAL, "bits must be a positive multiple of 64 (got %u)", bits);
  if (bits > BDG_MAX_BITS) return set_error(BDG_EUNSUPPORTED, "bits > %u", BDG_MAX_BITS);
  if (K == 0 || d == 0 || S == 0 || P == 0 || N == 0)
    return set_error(BDG_EINVAL, "K, d, S, P and N must be >= 1");
  if (N > P) return set_error(BDG_EINVAL, "N must be <= P");
  if (P > 1024 || K > BDG_MAX_K_TILE) return set_error(BDG_EUNSUPPORTED, "P > 1024 or K > %u", BDG_MAX_K_TILE);
  if (n == 0xFFFFFFFFu || n > 0x7FFFFFFFu) return set_error(BDG_EUNSUPPORTED, "n must be < 2^31");
  if (nq == 0 || n == 0) return BDG_OK;
  if (!codes || !graph || !feats || !q_codes || !q_feats || !entries || !out_idx || !out_dist)
    return set_error(BDG_EINVAL, "null pointer");
  const uint32_t words = bits / 64;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  // visited bitmaps for a batch of queries, at most about 1 GiB of scratch
  const size_t per_q = bdg::search_map_words(n) * sizeof(uint32_t);
  size_t batch = ((size_t)1 << 30) / per_q;
  if (batch < 1) batch = 1;
  if (batch > nq) batch = nq;
  uint32_t* maps = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&maps), batch * per_q, st);
  if (e != hipSuccess) return set_error(BDG_ENOMEM, "scratch: %s", hipGetErrorString(e));
  for (uint32_t q0 = 0; q0 < nq && e == hipSuccess; q0 += (uint32_t)batch) {
    const uint32_t nb = (uint32_t)((nq - q0) < batch ? (nq - q0) : batch);
    e = bdg::launch_search(codes, n, words, graph, K, feats, d, q_codes, q_feats, q_exclude, q0, nb,
                           entries, S, P, N, maps, out_idx, out_dist, out_visited, st);
  }
  hipError_t f = hipFreeAsync(maps, st);
  if (e != hipSuccess) return device_error(e, "search launch");
  if (f != hipSuccess) return device_error(f, "search scratch");
  return BDG_OK;
}

}  // extern "C"
