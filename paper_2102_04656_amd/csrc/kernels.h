// Internal interface between the host driver (bdg_api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bdg {

enum TilePath { kPathPopc = 1, kPathMfma = 2 };

// One launch of a distance tile: rows [row0, row0 + nrows) of `codes` are the
// queries; columns [col0, col1) are split into blocks of `col_block` columns,
// one grid row per block. Block b writes its per-row top-K lists to
//   out_idx/out_dist + (b * nrows + r) * K     (r = row - row0)
// with global column indices.
struct TileArgs {
  const uint64_t* codes;
  uint32_t words;  // bits / 64
  uint32_t K;
  uint32_t row0, nrows;
  uint32_t col0, col1, col_block;
  uint32_t* out_idx;
  uint16_t* out_dist;
};

bool tile_supported(int path, uint32_t words, uint32_t K);
// Rows of one tile (work-group) for a path.
uint32_t tile_rows(int path, uint32_t words);
hipError_t launch_tile(int path, const TileArgs& a, hipStream_t stream);

// Merge of L sorted lists per row; dedup = 0 when lists are known disjoint.
hipError_t launch_merge(const uint32_t* in_idx, const uint16_t* in_dist, uint32_t n, uint32_t L,
                        uint32_t K_in, uint32_t K, uint32_t* out_idx, uint16_t* out_dist,
                        int dedup, hipStream_t stream);

// One round of neighbourhood propagation (propagate.hip): row r of out =
// the K nearest distinct entries of r's list in in_idx and of the lists of
// its entries (distances recomputed from the codes). in_idx and out must not
// overlap.
hipError_t launch_propagate(const uint64_t* codes, uint32_t n, uint32_t words, uint32_t K,
                            const uint32_t* in_idx, uint32_t* out_idx, uint16_t* out_dist,
                            hipStream_t stream);

// Single-pass divide-and-conquer (dac.hip). launch_bkmeans: centres =
// codes of rows init[0..m), then `iters` rounds of assignment of the rows
// sample[0..ns) and majority update (device scratch: home [ns], cnt
// [m][words][64], size [m]). launch_dac: the approximate graph (device
// scratch: top [n][T], size [m], off [m + 1], cursor [m], member [n],
// hcodes [n][words]). Row indices in sample / init must be < n.
size_t bkmeans_tile_scratch_bytes(uint32_t ns, uint32_t m, uint32_t words);
hipError_t launch_bkmeans(const uint64_t* codes, uint32_t words, const uint32_t* sample,
                          uint32_t ns, const uint32_t* init, uint32_t m, uint32_t iters,
                          uint64_t* centres, uint32_t* home, uint32_t* cnt, uint32_t* size,
                          void* tile_scratch, hipStream_t stream);
// top_scratch (dac_top_scratch_bytes, 256-aligned) lets the nearest-centre
// step run on the matrix cores; 0 bytes means the tile does not take the shape.
size_t dac_top_scratch_bytes(uint32_t n, uint32_t m, uint32_t words, uint32_t T);
hipError_t launch_dac(const uint64_t* codes, uint32_t n, uint32_t words, const uint64_t* centres,
                      uint32_t m, uint32_t T, uint32_t coarse_num, uint32_t K, uint32_t* top,
                      uint32_t* size, uint32_t* off, uint32_t* cursor, uint32_t* member,
                      uint64_t* hcodes, uint32_t* out_idx, uint16_t* out_dist, void* top_scratch,
                      hipStream_t stream);

// Online search (search.hip): queries q0..q0+nq of the arrays, visited
// bitmaps maps [nq][search_map_words(n)] (scratch, cleared here).
size_t search_map_words(uint32_t n);
hipError_t launch_search(const uint64_t* codes, uint32_t n, uint32_t words, const uint32_t* graph,
                         uint32_t K, const float* feats, uint32_t d, const uint64_t* qcodes,
                         const float* qfeats, const uint32_t* qexcl, uint32_t q0, uint32_t nq,
                         const uint32_t* entries, uint32_t S, uint32_t P, uint32_t N,
                         uint32_t* maps, uint32_t* out_idx, float* out_dist, uint32_t* out_vis,
                         hipStream_t stream);

// Running-merge tile on the int8 matrix cores (tile_mfma.hip). One launch
// merges columns [cb, ce) into the lists of rows [row0, row0 + nrows); the
// lists live in out_idx/out_dist (row r at (r - row0) * K), which hold the
// result of the earlier column blocks unless `fresh`. Keys carry the global
// column index in idx_bits = run_idx_bits(bits) bits, so n must fit.
struct RunArgs {
  const uint64_t* codes;  // packed codes (queries are expanded from these)
  const void* frags;      // prep output for the same codes
  uint32_t words, bits, K, idx_bits;
  uint32_t row0, nrows, cb, ce;
  int fresh;
  uint32_t* out_idx;
  uint16_t* out_dist;
  // Rows and columns are different code sets (codes: the rows; frags: the
  // columns), so no column is a row's own pair. K <= 64 only.
  int rect = 0;
};

uint32_t run_idx_bits(uint32_t bits);
bool run_supported(uint32_t n, uint32_t words, uint32_t K);
// Tile schedules of the persistent build and the batched launch, numbered as
// the API's BDG_SCHEDULE_* (they differ in pending-buffer size, stage-ring
// depth and where the running lists live, never in the result): 3 (lists in
// LDS) always; 1 (16-key buffers, deeper ring) for codes of 128, 256 or 512
// bits; 2 (lists in global memory, more rows per compute wave) for codes of
// 128, 256 or 512 bits with up to 128 keys. 0 is the default, resolved by
// resolve_schedule before anything is launched.
constexpr int kScheduleLds = 3;
constexpr int kTileSchedules = 4;  // values 0 .. kTileSchedules - 1
constexpr int kExplicitSchedules[] = {kScheduleLds, 1, 2};  // what a tuner sweeps
bool schedule_supported(uint32_t words, uint32_t K, int schedule);
// 0 -> 2 where built for (words, K), else 3; any other value unchanged.
int resolve_schedule(uint32_t words, uint32_t K, int schedule);
// Rows of one tile (work-group) of the persistent launches under a schedule;
// never fewer than run_rows_per_wg(K).
uint32_t sched_rows_per_wg(uint32_t K, int schedule);
uint32_t run_rows_per_wg(uint32_t K);
// Operand prep: {0, 1} int8 fragments of every code, prep_bytes(n, words) bytes.
size_t prep_bytes(uint32_t n, uint32_t words);
hipError_t launch_prep(const uint64_t* codes, uint32_t n, uint32_t words, void* frags,
                       hipStream_t stream);
hipError_t launch_mfma_run(const RunArgs& a, hipStream_t stream);

// Batched partitions (one persistent launch): work item = up to
// run_rows_per_wg(K) rows [row0, row0 + nrows) of the shard holding columns
// [lo, hi); output indices are shard-local (column - lo).
struct BatchItem {
  uint32_t row0, nrows, lo, hi;
};
struct BatchArgs {
  const uint64_t* codes;
  const void* frags;
  uint32_t words, bits, K, idx_bits;
  const BatchItem* items;  // device, nitems entries
  uint32_t nitems;
  uint32_t* counter;       // device scratch word (reset by the launch)
  uint32_t grid;           // persistent work-groups
  uint32_t* out_idx;
  uint16_t* out_dist;
  int schedule = kScheduleLds;  // tile schedule (resolved; schedule_supported)
  // Admission bounds (launch_bounds_pass) of the rows [bound_base, ...), or
  // nullptr: while a row's list is not full, only candidates at a distance of
  // at most its bound are admitted.
  const uint16_t* bound = nullptr;
  uint32_t bound_base = 0;
};
hipError_t launch_mfma_batched(const BatchArgs& a, hipStream_t stream);

// A whole build as one persistent launch: rows [row0, row0 + nrows) against
// columns [0, ncols), as work items (tile of run_rows_per_wg(K) rows, column
// block of col_block columns) taken column block by column block; an item
// merges its columns into the tile's lists in out_idx/out_dist (row r at
// (r - row0) * K) after the item of the previous column block has. ctl:
// sweep_ctl_words(nrows, K) device words (claim counter, stall flag, one
// progress word per tile), reset by the launch itself.
struct SweepArgs {
  const uint64_t* codes;
  const void* frags;
  uint32_t words, bits, K, idx_bits;
  uint32_t row0, nrows, ncols, col_block;
  uint32_t* ctl;
  uint32_t grid;  // persistent work-groups
  uint32_t* out_idx;
  uint16_t* out_dist;
  uint32_t spin_limit = 0;  // polls of one dependency wait before it gives up (0: default)
  int schedule = kScheduleLds;  // tile schedule (resolved; schedule_supported)
  const uint16_t* bound = nullptr;  // admission bounds of rows [0, ...), or nullptr
};
constexpr uint32_t kSweepStallWord = 1;  // ctl[1] != 0: a dependency wait ran out
size_t sweep_ctl_words(uint32_t nrows, uint32_t K);
hipError_t launch_mfma_sweep(const SweepArgs& a, hipStream_t stream);

// Admission bounds (bound.hip). Rows [seg[0], seg[nseg]) of `codes` form
// nseg segments (partitions; a row's neighbours are the other rows of its
// segment). Segment s has pivots = its rows seg[s] + j * group, j <
// ceil(size / group), numbered from pseg[s]; every row joins the group of its
// nearest pivot, and its bound is the K-th smallest distance to up to `cap`
// other members of that group and up to `cap` members of each of the groups
// of its second- and third-nearest pivots, or 0xFFFF where those are fewer
// than K. Any K other rows of the segment bound the K-th distance of the
// graph row from above, so a tile that admits only candidates at most the
// bound while a list is not full still computes the exact graph.
struct BoundArgs {
  const uint64_t* codes;
  uint32_t words, bits, K;
  uint32_t group;        // rows per pivot
  uint32_t cap;          // other group members measured per row, at most
  uint32_t nseg;
  const uint32_t* seg;   // device [nseg + 1] first rows (ascending); nullptr
                         // with nseg = 1: rows [base, base + total)
  const uint32_t* pseg;  // device [nseg + 1] first pivots; nullptr: [0, npiv)
  uint32_t base, total;  // seg[0] and seg[nseg] - seg[0] (host copies)
  uint32_t npiv;         // pseg[nseg] (host copy)
  void* scratch;         // bound_scratch_bytes(total, words, npiv), 256-aligned
  uint16_t* bound;       // [total] output: row base + i at bound[i]
  // one segment only: bound_rect_bytes(total, words, npiv) bytes (256-aligned)
  // let the nearest pivots come from the matrix-core tile; nullptr: vector ALUs
  void* rect_scratch = nullptr;
};
size_t bound_scratch_bytes(uint32_t total, uint32_t words, uint32_t npiv);
size_t bound_rect_bytes(uint32_t total, uint32_t words, uint32_t npiv);  // 0: not supported
uint32_t bound_pivots(uint32_t rows, uint32_t group);  // ceil(rows / group)
hipError_t launch_bounds_pass(const BoundArgs& a, hipStream_t stream);

}  // namespace bdg
