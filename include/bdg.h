/*
 * bdg.h -- C ABI of the MI355X (gfx950) exact Hamming kNN-graph builder.
 *
 * The library builds the k-nearest-neighbour graph of a set of binary codes
 * under Hamming distance, the offline graph of Binary Distributed Graph
 * (Sec. 3). Codes are the binary representation of Sec. 3.1; the graph of one
 * partition is what the first reduce of the single-pass divide-and-conquer
 * computes by exhaustive search (Sec. 3.2), and the merge of neighbour lists is
 * the second reduce's merge-sort (Sec. 3.2, Sec. 3.3).
 *
 * Conventions for every entry point
 *   - Pointers to codes, inputs (in_...) and outputs (out_...) are DEVICE
 *     pointers (from hipMalloc or any device allocation, such as the data
 *     pointer of a torch tensor), owned by the caller. The library never frees
 *     caller memory.
 *   - Code layout: a code of `bits` bits is bits/64 little-endian uint64 words;
 *     bit j of the code is bit (j % 64) of word (j / 64). Codes are rows of a
 *     row-major [n][bits/64] array.
 *   - Graph layout: out_idx [n][K] uint32 and out_dist [n][K] uint16, row i
 *     holding the K smallest (distance, index) pairs over j != i, ascending in
 *     distance then index. A row with fewer than K candidates is padded with
 *     index BDG_NO_IDX and distance BDG_NO_DIST.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     The *_ex / stream-taking calls only enqueue work and return; results are
 *     ready when the stream reaches that point.
 *   - Return value: BDG_OK (0) or a negative bdg_status. On an argument error
 *     (BDG_EINVAL, BDG_EUNSUPPORTED) nothing is enqueued and outputs are
 *     untouched. On BDG_EDEVICE / BDG_ENOMEM outputs are unspecified;
 *     bdg_last_error() gives the message (thread-local).
 *   - Calls on distinct streams may run concurrently from several threads.
 */
#ifndef BDG_H_
#define BDG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BDG_VERSION 10000 /* 1.0.0 */

#define BDG_NO_IDX 0xFFFFFFFFu
#define BDG_NO_DIST 0xFFFFu
#define BDG_MAX_BITS 1024u
#define BDG_MAX_K 1024u     /* builds on the vector-ALU path, list merges */
#define BDG_MAX_K_TILE 256u /* the matrix-core path, batched plans, divide-and-
                               conquer, propagation and search */

typedef enum bdg_status {
    BDG_OK = 0,
    BDG_EINVAL = -1,       /* null pointer, K == 0, bits % 64 != 0, L == 0, ... */
    BDG_EUNSUPPORTED = -2, /* bits > BDG_MAX_BITS, K > BDG_MAX_K, n == 0xFFFFFFFF */
    BDG_ENOMEM = -3,       /* workspace allocation failed or workspace too small */
    BDG_EDEVICE = -4       /* a HIP call failed (message in bdg_last_error) */
} bdg_status;

/* Which distance tile computes the Hamming distances. Both give identical
 * graphs: XOR + popcount on the vector ALUs, or an exact int8 matrix-core
 * contraction of {0, 1} candidate bytes a with +-1 query bytes 2q - 1, with
 * ham = popcount(q) - <a, 2q - 1>. */
typedef enum bdg_path {
    BDG_PATH_AUTO = 0,
    BDG_PATH_POPC = 1,
    BDG_PATH_MFMA = 2
} bdg_path;

/* Options. Zero-initialise and set struct_size = sizeof(bdg_knn_opts); every
 * zero field takes its default. */
typedef struct bdg_knn_opts {
    uint32_t struct_size;
    int32_t path;            /* bdg_path; default AUTO */
    uint32_t row_block;      /* rows per row block (default 131072) */
    uint32_t col_block;      /* columns per column block (default 262144 on
                                the matrix-core path, 131072 on the vector-ALU
                                path; at most 2097152) */
    void *workspace;         /* optional device scratch; if NULL the library
                                allocates stream-ordered and frees before return */
    size_t workspace_bytes;  /* size of `workspace` */
    uint32_t first_rowblock; /* resume: start at this row block (default 0) */
    uint32_t stop_rowblock;  /* stop before this row block (0 = run to the end) */
    uint32_t tile_variant;   /* batched plans: work order (BDG_ORDER_*); else 0 */
    uint32_t n_tile_events;  /* length of tile_events (0 = no timing) */
    void **tile_events;      /* optional caller-created hipEvent_t handles: for
                                the i-th tile launch of the call (vector-ALU
                                path: one per row block, in order; matrix-core
                                path: one launch for the whole call), events
                                [2i] and [2i + 1] are recorded on the stream
                                just before and just after it, while
                                2i + 1 < n_tile_events */
    uint32_t wait_limit;     /* matrix-core path: polls one dependency wait of
                                the persistent launch makes before it gives up
                                and sets the stall flag (0 = default, seconds;
                                a correct run never reaches it). Lowering it
                                is a test hook for the give-up path */
    uint32_t tile_schedule;  /* matrix-core tile schedule (BDG_SCHEDULE_*; the
                                graph is the same under every schedule);
                                default 0 (the library's choice), or the
                                autotuned one with path AUTO and col_block 0 */
    uint32_t bound_group;    /* matrix-core path: admission bounds before the
                                search (BDG_BOUND_*): 0 = default (on, pivot
                                groups of BDG_BOUND_GROUP_DEFAULT rows, or the
                                autotuned setting with path AUTO and col_block
                                0), BDG_BOUND_OFF, or rows per pivot group
                                (BDG_BOUND_GROUP_MIN..BDG_BOUND_GROUP_MAX).
                                The graph is the same either way */
    uint32_t reserved;
} bdg_knn_opts;

/* Admission bounds (matrix-core path). Before the exhaustive search every row
 * gets an upper bound on its K-th neighbour distance: the K-th smallest
 * distance to the other members of its group and of the groups of its second-
 * and third-nearest pivots, where pivots are every bound_group-th row of the
 * partition and each row joins its nearest pivot's group. Any K other rows of
 * the partition bound the final K-th distance from above, so admitting only
 * candidates at most the bound while a row's list is not full leaves the graph
 * unchanged; it spares the admissions of far candidates seen before the row's
 * own cluster (the first reduce of Sec. 3.2 searches a partition
 * exhaustively, in input order). Costs about n * n / bound_group pair
 * distances and (bits / 8 + 36) n bytes of workspace. */
#define BDG_BOUND_OFF 1u
#define BDG_BOUND_GROUP_DEFAULT 256u
#define BDG_BOUND_GROUP_MIN 16u
#define BDG_BOUND_GROUP_MAX (1u << 24)

/* Tile schedules of the matrix-core build and of batched plans. They differ
 * in where the rows' running lists live, the size of their pending-key
 * buffers and the depth of the stage ring of candidate operands, never in the
 * result. */
#define BDG_SCHEDULE_DEFAULT 0   /* the library's choice: GLOBAL_LISTS where it
                                    is built for the code length and K (the
                                    fastest measured there), else LDS_LISTS */
#define BDG_SCHEDULE_DEEP_RING 1 /* lists in LDS, 16 pending keys per row,
                                    more stages in flight; codes of 128, 256
                                    or 512 bits */
#define BDG_SCHEDULE_GLOBAL_LISTS 2 /* the rows' running lists are kept as
                                    keys in the output index rows instead
                                    of LDS, which leaves room for eight
                                    compute waves of 48 rows (each operand
                                    read feeds more products); codes of 128,
                                    256 or 512 bits with up to 128 keys.
                                    Until the build (or the resumed row
                                    range) completes, out_idx holds these
                                    intermediate keys */
#define BDG_SCHEDULE_LDS_LISTS 3 /* lists in LDS, 32 pending keys per row;
                                    every code length and K */

/* ---------------------------------------------------------------- build --- */

/*
 * Exact Hamming kNN graph of one partition (Sec. 3.2, first reduce: every
 * record of the partition is a query against all of its records).
 *   codes   [n][bits/64] uint64, device
 *   n       number of codes (0 is a no-op)
 *   bits    code length, a multiple of 64, at most BDG_MAX_BITS
 *   K       neighbours per row, 1..BDG_MAX_K (the matrix-core path takes
 *           K <= BDG_MAX_K_TILE; path AUTO picks the vector ALUs beyond)
 *   out_idx [n][K] uint32, out_dist [n][K] uint16, device
 * Runs on the default stream and returns after completion. It allocates its
 * workspace itself and, on the matrix-core path, checks the persistent
 * launch's stall flag afterwards (BDG_EDEVICE if set; never in a correct run).
 */
int bdg_build_knn(const uint64_t *codes, uint32_t n, uint32_t bits, uint32_t K,
                  uint32_t *out_idx, uint16_t *out_dist);

/* As bdg_build_knn, enqueued on `stream` with options (opts may be NULL). The
 * graph is built blockwise: row blocks x column blocks; each column block
 * yields per-row top-K lists that are merged (as bdg_merge_lists) into the
 * output. On the matrix-core path the blocks are the items of one persistent
 * launch (tiles of rows x column blocks, a tile's blocks merged in column
 * order); its workspace ends with control words (a claim counter, a stall
 * flag that is never set in a correct run, and one progress word per tile).
 * With opts->workspace set, the call allocates nothing. Calls on one
 * workspace must not overlap. */
int bdg_build_knn_ex(const uint64_t *codes, uint32_t n, uint32_t bits, uint32_t K,
                     uint32_t *out_idx, uint16_t *out_dist, const bdg_knn_opts *opts,
                     void *stream);

/* Workspace bytes bdg_build_knn_ex needs for these arguments (0 if none). */
int bdg_build_knn_workspace_size(uint32_t n, uint32_t bits, uint32_t K,
                                 const bdg_knn_opts *opts, size_t *bytes);

/*
 * Outcome of the last bdg_build_knn_ex enqueued with this caller workspace
 * (opts->workspace) and the same n, bits, K and opts: waits for `stream`,
 * then reads the persistent launch's stall flag from the workspace's control
 * words. BDG_OK if the build completed normally (or its path has no
 * persistent launch), BDG_EDEVICE if a dependency wait gave up (the lists
 * are then unspecified; never in a correct run), BDG_EINVAL for a NULL or too
 * small workspace. The workspace is only read. The async build has no other
 * way to report this: its return value is decided before the kernel runs.
 */
int bdg_build_knn_check(uint32_t n, uint32_t bits, uint32_t K, const bdg_knn_opts *opts,
                        void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * matrix-core build of bdg_build_knn_ex (default blocks) with its workspace
 * in a static device array of BDG_NOALLOC_SCRATCH_MB MiB inside the library,
 * one copy per device, held until the process ends. The call allocates
 * nothing; the caller still passes codes and outputs (device pointers, as
 * bdg_build_knn_ex) and the stream, on which the work is enqueued.
 * Limit: the build's workspace (bdg_build_knn_workspace_size with path MFMA:
 * about n x bits bytes of operand fragments plus control words) must fit,
 * e.g. n up to about 260,000 codes of 256 bits or 130,000 of 512 bits; larger
 * inputs return BDG_EUNSUPPORTED before anything is enqueued. Every call on a
 * device shares that device's array: calls that overlap on one device (two
 * streams, two threads) race and must be serialised by the caller. Errors as
 * bdg_build_knn_ex; the stall flag can be read with bdg_build_knn_check only
 * through a caller workspace, so this variant does not report it.
 */
#define BDG_NOALLOC_SCRATCH_MB 64
int bdg_build_knn_noalloc(const uint64_t *codes, uint32_t n, uint32_t bits, uint32_t K,
                          uint32_t *out_idx, uint16_t *out_dist, void *stream);

/*
 * Merge neighbour lists (Sec. 3.2 second reduce; Sec. 3.3 merge-sort).
 *   in_idx/in_dist  [L][n][K_in], each list sorted by (dist, idx) and possibly
 *                   padded with sentinels (BDG_NO_IDX, BDG_NO_DIST)
 *   out_idx/out_dist [n][K]
 * Row r of the output = the K smallest distinct (dist, idx) pairs of the
 * union of the L lists of row r, ascending, sentinel-padded. An index must
 * carry the same distance wherever it appears. K_in, K in 1..BDG_MAX_K.
 */
int bdg_merge_lists(const uint32_t *in_idx, const uint16_t *in_dist, uint32_t n, uint32_t L,
                    uint32_t K_in, uint32_t K, uint32_t *out_idx, uint16_t *out_dist,
                    void *stream);

/*
 * One round of neighbourhood propagation (Sec. 3.3): every row is compared
 * with all neighbours of its first-floor neighbours (the second floor), and
 * keeps the K nearest of its own list and that floor.
 *   codes    [n][bits/64] uint64, device (bits a multiple of 64, at most
 *            BDG_MAX_BITS)
 *   in_idx   [n][K] uint32, device: row r's neighbours, any order; entries
 *            equal to BDG_NO_IDX, >= n or equal to r are absent. Only the
 *            indices are read: every distance is recomputed from the codes.
 *   out_idx/out_dist [n][K], device, must not overlap in_idx
 * Row r of the output = the K smallest distinct (ham(r, z), z), z != r, over
 * z in in_idx[r] and in in_idx[y] for every y in in_idx[r], ascending,
 * sentinel-padded (BDG_NO_IDX, BDG_NO_DIST). The propagation filter of
 * Sec. 3.6 (3) (a second-floor candidate farther than the row's current K-th
 * distance is not merged; ties are) is applied inside and never changes the
 * result. An exact graph is returned unchanged. Enqueued on `stream`; the
 * caller owns every buffer. Errors: BDG_EINVAL (bits not a multiple of 64,
 * K = 0, null pointer, overlapping outputs), BDG_EUNSUPPORTED (bits or K
 * beyond the maxima, n = 2^32 - 1), BDG_EDEVICE (launch failure); outputs are
 * untouched on validation errors. n = 0 is a no-op.
 */
int bdg_propagate(const uint64_t *codes, uint32_t n, uint32_t bits, uint32_t K,
                  const uint32_t *in_idx, uint32_t *out_idx, uint16_t *out_dist, void *stream);

/*
 * Binary k-means centres for the single-pass divide-and-conquer (Sec. 3.2,
 * Eq. 1-2), run on a down-sample.
 *   codes    [n][bits/64] uint64, device
 *   sample   host array of ns row indices (< n): the down-sample
 *   init     host array of m row indices (< n): the starting centres
 *   iters    rounds of: each sample row joins its nearest centre (ties to the
 *            smaller centre index); bit b of a centre becomes 1 iff more than
 *            half of its rows have bit b set (a tie gives 0); a centre
 *            without rows keeps its bits
 *   centres  [m][bits/64] uint64, device, written
 * Scratch is allocated on `stream` and freed before return; the call returns
 * after the work completes. Errors: BDG_EINVAL (bits, m = 0, null pointer, an
 * index >= n), BDG_EUNSUPPORTED (bits > BDG_MAX_BITS, m > 2^20), BDG_ENOMEM,
 * BDG_EDEVICE.
 */
int bdg_bkmeans(const uint64_t *codes, uint32_t n, uint32_t bits, const uint32_t *sample,
                uint32_t ns, const uint32_t *init, uint32_t m, uint32_t iters,
                uint64_t *centres, void *stream);

/*
 * Approximate kNN graph of the single-pass divide-and-conquer (Sec. 3.2).
 * Home of a row = its nearest centre (ties to the smaller index); D_j = the
 * rows whose home is j. Row q takes its nearest centres in order (at most T),
 * adding |D_j| to a running total and stopping once it reaches coarse_num
 * (the centre that crosses the budget is included), and its output row is
 * the K smallest (ham(q, b), b), b != q, over the home rows of those centres,
 * ascending, sentinel-padded. With T >= m and coarse_num >= n this is the
 * exact graph.
 *   codes [n][bits/64], centres [m][bits/64] uint64, device
 *   out_idx [n][K] uint32, out_dist [n][K] uint16, device
 * T in 1..64, K in 1..BDG_MAX_K_TILE, m in 1..2^20, coarse_num >= 1. Scratch
 * (about n (4 T + 4 + bits/8) bytes) is allocated and freed on `stream`
 * (stream-ordered). Errors as bdg_build_knn_ex; BDG_EUNSUPPORTED for T > 64.
 */
/*
 * Exact Hamming kNN of query codes against a base set: the exhaustive search
 * of one partition's queries against its base records (Sec. 3.2, the first
 * reduce with queries and base kept apart) and the binary linear search used
 * as ground truth for queries outside the base (Sec. 4.5). Row q = the first K
 * of (ham(queries[q], base[j]), j) over every base row j, in (distance, index)
 * order, padded with BDG_NO_IDX / BDG_NO_DIST when nb < K; no row is left out
 * (a query equal to base row j finds j at distance 0). Runs on the matrix-core
 * tile in its rectangular mode.
 *   queries [nq][bits/64], base [nb][bits/64] uint64, device
 *   out_idx [nq][K] uint32, out_dist [nq][K] uint16, device
 * K in 1..64; nb below 2^(32 - bits needed for a distance) (4,194,303 at 512
 * bits). A workspace of the base's operand fragments (about nb * bits bytes) is
 * allocated and freed on `stream` (stream-ordered); enqueued on `stream`.
 * Errors: BDG_EINVAL (bits, K = 0, null pointer), BDG_EUNSUPPORTED (bits >
 * BDG_MAX_BITS, K > 64, nb too large), BDG_ENOMEM, BDG_EDEVICE. nq = 0 is a
 * no-op.
 */
int bdg_hamming_knn(const uint64_t *queries, uint32_t nq, const uint64_t *base, uint32_t nb,
                    uint32_t bits, uint32_t K, uint32_t *out_idx, uint16_t *out_dist,
                    void *stream);

int bdg_build_knn_dac(const uint64_t *codes, uint32_t n, uint32_t bits, const uint64_t *centres,
                      uint32_t m, uint32_t T, uint32_t coarse_num, uint32_t K, uint32_t *out_idx,
                      uint16_t *out_dist, void *stream);

/*
 * Online search on the graph (Sec. 3.5): for each query, the nearest of the
 * S sampled rows `entries` (Hamming; ties to the smaller index) is the entry
 * point; hill-climbing keeps a candidate pool of the P smallest
 * (ham, index) seen and repeatedly expands the smallest pool member not yet
 * expanded (every neighbour in its graph row not visited before is marked
 * visited, measured and offered to the pool) until every pool member is
 * expanded; the pool is then re-ranked by squared L2 of the real-valued
 * features in float32 (each operation rounded, dimensions in order, ties to
 * the smaller index) and the N best are returned.
 *   codes [n][bits/64] uint64, graph [n][K] uint32 (absent: BDG_NO_IDX or
 *   >= n), feats [n][d] float, q_codes [nq][bits/64], q_feats [nq][d],
 *   q_exclude [nq] uint32 or NULL (a row each query must not return, e.g.
 *   its own), entries [S] uint32: all device
 *   out_idx [nq][N] uint32, out_dist [nq][N] float (padding BDG_NO_IDX,
 *   +inf), out_visited [nq] uint32 or NULL (rows visited per query)
 * 1 <= N <= P <= 1024, n < 2^31. Visited bitmaps (n/8 bytes per query, in
 * batches of at most 1 GiB) are allocated and freed on `stream`. Errors:
 * BDG_EINVAL (bits, zero sizes, N > P, null pointer), BDG_EUNSUPPORTED
 * (P > 1024, K > BDG_MAX_K_TILE, bits > BDG_MAX_BITS, n >= 2^31), BDG_ENOMEM,
 * BDG_EDEVICE.
 */
int bdg_graph_search(const uint64_t *codes, uint32_t n, uint32_t bits, const uint32_t *graph,
                     uint32_t K, const float *feats, uint32_t d, const uint64_t *q_codes,
                     const float *q_feats, const uint32_t *q_exclude, uint32_t nq,
                     const uint32_t *entries, uint32_t S, uint32_t P, uint32_t N,
                     uint32_t *out_idx, float *out_dist, uint32_t *out_visited, void *stream);

/* ---------------------------------------------------- many partitions --- */

/*
 * Many independent partitions in one persistent launch. The single-pass
 * divide-and-conquer (Sec. 3.2) yields partitions of very uneven size, which
 * the paper balances over its reduce nodes (Sec. 3.6 (1)); here every
 * partition (shard) is an exact kNN problem of its own:
 *   shard s = rows [offsets[s], offsets[s + 1]) of `codes`, searched against
 *   the same rows only; output row r (global) holds shard-local neighbour
 *   indices (column - offsets[s]), in the graph layout above.
 * Rows outside every shard are not written. Work items of up to 256 rows of
 * one shard are taken from a shared counter by one work-group per CU, longest
 * first (or in shard order), so one launch balances the uneven shards.
 *
 * A plan holds the work list, a counter and the operand workspace (device
 * memory it allocates once, about bits bytes per row). Launching a plan
 * allocates nothing, so it can be captured in a HIP graph.
 */
typedef struct bdg_batch_plan bdg_batch_plan;

#define BDG_ORDER_LONGEST_FIRST 0 /* work items by decreasing rows x columns */
#define BDG_ORDER_SHARD 1         /* work items in shard order */

typedef struct bdg_batch_info {
    uint32_t shards, rows, work_items, workgroups;
    int32_t order;         /* BDG_ORDER_* */
    int32_t schedule;      /* BDG_SCHEDULE_* in force (never DEFAULT: the
                              value it resolved to) */
    uint32_t bound_group;  /* rows per pivot group of the admission bounds, or
                              BDG_BOUND_OFF */
    uint32_t reserved;
    uint64_t pairs;        /* sum over shards of n_s (n_s - 1) */
    size_t device_bytes;   /* device memory held by the plan */
} bdg_batch_info;

/*
 * Build a plan. offsets: HOST array of S + 1 non-decreasing row offsets
 * (offsets[S] = rows of `codes` used). bits, K as for bdg_build_knn; every
 * shard must fit the matrix-core path (at most 2^(32 - bits needed for a
 * distance) - 1 rows). opts may be NULL; opts->tile_variant = BDG_ORDER_SHARD
 * selects shard order. Allocates device memory (synchronously).
 */
int bdg_batch_plan_create(const uint64_t *offsets, uint32_t S, uint32_t bits, uint32_t K,
                          const bdg_knn_opts *opts, bdg_batch_plan **plan);
void bdg_batch_plan_destroy(bdg_batch_plan *plan);
int bdg_batch_plan_info(const bdg_batch_plan *plan, bdg_batch_info *info);
/* Change the tile schedule (BDG_SCHEDULE_*, DEFAULT resolved as for a build;
 * rebuilds the work items, whose rows follow the schedule's tile, and drops a
 * captured graph);
 * BDG_EUNSUPPORTED if the schedule is not built for the plan's code length. */
int bdg_batch_plan_set_schedule(bdg_batch_plan *plan, int schedule);
/* Change the admission bounds (bound_group as in bdg_knn_opts: 0 = default,
 * BDG_BOUND_OFF, or rows per pivot group; uploads the pivot table, drops a
 * captured graph, waits for queued work first). The graph is the same either
 * way. A plan whose shards all have at most K + 1 rows has no bounds. */
int bdg_batch_plan_set_bound(bdg_batch_plan *plan, uint32_t bound_group);
/* Diagnostics: caller-created hipEvent_t handles recorded on the stream just
 * before and just after the persistent kernel of every later
 * bdg_build_knn_batched_plan call (not of graph replays), so that the kernel
 * can be timed apart from the operand prep and the admission bounds. Both
 * NULL stops it; one NULL is BDG_EINVAL. The plan does not own the events. */
int bdg_batch_plan_set_timing(bdg_batch_plan *plan, void *start_event, void *stop_event);
/* Change the work order (re-uploads the work list; drops a captured graph).
 * Waits for all work queued on the device first, so a launch of the plan
 * still in flight on any stream finishes with the old list. A plan holds one
 * work counter: its launches must not overlap (enqueue them on one stream). */
int bdg_batch_plan_set_order(bdg_batch_plan *plan, int order);

/* Enqueue the build of every shard on `stream` (operand prep, counter reset,
 * persistent kernel). Allocates nothing. codes: device [offsets[S]][bits/64];
 * out_idx/out_dist: device [offsets[S]][K]. */
int bdg_build_knn_batched_plan(const bdg_batch_plan *plan, const uint64_t *codes,
                               uint32_t *out_idx, uint16_t *out_dist, void *stream);

/* As bdg_build_knn_batched_plan, through a HIP graph: the first call (or a
 * call with other pointers) captures the launch sequence on `stream` (which
 * must not be the default stream) and instantiates it; every call launches
 * the graph. */
int bdg_build_knn_batched_graph(bdg_batch_plan *plan, const uint64_t *codes, uint32_t *out_idx,
                                uint16_t *out_dist, void *stream);

/* One-shot: plan, enqueue on `stream`, wait for completion, free the plan. */
int bdg_build_knn_batched_ex(const uint64_t *codes, const uint64_t *offsets, uint32_t S,
                             uint32_t bits, uint32_t K, uint32_t *out_idx, uint16_t *out_dist,
                             const bdg_knn_opts *opts, void *stream);

/* ------------------------------------------------ binarisers, float kNN --- */

/*
 * Sign-of-random-projection codes (the plain binariser; features are mapped
 * to Hamming space preserving locality, Sec. 3.1): bit j of row i is 1 iff
 * <x_i, proj[:, j]> > 0 in FP32 (strictly). x: device float [n][d] (d a
 * multiple of 16), proj: device float [d][bits] (bits a multiple of 64, at
 * most BDG_MAX_BITS), out_codes: device uint64 [n][bits/64] in the code
 * layout. Enqueues on `stream`.
 */
int bdg_encode(const float *x, uint32_t n, uint32_t d, const float *proj, uint32_t bits,
               uint64_t *out_codes, void *stream);

/* Codes from real values: bit j of row i = [z[i][j] > 0]; z device float
 * [n][bits]. */
int bdg_pack_signs(const float *z, uint32_t n, uint32_t bits, uint64_t *out_codes, void *stream);

/*
 * Exact squared-L2 kNN in FP32, the real-valued ground truth of recall
 * (Sec. 4.2): row q = the first K of (||q - y_j||^2, j) over base rows j,
 * leaving out exclude[q] (device int32 [nq], -1 = none; NULL = none), ties to
 * the smaller index. Distances are assembled as |q|^2 + |y|^2 - 2 <q, y>, the
 * inner products on the FP32 matrix cores with the top-K fused (no distance
 * block goes to memory), so near-ties closer than FP32 rounding may order
 * differently from exact arithmetic. d a multiple of 4 up to 512 takes the
 * matrix cores; other d a plain vector-ALU kernel with direct sums. queries:
 * device float [nq][d] and base: device float [nb][d], rows 4-byte aligned;
 * out_idx uint32 [nq][K] and out_dist float [nq][K] (padding: 0xFFFFFFFF /
 * +inf). K in 1..128. Allocates a stream-ordered workspace of norms and, for
 * a wide base split over work-groups, partial lists (about splits x nq x K x
 * 8 bytes).
 */
int bdg_float_knn(const float *queries, uint32_t nq, const float *base, uint32_t nb, uint32_t d,
                  uint32_t K, const int32_t *exclude, uint32_t *out_idx, float *out_dist,
                  void *stream);

/*
 * The learned binariser: an MLP d -> h -> bits with tanh units,
 *   Z1 = X W1^T + b1, H1 = tanh Z1, Z2 = H1 W2^T + b2, H = tanh Z2,
 * code bit j = [Z2_j > 0]. Products run on the BF16 matrix cores with FP32
 * accumulation; master weights are FP32. All pointers are device memory owned
 * by the caller. Shapes: d % 32 == 0, h % 64 == 0, bits % 64 == 0 (<= 1024);
 * a batch holds rows_pad rows (a multiple of 32), of which `rows` are used.
 */
typedef struct bdg_mlp_params {
    uint32_t d, h, bits;
    float *W1, *b1;          /* [h][d], [h] */
    float *W2, *b2;          /* [bits][h], [bits] */
    uint16_t *W1b;           /* bf16 copy of W1, [h][d] (bdg_mlp_refresh) */
    uint16_t *W2b, *W2bt;    /* bf16 copies of W2, [bits][h] and transposed [h][bits] */
} bdg_mlp_params;

typedef struct bdg_mlp_acts {
    uint32_t rows, rows_pad;
    uint16_t *Xb, *Xt;       /* input, bf16 [rows_pad][d] and [d][rows_pad] (Xt may be NULL
                                for inference) */
    float *H1;               /* [rows_pad][h] */
    uint16_t *H1b, *H1t;     /* bf16 [rows_pad][h] and [h][rows_pad] */
    float *Z2, *H;           /* [rows_pad][bits] */
    uint16_t *dZ2b, *dZ2t;   /* bf16 [rows_pad][bits] and [bits][rows_pad] */
    uint16_t *dZ1t;          /* bf16 [h][rows_pad] */
} bdg_mlp_acts;

typedef struct bdg_mlp_grads {
    float *W1, *b1, *W2, *b2; /* shapes of the parameters */
} bdg_mlp_grads;

typedef struct bdg_loss_opts {
    float margin, tau, lam_q, lam_b;
} bdg_loss_opts;

/* Batch rows X[idx[r]] * scale (idx NULL: rows 0..rows-1; 0xFFFFFFFF: a zero
 * row) into a->Xb / a->Xt; sets a->rows. X: device float [*][d]. */
int bdg_mlp_gather(const float *X, uint32_t d, const uint32_t *idx, uint32_t rows, float scale,
                   bdg_mlp_acts *a, void *stream);
int bdg_mlp_forward(const bdg_mlp_params *p, bdg_mlp_acts *a, void *stream);
/* Triplet loss on relaxed Hamming distances d(u, v) = (bits - <h_u, h_v>) / 2
 * of the rows (anchors 0..T-1, positives T..2T-1, negatives 2T..3T-1):
 *   L = mean softplus((d_ap - d_an + margin) / tau)
 *       + lam_q mean (|h| - 1)^2 + lam_b sum_j (mean_rows h_j)^2.
 * Writes dL/dZ2 into a->dZ2b / a->dZ2t (padding rows zero), gb2 = its column
 * sums, mu [bits] = the column means, *loss (device float) = L. */
int bdg_triplet_loss(const bdg_mlp_acts *a, uint32_t bits, uint32_t T, const bdg_loss_opts *o,
                     float *mu, float *gb2, float *loss, void *stream);
/* Gradients of W2, W1, b1 from a->dZ2b / a->dZ2t (b2's come from the loss). */
int bdg_mlp_backward(const bdg_mlp_params *p, const bdg_mlp_acts *a, bdg_mlp_grads *g,
                     void *stream);
/* Adam with bias correction (step t counts from 1) on `count` floats. */
int bdg_adam_step(float *param, const float *grad, float *m, float *v, size_t count, uint32_t t,
                  float lr, float beta1, float beta2, float eps, void *stream);
/* Refresh the bf16 copies of the weights from the FP32 masters. */
int bdg_mlp_refresh(const bdg_mlp_params *p, void *stream);
/* Codes of n rows X * scale (device float [n][d]) through the network. */
int bdg_mlp_encode(const bdg_mlp_params *p, const float *X, uint32_t n, float scale,
                   uint64_t *out_codes, void *stream);
/* C [M][N] (ldc) = A B^T for bf16 A [M][lda] and B [N][ldb] (K % 32 == 0,
 * lda, ldb multiples of 8), FP32 accumulation: the product the network uses. */
int bdg_gemm_nt_bf16(const uint16_t *A, uint32_t lda, const uint16_t *B, uint32_t ldb, uint32_t M,
                     uint32_t N, uint32_t K, float *C, uint32_t ldc, void *stream);

/* ------------------------------------------------------------- autotune --- */

/*
 * Schedule autotuning. Candidates compute the same graph; they are timed with
 * HIP events on `stream` (one warm-up, then averaged runs) and the fastest is
 * kept. `report` (may be NULL) receives a JSON object describing the choice
 * and every candidate's time. With BDG_AUTOTUNE_CACHE set, each choice is
 * appended to that file as one JSON line (read back by later processes).
 *
 * bdg_autotune_build: a coordinate search from the defaults over the
 *   matrix-core tile's column block (131072 / 262144 / 524288 columns), tile
 *   schedule (BDG_SCHEDULE_*) and admission-bound group (256, off, 128, 512,
 *   64), then the vector-ALU tile; writes the winner into opts->path,
 *   opts->col_block, opts->tile_schedule and opts->bound_group
 *   (opts->row_block is used as given) and remembers it for (bits, K,
 *   floor(log2 n)), so later calls with path AUTO and col_block 0 take it.
 *   Runs the build several times into out_idx/out_dist (device, [n][K]);
 *   allocates a workspace for the duration.
 * bdg_autotune_batched: the same search over the work order, the tile
 *   schedule and the admission-bound group; keeps the fastest in the plan.
 * With BDG_AUTOTUNE_LOG set, every candidate's time is printed to stderr as
 * it is taken.
 */
int bdg_autotune_build(const uint64_t *codes, uint32_t n, uint32_t bits, uint32_t K,
                       uint32_t *out_idx, uint16_t *out_dist, bdg_knn_opts *opts, void *stream,
                       char *report, size_t report_len);
int bdg_autotune_batched(bdg_batch_plan *plan, const uint64_t *codes, uint32_t *out_idx,
                         uint16_t *out_dist, void *stream, char *report, size_t report_len);

/* ------------------------------------------------------------ diagnostics --- */

/*
 * Sustained rate of one execution unit, for the roofline denominators of the
 * two Hamming tiles (not part of the method): a fixed loop of independent
 * instructions over every CU, timed with events on `stream` after a warm-up
 * run; waits for completion. BDG_PEAK_VALU_INT32: 32-bit integer vector
 * instructions per second (XOR, popcount-accumulate, add; lane operations).
 * BDG_PEAK_MFMA_INT8: int8 matrix-core operations per second (2 per
 * multiply-accumulate) of v_mfma_i32_16x16x64_i8 on random {0, 1} x +-1
 * operand bytes, the matrix tile's operands. Errors: BDG_EINVAL (unit,
 * NULL), BDG_ENOMEM, BDG_EDEVICE.
 */
#define BDG_PEAK_VALU_INT32 0
#define BDG_PEAK_MFMA_INT8 1
int bdg_probe_peak(int unit, double *ops_per_second, void *stream);

const char *bdg_status_string(int status);
/* Message of the last failed call on this thread ("" if none). */
const char *bdg_last_error(void);
int bdg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BDG_H_ */
