"""CPU oracle for the Hamming kNN-graph builder -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` may import this package. The product path (the GPU library and
its binding) never imports, links or runs anything here, and nothing here uses
the GPU library: the two share no code. Inputs come from the seeded generators
in ``paper_2102_04656_amd.datagen``, which hold none of the method's arithmetic.

Contents
  * ``knn_tiny``          -- pure-Python per-bit brute force with a full sort
                             (tiny inputs only); the plain definition.
  * ``knn_rows``          -- the same definition in plain C (``hamming_oracle.c``),
                             for rows sampled from large inputs.
  * ``knn_blocks``        -- per-column-block lists (the partition search of the
                             reduce step, Sec. 3.2) by the same C routine.
  * ``merge_lists``       -- top-K of the deduplicated union of lists (the
                             merge-sort of the second reduce, Sec. 3.2 / 3.3).
  * ``knn_sharded_rows``  -- the definition applied per shard, local indices.
  * ``pair_distances``    -- Hamming distance of explicit pairs.
  * ``propagate``         -- one round of neighbourhood propagation (Sec. 3.3):
                             top-K of a row's list and its neighbours' lists.
  * ``propagate_filtered``-- the same with the paper's propagation filter
                             (Sec. 3.6 (3)) applied to the second floor.
  * ``knn_rect``          -- queries against a separate base set (the same
                             definition with no row left out).
  * ``bkmeans``, ``nearest_centres``, ``dac_graph`` -- the single-pass
                             divide-and-conquer (Sec. 3.2): binary centres,
                             budgeted multi-assignment, partition search.
  * ``graph_search``      -- one query of the online search (Sec. 3.5):
                             sampled entry, hill-climbing with a candidate
                             pool, float32 re-rank of the pool.
Floating-point parts (the binarisers, the float-kNN ground truth, the encoder
network, its loss and optimiser) live in ``oracle.learned``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

NO_IDX = 0xFFFFFFFF
NO_DIST = 0xFFFF

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hamming_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP). Portable x86-64 flags only: the
    library may run on another host than the one that built it."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-mpopcnt", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-Wextra", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            lib = ctypes.CDLL(_LIB)
            u32, u64, p = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
            lib.oracle_knn_rows.argtypes = [p, u32, u32, u32, u32, u32, p, u32, p, p]
            lib.oracle_knn_rows.restype = ctypes.c_int
            lib.oracle_pair_distances.argtypes = [p, u32, p, p, u64, p]
            lib.oracle_pair_distances.restype = None
            lib.oracle_threads.restype = ctypes.c_int
            lib.oracle_set_threads.argtypes = [ctypes.c_int]
            _lib = lib
    return _lib


def threads() -> int:
    return int(_load().oracle_threads())


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------
# Pure-Python definition (tiny inputs)
# --------------------------------------------------------------------------

def _bit(codes, i, j):
    """Bit j of code i: word j // 64, position j % 64 (little-endian)."""
    return (int(codes[i][j // 64]) >> (j % 64)) & 1


def hamming_tiny(codes, i, j) -> int:
    """Count of bit positions in which codes i and j differ (per-bit loop)."""
    bits = 64 * len(codes[0])
    return sum(1 for b in range(bits) if _bit(codes, i, b) != _bit(codes, j, b))


def knn_tiny(codes, K: int):
    """Row i = first K of sorted [(ham(i, j), j) for j != i], sentinel-padded.

    Plain definition with Python's sort; only for n of a few hundred at most.
    """
    codes = [[int(w) for w in row] for row in np.asarray(codes, dtype=np.uint64)]
    n = len(codes)
    idx = np.full((n, K), NO_IDX, dtype=np.uint32)
    dist = np.full((n, K), NO_DIST, dtype=np.uint16)
    for i in range(n):
        keys = sorted((hamming_tiny(codes, i, j), j) for j in range(n) if j != i)
        for r, (d, j) in enumerate(keys[:K]):
            idx[i, r] = j
            dist[i, r] = d
    return idx, dist


# --------------------------------------------------------------------------
# Plain C brute force
# --------------------------------------------------------------------------

def knn_rows(codes: np.ndarray, K: int, rows=None, cols=None):
    """Exact kNN rows of ``codes`` (``[n][W]`` uint64) against columns
    ``cols = (c0, c1)`` (default all), for ``rows`` (default all)."""
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    n, words = codes.shape
    c0, c1 = (0, n) if cols is None else (int(cols[0]), int(cols[1]))
    if rows is None:
        nrows, rptr, keep = n, None, None
    else:
        keep = np.ascontiguousarray(rows, dtype=np.uint32)
        nrows, rptr = keep.size, _ptr(keep)
    idx = np.empty((nrows, K), dtype=np.uint32)
    dist = np.empty((nrows, K), dtype=np.uint16)
    if nrows:
        rc = _load().oracle_knn_rows(_ptr(codes), n, words, K, c0, c1, rptr, nrows,
                                     _ptr(idx), _ptr(dist))
        if rc != 0:
            raise RuntimeError("oracle_knn_rows failed")
    return idx, dist


def knn_blocks(codes: np.ndarray, K: int, col_block: int, rows=None):
    """Per-column-block lists ``[L][nrows][K]`` (each block searched alone)."""
    n = codes.shape[0]
    bounds = [(c, min(n, c + col_block)) for c in range(0, n, col_block)]
    parts = [knn_rows(codes, K, rows=rows, cols=b) for b in bounds]
    return (np.stack([p[0] for p in parts]), np.stack([p[1] for p in parts]))


def pair_distances(codes: np.ndarray, a, b) -> np.ndarray:
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    out = np.empty(a.size, dtype=np.uint16)
    if a.size:
        _load().oracle_pair_distances(_ptr(codes), codes.shape[1], _ptr(a), _ptr(b),
                                      a.size, _ptr(out))
    return out


# --------------------------------------------------------------------------
# Merge of neighbour lists (second reduce: merge all lists of one label and
# sort out the final kNN)
# --------------------------------------------------------------------------

def merge_lists(in_idx: np.ndarray, in_dist: np.ndarray, K: int):
    """``in_idx/in_dist [L][n][K_in]`` -> top-K ``[n][K]`` of the union.

    Per row: drop sentinel entries (idx == 0xFFFFFFFF), remove repeated
    (dist, idx) pairs, sort ascending by (dist, idx), keep K, pad with
    sentinels. Lists that name one index with two different distances are
    outside the contract (distances are a function of the pair).
    """
    in_idx = np.asarray(in_idx, dtype=np.uint32)
    in_dist = np.asarray(in_dist, dtype=np.uint16)
    L, n, kin = in_idx.shape
    out_idx = np.full((n, K), NO_IDX, dtype=np.uint32)
    out_dist = np.full((n, K), NO_DIST, dtype=np.uint16)
    for r in range(n):
        pairs = set()
        for l in range(L):
            for t in range(kin):
                j = int(in_idx[l, r, t])
                if j != NO_IDX:
                    pairs.add((int(in_dist[l, r, t]), j))
        for k, (d, j) in enumerate(sorted(pairs)[:K]):
            out_idx[r, k] = j
            out_dist[r, k] = d
    return out_idx, out_dist


# --------------------------------------------------------------------------
# Many independent partitions (shards), indices local to the shard
# --------------------------------------------------------------------------

def knn_sharded_rows(codes: np.ndarray, offsets, K: int, shard: int, rows=None):
    """kNN rows of one shard; ``rows`` are shard-local row ids."""
    lo, hi = int(offsets[shard]), int(offsets[shard + 1])
    return knn_rows(codes[lo:hi], K, rows=rows)


# --------------------------------------------------------------------------
# Neighbourhood propagation (one more floor of neighbours)
# --------------------------------------------------------------------------

def _ham_row(codes: np.ndarray, x: int, cols) -> dict:
    """{j: Hamming distance of codes x and j} (the C pair routine)."""
    cols = sorted(cols)
    if not cols:
        return {}
    d = pair_distances(codes, np.full(len(cols), x, dtype=np.uint32), np.array(cols, dtype=np.uint32))
    return dict(zip(cols, d.tolist()))


def _floors(in_idx: np.ndarray, n: int, x: int):
    first = [int(j) for j in in_idx[x] if int(j) != NO_IDX and int(j) < n]
    second = []
    for y in first:
        second += [int(z) for z in in_idx[y] if int(z) != NO_IDX and int(z) < n]
    return first, second


def propagate(codes: np.ndarray, in_idx: np.ndarray, K: int, rows=None):
    """One round of neighbourhood propagation (Sec. 3.3), the plain definition.

    The flat, depth-one breadth-first step: row x compares itself with every
    neighbour of its first-floor neighbours (the second floor) and keeps, from
    its own list and that floor, the K smallest distinct (ham(x, z), z) with
    z != x, ascending, sentinel-padded. Distances are recomputed from the codes
    (the input distances are not used). Entries equal to 0xFFFFFFFF or >= n
    are absent. ``rows`` (optional) selects output rows: the result then has
    one row per entry of ``rows``. Small inputs or row samples only.
    """
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    in_idx = np.asarray(in_idx, dtype=np.uint32)
    n = codes.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    out_idx = np.full((rows.size, K), NO_IDX, dtype=np.uint32)
    out_dist = np.full((rows.size, K), NO_DIST, dtype=np.uint16)
    for r, x in enumerate(rows.tolist()):
        first, second = _floors(in_idx, n, x)
        cand = (set(first) | set(second)) - {x}
        d = _ham_row(codes, x, cand)
        for k, (dd, j) in enumerate(sorted((d[j], j) for j in cand)[:K]):
            out_idx[r, k] = j
            out_dist[r, k] = dd
    return out_idx, out_dist


def propagate_filtered(codes: np.ndarray, in_idx: np.ndarray, K: int):
    """As ``propagate``, with the propagation filter (Sec. 3.6 (3)): a
    second-floor candidate of x is dropped when its distance exceeds the
    largest distance between x and its first-floor neighbours (the reading
    taken: drop when strictly larger, keep ties, so that a tie at that distance
    with a smaller index can still enter). With K first-floor neighbours the
    filter cannot change the result; the tests check that it does not."""
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    in_idx = np.asarray(in_idx, dtype=np.uint32)
    n = codes.shape[0]
    out_idx = np.full((n, K), NO_IDX, dtype=np.uint32)
    out_dist = np.full((n, K), NO_DIST, dtype=np.uint16)
    for x in range(n):
        first, second = _floors(in_idx, n, x)
        first = [j for j in first if j != x]
        d1 = _ham_row(codes, x, set(first))
        full = len(set(first)) >= K
        maxd = max(d1.values()) if (full and d1) else None
        d2 = _ham_row(codes, x, set(second) - {x} - set(first))
        kept = {j: v for j, v in d2.items() if maxd is None or v <= maxd}
        allc = dict(d1)
        allc.update(kept)
        for k, (dd, j) in enumerate(sorted((v, j) for j, v in allc.items())[:K]):
            out_idx[x, k] = j
            out_dist[x, k] = dd
    return out_idx, out_dist


# --------------------------------------------------------------------------
# Single-pass divide-and-conquer (Sec. 3.2): binary k-means centres, each
# point's nearest centres under the coarse_num budget, and the search of
# every point against the home members of its selected centres
# --------------------------------------------------------------------------

def _ham_matrix(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """[len(a)][len(b)] Hamming distances by per-word XOR and a byte table."""
    table = np.array([bin(v).count("1") for v in range(256)], dtype=np.int32)
    out = np.zeros((a.shape[0], b.shape[0]), dtype=np.int32)
    for w in range(a.shape[1]):
        x = np.bitwise_xor(a[:, w][:, None], b[:, w][None, :])
        out += table[x.view(np.uint8).reshape(x.shape + (8,))].sum(axis=2)
    return out


def bkmeans(codes: np.ndarray, sample, init, iters: int) -> np.ndarray:
    """Binary k-means on the rows ``sample`` of ``codes`` (Sec. 3.2, Eq. 1-2).

    Centres start as the codes of rows ``init`` (m of them). Each iteration:
    assign every sample point to its nearest centre (Hamming; ties to the
    smaller centre index), then set bit b of centre j to 1 iff more than half
    of its points have bit b set (the majority form of c_j = sgn(sum x_i) on
    binary members; a tie gives 0); a centre with no point keeps its bits.
    """
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    S = codes[np.asarray(sample, dtype=np.int64)]
    C = codes[np.asarray(init, dtype=np.int64)].copy()
    W = codes.shape[1]
    bits = np.unpackbits(S.view(np.uint8), axis=1, bitorder="little").astype(np.int64)
    for _ in range(iters):
        D = _ham_matrix(S, C)
        home = np.argmin(D, axis=1)  # first minimum: the smaller index
        for j in range(C.shape[0]):
            members = bits[home == j]
            if members.shape[0] == 0:
                continue
            ones = members.sum(axis=0)
            newbits = (2 * ones > members.shape[0]).astype(np.uint8)
            C[j] = np.packbits(newbits, bitorder="little").view(np.uint64)[:W]
    return C


def nearest_centres(codes: np.ndarray, centres: np.ndarray, T: int):
    """Per point the T nearest centres, ascending by (distance, centre)."""
    D = _ham_matrix(np.ascontiguousarray(codes, dtype=np.uint64),
                    np.ascontiguousarray(centres, dtype=np.uint64))
    m = D.shape[1]
    order = np.lexsort((np.broadcast_to(np.arange(m), D.shape), D), axis=1)[:, :T]
    return order.astype(np.uint32), np.take_along_axis(D, order, axis=1).astype(np.uint16)


def knn_rect(queries: np.ndarray, base: np.ndarray, K: int):
    """Exact kNN of query codes against a base set (the exhaustive search of a
    partition's queries against its base records, Sec. 3.2; the binary linear
    search of Sec. 4.5): row q = the first K of (ham(q, b_j), j) over every
    base row j, ascending, padded with (NO_IDX, NO_DIST); no row left out."""
    nq = np.asarray(queries).shape[0]
    oi = np.full((nq, K), NO_IDX, dtype=np.uint32)
    od = np.full((nq, K), NO_DIST, dtype=np.uint16)
    if nq and np.asarray(base).shape[0]:
        i, d = nearest_centres(queries, base, K)
        oi[:, :i.shape[1]] = i
        od[:, :d.shape[1]] = d
    return oi, od


def dac_graph(codes: np.ndarray, centres: np.ndarray, T: int, coarse_num: int, K: int,
              rows=None):
    """The approximate kNN graph of the single-pass divide-and-conquer.

    Home of a point = its nearest centre; D_j = the points whose home is j.
    Point q selects its nearest centres in order, adding centre j and |D_j|
    to a running total and stopping once the total reaches coarse_num (the
    centre that crosses the budget is included), at most T centres. Its row
    = the K smallest (ham(q, b), b), b != q, over b in the union of D_j of the
    selected centres (disjoint sets, so the second reduce has nothing to
    deduplicate), sentinel-padded. ``rows`` selects output rows.
    """
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    n = codes.shape[0]
    top, _ = nearest_centres(codes, centres, T)
    home = top[:, 0].astype(np.int64)
    size = np.bincount(home, minlength=centres.shape[0])
    members = [np.nonzero(home == j)[0] for j in range(centres.shape[0])]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    out_idx = np.full((rows.size, K), NO_IDX, dtype=np.uint32)
    out_dist = np.full((rows.size, K), NO_DIST, dtype=np.uint16)
    for r, q in enumerate(rows.tolist()):
        cand, total = [], 0
        for j in top[q].tolist():
            cand.append(members[j])
            total += int(size[j])
            if total >= coarse_num:
                break
        c = np.concatenate(cand)
        c = c[c != q]
        if c.size == 0:
            continue
        d = pair_distances(codes, np.full(c.size, q, dtype=np.uint32), c.astype(np.uint32))
        order = np.lexsort((c, d))[:K]
        out_idx[r, : order.size] = c[order]
        out_dist[r, : order.size] = d[order]
    return out_idx, out_dist


# --------------------------------------------------------------------------
# Online search on the graph (Sec. 3.5): sampled entry points, hill-climbing
# with a candidate pool, re-rank of the pool by real-valued features
# --------------------------------------------------------------------------

def l2_f32(a: np.ndarray, b: np.ndarray) -> np.float32:
    """Squared L2 distance in float32, accumulated over the dimensions in
    order: acc = acc + (a_i - b_i)^2, every operation rounded to float32
    (no fused multiply-add)."""
    acc = np.float32(0.0)
    for ai, bi in zip(a.astype(np.float32), b.astype(np.float32)):
        t = np.float32(ai - bi)
        acc = np.float32(acc + np.float32(t * t))
    return acc


def graph_search(codes: np.ndarray, graph_idx: np.ndarray, feats: np.ndarray, q_code, q_feat,
                 entries, P: int, N: int, exclude=None, max_expand: int = 1 << 20,
                 trace: dict | None = None):
    """One query of the online search (Sec. 3.5).

    Entry point: the nearest of the sampled rows ``entries`` to the query
    (Hamming; ties to the smaller index); only it starts the pool and counts
    as visited (the other samples stay reachable through the graph).
    Hill-climbing with a candidate pool of the P smallest (ham, idx) seen:
    repeatedly expand the smallest pool member not yet expanded (every
    neighbour in its graph row not visited before is measured, marked
    visited and offered to the pool), until every pool member is expanded.
    ``exclude`` (the query's own row) is never measured. Re-rank: all pool
    members by ``l2_f32`` to the query's features, ties to the smaller
    index; returns (idx [N], dist float32 [N]) padded with (0xFFFFFFFF,
    inf), and the number of rows visited. If ``trace`` is a dict, it
    receives the expanded rows in order ("expand") and the final pool of
    (ham, idx) keys ("pool").
    """
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    n = codes.shape[0]
    q_code = np.asarray(q_code, dtype=np.uint64)

    def ham(j):
        return sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(q_code, codes[j]))

    visited = set() if exclude is None else {int(exclude)}
    best = None
    for e in [int(x) for x in entries]:
        if e in visited or e >= n:
            continue
        k = (ham(e), e)
        best = k if best is None or k < best else best
    if best is not None:
        visited.add(best[1])
    out_idx = np.full(N, NO_IDX, dtype=np.uint32)
    out_dist = np.full(N, np.inf, dtype=np.float32)
    if best is None:
        return out_idx, out_dist, len(visited)
    pool = [best]            # sorted (ham, idx), at most P
    expanded = set()
    steps = 0
    while steps < max_expand:
        cand = [k for k in pool if k[1] not in expanded]
        if not cand:
            break
        u = cand[0][1]
        expanded.add(u)
        if trace is not None:
            trace.setdefault("expand", []).append(u)
        steps += 1
        for v in [int(x) for x in graph_idx[u]]:
            if v == NO_IDX or v >= n or v in visited:
                continue
            visited.add(v)
            pool.append((ham(v), v))
        pool = sorted(pool)[:P]
    if trace is not None:
        trace["pool"] = list(pool)
    rr = sorted((l2_f32(feats[j], q_feat), j) for _, j in pool)[:N]
    for k, (d, j) in enumerate(rr):
        out_idx[k] = j
        out_dist[k] = d
    return out_idx, out_dist, len(visited)
