"""Pins of the CPU oracle to things other than itself (CPU only).

Each ``pin_*`` takes a kNN function ``knn(codes, K) -> (idx, dist)`` and checks
it against hand-derived fixtures, closed forms, degenerate cases, invariants or
a library route (numpy ``unpackbits`` + ``lexsort``). The oracle must pass all
of them; ``test_pins_catch_planted_mistakes`` plants plausible mistakes in a
copy of the definition and shows each is caught by at least one pin.
"""
from math import comb

import numpy as np
import pytest

import oracle
from paper_2102_04656_amd import datagen
from tests import golden_io

NO_IDX, NO_DIST = oracle.NO_IDX, oracle.NO_DIST


def c_knn(codes, K):
    return oracle.knn_rows(codes, K)


def np_distances(codes, rows):
    """Library route: unpack to bits and count differing positions."""
    u = datagen.unpack_bits(codes).astype(np.int16)
    return (u[rows][:, None, :] != u[None, :, :]).sum(axis=2)


# ----------------------------------------------------------------- pins

def pin_cube3(knn):
    layouts, exp_idx, exp_dist = golden_io.cube3()
    for bits, positions, background in layouts:
        codes = golden_io.cube3_codes(bits, positions, background)
        for K in (3, 7, 10):
            idx, dist = knn(codes, K)
            k = min(K, 7)
            if not (np.array_equal(idx[:, :k], exp_idx[:, :k])
                    and np.array_equal(dist[:, :k], exp_dist[:, :k])):
                return False
            if K > 7 and not ((idx[:, 7:] == NO_IDX).all() and (dist[:, 7:] == NO_DIST).all()):
                return False
    return True


def hypercube_codes(k, bits, seed):
    """All 2^k vertices of {0,1}^k written at k random bit positions spread over
    every word, on a random fixed background."""
    g = np.random.default_rng(seed)
    positions = g.choice(bits, size=k, replace=False)
    # make sure the last word holds a varying bit
    positions[-1] = bits - 1 - int(g.integers(0, 64))
    positions = list(dict.fromkeys(int(p) for p in positions))
    while len(positions) < k:
        p = int(g.integers(0, bits))
        if p not in positions:
            positions.append(p)
    background = g.integers(0, 2, size=bits)
    rows = np.tile(background, (2 ** k, 1)).astype(np.uint8)
    for v in range(2 ** k):
        for t, p in enumerate(positions):
            rows[v, p] = (v >> t) & 1
    return datagen.pack_bits(rows)


def pin_hypercube(knn):
    for k, bits, seed in ((6, 128, 0), (7, 512, 1), (5, 256, 2)):
        codes = hypercube_codes(k, bits, seed)
        n = 2 ** k
        idx, dist = knn(codes, n - 1)
        for i in range(n):
            # closed form on vertex labels: ham(i, j) = number of differing label bits
            expected = sorted((bin(i ^ j).count("1"), j) for j in range(n) if j != i)
            if [(int(d), int(j)) for d, j in zip(dist[i], idx[i])] != expected:
                return False
            hist = np.bincount(dist[i], minlength=k + 1)
            if any(hist[r] != comb(k, r) for r in range(1, k + 1)):
                return False
        idx1, dist1 = knn(codes, k)
        for i in range(n):
            if list(idx1[i]) != sorted(i ^ (1 << b) for b in range(k)) or (dist1[i] != 1).any():
                return False
    return True


def pin_identical(knn):
    codes = np.tile(datagen.uniform_codes(1, 128, seed=3), (40, 1))
    for K in (1, 7, 39, 45):
        idx, dist = knn(codes, K)
        for i in range(40):
            others = [j for j in range(40) if j != i][:K]
            m = len(others)
            if list(idx[i, :m]) != others or (dist[i, :m] != 0).any():
                return False
            if (idx[i, m:] != NO_IDX).any() or (dist[i, m:] != NO_DIST).any():
                return False
    return True


def pin_library_route(knn):
    """Whole graph equals numpy unpackbits distances + lexsort, on tie-heavy data."""
    for n, bits, p, K, seed in ((150, 64, 0.05, 9, 4), (120, 256, 0.2, 17, 5),
                                (90, 512, 0.25, 89, 6), (60, 192, 0.1, 64, 7)):
        codes = datagen.clustered_codes(n, bits, n_centres=6, p=p, seed=seed)
        idx, dist = knn(codes, K)
        D = np_distances(codes, np.arange(n))
        for i in range(n):
            cand = np.array([j for j in range(n) if j != i])
            order = np.lexsort((cand, D[i, cand]))[:K]
            m = order.size
            if not (np.array_equal(idx[i, :m], cand[order])
                    and np.array_equal(dist[i, :m], D[i, cand[order]])):
                return False
            if (idx[i, m:] != NO_IDX).any():
                return False
    return True


def pin_invariants(knn):
    """Invariants that hold for any correct output, on clustered data."""
    n, bits, K = 600, 256, 16
    codes = datagen.clustered_codes(n, bits, n_centres=12, p=0.2, seed=8)
    idx, dist = knn(codes, K)
    keys = dist.astype(np.int64) * n + idx.astype(np.int64)
    if not (np.diff(keys, axis=1) > 0).all():        # sorted, distinct
        return False
    if (idx == np.arange(n)[:, None]).any():         # no self
        return False
    D = np_distances(codes, np.arange(n))
    if not np.array_equal(D[np.arange(n)[:, None], idx], dist):
        return False
    # symmetry of the reported distances
    for i in range(n):
        for r in range(K):
            j = int(idx[i, r])
            hit = np.nonzero(idx[j] == i)[0]
            if hit.size and dist[j, hit[0]] != dist[i, r]:
                return False
    # triangle inequality over reported neighbour pairs
    g = np.random.default_rng(9)
    for _ in range(2000):
        i = int(g.integers(n))
        a, b = g.integers(K, size=2)
        j, l = int(idx[i, a]), int(idx[i, b])
        if D[j, l] > int(dist[i, a]) + int(dist[i, b]):
            return False
    # certificate: every j outside row i has (d_ij, j) > the last key
    for i in g.choice(n, size=40, replace=False):
        last = int(dist[i, -1]) * n + int(idx[i, -1])
        inside = set(int(v) for v in idx[i]) | {int(i)}
        for j in range(n):
            if j not in inside and int(D[i, j]) * n + j <= last:
                return False
    return True


PINS = [pin_cube3, pin_hypercube, pin_identical, pin_library_route, pin_invariants]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_c_oracle_pinned(pin):
    assert pin(c_knn)


@pytest.mark.parametrize("pin", [pin_cube3, pin_identical], ids=lambda f: f.__name__)
def test_tiny_oracle_pinned(pin):
    assert pin(oracle.knn_tiny)


@pytest.mark.parametrize("bits", [64, 128, 256, 512])
def test_c_oracle_equals_tiny(bits):
    n = 70
    codes = datagen.clustered_codes(n, bits, n_centres=5, p=0.1, seed=bits)
    for K in (1, 5, n - 1, n + 3):
        a = oracle.knn_rows(codes, K)
        b = oracle.knn_tiny(codes, K)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_row_subset_and_column_range():
    codes = datagen.clustered_codes(500, 128, n_centres=8, p=0.15, seed=11)
    full = oracle.knn_rows(codes, 12)
    rows = np.array([0, 7, 499, 250, 3], dtype=np.uint32)
    sub = oracle.knn_rows(codes, 12, rows=rows)
    assert np.array_equal(sub[0], full[0][rows]) and np.array_equal(sub[1], full[1][rows])
    # column range: library route restricted to [c0, c1)
    c0, c1 = 130, 377
    idx, dist = oracle.knn_rows(codes, 12, cols=(c0, c1))
    D = np_distances(codes, np.arange(500))
    for i in (0, 200, 376, 499):
        cand = np.array([j for j in range(c0, c1) if j != i])
        order = np.lexsort((cand, D[i, cand]))[:12]
        assert np.array_equal(idx[i], cand[order])


# ----------------------------------------------------------- identities

def test_pm1_dot_identity():
    """ham(a, b) = (bits - <s_a, s_b>) / 2 with s = 2y - 1, including all-0/all-1."""
    g = np.random.default_rng(12)
    for bits in (64, 128, 256, 512, 1024):
        codes = datagen.uniform_codes(64, bits, seed=bits)
        codes[0] = 0
        codes[1] = np.uint64(0xFFFFFFFFFFFFFFFF)
        s = 2 * datagen.unpack_bits(codes).astype(np.int64) - 1
        a = g.integers(64, size=500)
        b = g.integers(64, size=500)
        a[:2], b[:2] = [0, 0], [1, 0]
        ham = oracle.pair_distances(codes, a, b).astype(np.int64)
        dot = (s[a] * s[b]).sum(axis=1)
        assert np.array_equal(ham, (bits - dot) // 2)
        assert ham[0] == bits and ham[1] == 0


def test_eq1_squared_euclid_is_hamming():
    """On {0,1} vectors the squared Euclidean distance of Eq. 1 is Hamming."""
    codes = datagen.uniform_codes(100, 256, seed=13)
    y = datagen.unpack_bits(codes).astype(np.float64)
    g = np.random.default_rng(14)
    a, b = g.integers(100, size=300), g.integers(100, size=300)
    sq = ((y[a] - y[b]) ** 2).sum(axis=1)
    assert np.array_equal(sq.astype(np.int64), oracle.pair_distances(codes, a, b).astype(np.int64))


# ---------------------------------------------------------------- merge

def test_merge_golden():
    K, in_idx, in_dist, out_idx, out_dist = golden_io.merge_small()
    idx, dist = oracle.merge_lists(in_idx, in_dist, K)
    assert np.array_equal(idx, out_idx) and np.array_equal(dist, out_dist)


@pytest.mark.parametrize("col_block", [37, 128, 333, 1000])
def test_blocks_then_merge_equals_whole(col_block):
    """Any column blocking followed by the merge gives the whole-range graph."""
    codes = datagen.clustered_codes(1000, 128, n_centres=10, p=0.15, seed=15)
    K = 20
    rows = np.arange(0, 1000, 7, dtype=np.uint32)
    whole = oracle.knn_rows(codes, K, rows=rows)
    bi, bd = oracle.knn_blocks(codes, K, col_block, rows=rows)
    mi, md = oracle.merge_lists(bi, bd, K)
    assert np.array_equal(mi, whole[0]) and np.array_equal(md, whole[1])
    # duplicated lists change nothing
    mi2, md2 = oracle.merge_lists(np.concatenate([bi, bi[::-1]]),
                                  np.concatenate([bd, bd[::-1]]), K)
    assert np.array_equal(mi2, whole[0]) and np.array_equal(md2, whole[1])


def test_sharded_local_indices():
    codes, offsets = datagen.sharded_codes(n_shards=3, lo=20, hi=60, c_lo=2, c_hi=4,
                                           bits=128, p=0.2, seed=16)
    for s in range(3):
        n_s = int(offsets[s + 1] - offsets[s])
        idx, dist = oracle.knn_sharded_rows(codes, offsets, 8, s)
        t_idx, t_dist = oracle.knn_tiny(codes[int(offsets[s]):int(offsets[s + 1])], 8)
        assert np.array_equal(idx, t_idx) and np.array_equal(dist, t_dist)
        assert ((idx < n_s) | (idx == NO_IDX)).all()


# ----------------------------------------------- planted mistakes (CPU)

def _mutant(kind):
    """A copy of the definition with one plausible mistake planted."""
    def knn(codes, K):
        codes = np.asarray(codes, dtype=np.uint64)
        n, words = codes.shape
        u = datagen.unpack_bits(codes).astype(np.int16)
        if kind == "drop_last_word":
            u = u[:, : 64 * (words - 1)] if words > 1 else u[:, :32]
        if kind == "bit_order_msb":
            u = u.reshape(n, words, 64)[:, :, ::-1].reshape(n, -1)
            u = u[:, : u.shape[1] - 1]
        idx = np.full((n, K), NO_IDX, dtype=np.uint32)
        dist = np.full((n, K), NO_DIST, dtype=np.uint16)
        for i in range(n):
            d = (u[i][None, :] != u).sum(axis=1)
            cand = np.arange(n)
            if kind != "self_included":
                cand = cand[cand != i]
            tie = -cand if kind == "ties_to_larger" else cand
            order = np.lexsort((tie, d[cand]))
            if kind == "off_by_one_k":
                order = order[1:]
            order = order[:K]
            idx[i, :order.size] = cand[order]
            dist[i, :order.size] = d[cand[order]]
            if kind == "no_padding" and order.size < K:
                idx[i, order.size:] = 0
        return idx, dist
    return knn


@pytest.mark.parametrize("kind", ["drop_last_word", "ties_to_larger", "self_included",
                                  "off_by_one_k", "no_padding", "bit_order_msb"])
def test_pins_catch_planted_mistakes(kind):
    mutant = _mutant(kind)
    assert not all(pin(mutant) for pin in PINS), f"no pin caught mistake '{kind}'"


def test_unplanted_mutant_passes():
    """The harness itself: the copy without a planted mistake passes every pin."""
    ok = _mutant("none")
    assert all(pin(ok) for pin in PINS)


def test_rect_knn_pins():
    # queries against a separate base (no row left out): pinned to the plain
    # per-bit definition and to the graph's definition on the same codes
    g = np.random.default_rng(41)
    base = datagen.clustered_codes(60, 128, 4, 0.2, seed=41)
    queries = datagen.clustered_codes(9, 128, 4, 0.2, seed=42)
    K = 7
    oi, od = oracle.knn_rect(queries, base, K)
    for q in range(queries.shape[0]):
        # per-bit brute force with a full sort by (distance, index)
        d = [sum(((int(queries[q, w]) ^ int(base[j, w])) >> b) & 1
                 for w in range(2) for b in range(64)) for j in range(base.shape[0])]
        want = sorted(range(base.shape[0]), key=lambda j: (d[j], j))[:K]
        assert list(oi[q]) == want and list(od[q]) == [d[j] for j in want]
    # queries = the base itself: each row finds itself first at distance 0,
    # then exactly the graph's row (distinct codes)
    codes = np.unique(datagen.uniform_codes(80, 64, seed=43), axis=0)
    ri, rd = oracle.knn_rect(codes, codes, K + 1)
    gi, gd = oracle.knn_rows(codes, K)
    assert (ri[:, 0] == np.arange(codes.shape[0])).all() and (rd[:, 0] == 0).all()
    assert np.array_equal(ri[:, 1:], gi) and np.array_equal(rd[:, 1:], gd)
    # fewer base rows than K: padded; an empty base: all padding
    pi, pd = oracle.knn_rect(queries, base[:3], 5)
    assert (pi[:, 3:] == oracle.NO_IDX).all() and (pd[:, 3:] == oracle.NO_DIST).all()
    ei, ed = oracle.knn_rect(queries, base[:0], 4)
    assert (ei == oracle.NO_IDX).all() and (ed == oracle.NO_DIST).all()
