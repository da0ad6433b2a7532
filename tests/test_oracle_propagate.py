"""Pins of the propagation oracle to things other than itself (CPU only).

``oracle.propagate`` walks the two floors of a row as sets. The pins check it
against: the exact graph being a fixed point (a property of the definition),
an adjacency-matrix formulation (second floor = A @ A, distances by numpy
``unpackbits``), the paper's filter leaving the result unchanged, the K-th
distance never growing, and absent entries being ignored. A plausible
mistake in the walk (dropping the first floor, keeping the row itself, no
dedup, a wrong tie order) fails at least one of them
(``test_pins_catch_planted_mistakes``).
"""
import numpy as np
import pytest

import oracle
from paper_2102_04656_amd import datagen

NO_IDX, NO_DIST = oracle.NO_IDX, oracle.NO_DIST


def np_ham(codes, x, cols):
    u = datagen.unpack_bits(codes).astype(np.int16)
    return (u[x][None, :] != u[cols]).sum(axis=1)


def approx_graph(codes, K, seed, keep=0.5):
    """A valid but inexact input graph: each row keeps a random part of its
    exact list and fills up with random other rows; distances by the oracle,
    rows sorted by (dist, idx)."""
    n = codes.shape[0]
    ei, _ = oracle.knn_rows(codes, K)
    g = np.random.default_rng(seed)
    idx = np.full((n, K), NO_IDX, np.uint32)
    dist = np.full((n, K), NO_DIST, np.uint16)
    for x in range(n):
        kept = [int(j) for j in ei[x] if g.random() < keep]
        pool = [j for j in g.permutation(n)[: 4 * K] if j != x and j not in kept]
        row = (kept + [int(j) for j in pool])[:K]
        d = oracle.pair_distances(codes, np.full(len(row), x), np.array(row))
        order = sorted(zip(d.tolist(), row))
        idx[x, : len(order)] = [j for _, j in order]
        dist[x, : len(order)] = [dd for dd, _ in order]
    return idx, dist


def matrix_route(codes, in_idx, K):
    """Second floor by the boolean adjacency matrix: M = A | (A @ A), no
    diagonal; row x keeps the K smallest (ham, j) over M[x]."""
    n = codes.shape[0]
    A = np.zeros((n, n), dtype=np.int64)
    for x in range(n):
        for j in in_idx[x]:
            if int(j) != NO_IDX and int(j) < n:
                A[x, int(j)] = 1
    M = (A + A @ A) > 0
    np.fill_diagonal(M, False)
    out_i = np.full((n, K), NO_IDX, np.uint32)
    out_d = np.full((n, K), NO_DIST, np.uint16)
    for x in range(n):
        cols = np.nonzero(M[x])[0]
        d = np_ham(codes, x, cols)
        order = np.lexsort((cols, d))[:K]
        out_i[x, : order.size] = cols[order]
        out_d[x, : order.size] = d[order]
    return out_i, out_d


# ----------------------------------------------------------------- pins

def pin_fixed_point(prop):
    for n, bits, K, seed in ((300, 128, 8, 1), (240, 64, 16, 2)):
        codes = datagen.clustered_codes(n, bits, 8, 0.15, seed)
        ei, ed = oracle.knn_rows(codes, K)
        pi, pd = prop(codes, ei, K)
        if not (np.array_equal(pi, ei) and np.array_equal(pd, ed)):
            return f"exact graph not a fixed point (n={n}, K={K})"
    return None


def pin_matrix_route(prop):
    for n, bits, K, seed in ((160, 128, 6, 3), (120, 192, 10, 4)):
        codes = datagen.clustered_codes(n, bits, 6, 0.2, seed)
        gi, _ = approx_graph(codes, K, seed)
        pi, pd = prop(codes, gi, K)
        mi, md = matrix_route(codes, gi, K)
        if not (np.array_equal(pi, mi) and np.array_equal(pd, md)):
            return f"differs from the adjacency-matrix route (n={n}, K={K})"
    return None


def pin_kth_never_grows(prop):
    codes = datagen.clustered_codes(200, 128, 6, 0.2, 5)
    K = 8
    gi, gd = approx_graph(codes, K, 5, keep=0.3)
    pi, pd = prop(codes, gi, K)
    for x in range(codes.shape[0]):
        if pd[x, K - 1] > gd[x, K - 1]:
            return f"row {x}: K-th distance grew"
        row = [(int(d), int(j)) for d, j in zip(pd[x], pi[x]) if int(j) != NO_IDX]
        if row != sorted(set(row)) or any(j == x for _, j in row):
            return f"row {x}: not ascending, distinct and self-free"
    return None


def pin_absent_entries(prop):
    codes = datagen.clustered_codes(120, 64, 5, 0.2, 6)
    K = 6
    gi, _ = approx_graph(codes, K, 6)
    holed = gi.copy()
    holed[::3, K - 2:] = NO_IDX
    holed[1::5, 0] = codes.shape[0] + 7  # out of range: absent
    pi, pd = prop(codes, holed, K)
    mi, md = matrix_route(codes, holed, K)
    if not (np.array_equal(pi, mi) and np.array_equal(pd, md)):
        return "sentinel or out-of-range entries not ignored"
    return None


PINS = (pin_fixed_point, pin_matrix_route, pin_kth_never_grows, pin_absent_entries)


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_oracle_propagate_pins(pin):
    assert pin(oracle.propagate) is None


def test_filter_is_lossless():
    for n, K, seed, keep in ((200, 8, 7, 0.5), (160, 12, 8, 0.2), (150, 8, 9, 1.0)):
        codes = datagen.clustered_codes(n, 128, 6, 0.2, seed)
        gi, _ = approx_graph(codes, K, seed, keep=keep)
        a = oracle.propagate(codes, gi, K)
        b = oracle.propagate_filtered(codes, gi, K)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_propagation_raises_recall():
    codes = datagen.clustered_codes(300, 128, 8, 0.2, 10)
    K = 8
    ei, _ = oracle.knn_rows(codes, K)
    gi, _ = approx_graph(codes, K, 10, keep=0.3)
    pi, _ = oracle.propagate(codes, gi, K)

    def recall(g):
        return np.mean([len(set(g[x]) & set(ei[x])) / K for x in range(codes.shape[0])])

    assert recall(pi) > recall(gi) + 0.2


# --------------------------------------------------- planted mistakes

def _mistake(kind):
    def prop(codes, in_idx, K):
        codes = np.ascontiguousarray(codes, dtype=np.uint64)
        n = codes.shape[0]
        out_i = np.full((n, K), NO_IDX, np.uint32)
        out_d = np.full((n, K), NO_DIST, np.uint16)
        for x in range(n):
            first = [int(j) for j in in_idx[x] if int(j) != NO_IDX and int(j) < n]
            second = [int(z) for y in first for z in in_idx[y] if int(z) != NO_IDX and int(z) < n]
            if kind == "no_first_floor":
                cand = list(set(second) - {x})
            elif kind == "keeps_self":
                cand = list(set(first) | set(second))
            elif kind == "no_dedup":
                cand = [j for j in first + second if j != x]
            else:
                cand = list((set(first) | set(second)) - {x})
            d = oracle.pair_distances(codes, np.full(len(cand), x), np.array(cand, dtype=np.uint32))
            pairs = list(zip(d.tolist(), cand))
            key = (lambda p: (p[0], -p[1])) if kind == "tie_larger_index" else (lambda p: p)
            for k, (dd, j) in enumerate(sorted(pairs, key=key)[:K]):
                out_i[x, k] = j
                out_d[x, k] = dd
        return out_i, out_d
    return prop


@pytest.mark.parametrize("kind", ["no_first_floor", "keeps_self", "no_dedup", "tie_larger_index"])
def test_pins_catch_planted_mistakes(kind):
    prop = _mistake(kind)
    failures = [p.__name__ for p in PINS if p(prop) is not None]
    assert failures, f"planted mistake {kind} passed every pin"
