"""Pins of the online-search oracle (CPU only): with a pool larger than the
data and a connected graph the search visits every row, so its answer is the
exact float kNN (checked against the float64 library route of
``oracle.learned.float_knn``); a pool of one is greedy descent, ending at a
row no neighbour of which is closer; the float32 re-rank distance is the
float64 distance up to rounding; the row excluded never appears. A
hand-derived trace on a 9-row graph with a pool of 3
(``tests/golden/search_small.txt``) fixes the best-first expansion order, the
final pool, the visited count and the re-ranked answer, and planted mistakes
(expanding the worst member, an unbounded pool, ties to the larger index, the
first sampled entry instead of the nearest) each fail it."""
import numpy as np
import pytest

import oracle
from oracle import learned
from paper_2102_04656_amd import datagen
from tests import golden_io


def small_world(n, d, bits, K, seed):
    g = np.random.default_rng(seed)
    feats = g.standard_normal((n, d)).astype(np.float32)
    proj = g.standard_normal((d, bits)).astype(np.float32)
    codes = learned.srp_encode(feats, proj)
    gi, _ = oracle.knn_rows(codes, K)
    gi = gi.copy()
    gi[:, K - 1] = (np.arange(n) + 1) % n  # a ring: every row reachable
    return feats, codes, gi


def test_full_pool_gives_exact_float_knn():
    feats, codes, gi = small_world(300, 16, 64, 8, 1)
    entries = np.arange(0, 300, 37)
    want, _ = learned.float_knn(feats[:12], feats, 10, exclude=np.arange(12))
    for q in range(12):
        idx, dist, nvis = oracle.graph_search(codes, gi, feats, codes[q], feats[q], entries,
                                              P=400, N=10, exclude=q)
        assert nvis == 300
        assert list(idx) == list(want[q])


def test_pool_of_one_is_greedy_descent():
    feats, codes, gi = small_world(400, 16, 128, 10, 2)
    u = datagen.unpack_bits(codes).astype(np.int16)
    for q in range(20):
        idx, _, _ = oracle.graph_search(codes, gi, feats, codes[q], feats[q], [5, 100, 250],
                                        P=1, N=1, exclude=q)
        x = int(idx[0])
        hx = int((u[x] != u[q]).sum())
        for v in gi[x]:
            if int(v) != q:
                assert int((u[int(v)] != u[q]).sum()) >= hx


def test_l2_f32_close_to_float64():
    g = np.random.default_rng(3)
    a, b = g.standard_normal(512), g.standard_normal(512)
    exact = float(((a.astype(np.float32).astype(np.float64) - b.astype(np.float32)) ** 2).sum())
    assert abs(float(oracle.l2_f32(a, b)) - exact) <= 1e-5 * exact


def test_planted_missing_exclusion_caught():
    feats, codes, gi = small_world(200, 16, 64, 8, 4)
    q = 7
    idx, _, _ = oracle.graph_search(codes, gi, feats, codes[q], feats[q], [0, 50], P=300, N=5,
                                    exclude=None)
    # without the exclusion the query's own row (distance 0) comes first,
    # which the exact float kNN with the row excluded does not contain
    want, _ = learned.float_knn(feats[q:q + 1], feats, 5, exclude=np.array([q]))
    assert int(idx[0]) == q and list(idx) != list(want[0])


# ------------------------------------------------ hand-derived trace (Sec. 3.5)


def _fixture_pin(search):
    """Run `search` on both hand-derived cases; return a description of the
    first mismatch with the fixture, or None."""
    codes, gi, feats, entries, cases = golden_io.search_small()
    q_code = np.zeros(1, dtype=np.uint64)
    q_feat = np.zeros(feats.shape[1], dtype=np.float32)
    for name, c in cases.items():
        tr = {}
        idx, dist, nvis = search(codes, gi, feats, q_code, q_feat, entries, P=c["P"], N=c["N"],
                                 exclude=c["exclude"], trace=tr)
        got = dict(expand=tr.get("expand"), pool=[tuple(k) for k in tr.get("pool", [])],
                   visited=nvis, answer=[(int(i), float(d)) for i, d in zip(idx, dist)])
        for key in ("expand", "pool", "visited", "answer"):
            if got[key] != c[key]:
                return f"case {name}: {key} {got[key]} != {c[key]}"
    return None


def test_search_matches_hand_derived_trace():
    assert _fixture_pin(oracle.graph_search) is None


def _planted_search(kind):
    """A copy of the search with one plausible mistake planted (CPU only)."""
    def search(codes, graph_idx, feats, q_code, q_feat, entries, P, N, exclude=None, trace=None):
        n = codes.shape[0]

        def ham(j):
            return sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(q_code, codes[j]))

        visited = set() if exclude is None else {int(exclude)}
        ents = [int(e) for e in entries if int(e) not in visited and int(e) < n]
        if kind == "first_entry":
            best = (ham(ents[0]), ents[0])
        else:
            best = min((ham(e), e) for e in ents)
        visited.add(best[1])
        order = (lambda k: (k[0], -k[1])) if kind == "ties_larger_index" else (lambda k: k)
        pool, expanded = [best], set()
        while True:
            cand = [k for k in pool if k[1] not in expanded]
            if not cand:
                break
            u = (cand[-1] if kind == "expand_worst" else cand[0])[1]
            expanded.add(u)
            trace.setdefault("expand", []).append(u)
            for v in [int(x) for x in graph_idx[u]]:
                if v >= n or v in visited:
                    continue
                visited.add(v)
                pool.append((ham(v), v))
            pool = sorted(pool, key=order)
            if kind != "pool_unbounded":
                pool = pool[:P]
        trace["pool"] = list(pool)
        rr = sorted((oracle.l2_f32(feats[j], q_feat), j) for _, j in pool)[:N]
        idx = np.array([j for _, j in rr], dtype=np.uint32)
        dist = np.array([d for d, _ in rr], dtype=np.float32)
        return idx, dist, len(visited)
    return search


@pytest.mark.parametrize("kind", ["expand_worst", "pool_unbounded", "ties_larger_index",
                                  "first_entry"])
def test_trace_pin_catches_planted_mistakes(kind):
    assert _planted_search("none") is not None
    assert _fixture_pin(_planted_search(kind)) is not None, \
        f"planted mistake {kind} passed the hand-derived trace"


def test_planted_copy_without_mistake_passes():
    # the copy used for planting is itself faithful, so each failure above is
    # the planted mistake's
    assert _fixture_pin(_planted_search("none")) is None
