"""Readers for the hand-derived fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def cube3():
    """-> (layouts, expected_idx [8][7], expected_dist [8][7]).

    Each layout is (bits, positions, background)."""
    layouts, rows = [], {}
    for line in _lines("cube3_knn.txt"):
        if line.startswith("layout"):
            kv = dict(tok.split("=") for tok in line.split()[1:])
            layouts.append((int(kv["bits"]), [int(p) for p in kv["positions"].split(",")],
                            int(kv["background"])))
        elif line.startswith("row"):
            head, body = line.split(":", 1)
            idx_s, dist_s = body.split("|")
            rows[int(head.split()[1])] = ([int(t) for t in idx_s.split()],
                                          [int(t) for t in dist_s.split()])
    idx = np.array([rows[r][0] for r in range(8)], dtype=np.uint32)
    dist = np.array([rows[r][1] for r in range(8)], dtype=np.uint16)
    return layouts, idx, dist


def cube3_codes(bits, positions, background):
    """Codes of the 8 vertices in a given layout (written bit by bit)."""
    words = bits // 64
    codes = np.zeros((8, words), dtype=np.uint64)
    for i in range(8):
        for b in range(bits):
            val = background
            if b in positions:
                val = (i >> positions.index(b)) & 1
            if val:
                codes[i, b // 64] |= np.uint64(1) << np.uint64(b % 64)
    return codes


def merge_small():
    """-> (K, in_idx [L][n][K_in], in_dist, out_idx [n][K], out_dist)."""
    ins, outs, K = {}, {}, None
    for line in _lines("merge_small.txt"):
        if line.startswith("K "):
            K = int(line.split()[1])
            continue
        head, body = line.split(":", 1)
        pairs = [tuple(int(v) for v in tok.split(",")) for tok in body.split()]
        parts = head.split()
        if parts[0] == "in":
            ins[(int(parts[1]), int(parts[2]))] = pairs
        else:
            outs[int(parts[1])] = pairs
    n = 1 + max(r for r, _ in ins)
    L = 1 + max(l for _, l in ins)
    kin = len(next(iter(ins.values())))
    in_idx = np.zeros((L, n, kin), dtype=np.uint32)
    in_dist = np.zeros((L, n, kin), dtype=np.uint16)
    for (r, l), pairs in ins.items():
        in_dist[l, r] = [p[0] for p in pairs]
        in_idx[l, r] = [p[1] for p in pairs]
    out_idx = np.array([[p[1] for p in outs[r]] for r in range(n)], dtype=np.uint32)
    out_dist = np.array([[p[0] for p in outs[r]] for r in range(n)], dtype=np.uint16)
    return K, in_idx, in_dist, out_idx, out_dist


def search_small():
    """-> (codes [n][1] uint64, graph [n][K] uint32, feats [n][d] float32,
    entries, cases) from search_small.txt; each case is a dict with P, N,
    exclude (None or a row), expand (rows in order), pool [(ham, idx)],
    visited and answer [(idx, dist)]."""
    nodes, graph, feats, entries, cases = {}, {}, {}, None, {}
    for line in _lines("search_small.txt"):
        line = line.split("#", 1)[0].strip()
        if not line or line.startswith("bits"):
            continue
        head, _, body = line.partition(":")
        parts = head.split()
        if parts[0] == "node":
            nodes[int(parts[1])] = [] if body.strip() == "-" else [int(t) for t in body.split()]
        elif parts[0] == "graph":
            graph[int(parts[1])] = [int(t) for t in body.split()]
        elif parts[0] == "feat":
            feats[int(parts[1])] = [float(t) for t in body.split()]
        elif parts[0] == "entries":
            entries = [int(t) for t in parts[1:]]
        elif parts[0] == "case":
            kv = dict(tok.split("=") for tok in parts[2:])
            cases[parts[1]] = dict(P=int(kv["P"]), N=int(kv["N"]),
                                   exclude=None if kv["exclude"] == "-" else int(kv["exclude"]))
        elif parts[0] == "expand":
            cases[parts[1]]["expand"] = [int(t) for t in body.split()]
        elif parts[0] == "pool":
            cases[parts[1]]["pool"] = [tuple(int(v) for v in t.split(",")) for t in body.split()]
        elif parts[0] == "visited":
            cases[parts[1]]["visited"] = int(body)
        elif parts[0] == "answer":
            cases[parts[1]]["answer"] = [(int(t.split(",")[0]), float(t.split(",")[1]))
                                         for t in body.split()]
    n = len(nodes)
    codes = np.zeros((n, 1), dtype=np.uint64)
    for i, pos in nodes.items():
        for b in pos:
            codes[i, 0] |= np.uint64(1) << np.uint64(b)
    g = np.array([graph[i] for i in range(n)], dtype=np.uint32)
    f = np.array([feats[i] for i in range(n)], dtype=np.float32)
    return codes, g, f, entries, cases
