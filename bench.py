#!/usr/bin/env python3
"""Benchmark of the exact Hamming kNN-graph build on one MI355X.

One step = one ``bdg_build_knn_ex`` call over the whole workload: operand
prep, every (row tile x column block) distance tile with its fused top-K, the
running merge of the per-column-block lists, and the output rows. Codes are
resident in HBM before the timed region starts.

Default workload: one GPU's partition at production shape -- 4,000,000 codes
of 512 bits from 20,000 random centres with bit-flip probability 0.25, exact
K = 100 graph (row blocks of 250,000, column blocks of 262,144). The vector-ALU
path is timed beside it (one step by default), and the 1,000,000 x 256-bit,
K = 64 workload is timed as a secondary object.

Prints ONE JSON line on stdout. ``value`` = n (n - 1) / seconds per step
(pair distances per second). ``roofline`` is for the dominant kernel (the
distance tile), timed live with HIP events recorded around every tile launch on
the launch stream. ``stall`` is the persistent launch's stall flag after the
timed builds (``bdg_build_knn_check``; 0 in a correct run). ``cpu_baseline``
times the CPU oracle on a bounded seeded row sample of the same workload, on
all host threads and on one.

    python bench.py [--steps 5] [--warmup 2] [--path auto|mfma|popc]
                    [--workload NAME] [--secondary NAME|none]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_INT8_TOPS = 5000.0           # dense int8 matrix, TOP/s
PEAK_FP32_MFMA_TFLOPS = 157.3     # dense FP32 matrix, TFLOP/s
CU, LANES, CLOCK = 256, 64, 2.4e9
PEAK_VALU_TOPS = CU * LANES * CLOCK / 1e12  # 32-bit integer vector ops, TOP/s (derived)
METRIC = "Hamming kNN-graph build pair-dist/s + % peak; recall@K learned vs plain codes"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources that define each timed kernel: a recorded HBM-traffic figure is
# reported only while they are unchanged since the counters were taken.
KERNEL_SOURCES = {
    "knn_mfma_sweep_kernel": ["tile_mfma_kern.h", "wave_topk.h", "tile_mfma.hip", "kernels.h"],
    "knn_mfma_batched_kernel": ["tile_mfma_kern.h", "wave_topk.h", "tile_mfma.hip", "kernels.h"],
    "knn_popc_kernel": ["knn_tiles.hip", "wave_topk.h", "kernels.h"],
    "propagate_kernel": ["propagate.hip", "wave_topk64.h", "kernels.h"],
}
CALIB_BYTES = 256 << 20


def kernel_source_hash(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2102_04656_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary
    of this kernel and workload (scaled by the copy-kernel calibration), or
    None if there is none or the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic__{kernel}__{workload}.md")
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic-record: "):
                rec = json.loads(line[len("traffic-record: "):])
    if not rec or rec.get("source_sha256_16") != kernel_source_hash(kernel):
        return None
    return rec


def copy_calibration():
    """A plain streaming kernel of known size for counter calibration:
    CALIB_BYTES read and CALIB_BYTES written (run outside the timed region)."""
    import torch
    src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


class HipEvents:
    """hipEvent_t handles created through the HIP runtime's C API."""

    def __init__(self, count: int):
        self.rt = ctypes.CDLL("libamdhip64.so")
        self.rt.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.rt.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                ctypes.c_void_p]
        self.rt.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.handles = (ctypes.c_void_p * count)()
        for i in range(count):
            h = ctypes.c_void_p()
            if self.rt.hipEventCreate(ctypes.byref(h)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.handles[i] = h.value

    def slice_ptr(self, start: int) -> int:
        return ctypes.addressof(self.handles) + start * ctypes.sizeof(ctypes.c_void_p)

    def elapsed_ms(self, a: int, b: int) -> float:
        ms = ctypes.c_float()
        if self.rt.hipEventElapsedTime(ctypes.byref(ms), self.handles[a], self.handles[b]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def close(self):
        for h in self.handles:
            self.rt.hipEventDestroy(h)


def run_path(codes_dev, n, bits, K, path, row_block, col_block, steps, warmup, schedule=0,
             bound_group=0):
    """Time `steps` full builds; returns (ms/step, tile kernel stats, outputs).

    The distance-tile launches of one build are, in order: one per row block
    (popc: all columns, per-block lists merged afterwards) or a single
    persistent launch (mfma: (row tile, column block) items, lists carried
    across column blocks)."""
    import torch
    from paper_2102_04656_amd import bdg

    nrb = (n + row_block - 1) // row_block
    if path == bdg.PATH_MFMA:
        shapes = [(n, n)]  # one persistent launch over all (row tile, column block) items
    else:
        shapes = [(min(row_block, n - r * row_block), n) for r in range(nrb)]
    nl = len(shapes)
    idx = torch.empty((n, K), dtype=torch.int32, device="cuda")
    dist = torch.empty((n, K), dtype=torch.int16, device="cuda")
    stream = torch.cuda.current_stream()
    ev = HipEvents(2 * nl * steps)
    # workspace allocated once, outside the timed region
    o = bdg.make_opts(path=path, row_block=row_block, col_block=col_block, tile_schedule=schedule,
                      bound_group=bound_group)
    ws_bytes = bdg.bdg_build_knn_workspace_size(n, bits, K, o)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device="cuda")

    def step(s):
        op = bdg.make_opts(path=path, row_block=row_block, col_block=col_block,
                           tile_schedule=schedule, bound_group=bound_group,
                           workspace=ws.data_ptr(), workspace_bytes=ws_bytes)
        if s is not None:
            op.n_tile_events = 2 * nl
            op.tile_events = ev.slice_ptr(2 * nl * s)
        st = bdg.bdg_build_knn_ex(codes_dev, n, bits, K, idx, dist, op, stream)
        if st != 0:
            raise RuntimeError(f"bdg_build_knn_ex failed: {st} {bdg.last_error()}")

    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        step(s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / steps
    # outcome of the last build on this workspace: the persistent launch's
    # stall flag (never set in a correct run)
    chk = bdg.make_opts(path=path, row_block=row_block, col_block=col_block,
                        tile_schedule=schedule, bound_group=bound_group,
                        workspace=ws.data_ptr(), workspace_bytes=ws_bytes)
    stall = bdg.bdg_build_knn_check(n, bits, K, chk, stream)
    if stall != 0:
        raise RuntimeError(f"bdg_build_knn_check: {stall} {bdg.last_error()}")
    durs, pairs = [], []
    for s in range(steps):
        for i, (rows, cols) in enumerate(shapes):
            e = 2 * nl * s + 2 * i
            durs.append(ev.elapsed_ms(e, e + 1))
            pairs.append(rows * cols)
    ev.close()
    # pairs per launch x launches / total kernel time = pairs / (average duration)
    return ms_step, dict(launches=len(durs), avg_ms=float(np.mean(durs)),
                         pairs_per_launch=float(np.mean(pairs)),
                         total_ms=float(np.sum(durs)), stall=stall), (idx, dist)


def cpu_baseline(codes, K, gpu_out, target_s):
    """Time the CPU oracle on a bounded seeded row sample of the workload."""
    import oracle
    from paper_2102_04656_amd import bdg
    n = codes.shape[0]
    g = np.random.default_rng(2021)
    calib = max(32, 2 * oracle.threads())
    rows = np.sort(g.choice(n, size=calib, replace=False)).astype(np.uint32)
    t0 = time.perf_counter()
    oracle.knn_rows(codes, K, rows=rows)
    t_cal = time.perf_counter() - t0
    R = int(min(n, max(calib, calib * target_s / max(t_cal, 1e-3))))
    rows = np.sort(g.choice(n, size=R, replace=False)).astype(np.uint32)
    t0 = time.perf_counter()
    oi, od = oracle.knn_rows(codes, K, rows=rows)
    t = time.perf_counter() - t0
    gi, gd = bdg.to_numpy_graph(*gpu_out)
    parity = bool(np.array_equal(gi[rows], oi) and np.array_equal(gd[rows], od))
    cores = oracle.threads()
    # the same oracle on one thread, on a share of the sample sized for about
    # a third of the time budget
    r1 = int(max(4, min(R, R * (target_s / 3) / max(t, 1e-3) / max(cores, 1))))
    rows1 = rows[:r1]
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        o1i, o1d = oracle.knn_rows(codes, K, rows=rows1)
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    parity = parity and bool(np.array_equal(o1i, oi[:r1]) and np.array_equal(o1d, od[:r1]))
    return dict(value=R * (n - 1) / t, unit="pair-dist/s", cores=cores,
                kind="oracle", seconds=t,
                sample=f"{R} seeded rows x all {n} columns of the same workload "
                       f"(exact K={K} rows by the C oracle)",
                parity_on_sample=parity,
                single_thread={"value": r1 * (n - 1) / t1, "seconds": t1,
                               "sample": f"the first {r1} rows of the same sample"},
                host={"cpu_model": cpu_model(), "affinity_cores": len(os.sched_getaffinity(0)),
                      "oracle_build": "gcc -O2 -mpopcnt -fopenmp (portable x86-64 flags)"})


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def recall_leg():
    """Learned vs sign-of-random-projection codes at equal length on the 1M x 512
    Gaussian mixture: recall@64 (Eq. 3) of the exact Hamming graph of each
    code set against exact float kNN over 10k sampled rows. Not timed as
    part of the build; the encode and graph times are reported beside it."""
    from paper_2102_04656_amd import datagen, learned_codes
    w = datagen.WORKLOADS["gmm-1m-512d"]
    log("[bench] recall leg: training the encoder on gmm-1m-512d")
    res, _ = learned_codes.experiment(
        n=w["n"], d=w["d"], n_comp=w["n_comp"], centre_std=w["centre_std"], seed=w["seed"],
        proj_seed=w["proj_seed"], bits=w["code_bits"], K_train=w["K_train"],
        K_eval=w["K_eval"], train_rows=w["train_rows"], eval_queries=w["eval_queries"])
    K = w["K_eval"]
    return {"workload": "gmm-1m-512d", "K": K, "bits": w["code_bits"],
            "learned": res["recall_learned"], "srp": res["recall_srp"],
            "gain": res["recall_learned"] - res["recall_srp"],
            "train_steps": res["steps"], "train_seconds": res["train_seconds"],
            "encode_ms_learned": res["encode_seconds_learned"] * 1e3,
            "encode_ms_srp": res["encode_seconds_srp"] * 1e3,
            "graph_ms_learned": res["graph_seconds_learned"] * 1e3,
            "graph_ms_srp": res["graph_seconds_srp"] * 1e3,
            "float_knn": {k: dict(v, kernel="fknn_mfma_kernel (+ norms, split merge)",
                                  roofline={"bound": "mfma", "achieved": v["tflops"],
                                            "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                                            "frac": v["tflops"] / PEAK_FP32_MFMA_TFLOPS})
                          for k, v in res["float_knn"].items()},
            "search_recall_at_60": {"srp": res["search_srp"], "learned": res["search_learned"]}}


def propagation_leg(codes, codes_dev, exact, bits, K, with_oracle, workload, steps=3):
    """One round of neighbourhood propagation (Sec. 3.3) on the workload's
    codes, from an inexact graph: the exact graph with half of every row's
    entries replaced by seeded random rows. Reports the kernel time (HIP
    events on the launch stream), recall@K of the input and of the output
    against the exact graph, the bytes the kernel moves through HBM (from the
    committed FETCH_SIZE / WRITE_SIZE record of this kernel and workload, if
    its sources are unchanged) against the HBM peak with the algorithmic
    gather bytes beside them, and the oracle on a seeded row sample (parity
    and rate). The kernel is latency-bound (random gathers of lists and
    codes, most served from L2 and the Infinity Cache)."""
    import torch
    from paper_2102_04656_amd import bdg
    n = exact.shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(2102)
    repl = torch.rand((n, K), generator=g, device="cuda") < 0.5
    rnd = torch.randint(0, n, (n, K), generator=g, device="cuda", dtype=torch.int32)
    in_idx = torch.where(repl, rnd, exact).contiguous()
    out = bdg.propagate(codes_dev, in_idx, bits=bits)  # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out = bdg.propagate(codes_dev, in_idx, bits=bits)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.mean(times))

    def recall(gr):
        return graph_recall(gr, exact)

    words = bits // 64
    cand = K + K * K  # first and second floor per row
    row_bytes = 4 * K + K * 4 * K + cand * 8 * words + 6 * K
    achieved = n * row_bytes / (ms * 1e-3) / 1e9
    res = {"workload": "exact graph with half of each row replaced by random rows (seed 2102)",
           "n": n, "K": K, "bits": bits, "ms": ms, "kernel": "propagate_kernel",
           "candidates_per_s": n * cand / (ms * 1e-3),
           "recall_in": recall(in_idx), "recall_out": recall(out[0]),
           "roofline": {"bound": "latency", "achieved": None, "peak": 8000.0, "unit": "GB/s",
                        "frac": None, "traffic": None,
                        "algorithmic_bytes_per_row": row_bytes,
                        "algorithmic_gb_per_s": achieved,
                        "note": "random gathers of lists and codes; the per-wave hash set "
                                "gathers each distinct candidate once and most reads hit "
                                "L2/MALL, so HBM is far from the bound"}}
    rec = recorded_traffic("propagate_kernel", workload)
    if rec is not None:
        hbm = rec["bytes_per_launch"] / (ms * 1e-3) / 1e9
        res["roofline"].update(achieved=hbm, frac=hbm / 8000.0, traffic=rec["bytes_per_launch"],
                               traffic_source=f"profiles/traffic__propagate_kernel__{workload}.md")
    if with_oracle:
        import oracle
        rows = np.sort(np.random.default_rng(2102).choice(n, size=256, replace=False))
        gin = in_idx.cpu().numpy().view(np.uint32)
        t0 = time.perf_counter()
        oi, od = oracle.propagate(codes, gin, K, rows=rows)
        t = time.perf_counter() - t0
        gi, gd = bdg.to_numpy_graph(*out)
        res["cpu_baseline"] = {"value": rows.size * cand / t, "unit": "candidates/s",
                               "cores": 1, "kind": "oracle", "seconds": t,
                               "sample": f"{rows.size} seeded rows of the same input graph"}
        res["parity_on_sample"] = bool(np.array_equal(gi[rows], oi) and np.array_equal(gd[rows], od))
    return res


def graph_recall(graph, exact):
    """Mean over rows of |graph row ∩ exact row| / K (GPU tensors, chunked)."""
    n, K = exact.shape
    hits = 0
    for r0 in range(0, n, 65536):
        a = graph[r0:r0 + 65536].long()
        b = exact[r0:r0 + 65536].long()
        hits += int((a[:, :, None] == b[:, None, :]).any(dim=2).sum().item())
    return hits / (n * K)


def dac_leg(codes_dev, exact, bits, K, m=1024, iters=8, T=16, coarse_num=8192):
    """The paper's construction pipeline on the workload's codes (Sec. 3.2 then
    3.3): binary k-means centres on a 10 % seeded sample, the approximate graph
    of the single-pass divide-and-conquer, then one round of neighbourhood
    propagation; recall@K of each graph against the exact one and the time of
    each step. Parity of these steps with the oracle is covered by the tests
    (the oracle's nearest-centre step over all rows is too slow here)."""
    import torch
    from paper_2102_04656_amd import bdg
    n = exact.shape[0]
    g = np.random.default_rng(2103)
    sample = np.sort(g.choice(n, size=n // 10, replace=False)).astype(np.uint32)
    init = sample[np.sort(g.choice(sample.size, size=m, replace=False))]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    C = bdg.bkmeans(codes_dev, sample, init, iters, bits=bits)
    torch.cuda.synchronize()
    t_bk = (time.perf_counter() - t0) * 1e3
    gi, _ = bdg.build_knn_dac(codes_dev, C, K, T, coarse_num, bits=bits)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    gi, gd = bdg.build_knn_dac(codes_dev, C, K, T, coarse_num, bits=bits)
    e1.record()
    torch.cuda.synchronize()
    t_dac = e0.elapsed_time(e1)
    e0.record()
    pi, pd = bdg.propagate(codes_dev, gi, bits=bits)
    e1.record()
    torch.cuda.synchronize()
    t_prop = e0.elapsed_time(e1)
    res = {"centres": m, "sample_rows": int(sample.size), "kmeans_iters": iters, "T": T,
           "coarse_num": coarse_num, "K": K,
           "kmeans_ms": t_bk, "dac_ms": t_dac, "propagate_ms": t_prop,
           "recall_dac": graph_recall(gi, exact), "recall_dac_propagated": graph_recall(pi, exact),
           "parity": "tests/test_gpu_dac.py and tests/test_gpu_propagate.py (oracle, n <= 20k)"}
    sweep = []
    for cn in (coarse_num // 16, coarse_num // 8, coarse_num // 4, coarse_num // 2):
        # the candidate budget against recall (Sec. 4.5)
        e0.record()
        gi, _ = bdg.build_knn_dac(codes_dev, C, K, T, cn, bits=bits)
        e1.record()
        torch.cuda.synchronize()
        td = e0.elapsed_time(e1)
        e0.record()
        pi, _ = bdg.propagate(codes_dev, gi, bits=bits)
        e1.record()
        torch.cuda.synchronize()
        sweep.append({"coarse_num": cn, "dac_ms": td, "recall_dac": graph_recall(gi, exact),
                      "propagate_ms": e0.elapsed_time(e1), "recall_propagated": graph_recall(pi, exact)})
    res["coarse_num_sweep"] = sweep
    return res


def batched_popc_leg(d, offsets, sizes, bits, K, pairs, out, stream):
    """The vector-ALU path on the same shards: one bdg_build_knn_ex per shard
    (shard-local indices by construction), one untimed and one timed pass;
    its graph is compared with the batched launch's on every row."""
    import torch
    from paper_2102_04656_amd import bdg
    pi, pd = torch.empty_like(out[0]), torch.empty_like(out[1])
    nmax = int(sizes.max())
    ws_bytes = bdg.bdg_build_knn_workspace_size(nmax, bits, K, bdg.make_opts(path=bdg.PATH_POPC))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device="cuda")
    o = bdg.make_opts(path=bdg.PATH_POPC, workspace=ws.data_ptr(), workspace_bytes=ws_bytes)

    def one_pass():
        for s in range(len(sizes)):
            lo, hi = int(offsets[s]), int(offsets[s + 1])
            if hi > lo:
                st = bdg.bdg_build_knn_ex(d[lo:hi], hi - lo, bits, K, pi[lo:hi], pd[lo:hi], o,
                                          stream)
                if st != 0:
                    raise RuntimeError(f"shard {s}: bdg_build_knn_ex failed: {st} "
                                       f"{bdg.last_error()}")

    log("[bench] vector-ALU path, one build per shard")
    one_pass()
    stream.synchronize()
    t0 = time.perf_counter()
    one_pass()
    stream.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    same = bool(torch.equal(pi, out[0]) and torch.equal(pd, out[1]))
    ops = pairs * 2 * bits // 32
    log(f"[bench] vector-ALU path: {ms:.1f} ms, graph identical to the batched launch: {same}")
    peak = MEASURED_PEAKS.get("valu_int32", PEAK_VALU_TOPS)
    return {"value": pairs / (ms * 1e-3), "ms_per_step": ms, "steps": 1,
            "kernel": "knn_popc_kernel + merge_lists_kernel, one bdg_build_knn_ex per shard",
            "achieved": ops / (ms * 1e-3) / 1e12, "peak": peak, "unit": "T ops/s",
            "frac": ops / (ms * 1e-3) / 1e12 / peak, "peak_derived": PEAK_VALU_TOPS,
            "timing": "end to end, host clock", "identical_to_batched_graph": same}


def bench_batched(args, w):
    """Many shards in one persistent launch, replayed as a HIP graph (schedule
    autotuned once, outside the timed region)."""
    import torch
    from paper_2102_04656_amd import bdg, datagen
    log(f"[bench] generating {args.workload}")
    t0 = time.perf_counter()
    codes, offsets = datagen.sharded_codes(n_shards=w["n_shards"], lo=w["lo"], hi=w["hi"],
                                           c_lo=w["c_lo"], c_hi=w["c_hi"], bits=w["bits"],
                                           p=w["p"], seed=w["seed"])
    bits, K = w["bits"], w["K"]
    peaks = measure_peaks()
    sizes = np.diff(offsets.astype(np.int64))
    pairs = int((sizes * (sizes - 1)).sum())
    log(f"[bench] generated {int(offsets[-1])} rows in {time.perf_counter() - t0:.1f}s; "
        f"{pairs:.4g} pairs")
    d = torch.from_numpy(codes.view(np.int64)).cuda()
    plan = bdg.BatchPlan(offsets, bits, K, bound_group=args.bound_group, schedule=args.schedule)
    out = plan.outputs()
    stream = torch.cuda.Stream()
    report = None
    if args.tune_batched:
        with torch.cuda.stream(stream):
            report = plan.autotune(d, out=out, stream=stream)
        stream.synchronize()
        log(f"[bench] autotune: {report}")
    ev = HipEvents(2 * args.steps)
    rt = ev.rt
    rt.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    sptr = stream.cuda_stream
    for _ in range(args.warmup):
        plan.build(d, out=out, stream=stream, graph=True)
    stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        rt.hipEventRecord(ev.handles[2 * s], sptr)
        plan.build(d, out=out, stream=stream, graph=True)
        rt.hipEventRecord(ev.handles[2 * s + 1], sptr)
    stream.synchronize()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    launch_ms = float(np.mean([ev.elapsed_ms(2 * s, 2 * s + 1) for s in range(args.steps)]))
    ev.close()
    # the persistent kernel alone (events around it, eager enqueues of the same
    # plan), apart from the operand prep and the admission bounds of a replay
    kev = HipEvents(2 * args.steps)
    for s in range(args.steps):
        plan.set_timing(kev.handles[2 * s], kev.handles[2 * s + 1])
        plan.build(d, out=out, stream=stream)
    stream.synchronize()
    plan.set_timing(None, None)
    kernel_ms = float(np.mean([kev.elapsed_ms(2 * s, 2 * s + 1) for s in range(args.steps)]))
    kev.close()
    info = plan.info()
    achieved = pairs * 2 * bits / (kernel_ms * 1e-3) / 1e12
    result = {
        "metric": METRIC, "value": pairs / (ms * 1e-3), "unit": "pair-dist/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i8", "data": "synthetic",
        "config": {"workload": args.workload, "shards": int(w["n_shards"]),
                   "rows": int(offsets[-1]), "bits": bits, "K": K, "pairs": pairs,
                   "work_items": info.work_items, "workgroups": info.workgroups,
                   "order": "longest-first" if info.order == 0 else "shard",
                   "schedule": info.schedule, "bound_group": info.bound_group,
                   "launch": "hip-graph (operand prep, admission bounds, persistent kernel); "
                             "kernel_avg_ms times the persistent kernel alone in eager builds, "
                             "replay_avg_ms the whole replay"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_INT8_TOPS,
                     "unit": "TOP/s", "frac": achieved / PEAK_INT8_TOPS, "traffic": None,
                     "kernel": "knn_mfma_batched_kernel", "kernel_avg_ms": kernel_ms,
                     "replay_avg_ms": launch_ms,
                     "frac_replay": pairs * 2 * bits / (launch_ms * 1e-3) / 1e12 / PEAK_INT8_TOPS,
                     "ops_per_pair": 2 * bits, "pairs_per_launch": pairs,
                     "sustained_probe": peaks["mfma_int8"]},
        "measured_peaks_tops": peaks,
    }
    if report:
        result["autotune"] = json.loads(report)
    rec = recorded_traffic("knn_mfma_batched_kernel", args.workload)
    if rec is not None:
        result["roofline"]["traffic"] = rec["bytes_per_launch"]
        result["roofline"]["traffic_source"] = (
            f"profiles/traffic__knn_mfma_batched_kernel__{args.workload}.md (FETCH_SIZE + "
            f"WRITE_SIZE per launch, copy-calibrated)")
    if args.other_path:
        result["popc_path"] = batched_popc_leg(d, offsets, sizes, bits, K, pairs, out, stream)
    if args.copy_calibration:
        copy_calibration()
    if not args.no_cpu_baseline:
        import oracle
        g = np.random.default_rng(2021)
        gi, gd = bdg.to_numpy_graph(*out)
        done_pairs, t_cpu, ok, nrows = 0, 0.0, True, 0
        order = g.permutation(len(sizes))
        for s in order:
            lo, hi = int(offsets[s]), int(offsets[s + 1])
            rows = np.sort(g.choice(hi - lo, size=min(hi - lo, 64), replace=False))
            t0 = time.perf_counter()
            oi, od = oracle.knn_rows(codes[lo:hi], K, rows=rows.astype(np.uint32))
            t_cpu += time.perf_counter() - t0
            ok &= bool(np.array_equal(gi[lo + rows], oi) and np.array_equal(gd[lo + rows], od))
            done_pairs += rows.size * (hi - lo - 1)
            nrows += rows.size
            if t_cpu > args.cpu_seconds:
                break
        result["cpu_baseline"] = {
            "value": done_pairs / t_cpu, "unit": "pair-dist/s", "cores": oracle.threads(),
            "kind": "oracle", "seconds": t_cpu,
            "sample": f"{nrows} seeded rows (up to 64 per shard, shards in seeded order) "
                      f"against their whole shards", "parity_on_sample": ok}
    print(json.dumps(result), flush=True)
    plan.close()


MEASURED_PEAKS = {}  # filled by main(): sustained rates from bdg_probe_peak, T ops/s


def measure_peaks():
    """Sustained rates of the two units (bdg_probe_peak), T ops/s: 32-bit
    integer vector instructions and int8 matrix-core operations on the tile's
    operand bytes."""
    from paper_2102_04656_amd import bdg
    MEASURED_PEAKS["valu_int32"] = bdg.probe_peak(bdg.PEAK_VALU_INT32) / 1e12
    MEASURED_PEAKS["mfma_int8"] = bdg.probe_peak(bdg.PEAK_MFMA_INT8) / 1e12
    log(f"[bench] measured peaks (T ops/s): {MEASURED_PEAKS}")
    return dict(MEASURED_PEAKS)


def resolved_schedule(schedule, bits, K):
    """The BDG_SCHEDULE_* value a build runs under: DEFAULT resolves to the
    global-lists schedule where the library builds it, else the LDS lists."""
    from paper_2102_04656_amd import bdg
    if schedule != bdg.SCHEDULE_DEFAULT:
        return schedule
    try:
        bdg.bdg_build_knn_workspace_size(1000, bits, K, bdg.make_opts(
            path=bdg.PATH_MFMA, tile_schedule=bdg.SCHEDULE_GLOBAL_LISTS))
        return bdg.SCHEDULE_GLOBAL_LISTS
    except bdg.BdgError:
        return bdg.SCHEDULE_LDS_LISTS


def time_build(w, workload, path, steps, warmup, other_steps, other_warmup, other_path,
               autotune=False, bound_group=0, schedule=0):
    """Generate one single-partition workload, time its build on `path` (and
    the other distance path for `other_steps`), return (codes, codes_dev,
    outputs of the main path, result fields). With `autotune` the schedule
    (path, column block, tile schedule) is first tuned by bdg_autotune_build,
    outside the timed region, and the timed builds take the winner."""
    import torch
    from paper_2102_04656_amd import bdg, datagen
    n, bits, K = w["n"], w["bits"], w["K"]
    row_block, col_block = w.get("row_block", 131072), w.get("col_block", 131072)
    log(f"[bench] generating {workload}: n={n} bits={bits} K={K}")
    t0 = time.perf_counter()
    codes = datagen.clustered_codes(n, bits, w["n_centres"], w["p"], w["seed"])
    log(f"[bench] generated in {time.perf_counter() - t0:.1f}s")
    codes_dev = torch.from_numpy(codes.view(np.int64)).cuda()
    torch.cuda.synchronize()

    paths = {"mfma": bdg.PATH_MFMA, "popc": bdg.PATH_POPC}
    tuned = None
    if autotune:
        log(f"[bench] {workload}: autotuning the build schedule")
        os.environ.setdefault("BDG_AUTOTUNE_LOG", "1")  # one stderr line per candidate
        t0 = time.perf_counter()
        o, rep = bdg.autotune_build(codes_dev, K, bits=bits, row_block=row_block)
        torch.cuda.synchronize()
        tuned = json.loads(rep)
        tuned["tuning_s"] = time.perf_counter() - t0
        log(f"[bench] autotune ({tuned['tuning_s']:.1f} s): {rep}")
        path = {bdg.PATH_MFMA: "mfma", bdg.PATH_POPC: "popc"}[o.path]
        col_block, schedule, bound_group = o.col_block, o.tile_schedule, o.bound_group
    runs, outs = {}, None
    order = [path] + ([p for p in paths if p != path] if other_path else [])
    for name in order:
        st, wu = (steps, warmup) if name == path else (other_steps, other_warmup)
        log(f"[bench] {workload}: timing path {name}: {st} steps after {wu} warmup")
        ms, kern, out = run_path(codes_dev, n, bits, K, paths[name], row_block, col_block, st, wu,
                                 schedule if name == path else 0,
                                 bound_group if name == path else 0)
        runs[name] = dict(ms_per_step=ms, kernel=kern, steps=st)
        if name == path:
            outs = out
        else:
            del out
        log(f"[bench] {name}: {ms:.2f} ms/step; tile kernel avg {kern['avg_ms']:.3f} ms "
            f"x {kern['launches'] // st} launches/step")

    pairs = n * (n - 1)

    def roof(name):
        kern = runs[name]["kernel"]
        if name == "mfma":
            ops_pair, peak, bound, kname = 2 * bits, PEAK_INT8_TOPS, "mfma", "knn_mfma_sweep_kernel"
        else:
            # the vector-ALU peak is the measured one (bdg_probe_peak); the
            # derivation from unit counts and clock is reported beside it
            ops_pair, bound, kname = 2 * bits // 32, "alu", "knn_popc_kernel"
            peak = MEASURED_PEAKS.get("valu_int32", PEAK_VALU_TOPS)
        achieved = kern["pairs_per_launch"] * ops_pair / (kern["avg_ms"] * 1e-3) / 1e12
        r = {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TOP/s",
             "frac": achieved / peak, "traffic": None, "kernel": kname,
             "kernel_avg_ms": kern["avg_ms"], "ops_per_pair": ops_pair,
             "pairs_per_launch": kern["pairs_per_launch"]}
        if name == "mfma" and "mfma_int8" in MEASURED_PEAKS:
            r["sustained_probe"] = MEASURED_PEAKS["mfma_int8"]
            r["frac_of_probe"] = achieved / MEASURED_PEAKS["mfma_int8"]
        if name != "mfma":
            r["peak_source"] = "measured (bdg_probe_peak, XOR + popcount-accumulate + add)"
            r["peak_derived"] = PEAK_VALU_TOPS
        rec = recorded_traffic(kname, workload)
        if rec is not None:
            r["traffic"] = rec["bytes_per_launch"]
            r["traffic_source"] = (f"profiles/traffic__{kname}__{workload}.md (FETCH_SIZE + "
                                   f"WRITE_SIZE per launch, copy-calibrated)")
        return r

    res = {"value": pairs / (runs[path]["ms_per_step"] * 1e-3),
           "ms_per_step": runs[path]["ms_per_step"],
           "dtype": "i8" if path == "mfma" else "u32",
           "config": {"workload": workload, "n": n, "bits": bits, "K": K,
                      "row_block": row_block, "col_block": col_block, "path": path,
                      "tile_schedule": resolved_schedule(schedule, bits, K) if path == "mfma"
                      else None,
                      "bound_group": bound_group or bdg.BOUND_GROUP_DEFAULT,
                      "centres": w["n_centres"], "flip_p": w["p"], "seed": w["seed"]},
           "roofline": roof(path), "stall": runs[path]["kernel"]["stall"]}
    if tuned is not None:
        res["autotune"] = tuned
    for name, r in runs.items():
        if name != path:
            rr = roof(name)
            res[f"{name}_path"] = {"value": pairs / (r["ms_per_step"] * 1e-3),
                                   "ms_per_step": r["ms_per_step"], "steps": r["steps"],
                                   "kernel_avg_ms": r["kernel"]["avg_ms"],
                                   "achieved": rr["achieved"], "peak": rr["peak"],
                                   "frac": rr["frac"], "stall": r["kernel"]["stall"]}
            for key in ("peak_source", "peak_derived"):
                if key in rr:
                    res[f"{name}_path"][key] = rr[key]
    return codes, codes_dev, outs, res


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--path", choices=["auto", "mfma", "popc"], default="auto")
    ap.add_argument("--workload", default="clustered-4m-512b-k100")
    ap.add_argument("--secondary", default="clustered-1m-256b-k64",
                    help="a second single-partition workload timed on the matrix-core path "
                         "with the same steps (reported, not the value); 'none' to skip")
    ap.add_argument("--other-path", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the other distance path (reported, not the value)")
    ap.add_argument("--other-steps", type=int, default=1,
                    help="timed steps of the other distance path")
    ap.add_argument("--other-warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--schedule", type=int, default=0,
                    help="tile schedule of the builds (BDG_SCHEDULE_*; the graph is the same "
                         "under each); 0: the library's default; --autotune overrides it")
    ap.add_argument("--bound-group", type=int, default=0,
                    help="admission bounds of the matrix-core build: rows per pivot group "
                         "(0: the library default, 1: off)")
    ap.add_argument("--tune-batched", action=argparse.BooleanOptionalAction, default=True,
                    help="batched workloads: tune the plan (work order, tile schedule, bound "
                         "group) before the timed replays")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the build schedule (bdg_autotune_build) before the timed builds, "
                         "outside the timed region, and time the winner")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed builds, run a streaming kernel of known size "
                         "(for scaling hardware byte counters)")
    ap.add_argument("--propagate", action=argparse.BooleanOptionalAction, default=True,
                    help="after the timed builds, run one round of neighbourhood propagation "
                         "from a degraded copy of the graph (reported, not the value)")
    ap.add_argument("--dac", action=argparse.BooleanOptionalAction, default=True,
                    help="after the timed builds, run the divide-and-conquer pipeline (binary "
                         "k-means, approximate graph, one propagation round) and report recall")
    ap.add_argument("--recall", action=argparse.BooleanOptionalAction, default=True,
                    help="after the timed builds, train the learned encoder on the 1M x 512 "
                         "mixture and report recall@64 of learned vs SRP codes (~30 s)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the graph build of one partition runs on a single "
              "MI355X, and multi-GPU runs are not part of this library; use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2102_04656_amd import bdg, datagen
    bdg.lib()
    w = datagen.WORKLOADS[args.workload]
    if "n_shards" in w:
        return bench_batched(args, w)
    main_path = "mfma" if args.path == "auto" else args.path
    peaks = measure_peaks()
    codes, codes_dev, outs, res = time_build(w, args.workload, main_path, args.steps, args.warmup,
                                             args.other_steps, args.other_warmup, args.other_path,
                                             autotune=args.autotune, bound_group=args.bound_group,
                                             schedule=args.schedule)
    n, bits, K = w["n"], w["bits"], w["K"]
    result = {
        "metric": METRIC,
        "value": res.pop("value"),
        "unit": "pair-dist/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": res.pop("dtype"),
        "data": "synthetic",
    }
    result.update(res)
    result["measured_peaks_tops"] = peaks
    if args.copy_calibration:
        copy_calibration()
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline (~{args.cpu_seconds:.0f}s sample)")
        result["cpu_baseline"] = cpu_baseline(codes, K, outs, args.cpu_seconds)
        log(f"[bench] cpu baseline: {result['cpu_baseline']['value']:.3e} pair-dist/s on "
            f"{result['cpu_baseline']['cores']} threads")
    if args.propagate:
        log("[bench] propagation leg")
        result["propagation"] = propagation_leg(codes, codes_dev, outs[0], bits, K,
                                                with_oracle=not args.no_cpu_baseline,
                                                workload=args.workload)
        log(f"[bench] propagation: {result['propagation']['ms']:.2f} ms, recall "
            f"{result['propagation']['recall_in']:.3f} -> {result['propagation']['recall_out']:.3f}")
    if args.dac:
        log("[bench] divide-and-conquer leg")
        # m is the knob the paper tunes (Sec. 4.5): on these synthetic codes recall needs
        # about as many centres as true clusters (1,000 at 1M rows; 20,000 at 4M rows)
        big = n > 2_000_000
        result["dac"] = dac_leg(codes_dev, outs[0], bits, K, m=32768 if big else 1024,
                                T=32 if big else 16, coarse_num=4096 if big else 8192)
        d = result["dac"]
        log(f"[bench] dac: kmeans {d['kmeans_ms']:.1f} ms, graph {d['dac_ms']:.1f} ms (recall "
            f"{d['recall_dac']:.3f}), + propagation {d['propagate_ms']:.1f} ms (recall "
            f"{d['recall_dac_propagated']:.3f})")
    del outs, codes_dev, codes
    torch.cuda.empty_cache()
    if args.secondary != "none" and args.secondary != args.workload:
        w2 = datagen.WORKLOADS[args.secondary]
        _, _, o2, r2 = time_build(w2, args.secondary, "mfma", args.steps, args.warmup, 0, 0,
                                  other_path=False, autotune=args.autotune,
                                  bound_group=args.bound_group, schedule=args.schedule)
        del o2
        result["secondary"] = r2
    if args.recall:
        result["recall"] = recall_leg()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
