"""Thin ctypes binding of ``libbdg.so`` (declared in ``include/bdg.h``).

Argument marshalling only: every step of the graph build runs in the HIP
library. PyTorch supplies device memory and streams. The functions named
``bdg_*`` mirror the C entry points one to one; ``build_knn`` and
``merge_lists`` allocate the outputs and raise on error.

Device arrays are torch tensors on the GPU, with the bit patterns of the C
types: codes as int64 (uint64 words), indices as int32 (uint32), distances as
int16 (uint16).

Loading fails loudly (``BdgLibraryMissing``) when the library has not been
built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbdg.so")

BDG_OK, BDG_EINVAL, BDG_EUNSUPPORTED, BDG_ENOMEM, BDG_EDEVICE = 0, -1, -2, -3, -4
PATH_AUTO, PATH_POPC, PATH_MFMA = 0, 1, 2
NO_IDX, NO_DIST = 0xFFFFFFFF, 0xFFFF
MAX_BITS, MAX_K, MAX_K_TILE = 1024, 1024, 256


class BdgLibraryMissing(ImportError):
    pass


class BdgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"bdg status {status}: {message}")
        self.status = status


class KnnOpts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("path", ctypes.c_int32),
        ("row_block", ctypes.c_uint32),
        ("col_block", ctypes.c_uint32),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("first_rowblock", ctypes.c_uint32),
        ("stop_rowblock", ctypes.c_uint32),
        ("tile_variant", ctypes.c_uint32),
        ("n_tile_events", ctypes.c_uint32),
        ("tile_events", ctypes.c_void_p),
        ("wait_limit", ctypes.c_uint32),
        ("tile_schedule", ctypes.c_uint32),
        ("bound_group", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("shards", ctypes.c_uint32),
        ("rows", ctypes.c_uint32),
        ("work_items", ctypes.c_uint32),
        ("workgroups", ctypes.c_uint32),
        ("order", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("bound_group", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("pairs", ctypes.c_uint64),
        ("device_bytes", ctypes.c_size_t),
    ]


ORDER_LONGEST_FIRST, ORDER_SHARD = 0, 1
SCHEDULE_DEFAULT, SCHEDULE_DEEP_RING, SCHEDULE_GLOBAL_LISTS, SCHEDULE_LDS_LISTS = 0, 1, 2, 3
BOUND_OFF, BOUND_GROUP_DEFAULT, BOUND_GROUP_MIN, BOUND_GROUP_MAX = 1, 256, 16, 1 << 24


class MlpParams(ctypes.Structure):
    _fields_ = [("d", ctypes.c_uint32), ("h", ctypes.c_uint32), ("bits", ctypes.c_uint32),
                ("W1", ctypes.c_void_p), ("b1", ctypes.c_void_p),
                ("W2", ctypes.c_void_p), ("b2", ctypes.c_void_p),
                ("W1b", ctypes.c_void_p), ("W2b", ctypes.c_void_p), ("W2bt", ctypes.c_void_p)]


class MlpActs(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_uint32), ("rows_pad", ctypes.c_uint32),
                ("Xb", ctypes.c_void_p), ("Xt", ctypes.c_void_p), ("H1", ctypes.c_void_p),
                ("H1b", ctypes.c_void_p), ("H1t", ctypes.c_void_p), ("Z2", ctypes.c_void_p),
                ("H", ctypes.c_void_p), ("dZ2b", ctypes.c_void_p), ("dZ2t", ctypes.c_void_p),
                ("dZ1t", ctypes.c_void_p)]


class MlpGrads(ctypes.Structure):
    _fields_ = [("W1", ctypes.c_void_p), ("b1", ctypes.c_void_p), ("W2", ctypes.c_void_p),
                ("b2", ctypes.c_void_p)]


class LossOpts(ctypes.Structure):
    _fields_ = [("margin", ctypes.c_float), ("tau", ctypes.c_float), ("lam_q", ctypes.c_float),
                ("lam_b", ctypes.c_float)]


def make_opts(**kw) -> KnnOpts:
    o = KnnOpts()
    o.struct_size = ctypes.sizeof(KnnOpts)
    for k, v in kw.items():
        if v is not None:
            setattr(o, k, v)
    return o


_lock = threading.Lock()
_lib = None

_u32, _u64, _i32, _p, _sz = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32,
                            ctypes.c_void_p, ctypes.c_size_t)
_SIGS = {
    "bdg_build_knn": [_p, _u32, _u32, _u32, _p, _p],
    "bdg_build_knn_ex": [_p, _u32, _u32, _u32, _p, _p, _p, _p],
    "bdg_build_knn_workspace_size": [_u32, _u32, _u32, _p, _p],
    "bdg_build_knn_check": [_u32, _u32, _u32, _p, _p],
    "bdg_build_knn_noalloc": [_p, _u32, _u32, _u32, _p, _p, _p],
    "bdg_probe_peak": [ctypes.c_int, _p, _p],
    "bdg_merge_lists": [_p, _p, _u32, _u32, _u32, _u32, _p, _p, _p],
    "bdg_propagate": [_p, _u32, _u32, _u32, _p, _p, _p, _p],
    "bdg_bkmeans": [_p, _u32, _u32, _p, _u32, _p, _u32, _u32, _p, _p],
    "bdg_build_knn_dac": [_p, _u32, _u32, _p, _u32, _u32, _u32, _u32, _p, _p, _p],
    "bdg_hamming_knn": [_p, _u32, _p, _u32, _u32, _u32, _p, _p, _p],
    "bdg_graph_search": [_p, _u32, _u32, _p, _u32, _p, _u32, _p, _p, _p, _u32, _p, _u32, _u32,
                         _u32, _p, _p, _p, _p],
    "bdg_batch_plan_create": [_p, _u32, _u32, _u32, _p, _p],
    "bdg_batch_plan_destroy": [_p],
    "bdg_batch_plan_info": [_p, _p],
    "bdg_batch_plan_set_order": [_p, ctypes.c_int],
    "bdg_batch_plan_set_schedule": [_p, ctypes.c_int],
    "bdg_batch_plan_set_bound": [_p, ctypes.c_uint32],
    "bdg_batch_plan_set_timing": [_p, _p, _p],
    "bdg_build_knn_batched_plan": [_p, _p, _p, _p, _p],
    "bdg_build_knn_batched_graph": [_p, _p, _p, _p, _p],
    "bdg_build_knn_batched_ex": [_p, _p, _u32, _u32, _u32, _p, _p, _p, _p],
    "bdg_autotune_build": [_p, _u32, _u32, _u32, _p, _p, _p, _p, _p, _sz],
    "bdg_autotune_batched": [_p, _p, _p, _p, _p, _p, _sz],
    "bdg_encode": [_p, _u32, _u32, _p, _u32, _p, _p],
    "bdg_pack_signs": [_p, _u32, _u32, _p, _p],
    "bdg_float_knn": [_p, _u32, _p, _u32, _u32, _u32, _p, _p, _p, _p],
    "bdg_mlp_gather": [_p, _u32, _p, _u32, ctypes.c_float, _p, _p],
    "bdg_mlp_forward": [_p, _p, _p],
    "bdg_triplet_loss": [_p, _u32, _u32, _p, _p, _p, _p, _p],
    "bdg_mlp_backward": [_p, _p, _p, _p],
    "bdg_adam_step": [_p, _p, _p, _p, _sz, _u32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                      ctypes.c_float, _p],
    "bdg_mlp_refresh": [_p, _p],
    "bdg_mlp_encode": [_p, _p, _u32, ctypes.c_float, _p, _p],
    "bdg_gemm_nt_bf16": [_p, _u32, _p, _u32, _u32, _u32, _u32, _p, _u32, _p],
    "bdg_status_string": [ctypes.c_int],
    "bdg_last_error": [],
    "bdg_version": [],
}


def lib():
    """Load libbdg.so (once). Raises BdgLibraryMissing if it is not built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise BdgLibraryMissing(
                    f"{LIB_PATH} is missing: build it with "
                    "`python -m paper_2102_04656_amd.build`")
            L = ctypes.CDLL(LIB_PATH)
            for name, args in _SIGS.items():
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = ctypes.c_int
            L.bdg_status_string.restype = ctypes.c_char_p
            L.bdg_batch_plan_destroy.restype = None
            L.bdg_last_error.restype = ctypes.c_char_p
            _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def last_error() -> str:
    return lib().bdg_last_error().decode()


def _check(status: int):
    if status != BDG_OK:
        raise BdgError(status, last_error())
    return status


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------ raw entry points

def bdg_build_knn(codes, n, bits, K, out_idx, out_dist) -> int:
    return lib().bdg_build_knn(_ptr(codes), n, bits, K, _ptr(out_idx), _ptr(out_dist))


def bdg_build_knn_ex(codes, n, bits, K, out_idx, out_dist, opts=None, stream=None) -> int:
    op = ctypes.byref(opts) if opts is not None else None
    return lib().bdg_build_knn_ex(_ptr(codes), n, bits, K, _ptr(out_idx), _ptr(out_dist), op,
                                  _stream(stream))


def bdg_build_knn_check(n, bits, K, opts, stream=None) -> int:
    """Status of the last build enqueued with this caller workspace (waits
    for the stream): 0, or BDG_EDEVICE if the persistent launch's stall flag
    is set."""
    return lib().bdg_build_knn_check(n, bits, K, ctypes.byref(opts), _stream(stream))


def bdg_build_knn_noalloc(codes, n, bits, K, out_idx, out_dist, stream=None) -> int:
    """The matrix-core build with the library's static workspace (allocates
    nothing; inputs up to the static scratch size)."""
    return lib().bdg_build_knn_noalloc(_ptr(codes), n, bits, K, _ptr(out_idx), _ptr(out_dist),
                                       _stream(stream))


PEAK_VALU_INT32, PEAK_MFMA_INT8 = 0, 1


def probe_peak(unit: int, stream=None) -> float:
    """Measured sustained rate of a unit (operations per second)."""
    v = ctypes.c_double()
    _check(lib().bdg_probe_peak(unit, ctypes.byref(v), _stream(stream)))
    return v.value


def bdg_build_knn_workspace_size(n, bits, K, opts=None) -> int:
    out = ctypes.c_size_t(0)
    op = ctypes.byref(opts) if opts is not None else None
    _check(lib().bdg_build_knn_workspace_size(n, bits, K, op, ctypes.byref(out)))
    return out.value


def bdg_merge_lists(in_idx, in_dist, n, L, K_in, K, out_idx, out_dist, stream=None) -> int:
    return lib().bdg_merge_lists(_ptr(in_idx), _ptr(in_dist), n, L, K_in, K, _ptr(out_idx),
                                 _ptr(out_dist), _stream(stream))


def bdg_propagate(codes, n, bits, K, in_idx, out_idx, out_dist, stream=None) -> int:
    return lib().bdg_propagate(_ptr(codes), n, bits, K, _ptr(in_idx), _ptr(out_idx),
                               _ptr(out_dist), _stream(stream))


def bdg_status_string(status: int) -> str:
    return lib().bdg_status_string(status).decode()


def bdg_version() -> int:
    return lib().bdg_version()


# ------------------------------------------------------------- conveniences

def build_knn(codes, K: int, bits: int | None = None, path: int = PATH_AUTO,
              row_block: int = 0, col_block: int = 0, stream=None, out=None,
              schedule: int = SCHEDULE_DEFAULT, bound_group: int = 0):
    """Exact Hamming kNN graph of ``codes`` (int64 ``[n][W]`` on the GPU).

    Returns ``(idx int32 [n][K], dist int16 [n][K])`` on the GPU (uint32 /
    uint16 bit patterns)."""
    import torch
    n, words = codes.shape
    bits = bits or 64 * words
    if out is None:
        out = (torch.empty((n, K), dtype=torch.int32, device=codes.device),
               torch.empty((n, K), dtype=torch.int16, device=codes.device))
    opts = make_opts(path=path, row_block=row_block, col_block=col_block, tile_schedule=schedule,
                     bound_group=bound_group)
    _check(bdg_build_knn_ex(codes, n, bits, K, out[0], out[1], opts, stream))
    return out


def merge_lists(in_idx, in_dist, K: int, stream=None):
    """Merge ``[L][n][K_in]`` lists into ``[n][K]`` (GPU tensors)."""
    import torch
    L, n, kin = in_idx.shape
    out = (torch.empty((n, K), dtype=torch.int32, device=in_idx.device),
           torch.empty((n, K), dtype=torch.int16, device=in_idx.device))
    _check(bdg_merge_lists(in_idx, in_dist, n, L, kin, K, out[0], out[1], stream))
    return out


def propagate(codes, in_idx, bits: int | None = None, stream=None):
    """One round of neighbourhood propagation of the graph ``in_idx [n][K]``
    (GPU tensors; codes ``[n][bits/64]`` int64/uint64). Returns new
    ``(idx int32 [n][K], dist int16 [n][K])``."""
    import torch
    n, K = in_idx.shape
    bits = bits or codes.shape[1] * 64
    out = (torch.empty((n, K), dtype=torch.int32, device=in_idx.device),
           torch.empty((n, K), dtype=torch.int16, device=in_idx.device))
    _check(bdg_propagate(codes, n, bits, K, in_idx, out[0], out[1], stream))
    return out


def bkmeans(codes, sample, init, iters: int, bits: int | None = None, stream=None):
    """Binary k-means centres (GPU): ``sample`` and ``init`` are host arrays of
    row indices; returns a ``[m][bits/64]`` int64 GPU tensor."""
    import numpy as np
    import torch
    n = codes.shape[0]
    bits = bits or codes.shape[1] * 64
    s = np.ascontiguousarray(sample, dtype=np.uint32)
    i = np.ascontiguousarray(init, dtype=np.uint32)
    out = torch.empty((i.size, bits // 64), dtype=torch.int64, device=codes.device)
    _check(lib().bdg_bkmeans(_ptr(codes), n, bits, s.ctypes.data, s.size, i.ctypes.data, i.size,
                             iters, _ptr(out), _stream(stream)))
    return out


def hamming_knn(queries, base, K: int, bits: int | None = None, stream=None):
    """Exact Hamming kNN of ``queries`` against ``base`` (int64 ``[n][W]`` on the
    GPU); returns ``(idx int32 [nq][K], dist int16 [nq][K])``."""
    import torch
    nq, words = queries.shape
    bits = bits or 64 * words
    out = (torch.empty((nq, K), dtype=torch.int32, device=queries.device),
           torch.empty((nq, K), dtype=torch.int16, device=queries.device))
    _check(lib().bdg_hamming_knn(_ptr(queries), nq, _ptr(base), base.shape[0], bits, K,
                                 _ptr(out[0]), _ptr(out[1]), _stream(stream)))
    return out


def build_knn_dac(codes, centres, K: int, T: int, coarse_num: int, bits: int | None = None,
                  stream=None):
    """Approximate graph of the single-pass divide-and-conquer (GPU tensors)."""
    import torch
    n = codes.shape[0]
    bits = bits or codes.shape[1] * 64
    out = (torch.empty((n, K), dtype=torch.int32, device=codes.device),
           torch.empty((n, K), dtype=torch.int16, device=codes.device))
    _check(lib().bdg_build_knn_dac(_ptr(codes), n, bits, _ptr(centres), centres.shape[0], T,
                                   coarse_num, K, _ptr(out[0]), _ptr(out[1]), _stream(stream)))
    return out


def graph_search(codes, graph, feats, q_codes, q_feats, entries, P: int, N: int,
                 q_exclude=None, bits: int | None = None, stream=None):
    """Online search (GPU tensors): returns (idx int32 [nq][N], dist float32
    [nq][N], visited int32 [nq])."""
    import torch
    n, K = graph.shape
    d = feats.shape[1]
    nq = q_codes.shape[0]
    bits = bits or codes.shape[1] * 64
    dev = codes.device
    out = (torch.empty((nq, N), dtype=torch.int32, device=dev),
           torch.empty((nq, N), dtype=torch.float32, device=dev),
           torch.empty((nq,), dtype=torch.int32, device=dev))
    _check(lib().bdg_graph_search(
        _ptr(codes), n, bits, _ptr(graph), K, _ptr(feats), d, _ptr(q_codes), _ptr(q_feats),
        _ptr(q_exclude) if q_exclude is not None else None, nq, _ptr(entries), entries.shape[0],
        P, N, _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _stream(stream)))
    return out


def to_numpy_graph(idx, dist):
    """GPU (int32, int16) graph -> host numpy (uint32, uint16)."""
    import numpy as np
    return (idx.cpu().numpy().view(np.uint32), dist.cpu().numpy().view(np.uint16))


# ------------------------------------------------------------ many partitions

def _host_offsets(offsets):
    import numpy as np
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    return off, ctypes.c_void_p(off.ctypes.data)


class BatchPlan:
    """A plan for building the graphs of many shards in one persistent launch
    (``bdg_batch_plan_*``). ``offsets`` is a host array of S + 1 row offsets."""

    def __init__(self, offsets, bits: int, K: int, order: int = ORDER_LONGEST_FIRST,
                 schedule: int = SCHEDULE_DEFAULT, bound_group: int = 0):
        off, ptr = _host_offsets(offsets)
        self.offsets, self.bits, self.K = off, bits, K
        self.S = off.size - 1
        h = ctypes.c_void_p()
        o = make_opts(tile_variant=order, tile_schedule=schedule, bound_group=bound_group)
        _check(lib().bdg_batch_plan_create(ptr, self.S, bits, K, ctypes.byref(o), ctypes.byref(h)))
        self.handle = h

    def info(self) -> BatchInfo:
        i = BatchInfo()
        _check(lib().bdg_batch_plan_info(self.handle, ctypes.byref(i)))
        return i

    def set_order(self, order: int):
        _check(lib().bdg_batch_plan_set_order(self.handle, order))

    def set_schedule(self, schedule: int):
        _check(lib().bdg_batch_plan_set_schedule(self.handle, schedule))

    def set_bound(self, bound_group: int):
        _check(lib().bdg_batch_plan_set_bound(self.handle, bound_group))

    def set_timing(self, start_event, stop_event):
        """hipEvent_t handles (ints) recorded around the persistent kernel of
        eager builds; (None, None) stops."""
        _check(lib().bdg_batch_plan_set_timing(self.handle, start_event, stop_event))

    def outputs(self, device="cuda"):
        import torch
        n = int(self.offsets[-1])
        return (torch.empty((n, self.K), dtype=torch.int32, device=device),
                torch.empty((n, self.K), dtype=torch.int16, device=device))

    def build(self, codes, out=None, stream=None, graph: bool = False):
        """Enqueue the build (through a HIP graph if ``graph``); returns (idx, dist)."""
        out = out if out is not None else self.outputs(codes.device)
        fn = lib().bdg_build_knn_batched_graph if graph else lib().bdg_build_knn_batched_plan
        _check(fn(self.handle, _ptr(codes), _ptr(out[0]), _ptr(out[1]), _stream(stream)))
        return out

    def autotune(self, codes, out=None, stream=None) -> str:
        out = out if out is not None else self.outputs(codes.device)
        rep = ctypes.create_string_buffer(4096)
        _check(lib().bdg_autotune_batched(self.handle, _ptr(codes), _ptr(out[0]), _ptr(out[1]),
                                          _stream(stream), rep, len(rep)))
        return rep.value.decode()

    def close(self):
        if getattr(self, "handle", None):
            lib().bdg_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bdg_build_knn_batched_ex(codes, offsets, S, bits, K, out_idx, out_dist, opts=None,
                             stream=None) -> int:
    off, ptr = _host_offsets(offsets)
    op = ctypes.byref(opts) if opts is not None else None
    return lib().bdg_build_knn_batched_ex(_ptr(codes), ptr, S, bits, K, _ptr(out_idx),
                                          _ptr(out_dist), op, _stream(stream))


def autotune_build(codes, K: int, bits: int | None = None, row_block: int = 0, stream=None):
    """Tune the single-partition schedule; returns (opts, report_json)."""
    import torch
    n, words = codes.shape
    bits = bits or 64 * words
    out = (torch.empty((n, K), dtype=torch.int32, device=codes.device),
           torch.empty((n, K), dtype=torch.int16, device=codes.device))
    o = make_opts(row_block=row_block)
    rep = ctypes.create_string_buffer(8192)
    _check(lib().bdg_autotune_build(_ptr(codes), n, bits, K, _ptr(out[0]), _ptr(out[1]),
                                    ctypes.byref(o), _stream(stream), rep, len(rep)))
    return o, rep.value.decode()


# ---------------------------------------------------- binarisers, float kNN

def encode_srp(x, proj, stream=None):
    """Sign-of-random-projection codes of x (float32 [n][d]) with proj
    (float32 [d][bits]), on the GPU: int64 [n][bits/64] (uint64 bit patterns)."""
    import torch
    n, d = x.shape
    bits = proj.shape[1]
    out = torch.empty((n, bits // 64), dtype=torch.int64, device=x.device)
    _check(lib().bdg_encode(_ptr(x), n, d, _ptr(proj), bits, _ptr(out), _stream(stream)))
    return out


def pack_signs(z, stream=None):
    import torch
    n, bits = z.shape
    out = torch.empty((n, bits // 64), dtype=torch.int64, device=z.device)
    _check(lib().bdg_pack_signs(_ptr(z), n, bits, _ptr(out), _stream(stream)))
    return out


def float_knn(queries, base, K: int, exclude=None, stream=None):
    """Exact squared-L2 kNN in FP32: (idx int32 [nq][K], dist float32 [nq][K])."""
    import torch
    nq, d = queries.shape
    out = (torch.empty((nq, K), dtype=torch.int32, device=queries.device),
           torch.empty((nq, K), dtype=torch.float32, device=queries.device))
    _check(lib().bdg_float_knn(_ptr(queries), nq, _ptr(base), base.shape[0], d, K,
                               _ptr(exclude), _ptr(out[0]), _ptr(out[1]), _stream(stream)))
    return out


def gemm_nt_bf16(A, B, stream=None):
    """C = A B^T for bf16 bit patterns A [M][K], B [N][K] (int16 tensors): float32 [M][N]."""
    import torch
    M, K = A.shape
    N = B.shape[0]
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(lib().bdg_gemm_nt_bf16(_ptr(A), K, _ptr(B), K, M, N, K, _ptr(C), N, _stream(stream)))
    return C


class Mlp:
    """Device state of the learned encoder d -> h -> bits (tanh) and its
    training step, all through the C ABI (bdg_mlp_*, bdg_triplet_loss,
    bdg_adam_step). Weights: W1 [h][d], W2 [bits][h] (FP32 masters)."""

    def __init__(self, W1, b1, W2, b2, device="cuda"):
        import torch
        f32 = dict(dtype=torch.float32, device=device)
        self.W1 = torch.as_tensor(W1, **f32).contiguous()
        self.b1 = torch.as_tensor(b1, **f32).contiguous()
        self.W2 = torch.as_tensor(W2, **f32).contiguous()
        self.b2 = torch.as_tensor(b2, **f32).contiguous()
        self.h, self.d = self.W1.shape
        self.bits = self.W2.shape[0]
        i16 = dict(dtype=torch.int16, device=device)
        self.W1b = torch.empty((self.h, self.d), **i16)
        self.W2b = torch.empty((self.bits, self.h), **i16)
        self.W2bt = torch.empty((self.h, self.bits), **i16)
        self.params = MlpParams(self.d, self.h, self.bits, _vp(self.W1), _vp(self.b1),
                                _vp(self.W2), _vp(self.b2), _vp(self.W1b), _vp(self.W2b),
                                _vp(self.W2bt))
        self.grads_t = [torch.zeros_like(t) for t in (self.W1, self.b1, self.W2, self.b2)]
        self.grads = MlpGrads(*[_vp(t) for t in self.grads_t])
        self.moments = [(torch.zeros_like(t), torch.zeros_like(t))
                        for t in (self.W1, self.b1, self.W2, self.b2)]
        self.step_count = 0
        self.refresh()

    def refresh(self, stream=None):
        _check(lib().bdg_mlp_refresh(ctypes.byref(self.params), _stream(stream)))

    def acts(self, rows_pad, train=True, device="cuda"):
        import torch
        assert rows_pad % 32 == 0
        i16 = dict(dtype=torch.int16, device=device)
        f32 = dict(dtype=torch.float32, device=device)
        t = dict(Xb=torch.empty((rows_pad, self.d), **i16),
                 Xt=torch.empty((self.d, rows_pad), **i16) if train else None,
                 H1=torch.empty((rows_pad, self.h), **f32),
                 H1b=torch.empty((rows_pad, self.h), **i16),
                 H1t=torch.empty((self.h, rows_pad), **i16),
                 Z2=torch.empty((rows_pad, self.bits), **f32),
                 H=torch.empty((rows_pad, self.bits), **f32),
                 dZ2b=torch.empty((rows_pad, self.bits), **i16) if train else None,
                 dZ2t=torch.empty((self.bits, rows_pad), **i16) if train else None,
                 dZ1t=torch.empty((self.h, rows_pad), **i16) if train else None,
                 mu=torch.empty(self.bits, **f32), loss=torch.zeros(1, **f32))
        a = MlpActs(0, rows_pad, *[_vp(t[k]) for k in ("Xb", "Xt", "H1", "H1b", "H1t", "Z2", "H",
                                                       "dZ2b", "dZ2t", "dZ1t")])
        return a, t

    def gather(self, a, X, idx, rows, scale=1.0, stream=None):
        _check(lib().bdg_mlp_gather(_ptr(X), self.d, _ptr(idx), rows, float(scale),
                                    ctypes.byref(a), _stream(stream)))

    def forward(self, a, stream=None):
        _check(lib().bdg_mlp_forward(ctypes.byref(self.params), ctypes.byref(a), _stream(stream)))

    def loss(self, a, t, T, margin=2.0, tau=4.0, lam_q=0.1, lam_b=0.01, stream=None):
        o = LossOpts(margin, tau, lam_q, lam_b)
        _check(lib().bdg_triplet_loss(ctypes.byref(a), self.bits, T, ctypes.byref(o),
                                      _ptr(t["mu"]), _vp(self.grads_t[3]), _ptr(t["loss"]),
                                      _stream(stream)))

    def backward(self, a, stream=None):
        _check(lib().bdg_mlp_backward(ctypes.byref(self.params), ctypes.byref(a),
                                      ctypes.byref(self.grads), _stream(stream)))

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step_count += 1
        for p, g, (m, v) in zip((self.W1, self.b1, self.W2, self.b2), self.grads_t, self.moments):
            _check(lib().bdg_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(),
                                       self.step_count, lr, beta1, beta2, eps, _stream(stream)))
        self.refresh(stream)

    def encode(self, X, scale=1.0, stream=None):
        import torch
        out = torch.empty((X.shape[0], self.bits // 64), dtype=torch.int64, device=X.device)
        _check(lib().bdg_mlp_encode(ctypes.byref(self.params), _ptr(X), X.shape[0], float(scale),
                                    _ptr(out), _stream(stream)))
        return out


def _vp(t):
    return None if t is None else t.data_ptr()
