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
MAX_BITS, MAX_K = 1024, 256


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
        ("reserved", ctypes.c_uint32 * 4),
    ]


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("shards", ctypes.c_uint32),
        ("rows", ctypes.c_uint32),
        ("work_items", ctypes.c_uint32),
        ("workgroups", ctypes.c_uint32),
        ("order", ctypes.c_int32),
        ("pairs", ctypes.c_uint64),
        ("device_bytes", ctypes.c_size_t),
    ]


ORDER_LONGEST_FIRST, ORDER_SHARD = 0, 1


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
    "bdg_merge_lists": [_p, _p, _u32, _u32, _u32, _u32, _p, _p, _p],
    "bdg_batch_plan_create": [_p, _u32, _u32, _u32, _p, _p],
    "bdg_batch_plan_destroy": [_p],
    "bdg_batch_plan_info": [_p, _p],
    "bdg_batch_plan_set_order": [_p, ctypes.c_int],
    "bdg_build_knn_batched_plan": [_p, _p, _p, _p, _p],
    "bdg_build_knn_batched_graph": [_p, _p, _p, _p, _p],
    "bdg_build_knn_batched_ex": [_p, _p, _u32, _u32, _u32, _p, _p, _p, _p],
    "bdg_autotune_build": [_p, _u32, _u32, _u32, _p, _p, _p, _p, _p, _sz],
    "bdg_autotune_batched": [_p, _p, _p, _p, _p, _p, _sz],
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


def bdg_build_knn_workspace_size(n, bits, K, opts=None) -> int:
    out = ctypes.c_size_t(0)
    op = ctypes.byref(opts) if opts is not None else None
    _check(lib().bdg_build_knn_workspace_size(n, bits, K, op, ctypes.byref(out)))
    return out.value


def bdg_merge_lists(in_idx, in_dist, n, L, K_in, K, out_idx, out_dist, stream=None) -> int:
    return lib().bdg_merge_lists(_ptr(in_idx), _ptr(in_dist), n, L, K_in, K, _ptr(out_idx),
                                 _ptr(out_dist), _stream(stream))


def bdg_status_string(status: int) -> str:
    return lib().bdg_status_string(status).decode()


def bdg_version() -> int:
    return lib().bdg_version()


# ------------------------------------------------------------- conveniences

def build_knn(codes, K: int, bits: int | None = None, path: int = PATH_AUTO,
              row_block: int = 0, col_block: int = 0, stream=None, out=None):
    """Exact Hamming kNN graph of ``codes`` (int64 ``[n][W]`` on the GPU).

    Returns ``(idx int32 [n][K], dist int16 [n][K])`` on the GPU (uint32 /
    uint16 bit patterns)."""
    import torch
    n, words = codes.shape
    bits = bits or 64 * words
    if out is None:
        out = (torch.empty((n, K), dtype=torch.int32, device=codes.device),
               torch.empty((n, K), dtype=torch.int16, device=codes.device))
    opts = make_opts(path=path, row_block=row_block, col_block=col_block)
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

    def __init__(self, offsets, bits: int, K: int, order: int = ORDER_LONGEST_FIRST):
        off, ptr = _host_offsets(offsets)
        self.offsets, self.bits, self.K = off, bits, K
        self.S = off.size - 1
        h = ctypes.c_void_p()
        o = make_opts(tile_variant=order)
        _check(lib().bdg_batch_plan_create(ptr, self.S, bits, K, ctypes.byref(o), ctypes.byref(h)))
        self.handle = h

    def info(self) -> BatchInfo:
        i = BatchInfo()
        _check(lib().bdg_batch_plan_info(self.handle, ctypes.byref(i)))
        return i

    def set_order(self, order: int):
        _check(lib().bdg_batch_plan_set_order(self.handle, order))

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
    rep = ctypes.create_string_buffer(4096)
    _check(lib().bdg_autotune_build(_ptr(codes), n, bits, K, _ptr(out[0]), _ptr(out[1]),
                                    ctypes.byref(o), _stream(stream), rep, len(rep)))
    return o, rep.value.decode()
