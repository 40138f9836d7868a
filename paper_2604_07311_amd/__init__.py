"""MI355X (gfx950) strided tensor contraction -- Python binding.

Thin ctypes layer over ``libfamlies.so`` (C ABI in ``include/famlies.h``):
argument marshalling only.  Every step of the contraction runs in the
library's HIP kernels and host planner; PyTorch supplies device memory and
streams.  There is no CPU fallback: if the library is missing or the GPU is
not a gfx950, calls raise.

Low-level functions keep the C names (``famlies_create``,
``famlies_plan_contract``, ``famlies_execute`` ...).  The convenience layer:

* :func:`contract` -- ``C = alpha * A.B + beta * C`` on torch tensors with
  labelled modes, e.g. ``contract(1.0, W, "abef", T, "efij", 1.0, C, "abij")``.
  Any strides (views, permutations, negative-free) are used as they are: no
  tensor is copied or transposed.
* :class:`ContractFn` -- autograd Function whose backward is two more
  contractions on the same engine.
"""
from __future__ import annotations

import ctypes
import os
import threading
from collections import OrderedDict
from typing import Dict, Optional, Sequence, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfamlies.so")

FAMLIES_OK = 0
FAMLIES_ERR_INVALID_ARG = -1
FAMLIES_ERR_SHAPE_MISMATCH = -2
FAMLIES_ERR_LABEL = -3
FAMLIES_ERR_UNSUPPORTED = -4
FAMLIES_ERR_ALIAS = -5
FAMLIES_ERR_ALIGN = -6
FAMLIES_ERR_ALLOC = -7
FAMLIES_ERR_DEVICE = -8
FAMLIES_ERR_BOUNDS = -9
FAMLIES_MAX_RANK = 8
FAMLIES_F64 = 1
FAMLIES_F32 = 2
FAMLIES_NATIVE = 0
FAMLIES_BF16X3 = 1
FAMLIES_BF16X6 = 2
FAMLIES_INT8X3 = 19   # FP64 emulated on INT8 MFMA with 3..7 digit slices (FAMLIES_F64 only)
FAMLIES_INT8X4 = 20
FAMLIES_INT8X5 = 21
FAMLIES_INT8X6 = 22
FAMLIES_INT8X7 = 23
FAMLIES_TUNE_QUICK = 1
FAMLIES_TUNE_BATCH_ONLY = 2
FAMLIES_TUNE_PLAIN_ONLY = 4

ERROR_NAMES = {
    FAMLIES_ERR_INVALID_ARG: "INVALID_ARG", FAMLIES_ERR_SHAPE_MISMATCH: "SHAPE_MISMATCH",
    FAMLIES_ERR_LABEL: "LABEL", FAMLIES_ERR_UNSUPPORTED: "UNSUPPORTED", FAMLIES_ERR_ALIAS: "ALIAS",
    FAMLIES_ERR_ALIGN: "ALIGN", FAMLIES_ERR_ALLOC: "ALLOC", FAMLIES_ERR_DEVICE: "DEVICE",
    FAMLIES_ERR_BOUNDS: "BOUNDS",
}


class famlies_tensor(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("extents", ctypes.POINTER(ctypes.c_int64)),
                ("strides", ctypes.POINTER(ctypes.c_int64)),
                ("labels", ctypes.POINTER(ctypes.c_int32))]


class famlies_plan_info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("batch", ctypes.c_int64),
                ("swapped", ctypes.c_int32), ("x_kfast", ctypes.c_int32),
                ("y_kfast", ctypes.c_int32), ("n_i", ctypes.c_int32), ("n_j", ctypes.c_int32),
                ("n_p", ctypes.c_int32), ("n_batch", ctypes.c_int32), ("n_trace", ctypes.c_int32),
                ("n_diag", ctypes.c_int32), ("tile_m", ctypes.c_int32), ("tile_n", ctypes.c_int32),
                ("tile_k", ctypes.c_int32), ("split_k", ctypes.c_int32),
                ("index_bits", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("split_tiles", ctypes.c_int32), ("flops", ctypes.c_double),
                ("index_elements", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


EXPORTS = [
    "famlies_create", "famlies_destroy", "famlies_plan_contract", "famlies_execute",
    "famlies_plan_destroy", "famlies_plan_get_info", "famlies_analyze", "famlies_batch_plan",
    "famlies_batch_execute", "famlies_tune", "famlies_load_tune_table", "famlies_last_error",
    "famlies_version", "famlies_pack_size", "famlies_pack", "famlies_execute_packed",
    "famlies_network_create", "famlies_network_add_tensor", "famlies_network_add_contraction",
    "famlies_network_compile", "famlies_network_bind", "famlies_network_tensor_ptr",
    "famlies_network_execute", "famlies_network_destroy", "famlies_contract_noalloc",
    "famlies_batch_plan_tiles",
]
FAMLIES_NET_PACK_A = 1
FAMLIES_NET_PACK_B = 2


class FamliesError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__("%s failed: %s (%s)" % (where, ERROR_NAMES.get(code, code), msg))
        self.code = code


_lib = None
_lib_lock = threading.Lock()


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise ImportError("libfamlies.so not built: run `python -m paper_2604_07311_amd.build` "
                              "(this package has no CPU fallback)")
        lib = ctypes.CDLL(path)
        T = ctypes.POINTER(famlies_tensor)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        sig = {
            "famlies_create": ([ctypes.POINTER(vp), i32], i32),
            "famlies_destroy": ([vp], i32),
            "famlies_plan_contract": ([vp, ctypes.POINTER(vp), i32, i32, T, T, T], i32),
            "famlies_execute": ([vp, dbl, vp, vp, dbl, vp, vp], i32),
            "famlies_plan_destroy": ([vp], i32),
            "famlies_plan_get_info": ([vp, ctypes.POINTER(famlies_plan_info)], i32),
            "famlies_analyze": ([i32, i32, T, T, T, ctypes.POINTER(famlies_plan_info),
                                 ctypes.POINTER(ctypes.c_int64), i64], i32),
            "famlies_batch_plan": ([vp, ctypes.POINTER(vp), i32, i64, T, T, T], i32),
            "famlies_batch_execute": ([vp, dbl, dbl, vp, vp, vp, vp], i32),
            "famlies_batch_plan_tiles": ([vp, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32), i64], i32),
            "famlies_tune": ([vp, ctypes.c_char_p, i32], i32),
            "famlies_load_tune_table": ([vp, ctypes.c_char_p], i32),
            "famlies_pack_size": ([vp, i32, ctypes.POINTER(ctypes.c_size_t)], i32),
            "famlies_pack": ([vp, i32, vp, vp, vp], i32),
            "famlies_execute_packed": ([vp, dbl, vp, vp, dbl, vp, i32, vp], i32),
            "famlies_network_create": ([vp, ctypes.POINTER(vp), i32, i32], i32),
            "famlies_network_add_tensor": ([vp, T, i32, ctypes.POINTER(ctypes.c_int32)], i32),
            "famlies_network_add_contraction": ([vp, dbl, i32, i32, dbl, i32, i32], i32),
            "famlies_network_compile": ([vp], i32),
            "famlies_network_bind": ([vp, i32, vp], i32),
            "famlies_network_tensor_ptr": ([vp, i32, ctypes.POINTER(vp)], i32),
            "famlies_network_execute": ([vp, vp], i32),
            "famlies_network_destroy": ([vp], i32),
            "famlies_contract_noalloc": ([vp, i32, i32, dbl, T, vp, T, vp, dbl, T, vp, vp], i32),
            "famlies_last_error": ([], ctypes.c_char_p),
            "famlies_version": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        return lib


def _check(st: int, where: str):
    if st != FAMLIES_OK:
        raise FamliesError(st, where, famlies_last_error())


# ---------------------------------------------------------------- raw C names
def famlies_last_error() -> str:
    return load_library().famlies_last_error().decode()


def famlies_version() -> str:
    return load_library().famlies_version().decode()


def famlies_create(device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load_library().famlies_create(ctypes.byref(h), int(device)), "famlies_create")
    return h.value


def famlies_destroy(handle: int) -> None:
    _check(load_library().famlies_destroy(handle), "famlies_destroy")


def make_desc(extents: Sequence[int], strides: Sequence[int], labels) -> famlies_tensor:
    """A famlies_tensor that keeps its arrays alive.  ``labels`` is a string
    (one label per character) or a sequence of ints."""
    labs = [ord(c) for c in labels] if isinstance(labels, str) else [int(x) for x in labels]
    r = len(extents)
    if len(strides) != r or len(labs) != r:
        raise ValueError("extents, strides and labels must have the same length")
    e = (ctypes.c_int64 * max(r, 1))(*[int(x) for x in extents])
    s = (ctypes.c_int64 * max(r, 1))(*[int(x) for x in strides])
    lab = (ctypes.c_int32 * max(r, 1))(*labs)
    d = famlies_tensor(r, e, s, lab)
    d._keep = (e, s, lab)
    return d


def famlies_plan_contract(handle: int, dtype: int, compute: int, A: famlies_tensor,
                          B: famlies_tensor, C: famlies_tensor) -> int:
    p = ctypes.c_void_p()
    _check(load_library().famlies_plan_contract(handle, ctypes.byref(p), dtype, compute,
                                                ctypes.byref(A), ctypes.byref(B), ctypes.byref(C)),
           "famlies_plan_contract")
    return p.value


def famlies_execute(plan: int, alpha: float, A_ptr: int, B_ptr: int, beta: float, C_ptr: int,
                    stream: int = 0) -> None:
    _check(load_library().famlies_execute(plan, float(alpha), A_ptr, B_ptr, float(beta), C_ptr,
                                          stream), "famlies_execute")


def famlies_contract_noalloc(handle: int, dtype: int, compute: int, alpha: float, A: famlies_tensor,
                             A_ptr: int, B: famlies_tensor, B_ptr: int, beta: float, C: famlies_tensor,
                             C_ptr: int, stream: int = 0) -> None:
    _check(load_library().famlies_contract_noalloc(handle, dtype, compute, float(alpha), ctypes.byref(A), A_ptr,
                                                   ctypes.byref(B), B_ptr, float(beta), ctypes.byref(C), C_ptr,
                                                   stream), "famlies_contract_noalloc")


def famlies_pack_size(plan: int, operand: int) -> int:
    n = ctypes.c_size_t()
    _check(load_library().famlies_pack_size(plan, int(operand), ctypes.byref(n)), "famlies_pack_size")
    return n.value


def famlies_pack(plan: int, operand: int, src_ptr: int, dst_ptr: int, stream: int = 0) -> None:
    _check(load_library().famlies_pack(plan, int(operand), src_ptr, dst_ptr, stream), "famlies_pack")


def famlies_execute_packed(plan: int, alpha: float, A_ptr: int, B_ptr: int, beta: float, C_ptr: int,
                           packed: int, stream: int = 0) -> None:
    _check(load_library().famlies_execute_packed(plan, float(alpha), A_ptr, B_ptr, float(beta), C_ptr,
                                                 int(packed), stream), "famlies_execute_packed")


class Network:
    """Thin wrapper over the famlies_network_* calls (same names underneath).

    >>> net = Network(FAMLIES_F64)
    >>> w = net.tensor(W.shape, W.stride(), "abef")          # bound by the caller
    >>> i1 = net.tensor(shape, strides, "abij", intermediate=True)
    >>> net.contract(1.0, w, t, 0.0, i1, pack_a=True)
    >>> net.compile(); net.bind(w, W.data_ptr()); net.execute(stream)
    """

    def __init__(self, dtype: int, compute: int = FAMLIES_NATIVE, device: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.famlies_network_create(handle(device), ctypes.byref(h), dtype, compute),
               "famlies_network_create")
        self.ptr = h.value

    def tensor(self, extents, strides, labels, intermediate: bool = False) -> int:
        i = ctypes.c_int32()
        d = make_desc(extents, strides, labels)
        _check(load_library().famlies_network_add_tensor(self.ptr, ctypes.byref(d), int(intermediate),
                                                         ctypes.byref(i)), "famlies_network_add_tensor")
        return i.value

    def contract(self, alpha, a: int, b: int, beta, c: int, pack_a: bool = False, pack_b: bool = False):
        flags = (FAMLIES_NET_PACK_A if pack_a else 0) | (FAMLIES_NET_PACK_B if pack_b else 0)
        _check(load_library().famlies_network_add_contraction(self.ptr, float(alpha), a, b, float(beta), c,
                                                              flags), "famlies_network_add_contraction")

    def compile(self):
        _check(load_library().famlies_network_compile(self.ptr), "famlies_network_compile")

    def bind(self, tid: int, ptr: int):
        _check(load_library().famlies_network_bind(self.ptr, tid, ptr), "famlies_network_bind")

    def tensor_ptr(self, tid: int) -> int:
        q = ctypes.c_void_p()
        _check(load_library().famlies_network_tensor_ptr(self.ptr, tid, ctypes.byref(q)),
               "famlies_network_tensor_ptr")
        return q.value

    def execute(self, stream: int = 0):
        _check(load_library().famlies_network_execute(self.ptr, stream), "famlies_network_execute")

    def close(self):
        if self.ptr:
            _check(load_library().famlies_network_destroy(self.ptr), "famlies_network_destroy")
            self.ptr = None


def famlies_plan_destroy(plan: int) -> None:
    _check(load_library().famlies_plan_destroy(plan), "famlies_plan_destroy")


def famlies_plan_get_info(plan: int) -> dict:
    info = famlies_plan_info()
    _check(load_library().famlies_plan_get_info(plan, ctypes.byref(info)), "famlies_plan_get_info")
    return info.as_dict()


def famlies_analyze(dtype: int, compute: int, A: famlies_tensor, B: famlies_tensor,
                    C: famlies_tensor, want_offsets: bool = False):
    """Host-only planner dry run.  Returns (info dict, offsets) where offsets
    is None or a dict of the nine indexing vectors (numpy int64)."""
    lib = load_library()
    info = famlies_plan_info()
    st = lib.famlies_analyze(dtype, compute, ctypes.byref(A), ctypes.byref(B), ctypes.byref(C),
                             ctypes.byref(info), None, 0)
    _check(st, "famlies_analyze")
    if not want_offsets:
        return info.as_dict(), None
    import numpy as np
    m, n, k, l = info.m, info.n, info.k, info.batch
    buf = np.zeros(2 * (m + n + k) + 3 * l, dtype=np.int64)
    st = lib.famlies_analyze(dtype, compute, ctypes.byref(A), ctypes.byref(B), ctypes.byref(C),
                             ctypes.byref(info), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                             buf.size)
    _check(st, "famlies_analyze")
    names = ["xrow", "xk", "yk", "ycol", "crow", "ccol", "xbatch", "ybatch", "cbatch"]
    lens = [m, k, k, n, m, n, l, l, l]
    out, pos = {}, 0
    for nm, ln in zip(names, lens):
        out[nm] = buf[pos:pos + ln].copy()
        pos += ln
    return info.as_dict(), out


def famlies_batch_plan(handle: int, dtype: int, descs_a, descs_b, descs_c) -> int:
    n = len(descs_a)
    if len(descs_b) != n or len(descs_c) != n:
        raise ValueError("descriptor lists differ in length")
    arr = [(famlies_tensor * max(n, 1))(*[(d.rank, d.extents, d.strides, d.labels) for d in ds])
           for ds in (descs_a, descs_b, descs_c)]
    p = ctypes.c_void_p()
    _check(load_library().famlies_batch_plan(handle, ctypes.byref(p), dtype, n, arr[0], arr[1],
                                             arr[2]), "famlies_batch_plan")
    return p.value


def famlies_batch_plan_tiles(plan: int, n: int):
    """Per-problem tile (tile_m, tile_n) of a batched plan of n problems."""
    tm = (ctypes.c_int32 * max(n, 1))()
    tn = (ctypes.c_int32 * max(n, 1))()
    _check(load_library().famlies_batch_plan_tiles(plan, tm, tn, n), "famlies_batch_plan_tiles")
    return [(tm[i], tn[i]) for i in range(n)]


def famlies_batch_execute(plan: int, alpha: float, beta: float, A_ptrs_dev: int, B_ptrs_dev: int,
                          C_ptrs_dev: int, stream: int = 0) -> None:
    _check(load_library().famlies_batch_execute(plan, float(alpha), float(beta), A_ptrs_dev,
                                                B_ptrs_dev, C_ptrs_dev, stream),
           "famlies_batch_execute")


def famlies_tune(handle: int, table_path: str, flags: int = 0) -> None:
    _check(load_library().famlies_tune(handle, table_path.encode(), flags), "famlies_tune")


def famlies_load_tune_table(handle: int, table_path: str) -> None:
    _check(load_library().famlies_load_tune_table(handle, table_path.encode()),
           "famlies_load_tune_table")


# ----------------------------------------------------------- torch-level API
_handles: Dict[int, int] = {}
# Plans keyed by device, stream, types, shapes, strides and labels.  A plan
# owns a split-K workspace that its launches share, so one plan serves one
# stream only: calls on unordered streams get plans of their own and never
# write partial sums into the same workspace.  Least recently used plans are
# destroyed beyond PLAN_CACHE_MAX entries (after the device has finished
# with them; never while a graph is being captured).
PLAN_CACHE_MAX = 256
_plan_cache: "OrderedDict[tuple, int]" = OrderedDict()
_cache_lock = threading.RLock()


def _torch():
    import torch
    return torch


def handle(device: int = 0) -> int:
    with _cache_lock:
        if device not in _handles:
            _handles[device] = famlies_create(device)
        return _handles[device]


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return FAMLIES_F64
    if t.dtype == torch.float32:
        return FAMLIES_F32
    raise TypeError("famlies supports float64 and float32 tensors, got %s" % t.dtype)


def _compute_code(compute: str) -> int:
    if compute in ("native", None):
        return FAMLIES_NATIVE
    if compute == "bf16x3":
        return FAMLIES_BF16X3
    if compute == "bf16x6":
        return FAMLIES_BF16X6
    if compute in ("int8x3", "int8x4", "int8x5", "int8x6", "int8x7"):
        return FAMLIES_INT8X3 + int(compute[-1]) - 3
    raise ValueError("compute must be 'native', 'bf16x3', 'bf16x6' or 'int8x3'..'int8x7'")


def _labels(l) -> Tuple[int, ...]:
    return tuple(ord(c) for c in l) if isinstance(l, str) else tuple(int(x) for x in l)


def _evict_locked() -> None:
    torch = _torch()
    if len(_plan_cache) <= PLAN_CACHE_MAX:
        return
    if torch.cuda.is_available() and torch.cuda.is_current_stream_capturing():
        return  # a captured graph may still refer to any cached plan
    victims = []
    while len(_plan_cache) > PLAN_CACHE_MAX:
        key, p = _plan_cache.popitem(last=False)
        victims.append((key[0], p))
    for dev in {d for d, _ in victims}:
        torch.cuda.synchronize(dev)  # launches still queued may use the plans
    for _, p in victims:
        famlies_plan_destroy(p)


def plan_for(A, la, B, lb, C, lc, compute: str = "native", stream: int = 0) -> int:
    """Cached plan for tensors of these shapes, strides and labels, to be
    launched on `stream` (a raw stream handle)."""
    dev = C.device.index or 0
    key = (dev, int(stream), _dtype_code(C), _compute_code(compute),
           tuple(A.shape), tuple(A.stride()), _labels(la),
           tuple(B.shape), tuple(B.stride()), _labels(lb),
           tuple(C.shape), tuple(C.stride()), _labels(lc))
    with _cache_lock:
        p = _plan_cache.get(key)
        if p is not None:
            _plan_cache.move_to_end(key)
            return p
        p = famlies_plan_contract(handle(dev), key[2], key[3],
                                  make_desc(A.shape, A.stride(), la),
                                  make_desc(B.shape, B.stride(), lb),
                                  make_desc(C.shape, C.stride(), lc))
        _plan_cache[key] = p
        _evict_locked()
        return p


def clear_plan_cache() -> None:
    with _cache_lock:
        plans = list(_plan_cache.items())
        _plan_cache.clear()
    torch = _torch()
    for dev in {k[0] for k, _ in plans}:
        torch.cuda.synchronize(dev)
    for _, p in plans:
        famlies_plan_destroy(p)


def contract(alpha: float, A, la, B, lb, beta: float = 0.0, C=None, lc=None, *,
             compute: str = "native", stream=None):
    """C = alpha * sum A*B + beta * C over labelled modes (in place on C).

    ``A``, ``B``, ``C`` are CUDA (HIP) torch tensors of one dtype (float64 or
    float32) with any strides; ``la``, ``lb``, ``lc`` give one label per mode.
    If ``C`` is None a new dense tensor is allocated (its modes ordered as in
    ``lc``) and beta must be 0.  Runs asynchronously on ``stream`` (default:
    torch's current stream) and returns C."""
    torch = _torch()
    if lc is None:
        raise ValueError("lc (labels of C) is required")
    if C is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs an input C")
        ext = {}
        for t, l in ((A, la), (B, lb)):
            for ch, e in zip(_labels(l), t.shape):
                ext[ch] = e
        C = torch.empty([ext[ch] for ch in _labels(lc)], dtype=A.dtype, device=A.device)
    for t in (A, B, C):
        if t.device.type != "cuda":
            raise TypeError("famlies.contract needs GPU tensors (no CPU fallback)")
    if not (A.dtype == B.dtype == C.dtype):
        raise TypeError("A, B and C must share one dtype")
    s = stream if stream is not None else torch.cuda.current_stream(C.device)
    p = plan_for(A, la, B, lb, C, lc, compute, s.cuda_stream)
    famlies_execute(p, alpha, A.data_ptr(), B.data_ptr(), beta, C.data_ptr(), s.cuda_stream)
    return C


from .autograd import ContractFn, contract_ad  # noqa: E402

__all__ = [n for n in EXPORTS] + ["contract", "ContractFn", "contract_ad", "make_desc",
                                  "load_library", "FamliesError", "plan_for", "Network"]
