"""FP64 CPU oracle for the strided tensor contraction -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and never imports it.

The arithmetic lives in ``oracle.c`` (plain nested loops, FP64); this module
only compiles it with gcc and marshals numpy buffers through ctypes.  See the
header of ``oracle.c`` for the definition it writes out and its conventions.

A strided tensor is passed as ``(buf, base, extents, strides)``: ``buf`` is a
1-D float64 numpy array (the storage), ``base`` the element offset of the
all-zero multi-index inside it, and element ``idx`` lives at
``buf[base + sum(idx[d] * strides[d])]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, ERR_ARG, ERR_SHAPE, ERR_LABEL = 0, -1, -2, -3


class _Tensor(ctypes.Structure):
    _fields_ = [
        ("rank", ctypes.c_int32),
        ("extents", ctypes.POINTER(ctypes.c_int64)),
        ("strides", ctypes.POINTER(ctypes.c_int64)),
        ("labels", ctypes.POINTER(ctypes.c_int32)),
    ]


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile ``oracle.c`` into a shared library with gcc (always rebuilds
    unless ``force`` is False and the library exists)."""
    if not force and os.path.exists(out):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-std=c99", src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_lib_cache = {}


def load(path: Optional[str] = None) -> ctypes.CDLL:
    path = path or _LIB
    if path in _lib_cache:
        return _lib_cache[path]
    if not os.path.exists(path):
        if path != _LIB:
            raise FileNotFoundError(path)
        build()
    lib = ctypes.CDLL(path)
    tp = ctypes.POINTER(_Tensor)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_contract.argtypes = [ctypes.c_double, tp, dp, tp, dp, ctypes.c_double, tp, dp,
                                    dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_contract.restype = ctypes.c_int
    lib.oracle_contract_entries.argtypes = [
        ctypes.c_double, tp, dp, tp, dp, ctypes.c_double, tp, dp,
        ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, dp, dp,
        ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_contract_entries.restype = ctypes.c_int
    lib.oracle_bf16_rne.argtypes = [ctypes.POINTER(ctypes.c_float),
                                    ctypes.POINTER(ctypes.c_float), ctypes.c_int64]
    lib.oracle_bf16_rne.restype = None
    lib.oracle_int8_digits.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_int, ctypes.POINTER(ctypes.c_int8)]
    lib.oracle_int8_digits.restype = None
    _lib_cache[path] = lib
    return lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__("oracle returned %d" % code)
        self.code = code


def _desc(extents: Sequence[int], strides: Sequence[int], labels: Sequence[int]):
    r = len(extents)
    if len(strides) != r or len(labels) != r:
        raise ValueError("extents/strides/labels length mismatch")
    e = (ctypes.c_int64 * max(r, 1))(*[int(x) for x in extents])
    s = (ctypes.c_int64 * max(r, 1))(*[int(x) for x in strides])
    lab = (ctypes.c_int32 * max(r, 1))(*[int(x) for x in labels])
    t = _Tensor(r, e, s, lab)
    t._keep = (e, s, lab)
    return t


def _labels(lbl) -> list:
    if isinstance(lbl, str):
        return [ord(ch) for ch in lbl]
    return [int(x) for x in lbl]


def _base_ptr(buf: Optional[np.ndarray], base: int):
    if buf is None:
        return None
    if buf.dtype != np.float64 or not buf.flags.c_contiguous or buf.ndim != 1:
        raise TypeError("oracle buffers must be 1-D contiguous float64")
    addr = buf.ctypes.data + 8 * int(base)
    return ctypes.cast(ctypes.c_void_p(addr), ctypes.POINTER(ctypes.c_double))


def _threads(nthreads):
    if nthreads is None:
        try:
            return len(os.sched_getaffinity(0))
        except AttributeError:  # pragma: no cover
            return os.cpu_count() or 1
    return int(nthreads)


def contract(alpha: float,
             a: Tuple[np.ndarray, int, Sequence[int], Sequence[int]], la,
             b: Tuple[np.ndarray, int, Sequence[int], Sequence[int]], lb,
             beta: float,
             c: Tuple[np.ndarray, int, Sequence[int], Sequence[int]], lc,
             *, split=False, compensated: bool = True,
             want_cond: bool = False, nthreads: Optional[int] = None,
             lib: Optional[ctypes.CDLL] = None):
    """Return a new storage array holding C = alpha*A.B + beta*C0 (C0 = c's
    buffer, which is not modified), and the condition tensor D (same storage
    layout) when ``want_cond``.  ``split``: False / 0 exact products, True / 1
    the bf16x3 split, 2 the bf16x6 split, int8_slices(s) FP64 emulated on
    8-bit integer products with s slices (see oracle.c)."""
    lib = lib or load()
    abuf, abase, aext, astr = a
    bbuf, bbase, bext, bstr = b
    cbuf, cbase, cext, cstr = c
    ta = _desc(aext, astr, _labels(la))
    tb = _desc(bext, bstr, _labels(lb))
    tc = _desc(cext, cstr, _labels(lc))
    out = np.array(cbuf, dtype=np.float64, copy=True)
    d = np.zeros_like(out) if want_cond else None
    rc = lib.oracle_contract(float(alpha), ctypes.byref(ta), _base_ptr(abuf, abase),
                             ctypes.byref(tb), _base_ptr(bbuf, bbase), float(beta),
                             ctypes.byref(tc), _base_ptr(out, cbase),
                             _base_ptr(d, cbase) if want_cond else None,
                             int(split), int(bool(compensated)), _threads(nthreads))
    if rc != OK:
        raise OracleError(rc)
    return (out, d) if want_cond else out


def contract_entries(alpha: float, a, la, b, lb, beta: float, c, lc,
                     cidx: np.ndarray, *, split=False, compensated: bool = True,
                     want_cond: bool = False, nthreads: Optional[int] = None,
                     lib: Optional[ctypes.CDLL] = None):
    """Compute only the C entries whose multi-indices are the rows of
    ``cidx`` (shape n x rank(C)); returns a length-n array (and D)."""
    lib = lib or load()
    abuf, abase, aext, astr = a
    bbuf, bbase, bext, bstr = b
    cbuf, cbase, cext, cstr = c
    ta = _desc(aext, astr, _labels(la))
    tb = _desc(bext, bstr, _labels(lb))
    tc = _desc(cext, cstr, _labels(lc))
    idx = np.ascontiguousarray(cidx, dtype=np.int64)
    n = idx.shape[0]
    out = np.zeros(n, dtype=np.float64)
    d = np.zeros(n, dtype=np.float64) if want_cond else None
    rc = lib.oracle_contract_entries(
        float(alpha), ctypes.byref(ta), _base_ptr(abuf, abase), ctypes.byref(tb),
        _base_ptr(bbuf, bbase), float(beta), ctypes.byref(tc), _base_ptr(cbuf, cbase),
        idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n,
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if want_cond else None,
        int(split), int(bool(compensated)), _threads(nthreads))
    if rc != OK:
        raise OracleError(rc)
    return (out, d) if want_cond else out


INT8_BASE = 16


def int8_slices(s: int) -> int:
    """The ``split`` code of FP64 emulated on 8-bit integer products with s
    slices (1 <= s <= 12; see oracle.c)."""
    if not 1 <= int(s) <= 12:
        raise ValueError("slices must be in 1..12")
    return INT8_BASE + int(s)


def int8_digits(x: np.ndarray, e: int, s: int, lib: Optional[ctypes.CDLL] = None) -> np.ndarray:
    """The s signed digits of each x * 2^-e (|x * 2^-e| <= 127/128), rounded
    to nearest, shape x.shape + (s,), int8."""
    lib = lib or load()
    src = np.ascontiguousarray(x, dtype=np.float64).ravel()
    out = np.zeros(src.size * int(s), dtype=np.int8)
    lib.oracle_int8_digits(src.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), src.size, int(e), int(s),
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
    return out.reshape(np.shape(x) + (int(s),))


def bf16_rne(x: np.ndarray, lib: Optional[ctypes.CDLL] = None) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even); returned
    as float32."""
    lib = lib or load()
    src = np.ascontiguousarray(x, dtype=np.float32).ravel()
    dst = np.empty_like(src)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.oracle_bf16_rne(src.ctypes.data_as(fp), dst.ctypes.data_as(fp), src.size)
    return dst.reshape(np.shape(x))
