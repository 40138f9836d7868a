"""Helpers shared by the tests: run a synthetic problem through the C ABI and
through the oracle, and the error bounds used to compare them."""
from __future__ import annotations

import math

import numpy as np

import synth

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def gamma(n: int, u: float) -> float:
    """Higham's gamma_n = n u / (1 - n u)."""
    return n * u / (1.0 - n * u)


def np_dtype(dtype: str):
    return {"f64": np.float64, "f32": np.float32}[dtype]


def round_inputs(p: synth.Problem, dtype: str) -> synth.Problem:
    """Round the problem's buffers to the element type (the oracle then sees
    the exact values the GPU sees)."""
    t = np_dtype(dtype)
    for name in ("abuf", "bbuf", "cbuf"):
        buf = getattr(p, name)
        if buf is not None:
            setattr(p, name, buf.astype(t).astype(np.float64))
    return p


def oracle_full(p: synth.Problem, alpha=None, beta=None, split=False):
    import oracle
    a, la, b, lb, c, lc = p.oracle_args()
    al = p.alpha if alpha is None else alpha
    be = p.beta if beta is None else beta
    return oracle.contract(al, a, la, b, lb, be, c, lc, split=split, want_cond=True)


def used_offsets(lay: synth.Strided) -> np.ndarray:
    """Storage offsets of every element of a layout, in column-major
    multi-index order."""
    off = np.full((1,), lay.base, dtype=np.int64)
    for e, s in zip(lay.extents, lay.strides):
        off = (np.arange(e, dtype=np.int64)[:, None] * s + off[None, :]).ravel()
    return off


class DeviceRunner:
    """Runs problems through the C ABI on cuda:0 with flat device buffers,
    so any strides (negative, zero, padded) can be used."""

    def __init__(self):
        import torch
        import paper_2604_07311_amd as fm
        self.torch = torch
        self.fm = fm
        self.h = fm.handle(0)

    def plan(self, p: synth.Problem, dtype: str, compute: str = "native"):
        fm = self.fm
        code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
        comp = fm._compute_code(compute)
        return fm.famlies_plan_contract(self.h, code, comp,
                                        fm.make_desc(p.a.extents, p.a.strides, p.la),
                                        fm.make_desc(p.b.extents, p.b.strides, p.lb),
                                        fm.make_desc(p.c.extents, p.c.strides, p.lc))

    def to_dev(self, buf: np.ndarray, dtype: str):
        t = self.torch.from_numpy(np.ascontiguousarray(buf.astype(np_dtype(dtype))))
        return t.to("cuda:0")

    def run(self, p: synth.Problem, dtype: str, compute: str = "native", alpha=None, beta=None,
            plan=None, keep=False):
        """Returns the whole C storage buffer after the call (float64 numpy)."""
        torch, fm = self.torch, self.fm
        es = 8 if dtype == "f64" else 4
        own = plan is None
        if own:
            plan = self.plan(p, dtype, compute)
        try:
            a = self.to_dev(p.abuf, dtype)
            b = self.to_dev(p.bbuf, dtype)
            c = self.to_dev(p.cbuf, dtype)
            al = p.alpha if alpha is None else alpha
            be = p.beta if beta is None else beta
            s = torch.cuda.current_stream()
            fm.famlies_execute(plan, al, a.data_ptr() + es * p.a.base, b.data_ptr() + es * p.b.base,
                               be, c.data_ptr() + es * p.c.base, s.cuda_stream)
            torch.cuda.synchronize()
            return c.cpu().numpy().astype(np.float64)
        finally:
            if own:
                fm.famlies_plan_destroy(plan)


def check_fp64(got: np.ndarray, want: np.ndarray, d: np.ndarray, K: int, where=None):
    """FP64 path: normwise relative error <= 1e-12 and componentwise
    |err| <= gamma_{K+2}(2^-53) * D."""
    idx = slice(None) if where is None else where
    g, w, dd = got[idx], want[idx], d[idx]
    nrm = np.linalg.norm(w)
    err = np.linalg.norm(g - w)
    assert err <= 1e-12 * nrm + 1e-300, "normwise %.3e" % (err / max(nrm, 1e-300))
    bound = gamma(K + 2, U64) * dd
    bad = np.abs(g - w) > bound
    assert not bad.any(), "componentwise bound violated at %d entries" % bad.sum()
    return err / max(nrm, 1e-300)


def check_fp32(got, want, d, K, where=None):
    """FP32 path: componentwise |err| <= gamma_{K+4}(2^-24) * D (K+2 for the
    dot products and the alpha/beta update, +2 for rounding alpha, beta and
    the final store)."""
    idx = slice(None) if where is None else where
    g, w, dd = got[idx], want[idx], d[idx]
    bound = gamma(K + 4, U32) * dd
    bad = np.abs(g - w) > bound
    assert not bad.any(), "componentwise bound violated at %d entries (max ratio %.3g)" % (
        bad.sum(), np.max(np.abs(g - w) / np.maximum(bound, 1e-300)))
    nrm = np.linalg.norm(w)
    return np.linalg.norm(g - w) / max(nrm, 1e-300)


def bf16x3_bound(K: int, d_prod: np.ndarray, d: np.ndarray) -> np.ndarray:
    """bf16x3 against the exact FP64 result: the dropped lo*lo term costs at
    most 3*2^-16*(1+2^-8) |a||b| per product; FP32 accumulation of the 2 split
    sums is bounded with u = 2^-23 (no assumption that the MFMA accumulator
    rounds to nearest); the FP64 epilogue and the FP32 store add 2^-23 * D.
    d_prod = |alpha| sum |a||b| (D without the beta term)."""
    return (3.0 * 2.0 ** -16 * (1 + 2.0 ** -8) + gamma(K, 2.0 ** -23) * (1 + 2.0 ** -7)) * d_prod \
        + 2.0 ** -23 * d
