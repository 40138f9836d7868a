"""Seeded synthetic inputs for the strided tensor contraction.

This module is shared by the oracle tests and the HIP-path tests/benchmark.
It holds no contraction arithmetic: it only draws storage layouts (extents,
strides, padding, storage orders) and element values from seeded numpy
generators, so the same seed gives the same tensors to both sides.

The workloads are the coupled-cluster-shaped contractions the paper's
quantum-chemistry motivation points at (Introduction, "Project Motivation";
Approach, "Supporting tensor computations"); the paper ships no data, so all
values are synthetic.

A tensor is described by a :class:`Strided` layout plus a flat float64 value
buffer ``buf``; element ``idx`` lives at ``buf[base + sum(idx[d]*strides[d])]``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np


@dataclass
class Strided:
    extents: List[int]
    strides: List[int]
    base: int
    size: int          # number of storage elements the buffer must hold

    @property
    def rank(self) -> int:
        return len(self.extents)


def layout(extents: Sequence[int], order: Optional[Sequence[int]] = None,
           pad: Optional[Sequence[int]] = None, fast_stride: int = 1,
           negate: Optional[Sequence[bool]] = None,
           zero: Optional[Sequence[bool]] = None) -> Strided:
    """Dense-with-padding storage.  ``order`` lists the modes from fastest to
    slowest (default: column-major, mode 0 fastest); ``pad[d]`` extra
    elements are left after each run of mode d; the fastest mode has stride
    ``fast_stride``.  ``negate[d]`` flips the sign of mode d's stride (the base
    moves so every element stays inside the buffer); ``zero[d]`` gives mode d
    stride 0 (broadcast; only meaningful for read-only operands)."""
    r = len(extents)
    order = list(range(r)) if order is None else list(order)
    pad = [0] * r if pad is None else list(pad)
    strides = [0] * r
    s = int(fast_stride)
    for d in order:
        strides[d] = s
        s *= max(int(extents[d]) + int(pad[d]), 1)
    if zero is not None:
        for d in range(r):
            if zero[d]:
                strides[d] = 0
    if negate is not None:
        for d in range(r):
            if negate[d]:
                strides[d] = -strides[d]
    base = sum(max(-st, 0) * max(int(e) - 1, 0) for st, e in zip(strides, extents))
    top = base + sum(max(st, 0) * max(int(e) - 1, 0) for st, e in zip(strides, extents))
    size = top + 1
    return Strided([int(e) for e in extents], strides, int(base), int(size))


def values(rng: np.random.Generator, n: int, dist: str) -> np.ndarray:
    """Flat float64 values.  ``uniform``: U[-1,1].  ``normal``: N(0,1).
    ``outliers``: N(0,1) with an i.i.d. Bernoulli(1e-3) mask scaled by 1e4.
    ``int``: integers uniform on [-8, 8] (all partial sums exact in FP32)."""
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, size=n)
    if dist == "normal":
        return rng.standard_normal(size=n)
    if dist == "outliers":
        x = rng.standard_normal(size=n)
        mask = rng.random(size=n) < 1e-3
        x[mask] *= 1e4
        return x
    if dist == "int":
        return rng.integers(-8, 9, size=n).astype(np.float64)
    if dist == "ones":
        return np.ones(n)
    raise ValueError(dist)


def fill(rng: np.random.Generator, lay: Strided, dist: str, dtype=np.float64) -> np.ndarray:
    """A storage buffer for ``lay``; padding elements get values too (they
    must never be read, and NaN there would show it: see ``poison``)."""
    buf = values(rng, lay.size, dist)
    return buf.astype(dtype)


def poison_padding(buf: np.ndarray, lay: Strided, value=np.nan) -> np.ndarray:
    """Set every storage element that no multi-index addresses to ``value``
    (used to show that padding is never read)."""
    used = np.zeros(buf.shape[0], dtype=bool)
    if all(e > 0 for e in lay.extents):
        off = np.full((1,), lay.base, dtype=np.int64)
        for e, s in zip(lay.extents, lay.strides):
            off = (off[:, None] + np.arange(e, dtype=np.int64)[None, :] * s).ravel()
        used[off] = True
    out = buf.copy()
    out[~used] = value
    return out


@dataclass
class Problem:
    """One labelled contraction C = alpha*A.B + beta*C0 with its data."""
    name: str
    la: str
    lb: str
    lc: str
    a: Strided
    b: Strided
    c: Strided
    alpha: float
    beta: float
    abuf: Optional[np.ndarray] = None
    bbuf: Optional[np.ndarray] = None
    cbuf: Optional[np.ndarray] = None
    meta: Dict = field(default_factory=dict)

    def oracle_args(self):
        return ((self.abuf, self.a.base, self.a.extents, self.a.strides), self.la,
                (self.bbuf, self.b.base, self.b.extents, self.b.strides), self.lb,
                (self.cbuf, self.c.base, self.c.extents, self.c.strides), self.lc)


def _ext(labels: str, dims: Dict[str, int]) -> List[int]:
    return [dims[ch] for ch in labels]


def plain16(seed: int = 1, dist: str = "uniform", n: int = 16, with_data: bool = True) -> Problem:
    """C[a,b,i,j] = sum_{e,f} A[a,e,i,f] B[e,b,f,j], every extent ``n``,
    dense column-major, alpha=1, beta=0.5."""
    dims = {ch: n for ch in "abijef"}
    p = Problem("plain%d" % n, "aeif", "ebfj", "abij",
                layout(_ext("aeif", dims)), layout(_ext("ebfj", dims)),
                layout(_ext("abij", dims)), 1.0, 0.5)
    if with_data:
        rng = np.random.default_rng(seed)
        p.abuf, p.bbuf, p.cbuf = (fill(rng, t, dist) for t in (p.a, p.b, p.c))
    return p


def ladder(v: int, o: int, seed: int = 2, dist: str = "uniform", c_dist: Optional[str] = None,
           with_data: bool = True, dtype=np.float64) -> Problem:
    """Particle-particle ladder C[a,b,i,j] += sum_{e,f} W[a,b,e,f] T[e,f,i,j].
    W is stored dense column-major in mode order (e,a,f,b), so no index order
    of it is contiguous for a plain GEMM; T and C are dense column-major.
    alpha = beta = 1."""
    dims = {"a": v, "b": v, "e": v, "f": v, "i": o, "j": o}
    # W[a,b,e,f]: storage order e (fastest), a, f, b
    w = layout(_ext("abef", dims), order=[2, 0, 3, 1])
    t = layout(_ext("efij", dims))
    c = layout(_ext("abij", dims))
    p = Problem("ladder_v%d_o%d" % (v, o), "abef", "efij", "abij", w, t, c, 1.0, 1.0,
                meta={"v": v, "o": o})
    if with_data:
        rng = np.random.default_rng(seed)
        cd = c_dist or ("normal" if dist == "outliers" else dist)
        p.abuf = fill_chunked(rng, w.size, dist, dtype)
        p.bbuf = fill_chunked(rng, t.size, dist, dtype)
        p.cbuf = fill_chunked(rng, c.size, cd, dtype)
    return p


def ring(o: int, v: int, seed: int = 4, dist: str = "outliers", with_data: bool = True,
         dtype=np.float64) -> Problem:
    """Ring term C[a,i,b,j] = sum_{k,c} X[a,k,i,c] Y[c,b,k,j], all dense
    column-major, a,b,c virtual (v) and i,j,k occupied (o); alpha=1, beta=0."""
    dims = {"a": v, "b": v, "c": v, "i": o, "j": o, "k": o}
    x = layout(_ext("akic", dims))
    y = layout(_ext("cbkj", dims))
    c = layout(_ext("aibj", dims))
    p = Problem("ring_o%d_v%d" % (o, v), "akic", "cbkj", "aibj", x, y, c, 1.0, 0.0,
                meta={"v": v, "o": o})
    if with_data:
        rng = np.random.default_rng(seed)
        p.abuf = fill_chunked(rng, x.size, dist, dtype)
        p.bbuf = fill_chunked(rng, y.size, dist, dtype)
        p.cbuf = fill_chunked(rng, c.size, "normal", dtype)
    return p


def autograd_case(o: int, v: int, seed: int = 6, with_data: bool = True) -> Problem:
    """C[a,b,i,j] = sum_{e,f} A[a,e,i,f] B[e,b,f,j] with a,b,e,f virtual (v)
    and i,j occupied (o); A, B uniform[-1,1], alpha=1, beta=0.  ``meta['G']``
    holds the upstream gradient G ~ N(0,1) in C's dense layout."""
    dims = {"a": v, "b": v, "e": v, "f": v, "i": o, "j": o}
    p = Problem("autograd_o%d_v%d" % (o, v), "aeif", "ebfj", "abij",
                layout(_ext("aeif", dims)), layout(_ext("ebfj", dims)),
                layout(_ext("abij", dims)), 1.0, 0.0, meta={"v": v, "o": o})
    if with_data:
        rng = np.random.default_rng(seed)
        p.abuf = fill(rng, p.a, "uniform")
        p.bbuf = fill(rng, p.b, "uniform")
        p.cbuf = np.zeros(p.c.size)
        p.meta["G"] = fill(rng, p.c, "normal")
    return p


def fill_chunked(rng: np.random.Generator, n: int, dist: str, dtype, chunk: int = 1 << 26):
    """Like :func:`fill` but generated in chunks straight into ``dtype`` so a
    multi-GB float32 tensor never exists in float64."""
    out = np.empty(n, dtype=dtype)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        out[s:e] = values(rng, e - s, dist)
    return out


# ---------------------------------------------------------------- batched
LABEL_POOL = "abcdefghijklmnopqrstuvwxyz"


def random_problem(rng: np.random.Generator, lo: int = 4, hi: int = 48,
                   n_i: int = 2, n_j: int = 2, n_p: int = 2, pad_hi: int = 3,
                   p_stride2: float = 0.25, alpha: float = 1.0, beta: float = 0.5) -> Problem:
    """One random labelled contraction: ``n_i`` labels in A and C only,
    ``n_j`` in B and C only, ``n_p`` in A and B only, each extent uniform on
    {lo..hi}.  Each tensor's mode order is a random permutation, and its
    storage is dense in a second random permutation with per-mode padding
    uniform on {0..pad_hi} and a fastest stride of 1 (prob. 3/4) or 2."""
    labs = list(rng.choice(list(LABEL_POOL), size=n_i + n_j + n_p, replace=False))
    I, J, P = labs[:n_i], labs[n_i:n_i + n_j], labs[n_i + n_j:]
    dims = {ch: int(rng.integers(lo, hi + 1)) for ch in labs}

    def mk(modes):
        modes = list(rng.permutation(modes))
        ext = [dims[ch] for ch in modes]
        order = list(rng.permutation(len(modes)))
        pad = [int(rng.integers(0, pad_hi + 1)) for _ in modes]
        fs = 2 if rng.random() < p_stride2 else 1
        return "".join(modes), layout(ext, order=order, pad=pad, fast_stride=fs)

    la, a = mk(I + P)
    lb, b = mk(P + J)
    lc, c = mk(I + J)
    return Problem("rand", la, lb, lc, a, b, c, alpha, beta, meta={"dims": dims})


def batched(n: int, seed: int = 5, lo: int = 4, hi: int = 48, with_data: bool = False,
            dist: str = "uniform") -> List[Problem]:
    """``n`` independent random 4-index contractions (see
    :func:`random_problem`), alpha=1, beta=0.5."""
    rng = np.random.default_rng(seed)
    probs = [random_problem(rng, lo, hi) for _ in range(n)]
    if with_data:
        for p in probs:
            p.abuf, p.bbuf, p.cbuf = (fill(rng, t, dist) for t in (p.a, p.b, p.c))
    return probs


def sizes(p: Problem):
    """(M, N, K) of a classical contraction: products of the extents of the
    labels in A&C, B&C and A&B respectively."""
    ea = dict(zip(p.la, p.a.extents))
    eb = dict(zip(p.lb, p.b.extents))
    M = N = K = 1
    for ch, e in ea.items():
        if ch in p.lc:
            M *= e
        elif ch in p.lb:
            K *= e
    for ch, e in eb.items():
        if ch in p.lc and ch not in p.la:
            N *= e
    return M, N, K
