"""Pins for the oracle's FP64 emulation on 8-bit integer products (CPU only).

The oracle (``split = oracle.int8_slices(s)``) scales each row of A's and
each column of B's GEMM view by a power of two into [-127/128, 127/128],
cuts the scaled values into s signed digits by exact rounding to nearest in
base 2^7, sums the digit products of the pairs (t, u) with t + u <= s + 1 as
exact integers and recombines them in FP64.  Each check ties it to something
other than itself: an exact-rational re-implementation of those steps
written here with ``fractions``, integer inputs (where one digit is exact and
the emulation must equal the plain contraction bit for bit), a closed form
with a Kronecker-delta operand (the emulation then returns A rounded to the
nearest multiple of 2^-7s of its row scale), power-of-two scaling, and the
error bound against the exact FP64 contraction."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from tests.brute import enumerate_contraction
from tests.test_oracle import _random_roles_problem


def _exp(vmax):
    """Smallest integer e with vmax <= (127/128) 2^e (0 for 0), from the
    definition."""
    if vmax == 0:
        return 0
    lim = Fraction(127, 128)
    e = 0
    while Fraction(vmax) > lim * Fraction(2) ** e:
        e += 1
    while Fraction(vmax) <= lim * Fraction(2) ** (e - 1):
        e -= 1
    return e


def _rne(w):
    """Nearest integer to the rational w, ties to the even one."""
    q = math.floor(w + Fraction(1, 2))
    if w + Fraction(1, 2) == q and q % 2:
        q -= 1
    return q


def _digits(x, e, s):
    """Digits of v = x 2^-e on exact rationals: repeatedly the nearest
    integer to 128 times the remainder."""
    v = Fraction(x) / Fraction(2) ** e
    assert abs(v) <= Fraction(127, 128)
    out = []
    for _ in range(s):
        v *= 128
        q = _rne(v)
        out.append(q)
        v -= q
    return out


def _brute_int8(alpha, a, la, b, lb, beta, c, lc, s):
    """Exact-rational emulation of every C entry (independent of oracle.c):
    rows and columns found by enumerating all label assignments."""
    abuf, abase, aext, astr = a
    bbuf, bbase, bext, bstr = b
    cbuf, cbase, cext, cstr = c
    ext = {}
    for labs, exts in ((lc, cext), (la, aext), (lb, bext)):
        for ch, e in zip(labs, exts):
            ext[ch] = e
    summed = sorted(set(la + lb) - set(lc))
    out = [float(x) for x in cbuf]
    for cvals in itertools.product(*[range(ext[ch]) for ch in lc]):
        fixed = dict(zip(lc, cvals))
        pairs = []
        for svals in itertools.product(*[range(ext[ch]) for ch in summed]):
            v = dict(fixed, **dict(zip(summed, svals)))
            ia = abase + sum(v[ch] * st for ch, st in zip(la, astr))
            ib = bbase + sum(v[ch] * st for ch, st in zip(lb, bstr))
            pairs.append((float(abuf[ia]), float(bbuf[ib])))
        ic = cbase + sum(x * st for x, st in zip(cvals, cstr))
        ea = _exp(max([abs(x) for x, _ in pairs], default=0.0))
        eb = _exp(max([abs(y) for _, y in pairs], default=0.0))
        S = {}
        for x, y in pairs:
            dx, dy = _digits(x, ea, s), _digits(y, eb, s)
            for t in range(1, s + 1):
                for u in range(1, s + 2 - t):
                    S[(t, u)] = S.get((t, u), 0) + dx[t - 1] * dy[u - 1]
        prod = sum((Fraction(S[k]) / Fraction(2) ** (7 * (k[0] + k[1])) for k in S), Fraction(0))
        prod *= Fraction(2) ** (ea + eb)
        r = 0.0 if alpha == 0 else float(Fraction(alpha) * prod)
        if beta != 0:
            r = r + beta * float(cbuf[ic])
        out[ic] = r
    return np.array(out)


def test_digits_definition(oracle_lib):
    rng = np.random.default_rng(11)
    ties = [(2 * k + 1) * 2.0 ** -8 for k in range(-63, 63)]   # v 2^7 = half-integers
    x = np.concatenate([rng.uniform(-1, 1, 300) * (127 / 128), ties,
                        [0.0, -0.0, 0.5, -0.5, 2.0 ** -30, 127 / 128, -127 / 128, 3 * 2.0 ** -15]])
    for s in (1, 3, 7, 9):
        d = oracle.int8_digits(x, 0, s)
        for i, xi in enumerate(x):
            assert list(d[i]) == _digits(xi, 0, s)
        assert np.all(np.abs(d[:, 0]) <= 127) and np.all(np.abs(d[:, 1:]) <= 64)
        # v = sum d_t 2^-7t + remainder, |remainder| <= 2^-7s / 2
        rec = (d.astype(np.float64) * 2.0 ** (-7 * np.arange(1, s + 1))).sum(axis=1)
        assert np.all(np.abs(x - rec) <= 2.0 ** (-7 * s - 1))
    # scaled rows: x 2^-e
    y = rng.uniform(-6, 6, 50)
    d = oracle.int8_digits(y, 3, 4)
    for i, yi in enumerate(y):
        assert list(d[i]) == _digits(yi, 3, 4)


@pytest.mark.parametrize("seed", range(16))
def test_bruteforce_exact_rational(oracle_lib, seed):
    """General labels (batch, summed inside one input, diagonals, negative,
    zero and padded strides) against the exact-rational re-implementation;
    the oracle's FP64 recombination may differ by rounding only."""
    rng = np.random.default_rng(2000 + seed)
    la, a, lb, b, lc, c = _random_roles_problem(rng)
    dist = ["uniform", "normal", "outliers", "uniform"][seed % 4]
    abuf = synth.values(rng, a.size, dist) * float(2.0 ** rng.integers(-8, 9))
    bbuf = synth.values(rng, b.size, dist)
    cbuf = synth.values(rng, c.size, "uniform")
    s = [2, 3, 5, 7][seed % 4]
    alpha, beta = [(1.0, 0.5), (-1.5, 0.0), (0.0, 2.0), (1.0, 1.0)][seed % 4]
    A, B, C = (abuf, a.base, a.extents, a.strides), (bbuf, b.base, b.extents, b.strides), \
        (cbuf, c.base, c.extents, c.strides)
    got, d = oracle.contract(alpha, A, la, B, lb, beta, C, lc, split=oracle.int8_slices(s), want_cond=True)
    want = _brute_int8(alpha, A, la, B, lb, beta, C, lc, s)
    used = synth_used(c)
    assert np.all(np.abs(got[used] - want[used]) <= 4 * 2.0 ** -53 * (np.abs(want[used]) + d[used]) + 1e-300)
    # storage outside C's elements untouched
    mask = np.ones(len(cbuf), bool)
    mask[used] = False
    np.testing.assert_array_equal(got[mask], cbuf[mask])


def synth_used(lay):
    off = np.full((1,), lay.base, dtype=np.int64)
    for e, st in zip(lay.extents, lay.strides):
        off = (np.arange(e, dtype=np.int64)[:, None] * st + off[None, :]).ravel()
    return off


@pytest.mark.parametrize("seed", range(12))
def test_integer_inputs_exact(oracle_lib, seed):
    """Integers in [-8, 8]: after scaling each value is one exact digit, so
    for every s the emulation equals the plain contraction bit for bit."""
    rng = np.random.default_rng(3000 + seed)
    la, a, lb, b, lc, c = _random_roles_problem(rng)
    A = (synth.values(rng, a.size, "int"), a.base, a.extents, a.strides)
    B = (synth.values(rng, b.size, "int"), b.base, b.extents, b.strides)
    C = (synth.values(rng, c.size, "int"), c.base, c.extents, c.strides)
    plain = np.array(enumerate_contraction(1.0, A, la, B, lb, 0.5, C, lc))
    for s in (1, 2, 7):
        got = oracle.contract(1.0, A, la, B, lb, 0.5, C, lc, split=oracle.int8_slices(s))
        np.testing.assert_array_equal(got, plain)


def test_kronecker_closed_form(oracle_lib):
    """B[e,b,f,j] = delta(e,b) delta(f,j): every column of B's view holds one
    1 (scale 2^1, digit 64), so the emulation returns each A entry rounded to
    the nearest multiple of 2^-7s of its row's scale 2^ea (ties to even):
    C[a,b,i,j] = alpha 2^(ea-7s) rint(A[a,b,i,j] 2^(7s-ea)) + beta C0, with
    ea the smallest e such that the row's max|A| <= (127/128) 2^e."""
    n = 4
    rng = np.random.default_rng(17)
    p = synth.plain16(seed=17, n=n)
    abuf = synth.values(rng, p.a.size, "outliers")
    A4w = abuf.reshape((n,) * 4, order="F")              # a view: writes go to abuf
    A4w[1, 2, 0, 3] = 0.999 * 8 * np.sign(A4w[1, 2, 0, 3]) * max(1.0, np.abs(A4w[1, :, 0, :]).max() / 8)
    A4w[3, :, 2, :] = A4w[3, :, 2, :] / np.abs(A4w[3, :, 2, :]).max() * (255 / 256)   # row max in (127/128, 1)
    bbuf = np.zeros(p.b.size)
    for e in range(n):
        for f in range(n):
            bbuf[p.b.base + e * p.b.strides[0] + e * p.b.strides[1] + f * p.b.strides[2]
                 + f * p.b.strides[3]] = 1.0
    cbuf = synth.values(rng, p.c.size, "uniform")
    A4 = abuf.reshape((n,) * 4, order="F")            # A[a,e,i,f]
    C0 = cbuf.reshape((n,) * 4, order="F")
    for s in (1, 2, 4):
        out = oracle.contract(1.0, (abuf, 0, p.a.extents, p.a.strides), "aeif",
                              (bbuf, 0, p.b.extents, p.b.strides), "ebfj", 0.5,
                              (cbuf, 0, p.c.extents, p.c.strides), "abij", split=oracle.int8_slices(s))
        want = np.empty((n,) * 4)
        for a_ in range(n):
            for i in range(n):
                row = A4[a_, :, i, :]
                ea = _exp(float(np.abs(row).max()))
                for b_ in range(n):
                    for j in range(n):
                        t = math.ldexp(float(np.rint(math.ldexp(float(A4[a_, b_, i, j]), 7 * s - ea))),
                                       ea - 7 * s)
                        want[a_, b_, i, j] = t + 0.5 * C0[a_, b_, i, j]
        np.testing.assert_array_equal(out.reshape((n,) * 4, order="F"), want)


def test_power_of_two_scaling(oracle_lib):
    """Scaling A by 2^k moves every row scale by k: results scale exactly."""
    p = synth.plain16(seed=19, n=6)
    rng = np.random.default_rng(19)
    abuf = synth.values(rng, p.a.size, "normal")
    bbuf = synth.values(rng, p.b.size, "normal")
    c = (np.zeros(p.c.size), 0, p.c.extents, p.c.strides)
    split = oracle.int8_slices(5)
    r0 = oracle.contract(1.0, (abuf, 0, p.a.extents, p.a.strides), p.la,
                         (bbuf, 0, p.b.extents, p.b.strides), p.lb, 0.0, c, p.lc, split=split)
    for k in (-40, -3, 5, 60):
        rk = oracle.contract(1.0, (abuf * 2.0 ** k, 0, p.a.extents, p.a.strides), p.la,
                             (bbuf, 0, p.b.extents, p.b.strides), p.lb, 0.0, c, p.lc, split=split)
        np.testing.assert_array_equal(rk, r0 * 2.0 ** k)


def test_error_bound_and_convergence(oracle_lib):
    """Against the exact FP64 contraction: each product is off by at most
    (s+4)/4 2^-7s 2^(ea+eb) (rounded digits: 2^-7s-1 per operand; dropped
    pairs: s-1 products of two digits <= 64 at weight 2^-7(s+2)), plus FP64
    rounding; and each extra slice shrinks the error by about 2^7."""
    p = synth.plain16(seed=23, n=8)
    rng = np.random.default_rng(23)
    abuf = synth.values(rng, p.a.size, "outliers")
    bbuf = synth.values(rng, p.b.size, "normal")
    A = (abuf, 0, p.a.extents, p.a.strides)
    B = (bbuf, 0, p.b.extents, p.b.strides)
    C = (np.zeros(p.c.size), 0, p.c.extents, p.c.strides)
    exact, d = oracle.contract(1.0, A, p.la, B, p.lb, 0.0, C, p.lc, want_cond=True)
    # row and column scales of the GEMM view: A[a,e,i,f] rows (a,i), B[e,b,f,j] columns (b,j)
    n = 8
    A4 = abuf.reshape((n,) * 4, order="F")
    B4 = bbuf.reshape((n,) * 4, order="F")
    ea = np.array([[_exp(float(np.abs(A4[a_, :, i, :]).max())) for i in range(n)] for a_ in range(n)])
    eb = np.array([[_exp(float(np.abs(B4[:, b_, :, j]).max())) for j in range(n)] for b_ in range(n)])
    scale = np.exp2(ea[:, None, :, None] + eb[None, :, None, :]).reshape(-1, order="F")   # C[a,b,i,j]
    K = n * n
    errs = []
    for s in (2, 3, 4, 5, 6, 7):
        got = oracle.contract(1.0, A, p.la, B, p.lb, 0.0, C, p.lc, split=oracle.int8_slices(s))
        err = np.abs(got - exact)
        bound = K * (s + 4) / 4 * 2.0 ** (-7 * s) * scale + 8 * 2.0 ** -53 * (d + np.abs(exact))
        assert np.all(err <= bound), s
        errs.append(np.linalg.norm(got - exact))
    for e0, e1 in zip(errs[:-2], errs[1:-1]):
        assert e1 < e0 / 32
    assert errs[-1] <= 1e-12 * np.linalg.norm(exact)


def test_nonfinite_rows_give_nan(oracle_lib):
    n = 3
    p = synth.plain16(seed=29, n=n)
    rng = np.random.default_rng(29)
    abuf = synth.values(rng, p.a.size, "uniform")
    bbuf = synth.values(rng, p.b.size, "uniform")
    abuf[p.a.base] = np.inf  # A[0,0,0,0]: the row (a=0, i=0)
    out = oracle.contract(1.0, (abuf, 0, p.a.extents, p.a.strides), "aeif",
                          (bbuf, 0, p.b.extents, p.b.strides), "ebfj", 0.0,
                          (np.zeros(p.c.size), 0, p.c.extents, p.c.strides), "abij",
                          split=oracle.int8_slices(3)).reshape((n,) * 4, order="F")
    assert np.all(np.isnan(out[0, :, 0, :]))
    mask = np.ones_like(out, bool)
    mask[0, :, 0, :] = False
    assert np.all(np.isfinite(out[mask]))


def test_bad_slice_counts(oracle_lib):
    p = synth.plain16(seed=1, n=2)
    args = p.oracle_args()
    for bad in (3, 15, 16, 29, -1):
        with pytest.raises(oracle.OracleError):
            oracle.contract(1.0, *args[:4], 0.0, *args[4:], split=bad)
    with pytest.raises(ValueError):
        oracle.int8_slices(0)
