"""Pins for the FP64 oracle (CPU only).  Each check ties the oracle to
something other than itself: a pure-Python enumerator, closed forms, a
library routine (numpy matmul after an explicit permutation, torch's bf16
rounding), or an algebraic invariant.  ``test_oracle_mutants.py`` shows that
plausible mistakes in the oracle fail these checks."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests.brute import enumerate_contraction

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random_roles_problem(rng, allow_general=True, max_ext=3):
    """A tiny problem with random label roles, strides and padding."""
    roles = ["I", "J", "P"]
    if allow_general:
        roles += ["batch", "traceA", "traceB"]
    nlab = int(rng.integers(1, 6))
    labs = list("abcdefgh"[:nlab])
    role = {ch: roles[int(rng.integers(0, len(roles)))] for ch in labs}
    ext = {ch: int(rng.integers(0 if rng.random() < 0.1 else 1, max_ext + 1)) for ch in labs}
    la = [ch for ch in labs if role[ch] in ("I", "P", "batch", "traceA")]
    lb = [ch for ch in labs if role[ch] in ("J", "P", "batch", "traceB")]
    lc = [ch for ch in labs if role[ch] in ("I", "J", "batch")]
    if allow_general and la and rng.random() < 0.3:
        la.append(la[int(rng.integers(0, len(la)))])   # a diagonal in A
    for lst in (la, lb, lc):
        rng.shuffle(lst)

    def lay(modes, inp):
        n = len(modes)
        order = list(rng.permutation(n))
        pad = [int(rng.integers(0, 2)) for _ in range(n)]
        neg = [bool(rng.random() < 0.3) for _ in range(n)]
        zero = [inp and bool(rng.random() < 0.15) for _ in range(n)]
        return synth.layout([ext[ch] for ch in modes], order=order, pad=pad,
                            fast_stride=int(rng.integers(1, 3)), negate=neg, zero=zero)

    a, b, c = lay(la, True), lay(lb, True), lay(lc, False)
    return "".join(la), a, "".join(lb), b, "".join(lc), c


@pytest.mark.parametrize("seed", range(60))
def test_bruteforce_integer_exact(oracle_lib, seed):
    """Integer inputs: every partial sum is exact, so the oracle must equal
    the independent enumerator bit for bit, whatever the order of summation."""
    rng = np.random.default_rng(1000 + seed)
    la, a, lb, b, lc, c = _random_roles_problem(rng)
    abuf = synth.values(rng, a.size, "int")
    bbuf = synth.values(rng, b.size, "int")
    cbuf = synth.values(rng, c.size, "int")
    alpha, beta = [(1.0, 0.5), (-2.0, 0.0), (0.0, 3.0), (1.0, 1.0)][seed % 4]
    A, B, C = (abuf, a.base, a.extents, a.strides), (bbuf, b.base, b.extents, b.strides), \
        (cbuf, c.base, c.extents, c.strides)
    got = oracle.contract(alpha, A, la, B, lb, beta, C, lc)
    want = enumerate_contraction(alpha, A, la, B, lb, beta, C, lc)
    np.testing.assert_array_equal(got, np.array(want))


@pytest.mark.parametrize("seed", range(20))
def test_bruteforce_real(oracle_lib, seed):
    """Real inputs: equal to the enumerator within the textbook bound for
    recursive summation, |err| <= gamma_{n+2} * D (Higham, gamma_n = nu/(1-nu))."""
    rng = np.random.default_rng(2000 + seed)
    la, a, lb, b, lc, c = _random_roles_problem(rng, max_ext=4)
    abuf, bbuf, cbuf = (synth.values(rng, t.size, "uniform") for t in (a, b, c))
    A, B, C = (abuf, a.base, a.extents, a.strides), (bbuf, b.base, b.extents, b.strides), \
        (cbuf, c.base, c.extents, c.strides)
    got, d = oracle.contract(0.75, A, la, B, lb, -0.25, C, lc, want_cond=True)
    want = np.array(enumerate_contraction(0.75, A, la, B, lb, -0.25, C, lc))
    n = 4 ** 6 + 2
    u = 2.0 ** -53
    gam = n * u / (1 - n * u)
    assert np.all(np.abs(got - want) <= 2 * gam * d + 1e-300)


def test_kronecker_delta_closed_form(oracle_lib):
    """B[e,b,f,j] = delta(e,b) delta(f,j)  =>  C[a,b,i,j] = alpha*A[a,b,i,j]
    + beta*C0 exactly."""
    n = 5
    rng = np.random.default_rng(7)
    p = synth.plain16(seed=7, n=n)
    abuf = synth.values(rng, p.a.size, "uniform")
    bbuf = np.zeros(p.b.size)
    for e in range(n):
        for f in range(n):
            bbuf[p.b.base + e * p.b.strides[0] + e * p.b.strides[1]
                 + f * p.b.strides[2] + f * p.b.strides[3]] = 1.0
    cbuf = synth.values(rng, p.c.size, "uniform")
    out = oracle.contract(1.0, (abuf, 0, p.a.extents, p.a.strides), "aeif",
                          (bbuf, 0, p.b.extents, p.b.strides), "ebfj", 0.5,
                          (cbuf, 0, p.c.extents, p.c.strides), "abij")
    A = abuf.reshape((n, n, n, n), order="F")        # A[a,e,i,f]
    C0 = cbuf.reshape((n, n, n, n), order="F")
    want = A.transpose(0, 1, 2, 3) + 0.5 * C0         # C[a,b,i,j] = A[a,b,i,j]
    np.testing.assert_array_equal(out.reshape((n,) * 4, order="F"), want)


def test_all_ones_closed_form(oracle_lib):
    """A = B = 1  =>  C = alpha*K + beta*C0 exactly (K = product of summed
    extents)."""
    p = synth.ladder(6, 3, with_data=False)
    rng = np.random.default_rng(3)
    cbuf = synth.values(rng, p.c.size, "int")
    out = oracle.contract(2.0, (np.ones(p.a.size), 0, p.a.extents, p.a.strides), p.la,
                          (np.ones(p.b.size), 0, p.b.extents, p.b.strides), p.lb, 0.5,
                          (cbuf, 0, p.c.extents, p.c.strides), p.lc)
    np.testing.assert_array_equal(out, 2.0 * 36 + 0.5 * cbuf)


def test_ones_times_random_is_marginal(oracle_lib):
    """A = 1, B random  =>  C[a,b,i,j] = sum_{e,f} B[e,b,f,j], independent
    of a and i (numpy's sum gives the marginal)."""
    n = 4
    p = synth.plain16(n=n, with_data=False)
    rng = np.random.default_rng(11)
    bbuf = synth.values(rng, p.b.size, "int")
    out = oracle.contract(1.0, (np.ones(p.a.size), 0, p.a.extents, p.a.strides), "aeif",
                          (bbuf, 0, p.b.extents, p.b.strides), "ebfj", 0.0,
                          (np.zeros(p.c.size), 0, p.c.extents, p.c.strides), "abij")
    Bt = bbuf.reshape((n,) * 4, order="F")           # B[e,b,f,j]
    marg = Bt.sum(axis=(0, 2))                       # [b, j]
    C = out.reshape((n,) * 4, order="F")             # C[a,b,i,j]
    for a in range(n):
        for i in range(n):
            np.testing.assert_array_equal(C[a, :, i, :], marg)


def _as_dense(buf, lay):
    """Gather a strided tensor into a dense numpy array by fancy indexing."""
    idx = np.full([max(e, 0) for e in lay.extents] or [], lay.base, dtype=np.int64)
    for d, (e, s) in enumerate(zip(lay.extents, lay.strides)):
        shape = [1] * len(lay.extents)
        shape[d] = e
        idx = idx + (np.arange(e, dtype=np.int64) * s).reshape(shape)
    return buf[idx]


def _permuted_gemm(p):
    """The explicit route: permute A to (I..., P...), B to (P..., J...),
    reshape to matrices, numpy.matmul in FP64, reshape back to C's order."""
    A = _as_dense(p.abuf, p.a)
    B = _as_dense(p.bbuf, p.b)
    I = [ch for ch in p.la if ch in p.lc]
    P = [ch for ch in p.la if ch in p.lb]
    J = [ch for ch in p.lb if ch in p.lc]
    Ap = np.transpose(A, [p.la.index(ch) for ch in I + P])
    Bp = np.transpose(B, [p.lb.index(ch) for ch in P + J])
    M = int(np.prod([Ap.shape[k] for k in range(len(I))]))
    K = int(np.prod(Ap.shape[len(I):]))
    N = int(np.prod(Bp.shape[len(P):]))
    Cm = Ap.reshape(M, K) @ Bp.reshape(K, N)
    Cl = Cm.reshape(Ap.shape[:len(I)] + Bp.shape[len(P):])
    return np.transpose(Cl, [(I + J).index(ch) for ch in p.lc])


@pytest.mark.parametrize("seed", range(12))
def test_agrees_with_permuted_gemm(oracle_lib, seed):
    rng = np.random.default_rng(300 + seed)
    p = synth.random_problem(rng, lo=2, hi=7)
    p.abuf, p.bbuf = synth.fill(rng, p.a, "uniform"), synth.fill(rng, p.b, "uniform")
    p.cbuf = synth.fill(rng, p.c, "uniform")
    out, d = oracle.contract(1.0, *p.oracle_args()[:4], 0.0, *p.oracle_args()[4:],
                             want_cond=True)
    got = _as_dense(out, p.c)
    want = _permuted_gemm(p)
    K = synth.sizes(p)[2]
    u = 2.0 ** -53
    bound = 2 * (K + 2) * u / (1 - (K + 2) * u) * _as_dense(d, p.c)
    assert np.all(np.abs(got - want) <= bound)


def test_permuted_gemm_integer_exact(oracle_lib):
    rng = np.random.default_rng(77)
    for _ in range(5):
        p = synth.random_problem(rng, lo=3, hi=9)
        p.abuf, p.bbuf = synth.fill(rng, p.a, "int"), synth.fill(rng, p.b, "int")
        p.cbuf = np.zeros(p.c.size)
        out = oracle.contract(1.0, *p.oracle_args()[:4], 0.0, *p.oracle_args()[4:])
        np.testing.assert_array_equal(_as_dense(out, p.c), _permuted_gemm(p))


def test_bilinearity_power_of_two_exact(oracle_lib):
    p = synth.plain16(seed=9, n=6)
    base = oracle.contract(1.0, *p.oracle_args()[:4], 0.0, *p.oracle_args()[4:])
    a2 = (p.abuf * 2.0, p.a.base, p.a.extents, p.a.strides)
    dbl = oracle.contract(1.0, a2, p.la, *p.oracle_args()[2:4], 0.0, *p.oracle_args()[4:])
    np.testing.assert_array_equal(dbl, 2.0 * base)


def test_swapping_operands_integer_exact(oracle_lib):
    p = synth.plain16(seed=10, n=5, dist="int")
    x = oracle.contract(1.0, *p.oracle_args()[:4], 0.5, *p.oracle_args()[4:])
    a, la, b, lb, c, lc = p.oracle_args()
    y = oracle.contract(1.0, b, lb, a, la, 0.5, c, lc)
    np.testing.assert_array_equal(x, y)


def test_blas_conventions_nan(oracle_lib):
    """beta == 0: C0 is not read (NaN there does not leak); alpha == 0: A and
    B are not read; NaN in A propagates to the C entries it feeds."""
    p = synth.plain16(seed=12, n=3)
    a, la, b, lb, c, lc = p.oracle_args()
    cn = (np.full_like(p.cbuf, np.nan), c[1], c[2], c[3])
    out, d = oracle.contract(1.0, a, la, b, lb, 0.0, cn, lc, want_cond=True)
    assert np.all(np.isfinite(out)) and np.all(np.isfinite(d))
    an = (np.full_like(p.abuf, np.nan), a[1], a[2], a[3])
    out = oracle.contract(0.0, an, la, b, lb, 2.0, c, lc)
    np.testing.assert_array_equal(out, 2.0 * p.cbuf)
    abuf = p.abuf.copy()
    abuf[0] = np.nan       # A[0,0,0,0] feeds C[0,:,0,:]
    out = oracle.contract(1.0, (abuf, a[1], a[2], a[3]), la, b, lb, 0.0, c, lc)
    C = out.reshape((3,) * 4, order="F")
    assert np.all(np.isnan(C[0, :, 0, :]))
    C[0, :, 0, :] = 0
    assert np.all(np.isfinite(C))


def test_empty_sum_and_empty_output(oracle_lib):
    lay0 = synth.layout([3, 0])
    a = (np.ones(max(lay0.size, 1)), 0, [3, 0], lay0.strides)
    b = (np.ones(1), 0, [0], [1])
    cbuf = np.array([1.0, 2.0, 3.0])
    out = oracle.contract(1.0, a, "ik", b, "k", 0.5, (cbuf, 0, [3], [1]), "i")
    np.testing.assert_array_equal(out, 0.5 * cbuf)
    out = oracle.contract(1.0, (np.ones(3), 0, [3], [1]), "k", (np.ones(3), 0, [3], [1]), "k",
                          0.5, (np.array([4.0]), 0, [], []), "")
    np.testing.assert_array_equal(out, [3.0 + 2.0])


def test_error_codes(oracle_lib):
    one = (np.ones(4), 0, [2, 2], [1, 2])
    with pytest.raises(oracle.OracleError) as e:
        oracle.contract(1.0, one, "ik", (np.ones(3), 0, [3], [1]), "k", 0.0,
                        (np.ones(2), 0, [2], [1]), "i")
    assert e.value.code == oracle.ERR_SHAPE
    with pytest.raises(oracle.OracleError) as e:
        oracle.contract(1.0, one, "ik", one, "kj", 0.0, (np.ones(4), 0, [2, 2], [1, 2]), "iz")
    assert e.value.code == oracle.ERR_LABEL
    with pytest.raises(oracle.OracleError) as e:
        oracle.contract(1.0, one, "ik", one, "kj", 0.0, (np.ones(4), 0, [2, 2], [1, 2]), "ii")
    assert e.value.code == oracle.ERR_LABEL


def test_compensated_summation(oracle_lib):
    """Terms 1e16, 1, -1e16: plain recursive summation loses the 1,
    Neumaier's compensated summation keeps it."""
    a = (np.array([1e16, 1.0, -1e16]), 0, [3], [1])
    b = (np.ones(3), 0, [3], [1])
    c = (np.zeros(1), 0, [], [])
    assert oracle.contract(1.0, a, "k", b, "k", 0.0, c, "", compensated=True)[0] == 1.0
    assert oracle.contract(1.0, a, "k", b, "k", 0.0, c, "", compensated=False)[0] == 0.0


def test_condition_tensor(oracle_lib):
    """Non-negative data: D = |alpha| sum|ab| + |beta||C0| equals C itself
    (up to rounding of the same sums)."""
    p = synth.plain16(seed=13, n=4)
    a, la, b, lb, c, lc = p.oracle_args()
    a = (np.abs(p.abuf), a[1], a[2], a[3])
    b = (np.abs(p.bbuf), b[1], b[2], b[3])
    c = (np.abs(p.cbuf), c[1], c[2], c[3])
    out, d = oracle.contract(1.0, a, la, b, lb, 0.5, c, lc, want_cond=True)
    np.testing.assert_allclose(out, d, rtol=1e-14)


def test_condition_tensor_mixed_signs(oracle_lib):
    """D = |alpha| * sum |A||B| + |beta||C0|, which numpy's einsum of the
    absolute values gives independently."""
    p = synth.plain16(seed=14, n=4)
    out, d = oracle.contract(-1.5, *p.oracle_args()[:4], -0.5, *p.oracle_args()[4:],
                             want_cond=True)
    A, B = np.abs(_as_dense(p.abuf, p.a)), np.abs(_as_dense(p.bbuf, p.b))
    want = 1.5 * np.einsum("aeif,ebfj->abij", A, B) + 0.5 * np.abs(_as_dense(p.cbuf, p.c))
    np.testing.assert_allclose(_as_dense(d, p.c), want, rtol=1e-13)
    assert np.all(_as_dense(d, p.c) >= np.abs(_as_dense(out, p.c)) * (1 - 1e-13))


def test_entries_match_full(oracle_lib):
    rng = np.random.default_rng(21)
    p = synth.random_problem(rng, lo=2, hi=6)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    full = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:])
    idx = np.stack([rng.integers(0, e, size=40) for e in p.c.extents], axis=1)
    vals = oracle.contract_entries(p.alpha, *p.oracle_args()[:4], p.beta,
                                   *p.oracle_args()[4:], idx)
    offs = p.c.base + idx @ np.array(p.c.strides)
    np.testing.assert_array_equal(vals, full[offs])


# ------------------------------------------------------------ bf16 split
def test_bf16_rne_matches_torch(oracle_lib):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32),
                        (rng.standard_normal(2000) * 1e30).astype(np.float32),
                        (rng.standard_normal(2000) * 1e-38).astype(np.float32),
                        np.array([0.0, -0.0, np.inf, -np.inf, 3.4e38, -3.4e38,
                                  1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8,
                                  1.0 + 2.0 ** -8 + 2.0 ** -20], dtype=np.float32)])
    ours = oracle.bf16_rne(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(ours.view(np.uint32), ref.view(np.uint32))
    nan = oracle.bf16_rne(np.array([np.nan], dtype=np.float32))
    assert np.isnan(nan[0])


def _split_ref_numpy(p):
    """The bf16x3 split written with torch's bf16 rounding and numpy einsum in
    FP64: hi*hi + hi*lo + lo*hi."""
    torch = pytest.importorskip("torch")

    def split(buf):
        x = torch.from_numpy(buf.astype(np.float32))
        hi = x.to(torch.bfloat16).to(torch.float32)
        lo = (x - hi).to(torch.bfloat16).to(torch.float32)
        return hi.numpy().astype(np.float64), lo.numpy().astype(np.float64)

    ah, al = split(p.abuf)
    bh, bl = split(p.bbuf)
    A = lambda buf: _as_dense(buf, p.a)
    B = lambda buf: _as_dense(buf, p.b)
    ein = "%s,%s->%s" % (p.la, p.lb, p.lc)
    return (np.einsum(ein, A(ah), B(bh)) + np.einsum(ein, A(ah), B(bl))
            + np.einsum(ein, A(al), B(bh)))


def test_split_reference_matches_library_split(oracle_lib):
    rng = np.random.default_rng(31)
    p = synth.plain16(seed=31, n=5)
    p.abuf = p.abuf.astype(np.float32).astype(np.float64)
    p.bbuf = p.bbuf.astype(np.float32).astype(np.float64)
    out, d = oracle.contract(1.0, *p.oracle_args()[:4], 0.0, *p.oracle_args()[4:],
                             split=True, want_cond=True)
    want = _split_ref_numpy(p)
    got = _as_dense(out, p.c)
    K = 25 * 3
    u = 2.0 ** -53
    assert np.all(np.abs(got - want) <= 2 * K * u * _as_dense(d, p.c) + 1e-300)
    exact = _as_dense(oracle.contract(1.0, *p.oracle_args()[:4], 0.0, *p.oracle_args()[4:]), p.c)
    # the dropped lo*lo term: |ab - (hh+hl+lh)| <= 3*2^-16*(1+2^-8)|a||b| per product
    dd = _as_dense(d, p.c)
    assert np.all(np.abs(got - exact) <= 3.0 * 2.0 ** -16 * (1 + 2.0 ** -8) * dd)
    assert np.any(got != exact)


def test_split_exact_when_inputs_are_bf16(oracle_lib):
    """Inputs already representable in bf16 have lo = 0, so the split result
    equals the plain result."""
    p = synth.plain16(seed=32, n=4)
    p.abuf = oracle.bf16_rne(p.abuf.astype(np.float32)).astype(np.float64)
    p.bbuf = oracle.bf16_rne(p.bbuf.astype(np.float32)).astype(np.float64)
    s = oracle.contract(1.0, *p.oracle_args()[:4], 0.5, *p.oracle_args()[4:], split=True)
    x = oracle.contract(1.0, *p.oracle_args()[:4], 0.5, *p.oracle_args()[4:])
    np.testing.assert_array_equal(s, x)


def _split6_ref_numpy(p):
    """The bf16x6 split with torch's bf16 rounding and numpy einsum in FP64:
    hh + hm + mh + hl + mm + lh."""
    torch = pytest.importorskip("torch")

    def split(buf):
        x = torch.from_numpy(buf.astype(np.float32))
        h = x.to(torch.bfloat16).to(torch.float32)
        r = x - h
        m = r.to(torch.bfloat16).to(torch.float32)
        l = (r - m).to(torch.bfloat16).to(torch.float32)
        return [t.numpy().astype(np.float64) for t in (h, m, l)]

    a = [_as_dense(t, p.a) for t in split(p.abuf)]
    b = [_as_dense(t, p.b) for t in split(p.bbuf)]
    ein = "%s,%s->%s" % (p.la, p.lb, p.lc)
    return sum(np.einsum(ein, a[i], b[j]) for i in range(3) for j in range(3) if i + j <= 2)


def test_bf16x6_split_matches_library_split(oracle_lib):
    p = synth.plain16(seed=41, n=5, dist="outliers")
    p.abuf = p.abuf.astype(np.float32).astype(np.float64)
    p.bbuf = p.bbuf.astype(np.float32).astype(np.float64)
    out, d = oracle.contract(1.0, *p.oracle_args()[:4], 0.0, *p.oracle_args()[4:],
                             split=2, want_cond=True)
    want = _split6_ref_numpy(p)
    assert np.all(np.abs(_as_dense(out, p.c) - want) <= 2 * 6 * 25 * 2.0 ** -53 * _as_dense(d, p.c))


def test_bf16x6_error_bound(oracle_lib):
    """Dropping m*l, l*m and l*l costs at most about 2^-23 |a||b| per product;
    the bf16x6 result is within 2^-22 D of the exact one and far closer than
    bf16x3."""
    p = synth.plain16(seed=42, n=6)
    p.abuf = p.abuf.astype(np.float32).astype(np.float64)
    p.bbuf = p.bbuf.astype(np.float32).astype(np.float64)
    args = (1.0, *p.oracle_args()[:4], 0.0, *p.oracle_args()[4:])
    exact, d = oracle.contract(*args, want_cond=True)
    s6 = oracle.contract(*args, split=2)
    s3 = oracle.contract(*args, split=1)
    assert np.all(np.abs(s6 - exact) <= 2.0 ** -22 * d)
    assert np.linalg.norm(s6 - exact) < np.linalg.norm(s3 - exact) / 64


def test_golden_fixtures(oracle_lib):
    """Hand-computed small contractions stored as text fixtures."""
    with open(os.path.join(GOLDEN, "tiny_contractions.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        args = []
        for key in ("A", "B", "C"):
            t = case[key]
            args.append((np.array(t["buf"], dtype=np.float64), t["base"], t["extents"],
                         t["strides"]))
        out = oracle.contract(case["alpha"], args[0], case["A"]["labels"], args[1],
                              case["B"]["labels"], case["beta"], args[2], case["C"]["labels"])
        np.testing.assert_array_equal(out, np.array(case["expect"], dtype=np.float64),
                                      err_msg=case["name"])
