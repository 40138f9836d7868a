"""GPU parity of the bf16x3 precision path (FP32 data, BF16 MFMA products,
FP64 recombination) against the oracle's exact and split-exact results."""
import numpy as np
import pytest

import oracle
import synth
from tests.famlies_testutil import DeviceRunner, bf16x3_bound, gamma, round_inputs, used_offsets

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def gpu():
    return DeviceRunner()


def _d_prod(p):
    """|alpha| * sum |a||b| per C entry (the oracle's D with beta = 0)."""
    a, la, b, lb, c, lc = p.oracle_args()
    _, d = oracle.contract(p.alpha, a, la, b, lb, 0.0, c, lc, want_cond=True)
    return d


def test_integer_inputs_exact(gpu):
    """Integers in [-8, 8] are exact in bf16 (lo = 0) and every partial sum
    is exact in FP32: bf16x3 equals the oracle bit for bit."""
    rng = np.random.default_rng(81)
    for seed in range(4):
        p = synth.random_problem(rng, lo=4, hi=30)
        p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "int") for t in (p.a, p.b, p.c))
        note("bf16x3 int-exact %d %s" % (seed, synth.sizes(p)))
        want = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:])
        got = gpu.run(p, "f32", compute="bf16x3")
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("case", ["ladder", "ring", "random"])
def test_bf16x3_bounds(gpu, case):
    rng = np.random.default_rng(82)
    if case == "ladder":
        p = synth.ladder(20, 6, seed=83, dist="outliers")
    elif case == "ring":
        p = synth.ring(6, 22, seed=84)
    else:
        p = synth.random_problem(rng, lo=6, hi=40)
        p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "outliers") for t in (p.a, p.b, p.c))
    p = round_inputs(p, "f32")
    K = synth.sizes(p)[2]
    used = np.zeros(p.cbuf.size, dtype=bool)
    used[used_offsets(p.c)] = True
    exact, d = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:],
                               want_cond=True)
    split, _ = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:],
                               split=True, want_cond=True)
    dp = _d_prod(p)
    got = gpu.run(p, "f32", compute="bf16x3")
    f32 = gpu.run(p, "f32")
    u = used
    # against the exact FP64 result
    bound = bf16x3_bound(K, dp, d)
    assert np.all(np.abs(got[u] - exact[u]) <= bound[u])
    # against the split-exact reference: only the FP32 accumulation differs
    acc = gamma(2 * K, 2.0 ** -23) * (1 + 2.0 ** -7) * dp + 2.0 ** -23 * d
    assert np.all(np.abs(got[u] - split[u]) <= acc[u])
    e3 = np.linalg.norm(got[u] - exact[u]) / np.linalg.norm(exact[u])
    e32 = np.linalg.norm(f32[u] - exact[u]) / np.linalg.norm(exact[u])
    note("%s K=%d  bf16x3 rel err %.3e   fp32 rel err %.3e" % (case, K, e3, e32))
    # bf16x3 keeps about 16 bits: well below bf16 (2^-8) and near FP32
    assert e3 < 1e-4


def test_bf16_exact_inputs_match_fp32_accumulation(gpu):
    """Inputs already representable in bf16 (lo = 0): the result is the
    FP32-accumulated exact products, within gamma_K(2^-23) * D of the oracle."""
    p = synth.plain16(seed=85, n=10)
    p.abuf = oracle.bf16_rne(p.abuf.astype(np.float32)).astype(np.float64)
    p.bbuf = oracle.bf16_rne(p.bbuf.astype(np.float32)).astype(np.float64)
    p = round_inputs(p, "f32")
    want, d = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:],
                              want_cond=True)
    got = gpu.run(p, "f32", compute="bf16x3")
    K = 100
    assert np.all(np.abs(got - want) <= (gamma(K, 2.0 ** -23) + 2.0 ** -23) * d)


def test_bf16x3_split_k(gpu):
    """Small C, long K: split-K partials are combined in FP64."""
    a = synth.layout([24, 4000])
    b = synth.layout([4000, 10], order=[1, 0])
    c = synth.layout([24, 10])
    p = synth.Problem("b3splitk", "ik", "kj", "ij", a, b, c, 1.0, 0.5)
    rng = np.random.default_rng(86)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "normal") for t in (p.a, p.b, p.c))
    p = round_inputs(p, "f32")
    info = gpu.fm.famlies_plan_get_info(gpu.plan(p, "f32", "bf16x3"))
    assert info["split_k"] > 1
    exact, d = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:],
                               want_cond=True)
    got = gpu.run(p, "f32", compute="bf16x3")
    assert np.all(np.abs(got - exact) <= bf16x3_bound(4000, _d_prod(p), d))


# ------------------------------------------------------------------ bf16x6
def test_bf16x6_integer_exact(gpu):
    rng = np.random.default_rng(87)
    p = synth.random_problem(rng, lo=4, hi=30)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "int") for t in (p.a, p.b, p.c))
    want = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:])
    np.testing.assert_array_equal(gpu.run(p, "f32", compute="bf16x6"), want)


@pytest.mark.parametrize("case", ["ladder", "random"])
def test_bf16x6_fp32_level_accuracy(gpu, case):
    """bf16x6 against the oracle's split-exact bf16x6 reference (only the FP32
    accumulation differs) and against the exact result at the FP32 bound."""
    rng = np.random.default_rng(88)
    if case == "ladder":
        p = synth.ladder(20, 6, seed=89, dist="outliers")
    else:
        p = synth.random_problem(rng, lo=6, hi=40)
        p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "outliers") for t in (p.a, p.b, p.c))
    p = round_inputs(p, "f32")
    K = synth.sizes(p)[2]
    used = np.zeros(p.cbuf.size, dtype=bool)
    used[used_offsets(p.c)] = True
    args = (p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:])
    exact, d = oracle.contract(*args, want_cond=True)
    split6 = oracle.contract(*args, split=2)
    dp = _d_prod(p)
    got = gpu.run(p, "f32", compute="bf16x6")
    f32 = gpu.run(p, "f32")
    u = used
    acc = gamma(3 * K, 2.0 ** -23) * (1 + 2.0 ** -7) * dp + 2.0 ** -23 * d
    assert np.all(np.abs(got[u] - split6[u]) <= acc[u])
    # dropped terms (m*l, l*m, l*l) add at most 2^-22 |a||b| per product
    assert np.all(np.abs(got[u] - exact[u]) <= (2.0 ** -22 * dp + acc)[u])
    e6 = np.linalg.norm(got[u] - exact[u]) / np.linalg.norm(exact[u])
    e32 = np.linalg.norm(f32[u] - exact[u]) / np.linalg.norm(exact[u])
    note("%s K=%d  bf16x6 rel err %.3e   fp32 rel err %.3e" % (case, K, e6, e32))
    assert e6 < 4 * e32 + 1e-7


@pytest.mark.parametrize("compute", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("k", [32, 64, 96, 40])
def test_split_kernels_short_k(gpu, compute, k):
    """Short K on the split kernels' two-slice pipeline (one, two and three
    slices; K = 40 also has a partial last slice and is gathered): each
    result agrees with the oracle's split-exact reference up to the FP32
    accumulation."""
    ext = {"k": k, "i": 200, "j": 136}
    lays = [synth.layout([ext[ch] for ch in lab]) for lab in ("ki", "kj", "ij")]
    p = synth.Problem("short_k", "ki", "kj", "ij", *lays, 1.0, 0.5)
    rng = np.random.default_rng(90 + k)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "outliers") for t in (p.a, p.b, p.c))
    p = round_inputs(p, "f32")
    args = (p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:])
    exact, d = oracle.contract(*args, want_cond=True)
    ref = oracle.contract(*args, split=1 if compute == "bf16x3" else 2)
    dp = _d_prod(p)
    got = gpu.run(p, "f32", compute=compute)
    parts = 2 if compute == "bf16x3" else 3
    acc = gamma(parts * k, 2.0 ** -23) * (1 + 2.0 ** -7) * dp + 2.0 ** -23 * d
    np.testing.assert_array_less(np.abs(got - ref), acc + 1e-300)
    note("%s K=%d max |got-ref|/D %.2e" % (compute, k, float(np.max(np.abs(got - ref) / np.maximum(d, 1e-300)))))
