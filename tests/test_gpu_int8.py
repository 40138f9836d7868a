"""FP64 emulated on INT8 MFMA (FAMLIES_INT8X3..7) against the oracle.

* Integer inputs in [-8, 8] over random layouts and labels: every value is
  one exact digit after scaling, so the GPU result must equal the plain
  oracle bit for bit (for every slice count).
* Real data: against the oracle's own slice emulation (oracle.int8_slices:
  the same exact integer digit sums, so the two differ only in how FP64
  recombines them) at gamma_{s+4}(2^-53) D', and against the exact FP64
  contraction within the bound K (s+4)/4 2^-7s 2^(ea+eb) |alpha| (rounded
  digits and dropped digit pairs), where ea, eb are the power-of-two scales
  of the entry's row of A and column of B (computed here from the dense
  tensors with numpy: the smallest e with max|v| <= (127/128) 2^e).
* Rows holding Inf give NaN; K beyond one exact int32 chunk; the full-size
  ladder v=128 o=32 on sampled entries (normwise <= 1e-12)."""
import numpy as np
import pytest

import oracle
import synth
from tests.famlies_testutil import DeviceRunner, U64, gamma, used_offsets
from tests.test_oracle import _random_roles_problem

pytestmark = pytest.mark.gpu

MODES = {3: "int8x3", 4: "int8x4", 5: "int8x5", 6: "int8x6", 7: "int8x7"}


def note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def runner():
    return DeviceRunner()


@pytest.mark.parametrize("seed", range(24))
def test_int8_integer_exact(runner, seed):
    rng = np.random.default_rng(7000 + seed)
    la, a, lb, b, lc, c = _random_roles_problem(rng, max_ext=9)
    p = synth.Problem("int", la, lb, lc, a, b, c, *[(1.0, 0.5), (-2.0, 0.0), (0.0, 3.0), (1.0, 1.0)][seed % 4])
    p.abuf = synth.values(rng, a.size, "int")
    p.bbuf = synth.values(rng, b.size, "int")
    p.cbuf = synth.values(rng, c.size, "int")
    s = [6, 3, 4, 5, 7][seed % 5]
    note("int8 integer seed %d s %d: %s %s -> %s" % (seed, s, la, lb, lc))
    got = runner.run(p, "f64", MODES[s])
    want = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:])
    used = used_offsets(p.c)
    np.testing.assert_array_equal(got[used], want[used])


def _scales(p, n):
    """2^(ea+eb) for every C entry of the plain16-shaped problem
    C[a,b,i,j] = sum_{e,f} A[a,e,i,f] B[e,b,f,j] (dense column-major)."""
    A = p.abuf.reshape((n,) * 4, order="F")
    B = p.bbuf.reshape((n,) * 4, order="F")
    def scale_exp(mx):
        f, e = np.frexp(mx)
        return np.where(f <= 127 / 128, e, e + 1)
    ea = scale_exp(np.abs(A).max(axis=(1, 3)))             # [a, i]
    eb = scale_exp(np.abs(B).max(axis=(0, 2)))             # [b, j]
    sc = np.exp2((ea[:, None, :, None] + eb[None, :, None, :]).astype(np.float64))  # [a, b, i, j]
    return sc.reshape(-1, order="F")


@pytest.mark.parametrize("s", [3, 4, 5, 6, 7])
@pytest.mark.parametrize("dist", ["uniform", "outliers"])
def test_int8_vs_oracle(runner, s, dist):
    n = 20  # M = N = K = 400: ragged tiles along M, N and K
    p = synth.plain16(seed=40 + s, n=n, dist=dist)
    got = runner.run(p, "f64", MODES[s])
    emul = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:], split=oracle.int8_slices(s))
    exact, d = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:], want_cond=True)
    K = n * n
    scale = _scales(p, n) * abs(p.alpha)
    dprime = d + K * scale * (2.0 ** (1 - 7 * s) + 2.0 ** (-14 * s))
    err_emul = np.abs(got - emul)
    assert np.all(err_emul <= gamma(s + 4, U64) * dprime), np.max(err_emul / (gamma(s + 4, U64) * dprime))
    err = np.abs(got - exact)
    bound = K * (s + 4) / 4 * 2.0 ** (-7 * s) * scale + gamma(s + 4, U64) * dprime
    assert np.all(err <= bound), np.max(err / bound)
    note("int8x%d %s: normwise vs exact %.3e, vs emulation %.3e" % (
        s, dist, np.linalg.norm(got - exact) / np.linalg.norm(exact),
        np.linalg.norm(got - emul) / np.linalg.norm(emul)))


def test_int8_batch_and_strides(runner):
    """Batch labels, a permuted and padded layout, beta = 0: against the
    oracle's emulation (general labels; the bound uses the exact D plus the
    digit terms with the largest possible scale, 2 max|A| max|B|)."""
    rng = np.random.default_rng(77)
    a = synth.layout([7, 5, 6, 3], order=[2, 0, 3, 1], pad=[1, 0, 2, 1])   # A[i,k,l,m]
    b = synth.layout([5, 9, 6, 3], order=[1, 3, 0, 2], pad=[0, 1, 0, 0])   # B[k,j,l,m]
    c = synth.layout([9, 7, 3], order=[1, 0, 2], pad=[0, 0, 1])           # C[j,i,m]
    p = synth.Problem("batch", "iklm", "kjlm", "jim", a, b, c, 1.5, 0.0)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "normal") for t in (a, b, c))
    got = runner.run(p, "f64", "int8x6")
    emul = oracle.contract(p.alpha, *p.oracle_args()[:4], 0.0, *p.oracle_args()[4:], split=oracle.int8_slices(6))
    exact, d = oracle.contract(p.alpha, *p.oracle_args()[:4], 0.0, *p.oracle_args()[4:], want_cond=True)
    used = used_offsets(c)
    K = 5 * 6
    big = 4 * np.abs(p.abuf).max() * np.abs(p.bbuf).max() * 1.5
    dprime = d[used] + K * big * 2.0 ** -41
    assert np.all(np.abs(got[used] - emul[used]) <= gamma(10, U64) * dprime)
    assert np.all(np.abs(got[used] - exact[used]) <= K * 8 * 2.0 ** -42 * big + gamma(10, U64) * dprime)


def test_int8_nonfinite_rows(runner):
    n = 8
    p = synth.plain16(seed=51, n=n)
    p.abuf = p.abuf.copy()
    p.abuf[p.a.base + 2 * p.a.strides[0] + 3 * p.a.strides[2]] = np.inf   # A[2,0,3,0]: row (a=2, i=3)
    got = runner.run(p, "f64", "int8x6").reshape((n,) * 4, order="F")
    assert np.all(np.isnan(got[2, :, 3, :]))
    mask = np.ones_like(got, bool)
    mask[2, :, 3, :] = False
    assert np.all(np.isfinite(got[mask]))


def test_int8_long_k_in_chunks(runner):
    """K = 32768 > 22144 (the exact int32 chunk of six slices): the GEMM runs
    as two launches, the second adding to C."""
    rng = np.random.default_rng(61)
    m, n, k = 96, 80, 32768
    a = synth.layout([m, k], order=[1, 0])
    b = synth.layout([k, n])
    c = synth.layout([m, n])
    p = synth.Problem("longk", "ik", "kj", "ij", a, b, c, 1.0, 0.5)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (a, b, c))
    got = runner.run(p, "f64", "int8x6")
    emul = oracle.contract(1.0, *p.oracle_args()[:4], 0.5, *p.oracle_args()[4:], split=oracle.int8_slices(6))
    exact, d = oracle.contract(1.0, *p.oracle_args()[:4], 0.5, *p.oracle_args()[4:], want_cond=True)
    dprime = d + 4 * k * 2.0 ** -40
    assert np.all(np.abs(got - emul) <= gamma(12, U64) * dprime)
    assert np.linalg.norm(got - exact) <= 1e-12 * np.linalg.norm(exact)


def test_int8_fullsize_ladder_v128_o32():
    """The benchmarked ladder, launched as bench.py does, on 2048 sampled
    entries: normwise <= 1e-12 against the exact FP64 oracle, and the
    oracle's slice emulation of the same entries at gamma_{10} D'."""
    import torch
    import paper_2604_07311_amd as fm
    p = synth.ladder(128, 32, seed=2, dtype=np.float64)
    plan = fm.famlies_plan_contract(fm.handle(0), fm.FAMLIES_F64, fm.FAMLIES_INT8X6,
                                    fm.make_desc(p.a.extents, p.a.strides, p.la),
                                    fm.make_desc(p.b.extents, p.b.strides, p.lb),
                                    fm.make_desc(p.c.extents, p.c.strides, p.lc))
    info = fm.famlies_plan_get_info(plan)
    assert info["kernel"] == 14
    dev = [torch.from_numpy(b).cuda() for b in (p.abuf, p.bbuf, p.cbuf)]
    fm.famlies_execute(plan, p.alpha, dev[0].data_ptr(), dev[1].data_ptr(), p.beta, dev[2].data_ptr(),
                       torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = dev[2].cpu().numpy()
    fm.famlies_plan_destroy(plan)
    del dev
    rng = np.random.default_rng(505)
    idx = np.stack([rng.integers(0, e, size=2048) for e in p.c.extents], axis=1)
    args = p.oracle_args()
    want, d = oracle.contract_entries(p.alpha, *args[:4], p.beta, *args[4:], idx, want_cond=True)
    emul = oracle.contract_entries(p.alpha, *args[:4], p.beta, *args[4:], idx, split=oracle.int8_slices(6))
    g = got[p.c.base + idx @ np.array(p.c.strides)]
    K = 128 * 128
    nrm = np.linalg.norm(g - want) / np.linalg.norm(want)
    note("int8x6 ladder v128 o32: normwise vs exact %.3e" % nrm)
    assert nrm <= 1e-12
    # U[-1,1] data: every row and column scale is at most 2^1
    assert np.all(np.abs(g - emul) <= gamma(10, U64) * (d + 4 * K * 2.0 ** -40))
    assert np.all(np.abs(g - want) <= 4 * K * 2.5 * 2.0 ** -42 + gamma(10, U64) * (d + 4 * K * 2.0 ** -40))
