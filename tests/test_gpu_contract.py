"""GPU parity of the plain FP64 / FP32 contraction against the FP64 oracle,
through the C ABI.  Sizes span several tiles with ragged tails; every input
is seeded and synthetic."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.famlies_testutil import (DeviceRunner, check_fp32, check_fp64, gamma, oracle_full,
                                    round_inputs, used_offsets)

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return DeviceRunner()


def _parity(gpu, p, dtype, alpha=None, beta=None):
    p = round_inputs(p, dtype)
    K = synth.sizes(p)[2]
    want, d = oracle_full(p, alpha, beta)
    got = gpu.run(p, dtype, alpha=alpha, beta=beta)
    # untouched storage (padding of C) must keep its value
    used = np.zeros(p.cbuf.size, dtype=bool)
    used[used_offsets(p.c)] = True
    np.testing.assert_array_equal(got[~used], p.cbuf[~used])
    if dtype == "f64":
        return check_fp64(got, want, d, K, where=used)
    return check_fp32(got, want, d, K, where=used)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_plain16_config(gpu, dtype):
    """C[a,b,i,j] = sum_{e,f} A[a,e,i,f] B[e,b,f,j], all extents 16,
    alpha=1, beta=0.5, U[-1,1]."""
    note("plain16 %s" % dtype)
    p = synth.plain16(seed=1)
    rel = _parity(gpu, p, dtype)
    note("plain16 %s rel err %.3e" % (dtype, rel))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("seed", range(12))
def test_integer_exact_random_layouts(gpu, dtype, seed):
    """Integer inputs make every partial sum exact: GPU == oracle bit for bit,
    on random mode orders, padding and stride-2 layouts."""
    rng = np.random.default_rng(9000 + seed)
    p = synth.random_problem(rng, lo=3, hi=24)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "int") for t in (p.a, p.b, p.c))
    note("int-exact %s seed %d %s" % (dtype, seed, synth.sizes(p)))
    want = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:])
    got = gpu.run(p, dtype)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("seed", range(8))
def test_random_layouts_real(gpu, dtype, seed):
    rng = np.random.default_rng(9100 + seed)
    p = synth.random_problem(rng, lo=4, hi=40)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    note("random %s seed %d %s" % (dtype, seed, synth.sizes(p)))
    _parity(gpu, p, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ladder_small_ragged(gpu, dtype):
    """Ladder shape with W stored (e,a,f,b), sizes not multiples of the tiles."""
    p = synth.ladder(19, 7, seed=22)
    note("ladder v19 o7 %s %s" % (dtype, synth.sizes(p)))
    _parity(gpu, p, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ring_small(gpu, dtype):
    p = synth.ring(9, 21, seed=23, dist="uniform")
    note("ring o9 v21 %s %s" % (dtype, synth.sizes(p)))
    _parity(gpu, p, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_split_k_path(gpu, dtype):
    """Small C, long K: the planner splits K; partial sums are reduced in a
    fixed order."""
    a = synth.layout([20, 3000])
    b = synth.layout([3000, 12], order=[1, 0])
    c = synth.layout([20, 12])
    p = synth.Problem("splitk", "ik", "kj", "ij", a, b, c, 1.0, -0.75)
    rng = np.random.default_rng(31)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    info = gpu.fm.famlies_plan_get_info(gpu.plan(p, dtype))
    assert info["split_k"] > 1
    note("split-k %s splits=%d" % (dtype, info["split_k"]))
    _parity(gpu, p, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_negative_zero_strides(gpu, dtype):
    a = synth.layout([37, 5, 11], order=[2, 0, 1], negate=[True, False, True])
    b = synth.layout([5, 11, 29, 3], negate=[False, True, False, False], zero=[False, False, False, True])
    c = synth.layout([29, 37, 3], order=[1, 0, 2], pad=[1, 0, 2], negate=[False, True, False])
    p = synth.Problem("negzero", "ikl", "klju", "jiu", a, b, c, 1.5, 0.25)
    rng = np.random.default_rng(32)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    note("neg/zero strides %s" % dtype)
    _parity(gpu, p, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_padding_never_read(gpu, dtype):
    """NaN in every padding element of A and B: results stay finite."""
    rng = np.random.default_rng(33)
    p = synth.random_problem(rng, lo=5, hi=30, pad_hi=3)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    p.abuf = synth.poison_padding(p.abuf, p.a)
    p.bbuf = synth.poison_padding(p.bbuf, p.b)
    note("poisoned padding %s" % dtype)
    got = gpu.run(p, dtype)
    assert np.all(np.isfinite(got[used_offsets(p.c)]))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_blas_conventions(gpu, dtype):
    p = synth.plain16(seed=34, n=9)
    p = round_inputs(p, dtype)
    note("beta=0 with NaN C0 %s" % dtype)
    p.cbuf = np.full_like(p.cbuf, np.nan)
    got = gpu.run(p, dtype, beta=0.0)
    assert np.all(np.isfinite(got))
    note("alpha=0 with NaN A %s" % dtype)
    p2 = synth.plain16(seed=35, n=9)
    p2 = round_inputs(p2, dtype)
    p2.abuf = np.full_like(p2.abuf, np.nan)
    got = gpu.run(p2, dtype, alpha=0.0, beta=0.5)
    np.testing.assert_array_equal(got, 0.5 * p2.cbuf)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_degenerate(gpu, dtype):
    rng = np.random.default_rng(36)
    note("K == 0 %s" % dtype)
    a = synth.layout([7, 0])
    b = synth.layout([0, 5])
    c = synth.layout([7, 5])
    p = synth.Problem("k0", "ik", "kj", "ij", a, b, c, 1.0, 0.5)
    p.abuf, p.bbuf = np.zeros(a.size), np.zeros(b.size)
    p.cbuf = synth.fill(rng, c, "int")
    np.testing.assert_array_equal(gpu.run(p, dtype), 0.5 * p.cbuf)
    np.testing.assert_array_equal(gpu.run(p, dtype, beta=0.0), np.zeros_like(p.cbuf))
    note("M == 0 %s" % dtype)
    p = synth.Problem("m0", "ik", "kj", "ij", synth.layout([0, 4]), synth.layout([4, 3]),
                      synth.layout([0, 3]), 1.0, 0.5)
    p.abuf, p.bbuf, p.cbuf = np.ones(1), np.ones(12), np.full(1, 7.0)
    np.testing.assert_array_equal(gpu.run(p, dtype), [7.0])
    note("dot product (rank-0 C) %s" % dtype)
    p = synth.Problem("dot", "k", "k", "", synth.layout([1000]), synth.layout([1000], fast_stride=3),
                      synth.layout([]), 2.0, -1.0)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "int") for t in (p.a, p.b, p.c))
    want = oracle.contract(2.0, *p.oracle_args()[:4], -1.0, *p.oracle_args()[4:])
    np.testing.assert_array_equal(gpu.run(p, dtype), want)
    note("outer product (K = 1) %s" % dtype)
    p = synth.Problem("outer", "i", "j", "ji", synth.layout([130]), synth.layout([70]),
                      synth.layout([70, 130]), 1.0, 0.0)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "int") for t in (p.a, p.b, p.c))
    want = oracle.contract(1.0, *p.oracle_args()[:4], 0.0, *p.oracle_args()[4:])
    np.testing.assert_array_equal(gpu.run(p, dtype), want)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_deterministic(gpu, dtype):
    rng = np.random.default_rng(37)
    p = synth.random_problem(rng, lo=10, hi=40)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    note("determinism %s" % dtype)
    x = gpu.run(p, dtype)
    y = gpu.run(p, dtype)
    np.testing.assert_array_equal(x, y)


def test_execute_errors(gpu):
    fm = gpu.fm
    torch = gpu.torch
    p = synth.plain16(seed=38, n=4)
    plan = gpu.plan(p, "f64")
    a = gpu.to_dev(p.abuf, "f64")
    c = gpu.to_dev(p.cbuf, "f64")
    with pytest.raises(fm.FamliesError) as e:
        fm.famlies_execute(plan, 1.0, a.data_ptr() + 4, a.data_ptr(), 0.0, c.data_ptr(), 0)
    assert e.value.code == fm.FAMLIES_ERR_ALIGN
    with pytest.raises(fm.FamliesError) as e:
        fm.famlies_execute(plan, 1.0, a.data_ptr(), c.data_ptr(), 0.0, c.data_ptr(), 0)
    assert e.value.code == fm.FAMLIES_ERR_ALIAS
    fm.famlies_plan_destroy(plan)
    with pytest.raises(fm.FamliesError) as e:
        fm.famlies_execute(plan, 1.0, a.data_ptr(), a.data_ptr(), 0.0, c.data_ptr(), 0)
    assert e.value.code == fm.FAMLIES_ERR_INVALID_ARG
    torch.cuda.synchronize()


def test_torch_level_contract(gpu):
    """contract() on torch views: permuted and sliced tensors are used with
    their strides, no copies."""
    import torch
    import paper_2604_07311_amd as fm
    g = torch.Generator().manual_seed(5)
    A = torch.rand(30, 17, 11, generator=g, dtype=torch.float64).cuda().permute(2, 0, 1)  # [k,i,l]
    B = torch.rand(11, 17, 40, generator=g, dtype=torch.float64).cuda()[:, :, ::2]      # [k,l,j]
    C = fm.contract(1.0, A, "kil", B, "klj", 0.0, None, "ij")
    ref = torch.einsum("kil,klj->ij", A.cpu(), B.cpu())
    torch.testing.assert_close(C.cpu(), ref, rtol=1e-13, atol=1e-13)


def _general_problem(rng, max_ext):
    """Random labels in every role: row, column, contracted, batch (in all
    three), summed inside one input, and a diagonal (repeated label)."""
    from tests.test_oracle import _random_roles_problem
    while True:
        la, a, lb, b, lc, c = _random_roles_problem(rng, allow_general=True, max_ext=max_ext)
        if a.size < 4_000_000 and b.size < 4_000_000 and c.size < 4_000_000:
            return synth.Problem("general", la, lb, lc, a, b, c, 1.5, -0.5)


@pytest.mark.parametrize("compute", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("seed", range(10))
def test_general_labels_integer_exact(gpu, compute, seed):
    """Batch labels, labels summed inside one input and diagonals, on
    random layouts: integer data, so every path equals the oracle bit for bit."""
    import paper_2604_07311_amd as fm
    rng = np.random.default_rng(9300 + seed)
    p = _general_problem(rng, max_ext=12)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "int") for t in (p.a, p.b, p.c))
    dtype = "f64" if compute == "f64" else "f32"
    comp = "bf16x3" if compute == "bf16x3" else "native"
    try:
        plan = gpu.plan(p, dtype, comp)
    except fm.FamliesError as e:
        assert e.code == fm.FAMLIES_ERR_ALIAS   # non-injective random C layouts
        return
    info = fm.famlies_plan_get_info(plan)
    note("general %s seed %d: %s%s%s batch=%d trace=%d diag=%d" % (
        compute, seed, p.la, ",", p.lb, info["batch"], info["n_trace"], info["n_diag"]))
    want = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:])
    got = gpu.run(p, dtype, compute=comp, plan=plan)
    fm.famlies_plan_destroy(plan)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_mode_real(gpu, dtype):
    """C[b,a,i] = sum_e A[a,e,b] B[e,i,b]: a batch label over several tiles."""
    a = synth.layout([70, 90, 5], order=[1, 0, 2])
    b = synth.layout([90, 130, 5], pad=[1, 0, 0])
    c = synth.layout([5, 70, 130], order=[2, 1, 0])
    p = synth.Problem("batchmode", "aeb", "eib", "bai", a, b, c, 1.0, 0.5)
    rng = np.random.default_rng(9400)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    note("batch mode %s" % dtype)
    _parity(gpu, p, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rank8_tensors(gpu, dtype):
    """The largest rank the interface takes: A, B and C of rank 8 (four row,
    four contracted and four column labels), permuted and padded storage,
    integer data, so the result is exact."""
    rng = np.random.default_rng(777)
    I, P, J = "abcd", "efgh", "ijkl"
    ext = {ch: int(rng.integers(2, 4)) for ch in I + P + J}

    def lay(labels):
        order = list(rng.permutation(len(labels)))
        pad = [int(rng.integers(0, 2)) for _ in labels]
        return synth.layout([ext[ch] for ch in labels], order=order, pad=pad)

    la, lb, lc = I[:2] + P + I[2:], P[::-1] + J, J[:2] + I + J[2:]
    p = synth.Problem("rank8", la, lb, lc, lay(la), lay(lb), lay(lc), 1.0, 0.5)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "int") for t in (p.a, p.b, p.c))
    note("rank-8 %s: %s" % (dtype, synth.sizes(p)))
    want = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:])
    got = gpu.run(p, dtype)
    used = used_offsets(p.c)
    np.testing.assert_array_equal(got[used], want[used])
