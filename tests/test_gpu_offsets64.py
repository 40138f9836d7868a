"""The 64-bit indexing path (operands spanning 4 GiB or more) on problems
small enough for the oracle: a tile-table entry forces 64-bit indexing
vectors, and every precision and label class is checked against the oracle
as on the 32-bit path."""
import numpy as np
import pytest

import oracle
import synth
from tests.famlies_testutil import GpuRunner, bf16x3_bound, check_fp32, check_fp64, round_inputs, used_offsets

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def gpu():
    return GpuRunner()


def _plan64(gpu, tmp_path, p, dtype, compute="native", bm=None):
    """A plan through a handle whose table forces 64-bit offsets (and, when
    bm is given, bm x bm tiles) for this problem's size class."""
    fm = gpu.fm
    code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
    comp = {"native": 0, "bf16x3": 1, "bf16x6": 2}[compute]
    descs = [fm.make_desc(t.extents, t.strides, lab) for t, lab in ((p.a, p.la), (p.b, p.lb), (p.c, p.lc))]
    info, _ = fm.famlies_analyze(code, comp, *descs)
    lg = lambda x: int(np.ceil(np.log2(max(x, 1))))
    b = bm or info["tile_m"]
    bk = 16 if (dtype == "f64" and compute == "native") else 32
    path = tmp_path / ("t64_%s_%s.txt" % (dtype, compute))
    path.write_text("plain %d %d %d %d %d %d %d %d %d 64\n" % (code, comp, lg(info["m"]), lg(info["n"]),
                                                              lg(info["k"]), b, b, bk, info["split_k"]))
    h = fm.famlies_create(0)
    fm.famlies_load_tune_table(h, str(path))
    plan = fm.famlies_plan_contract(h, code, comp, *descs)
    return h, plan


def _run64(gpu, tmp_path, p, dtype, compute="native", bm=None):
    h, plan = _plan64(gpu, tmp_path, p, dtype, compute, bm)
    info = gpu.fm.famlies_plan_get_info(plan)
    note("64-bit %s %s %s: tile %d split %d kernel %d" % (p.name, dtype, compute, info["tile_m"],
                                                        info["split_k"], info["kernel"]))
    assert info["index_bits"] == 64
    got = gpu.run(p, dtype, compute=compute, plan=plan)
    gpu.fm.famlies_plan_destroy(plan)
    gpu.fm.famlies_destroy(h)
    return got, info


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bm", [64, 128])
@pytest.mark.parametrize("v", [24, 32])
def test_ladder_64bit(gpu, tmp_path, dtype, bm, v):
    """v = 24: only T's fused K is read in affine blocks (W's e-runs of 24
    split the K slices); v = 32: both operands are."""
    p = round_inputs(synth.ladder(v, 8, seed=301), dtype)
    got, info = _run64(gpu, tmp_path, p, dtype, bm=bm)
    assert info["kernel"] & 48 == (48 if v == 32 else 16)
    want, d = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:], want_cond=True)
    (check_fp64 if dtype == "f64" else check_fp32)(got, want, d, v * v)


@pytest.mark.parametrize("seed", range(4))
def test_random_general_labels_64bit(gpu, tmp_path, seed):
    """Random layouts (padding, permutations, stride 2) through both
    precisions."""
    rng = np.random.default_rng(310 + seed)
    p = synth.random_problem(rng, lo=3, hi=24)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    K = synth.sizes(p)[2]
    used = np.zeros(p.cbuf.size, dtype=bool)
    used[used_offsets(p.c)] = True
    for dtype in ("f64", "f32"):
        q = synth.Problem(p.name, p.la, p.lb, p.lc, p.a, p.b, p.c, p.alpha, p.beta)
        q.abuf, q.bbuf, q.cbuf = p.abuf.copy(), p.bbuf.copy(), p.cbuf.copy()
        q = round_inputs(q, dtype)
        got, _ = _run64(gpu, tmp_path, q, dtype)
        want, d = oracle.contract(q.alpha, *q.oracle_args()[:4], q.beta, *q.oracle_args()[4:], want_cond=True)
        (check_fp64 if dtype == "f64" else check_fp32)(got, want, d, K, where=used)


def test_bf16x3_64bit(gpu, tmp_path):
    p = round_inputs(synth.ladder(24, 6, seed=320, dist="outliers"), "f32")
    K = 576
    exact, d = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:], want_cond=True)
    _, dp = oracle.contract(p.alpha, *p.oracle_args()[:4], 0.0, *p.oracle_args()[4:], want_cond=True)
    got, info = _run64(gpu, tmp_path, p, "f32", compute="bf16x3")
    assert info["kernel"] & 16             # T's fused K: affine blocks on the 64-bit path
    assert np.all(np.abs(got - exact) <= bf16x3_bound(K, dp, d))


def test_batch_modes_64bit(gpu, tmp_path):
    a = synth.layout([40, 30, 3], order=[1, 0, 2])
    b = synth.layout([30, 50, 3])
    c = synth.layout([3, 50, 40], order=[1, 2, 0])
    p = synth.Problem("batch64", "ikb", "kjb", "bji", a, b, c, 1.0, 0.5)
    rng = np.random.default_rng(330)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    got, _ = _run64(gpu, tmp_path, p, "f64")
    want, d = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:], want_cond=True)
    check_fp64(got, want, d, 30)
