"""The element-offset indexing forms (operands spanning 4 GiB or more) on
problems small enough for the oracle: a tile-table entry forces int64
element offsets ("64") or int32 element offsets ("e32", for operands past
4 GiB but under 2^31 elements), and every precision and label class is
checked against the oracle as on the byte-offset path."""
import numpy as np
import pytest

import oracle
import synth
from tests.famlies_testutil import DeviceRunner, bf16x3_bound, check_fp32, check_fp64, gamma, round_inputs, used_offsets

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def gpu():
    return DeviceRunner()


@pytest.fixture(params=["64", "e32"])
def form(request):
    return request.param


def _plan64(gpu, tmp_path, p, dtype, compute="native", bm=None, form="64"):
    """A plan through a handle whose table forces the element-offset form
    `form` (and, when bm is given, bm x bm tiles) for this problem's size
    class."""
    fm = gpu.fm
    code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
    comp = {"native": 0, "bf16x3": 1, "bf16x6": 2}[compute]
    descs = [fm.make_desc(t.extents, t.strides, lab) for t, lab in ((p.a, p.la), (p.b, p.lb), (p.c, p.lc))]
    info, _ = fm.famlies_analyze(code, comp, *descs)
    lg = lambda x: int(np.ceil(np.log2(max(x, 1))))
    b = bm or info["tile_m"]
    bk = 8 if (dtype == "f64" and compute == "native") else 32
    path = tmp_path / ("t%s_%s_%s.txt" % (form, dtype, compute))
    path.write_text("plain %d %d %d %d %d %d %d %d %d %s\n" % (code, comp, lg(info["m"]), lg(info["n"]),
                                                              lg(info["k"]), b, b, bk, info["split_k"], form))
    h = fm.famlies_create(0)
    fm.famlies_load_tune_table(h, str(path))
    plan = fm.famlies_plan_contract(h, code, comp, *descs)
    return h, plan


def _run64(gpu, tmp_path, p, dtype, compute="native", bm=None, form="64"):
    h, plan = _plan64(gpu, tmp_path, p, dtype, compute, bm, form)
    info = gpu.fm.famlies_plan_get_info(plan)
    note("%s %s %s %s: tile %d split %d kernel %d" % (form, p.name, dtype, compute, info["tile_m"],
                                                    info["split_k"], info["kernel"]))
    assert info["index_bits"] == (64 if form == "64" else 32) and info["index_elements"] == 1
    got = gpu.run(p, dtype, compute=compute, plan=plan)
    gpu.fm.famlies_plan_destroy(plan)
    gpu.fm.famlies_destroy(h)
    return got, info


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bm", [64, 128])
@pytest.mark.parametrize("v", [24, 32])
def test_ladder_64bit(gpu, tmp_path, dtype, bm, v, form):
    """v = 24: in FP32 only T's fused K is read in affine blocks (W's e-runs
    of 24 split the 32-wide K slices), in FP64 both are (8-wide slices);
    v = 32: both operands are."""
    p = round_inputs(synth.ladder(v, 8, seed=301), dtype)
    got, info = _run64(gpu, tmp_path, p, dtype, bm=bm, form=form)
    assert info["kernel"] & 48 == (48 if v == 32 or dtype == "f64" else 16)
    want, d = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:], want_cond=True)
    (check_fp64 if dtype == "f64" else check_fp32)(got, want, d, v * v)


@pytest.mark.parametrize("seed", range(4))
def test_random_general_labels_64bit(gpu, tmp_path, seed, form):
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
        got, _ = _run64(gpu, tmp_path, q, dtype, form=form)
        want, d = oracle.contract(q.alpha, *q.oracle_args()[:4], q.beta, *q.oracle_args()[4:], want_cond=True)
        (check_fp64 if dtype == "f64" else check_fp32)(got, want, d, K, where=used)


@pytest.mark.parametrize("compute", ["bf16x3", "bf16x6"])
def test_bf16x3_64bit(gpu, tmp_path, form, compute):
    p = round_inputs(synth.ladder(24, 6, seed=320, dist="outliers"), "f32")
    K = 576
    exact, d = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:], want_cond=True)
    _, dp = oracle.contract(p.alpha, *p.oracle_args()[:4], 0.0, *p.oracle_args()[4:], want_cond=True)
    got, info = _run64(gpu, tmp_path, p, "f32", compute=compute, form=form)
    assert info["kernel"] & 16             # T's fused K: affine blocks on the element-offset paths
    if compute == "bf16x3":
        bound = bf16x3_bound(K, dp, d)
    else:  # dropped products below 2^-22 |a||b|, FP32 sums of 3K products, FP32 store
        bound = (2.0 ** -22 + gamma(3 * K, 2.0 ** -23) * (1 + 2.0 ** -7)) * dp + 2.0 ** -23 * d
    assert np.all(np.abs(got - exact) <= bound)


def test_batch_modes_64bit(gpu, tmp_path, form):
    a = synth.layout([40, 30, 3], order=[1, 0, 2])
    b = synth.layout([30, 50, 3])
    c = synth.layout([3, 50, 40], order=[1, 2, 0])
    p = synth.Problem("batch64", "ikb", "kjb", "bji", a, b, c, 1.0, 0.5)
    rng = np.random.default_rng(330)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    got, _ = _run64(gpu, tmp_path, p, "f64", form=form)
    want, d = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:], want_cond=True)
    check_fp64(got, want, d, 30)
