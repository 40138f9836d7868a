"""Affine-block loads (the block strides of the block-scatter layout): an
operand gathered along K whose every K-slice is a unit-stride run with
16-byte aligned starts is read with 16-byte loads.  Checked against the
oracle with ragged K (the slice crossing K loads element by element), batch
modes, both tile sizes, and a base pointer that is not 16-byte aligned (the
plan then falls back to gathering)."""
import numpy as np
import pytest

import oracle
import synth
from tests.famlies_testutil import DeviceRunner, check_fp32, check_fp64, round_inputs

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def gpu():
    return DeviceRunner()


def _problem(la, lb, lc, ext, orders, seed, alpha=1.0, beta=0.5):
    lays = [synth.layout([ext[ch] for ch in lab], order=o) for lab, o in zip((la, lb, lc), orders)]
    p = synth.Problem("affine", la, lb, lc, *lays, alpha, beta)
    rng = np.random.default_rng(seed)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    return p


def _shift(p):
    """The same problem with every tensor one element further into its
    buffer: base pointers lose their 16-byte alignment."""
    q = synth.Problem(p.name + "_shifted", p.la, p.lb, p.lc,
                      *(synth.Strided(t.extents, t.strides, t.base + 1, t.size + 1) for t in (p.a, p.b, p.c)),
                      p.alpha, p.beta)
    q.abuf, q.bbuf, q.cbuf = (np.concatenate([[0.0], b]) for b in (p.abuf, p.bbuf, p.cbuf))
    return q


def _forced_plan(gpu, tmp_path, p, dtype, bm):
    """A plan whose handle's tile table forces bm x bm tiles, no split-K."""
    fm = gpu.fm
    code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
    descs = [fm.make_desc(t.extents, t.strides, lab) for t, lab in ((p.a, p.la), (p.b, p.lb), (p.c, p.lc))]
    info, _ = fm.famlies_analyze(code, 0, *descs)
    lg = lambda x: int(np.ceil(np.log2(max(x, 1))))
    path = tmp_path / ("tiles_%s_%d.txt" % (dtype, bm))
    path.write_text("plain %d 0 %d %d %d %d %d %d 1\n" % (code, lg(info["m"]), lg(info["n"]), lg(info["k"]), bm, bm,
                                                          8 if dtype == "f64" else 32))
    h = fm.famlies_create(0)
    fm.famlies_load_tune_table(h, str(path))
    plan = fm.famlies_plan_contract(h, code, 0, *descs)
    return h, plan


def _check(gpu, p, dtype, K, expect_kernel_bits, tmp_path=None, bm=None):
    p = round_inputs(p, dtype)
    h = None
    if bm:
        h, plan = _forced_plan(gpu, tmp_path, p, dtype, bm)
    else:
        plan = gpu.plan(p, dtype)
    info = gpu.fm.famlies_plan_get_info(plan)
    note("affine %s %s: kernel %d tile %d split %d m=%d n=%d k=%d" % (
        p.name, dtype, info["kernel"], info["tile_m"], info["split_k"], info["m"], info["n"], info["k"]))
    assert info["kernel"] & 48 == expect_kernel_bits
    if bm:
        assert info["tile_m"] == bm
    got = gpu.run(p, dtype, plan=plan)
    gpu.fm.famlies_plan_destroy(plan)
    if h is not None:
        gpu.fm.famlies_destroy(h)
    want, d = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:], want_cond=True)
    (check_fp64 if dtype == "f64" else check_fp32)(got, want, d, K)
    return got


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bm", [None, 128])
def test_fused_k_ragged(gpu, tmp_path, dtype, bm):
    """A[k,l,i] B[k,l,j] -> C[j,i]: K = 40*16 = 640 fuses to one unit-stride
    mode, a multiple of the K slice; then K = 36*13 = 468, a multiple of
    neither slice (8 FP64, 32 FP32 elements), and both operands are gathered
    (planned tiles, then forced 128 x 128)."""
    ext = {"k": 40, "l": 16, "i": 600, "j": 520}
    p = _problem("kli", "klj", "ji", ext, (None, None, None), seed=201)
    got = _check(gpu, p, dtype, 640, 48, tmp_path, bm)
    ext13 = dict(ext, k=36, l=13)
    _check(gpu, _problem("kli", "klj", "ji", ext13, (None, None, None), seed=205), dtype, 468, 0, tmp_path, bm)
    # unaligned base pointers: same plan shape, gathering path, same values up to rounding
    q = _shift(p)
    got_q = _check(gpu, q, dtype, 640, 48, tmp_path, bm)
    np.testing.assert_allclose(got_q[1:], got, rtol=0, atol=1e-12 if dtype == "f64" else 1e-4)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_unfused_k_blocks_and_small_tiles(gpu, dtype):
    """K modes that do not fuse (k unit stride, extent 64; l far away): every
    K-slice still lies inside one run of k.  Small M, N plan 64 x 64 tiles."""
    ext = {"k": 64, "l": 5, "i": 40, "j": 36}
    p = _problem("kil", "klj", "ij", ext, ([0, 1, 2], [0, 2, 1], [0, 1]), seed=202)
    _check(gpu, p, dtype, 320, 48)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_modes(gpu, dtype):
    """A batch label b in all three tensors: the batch offsets keep the run
    starts aligned."""
    ext = {"k": 96, "i": 130, "j": 70, "b": 3}
    p = _problem("kib", "kjb", "jib", ext, (None, None, None), seed=203)
    _check(gpu, p, dtype, 96, 48)


def test_row_offsets_decide(gpu):
    """Rows of A and B 34 elements apart (k extent 32 plus 2 padding): 16-byte
    runs for FP64 (2 elements) but not for FP32 (4 elements), where both are
    gathered."""
    ext = {"k": 32, "i": 200, "j": 64}
    lays = [synth.layout([ext[ch] for ch in lab], pad=pd) for lab, pd in (("ki", [2, 0]), ("kj", [2, 0]), ("ji", None))]
    p = synth.Problem("affine_rows34", "ki", "kj", "ji", *lays, 1.0, 0.5)
    rng = np.random.default_rng(204)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    _check(gpu, p, "f64", 32, 48)
    _check(gpu, p, "f32", 32, 0)
