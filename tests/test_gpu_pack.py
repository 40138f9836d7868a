"""Pre-packed operands: famlies_pack writes an operand in the plan's tile
order (split into bf16 parts for the split modes) and famlies_execute_packed
reads it.  The packed path runs the same products in the same order as the
gathering path, so the two results must agree bit for bit; the gathering
path itself is pinned to the oracle elsewhere (and again here)."""
import numpy as np
import pytest

import oracle
import synth
from tests.famlies_testutil import DeviceRunner, check_fp32, check_fp64, round_inputs, used_offsets

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def gpu():
    return DeviceRunner()


def _forced_handle(fm, tmp_path, p, dtype, compute, bm, split=1):
    """A handle whose tile table forces `bm` x 128 tiles (and `split`) for
    this problem's size class."""
    code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
    comp = {"native": 0, "bf16x3": 1, "bf16x6": 2}[compute]
    info, _ = fm.famlies_analyze(code, comp, fm.make_desc(p.a.extents, p.a.strides, p.la),
                                 fm.make_desc(p.b.extents, p.b.strides, p.lb),
                                 fm.make_desc(p.c.extents, p.c.strides, p.lc))
    lg = lambda x: int(np.ceil(np.log2(max(x, 1))))
    bk = 8 if dtype == "f64" else 32
    path = tmp_path / ("tiles_%s_%s.txt" % (dtype, compute))
    path.write_text("plain %d %d %d %d %d %d 128 %d %d\n" % (
        code, comp, lg(info["m"]), lg(info["n"]), lg(info["k"]), bm, bk, split))
    h = fm.famlies_create(0)
    fm.famlies_load_tune_table(h, str(path))
    return h


def _run(gpu, h, p, dtype, compute, pack_mask):
    """Gathered result and packed result of one problem (C storage)."""
    import torch
    fm = gpu.fm
    code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
    comp = {"native": 0, "bf16x3": 1, "bf16x6": 2}[compute]
    plan = fm.famlies_plan_contract(h, code, comp, fm.make_desc(p.a.extents, p.a.strides, p.la),
                                    fm.make_desc(p.b.extents, p.b.strides, p.lb),
                                    fm.make_desc(p.c.extents, p.c.strides, p.lc))
    info = fm.famlies_plan_get_info(plan)
    es = 8 if dtype == "f64" else 4
    a, b, c0 = gpu.to_dev(p.abuf, dtype), gpu.to_dev(p.bbuf, dtype), gpu.to_dev(p.cbuf, dtype)
    pa, pb = a.data_ptr() + es * p.a.base, b.data_ptr() + es * p.b.base
    s = torch.cuda.current_stream().cuda_stream
    c1 = c0.clone()
    fm.famlies_execute(plan, p.alpha, pa, pb, p.beta, c1.data_ptr() + es * p.c.base, s)
    bufs = {}
    for op in (0, 1):
        if pack_mask & (1 << op):
            n = fm.famlies_pack_size(plan, op)
            bufs[op] = torch.empty(n // 4 + 4, dtype=torch.int32, device="cuda")
            fm.famlies_pack(plan, op, pa if op == 0 else pb, bufs[op].data_ptr(), s)
    c2 = c0.clone()
    fm.famlies_execute_packed(plan, p.alpha, bufs[0].data_ptr() if 0 in bufs else pa,
                              bufs[1].data_ptr() if 1 in bufs else pb, p.beta,
                              c2.data_ptr() + es * p.c.base, pack_mask, s)
    torch.cuda.synchronize()
    fm.famlies_plan_destroy(plan)
    return info, c1.cpu().numpy().astype(np.float64), c2.cpu().numpy().astype(np.float64)


CASES = [("f64", "native", 128), ("f32", "native", 128), ("f32", "bf16x3", 128),
         ("f32", "bf16x3", 256), ("f32", "bf16x6", 128)]


@pytest.mark.parametrize("dtype,compute,bm", CASES)
@pytest.mark.parametrize("mask", [1, 2, 3])
def test_packed_equals_gathered_ladder(gpu, tmp_path, dtype, compute, bm, mask):
    """Ladder with ragged sizes (M = 15*13, N = K = 37*37)."""
    fm = gpu.fm
    p = round_inputs(synth.ladder(37, 13, seed=95, dist="outliers" if compute != "native" else "uniform"),
                     dtype)
    h = _forced_handle(fm, tmp_path, p, dtype, compute, bm)
    info, gathered, packed = _run(gpu, h, p, dtype, compute, mask)
    note("packed %s %s tile %dx%d mask %d: m=%d n=%d k=%d" % (
        dtype, compute, info["tile_m"], info["tile_n"], mask, info["m"], info["n"], info["k"]))
    assert info["tile_m"] == bm
    np.testing.assert_array_equal(packed, gathered)
    if compute == "native":
        want, d = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:],
                                  want_cond=True)
        (check_fp64 if dtype == "f64" else check_fp32)(packed, want, d, 37 * 37)
    fm.famlies_destroy(h)


@pytest.mark.parametrize("dtype,compute", [("f64", "native"), ("f32", "bf16x3")])
def test_packed_split_k_and_batch_modes(gpu, tmp_path, dtype, compute):
    """Batch labels (one packed plane per batch index) and split-K slices."""
    fm = gpu.fm
    a = synth.layout([130, 300, 3], order=[1, 0, 2])
    b = synth.layout([300, 150, 3])
    c = synth.layout([3, 150, 130], order=[1, 2, 0])
    p = synth.Problem("packbatch", "ikb", "kjb", "bji", a, b, c, 1.0, 0.5)
    rng = np.random.default_rng(96)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    p = round_inputs(p, dtype)
    h = _forced_handle(fm, tmp_path, p, dtype, compute, 128)
    info, gathered, packed = _run(gpu, h, p, dtype, compute, 3)
    assert info["batch"] == 3
    np.testing.assert_array_equal(packed, gathered)
    fm.famlies_destroy(h)
    # split-K (no batch modes)
    p2 = round_inputs(synth.ladder(30, 10, seed=97), dtype)
    h = _forced_handle(fm, tmp_path, p2, dtype, compute, 128, split=3)
    info, gathered, packed = _run(gpu, h, p2, dtype, compute, 3)
    note("packed split-K: splits=%d" % info["split_k"])
    assert info["split_k"] > 1
    np.testing.assert_array_equal(packed, gathered)
    fm.famlies_destroy(h)


@pytest.mark.parametrize("dtype,compute", [("f64", "native"), ("f32", "native"), ("f32", "bf16x3"),
                                           ("f32", "bf16x6")])
def test_packed_small_tiles(gpu, dtype, compute):
    """Small problems plan 64 x 64 tiles (and split-K); packed equals gathered."""
    p = round_inputs(synth.plain16(seed=99, n=9, dist="uniform"), dtype)
    h = gpu.fm.handle(0)
    info, gathered, packed = _run(gpu, h, p, dtype, compute, 3)
    note("small packed %s %s tile %d split %d" % (dtype, compute, info["tile_m"], info["split_k"]))
    np.testing.assert_array_equal(packed, gathered)


def test_pack_rejects_bad_arguments(gpu):
    fm = gpu.fm
    p = synth.plain16(seed=98, n=6)
    plan = gpu.plan(p, "f64")
    with pytest.raises(fm.FamliesError) as e:
        fm.famlies_pack_size(plan, 2)
    assert e.value.code == fm.FAMLIES_ERR_INVALID_ARG
    with pytest.raises(fm.FamliesError) as e:
        fm.famlies_execute_packed(plan, 1.0, 0, 0, 0.0, 0, 7, 0)
    assert e.value.code == fm.FAMLIES_ERR_INVALID_ARG
    fm.famlies_plan_destroy(plan)
