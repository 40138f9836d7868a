"""Tail split-K: the last tiles in tile order run as K slices whose partial
sums are reduced afterwards, the other tiles over all of K first.  Forced
through a tile-table entry on problems the oracle checks in full, with
ragged tiles, ragged K slices, beta = 0 and beta != 0."""
import numpy as np
import pytest

import synth
from tests.famlies_testutil import DeviceRunner, check_fp32, check_fp64, oracle_full, round_inputs, used_offsets

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def gpu():
    return DeviceRunner()


def _problems():
    ring = synth.ring(9, 21, seed=41, dist="uniform")          # M = N = K = 189
    rnd = synth.random_problem(np.random.default_rng(43), lo=8, hi=19, beta=-0.75)
    rng = np.random.default_rng(44)
    rnd.abuf, rnd.bbuf, rnd.cbuf = (synth.fill(rng, t, "uniform") for t in (rnd.a, rnd.b, rnd.c))
    return [ring, rnd]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bm", [64, 128])
@pytest.mark.parametrize("split,tail", [(2, 1), (3, -1), (4, 2)])
@pytest.mark.parametrize("which", [0, 1])
def test_tail_split_matches_oracle(gpu, tmp_path, dtype, bm, split, tail, which):
    fm = gpu.fm
    p = round_inputs(_problems()[which], dtype)
    M, N, K = synth.sizes(p)
    ntiles = -(-M // bm) * -(-N // bm)
    if ntiles < 2:
        pytest.skip("one tile: nothing to split off")
    tail = ntiles - 1 if tail < 0 else min(tail, ntiles - 1)
    code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
    bk = 8 if dtype == "f64" else 32
    descs = [fm.make_desc(t.extents, t.strides, lab) for t, lab in ((p.a, p.la), (p.b, p.lb), (p.c, p.lc))]
    info, _ = fm.famlies_analyze(code, 0, *descs)
    lg = lambda x: int(np.ceil(np.log2(max(x, 1))))
    path = tmp_path / "tail.txt"
    path.write_text("plain %d 0 %d %d %d %d %d %d %d 0 %d\n" % (code, lg(info["m"]), lg(info["n"]), lg(info["k"]),
                                                                bm, bm, bk, split, tail))
    h = fm.famlies_create(0)
    fm.famlies_load_tune_table(h, str(path))
    plan = fm.famlies_plan_contract(h, code, 0, *descs)
    pi = fm.famlies_plan_get_info(plan)
    note("tail split %s %s M%d N%d K%d: tile %d split %d of %d tiles split %d" % (
        p.name, dtype, M, N, K, pi["tile_m"], pi["split_k"], ntiles, pi["split_tiles"]))
    assert pi["tile_m"] == bm and pi["split_k"] > 1 and pi["split_tiles"] == tail
    try:
        for beta in (p.beta, 0.0):
            want, d = oracle_full(p, None, beta)
            got = gpu.run(p, dtype, beta=beta, plan=plan)
            used = np.zeros(p.cbuf.size, dtype=bool)
            used[used_offsets(p.c)] = True
            np.testing.assert_array_equal(got[~used], p.cbuf[~used])
            if dtype == "f64":
                check_fp64(got, want, d, K, where=used)
            else:
                check_fp32(got, want, d, K, where=used)
    finally:
        fm.famlies_plan_destroy(plan)
        fm.famlies_destroy(h)


def test_tail_split_same_bits_as_whole_split(gpu, tmp_path):
    """Each split tile sums the same K slices in the same order as when every
    tile is split, so its entries agree bit for bit; the whole tiles agree
    with the unsplit plan bit for bit."""
    fm = gpu.fm
    p = round_inputs(_problems()[0], "f32")
    code = fm.FAMLIES_F32
    descs = [fm.make_desc(t.extents, t.strides, lab) for t, lab in ((p.a, p.la), (p.b, p.lb), (p.c, p.lc))]
    info, _ = fm.famlies_analyze(code, 0, *descs)
    lg = lambda x: int(np.ceil(np.log2(max(x, 1))))
    outs = {}
    for name, split, tail in (("whole", 1, 0), ("all", 3, 0), ("tail", 3, 4)):
        path = tmp_path / ("t_%s.txt" % name)
        path.write_text("plain %d 0 %d %d %d 64 64 32 %d 0 %d\n" % (code, lg(info["m"]), lg(info["n"]),
                                                                   lg(info["k"]), split, tail))
        h = fm.famlies_create(0)
        fm.famlies_load_tune_table(h, str(path))
        plan = fm.famlies_plan_contract(h, code, 0, *descs)
        try:
            outs[name] = gpu.run(p, "f32", plan=plan)
        finally:
            fm.famlies_plan_destroy(plan)
            fm.famlies_destroy(h)
    # C's kernel view: rows of tile t = pm*64.., tile order M fastest; the
    # last 4 of the 9 tiles are split.  Compare via the C indexing vectors.
    _, offs = fm.famlies_analyze(code, 0, *descs, want_offsets=True)
    cm, cn = offs["crow"], offs["ccol"]
    M, N = len(cm), len(cn)
    tm = -(-M // 64)
    addr = p.c.base + cm[:, None] + cn[None, :]
    t = (np.arange(M)[:, None] // 64) + tm * (np.arange(N)[None, :] // 64)
    split_mask = t >= tm * -(-N // 64) - 4
    np.testing.assert_array_equal(outs["tail"][addr[split_mask]], outs["all"][addr[split_mask]])
    np.testing.assert_array_equal(outs["tail"][addr[~split_mask]], outs["whole"][addr[~split_mask]])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("split,tail", [(3, 0), (3, 2), (2, 5)])
def test_tail_split_affine_short_units(gpu, tmp_path, dtype, split, tail):
    """Both operands read in affine 16-byte blocks (two slices in flight) with
    K = 96 cut into K slices of one or two slices each: the pipeline's
    prologue and its clamped look-ahead loads on the shortest ranges."""
    fm = gpu.fm
    ext = {"k": 96, "i": 200, "j": 136}
    lays = [synth.layout([ext[ch] for ch in lab]) for lab in ("ki", "kj", "ij")]
    p = synth.Problem("affine_short", "ki", "kj", "ij", *lays, 1.0, 0.25)
    rng = np.random.default_rng(47)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "uniform") for t in (p.a, p.b, p.c))
    p = round_inputs(p, dtype)
    code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
    bk = 8 if dtype == "f64" else 32
    descs = [fm.make_desc(t.extents, t.strides, lab) for t, lab in ((p.a, p.la), (p.b, p.lb), (p.c, p.lc))]
    info, _ = fm.famlies_analyze(code, 0, *descs)
    lg = lambda x: int(np.ceil(np.log2(max(x, 1))))
    path = tmp_path / "short.txt"
    path.write_text("plain %d 0 %d %d %d 64 64 %d %d 0 %d\n" % (code, lg(info["m"]), lg(info["n"]), lg(info["k"]),
                                                               bk, split, tail))
    h = fm.famlies_create(0)
    fm.famlies_load_tune_table(h, str(path))
    plan = fm.famlies_plan_contract(h, code, 0, *descs)
    pi = fm.famlies_plan_get_info(plan)
    note("affine short units %s: kernel %d split %d split tiles %d" % (dtype, pi["kernel"], pi["split_k"],
                                                                       pi["split_tiles"]))
    try:
        assert pi["kernel"] & 48 == 48 and pi["split_k"] == split
        want, d = oracle_full(p)
        got = gpu.run(p, dtype, plan=plan)
        (check_fp64 if dtype == "f64" else check_fp32)(got, want, d, 96)
    finally:
        fm.famlies_plan_destroy(plan)
        fm.famlies_destroy(h)
