"""GPU parity of the persistent batched kernel: many uneven random 4-index
contractions in one launch, each checked against the oracle; graph capture
and replay give the eager bits."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.famlies_testutil import check_fp32, check_fp64, round_inputs, used_offsets

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)


class Batch:
    """Device buffers and pointer arrays for a list of problems."""

    def __init__(self, probs, dtype, handle=None):
        import torch
        import paper_2604_07311_amd as fm
        self.torch, self.fm = torch, fm
        self.probs = probs
        self.dtype = dtype
        npdt = np.float64 if dtype == "f64" else np.float32
        es = 8 if dtype == "f64" else 4
        self.bufs = []
        pa, pb, pc = [], [], []
        for p in probs:
            a = torch.from_numpy(p.abuf.astype(npdt)).cuda()
            b = torch.from_numpy(p.bbuf.astype(npdt)).cuda()
            c = torch.from_numpy(p.cbuf.astype(npdt)).cuda()
            self.bufs.append((a, b, c))
            pa.append(a.data_ptr() + es * p.a.base)
            pb.append(b.data_ptr() + es * p.b.base)
            pc.append(c.data_ptr() + es * p.c.base)
        self.pa = torch.tensor(pa, dtype=torch.int64, device="cuda")
        self.pb = torch.tensor(pb, dtype=torch.int64, device="cuda")
        self.pc = torch.tensor(pc, dtype=torch.int64, device="cuda")
        code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
        self.plan = fm.famlies_batch_plan(
            fm.handle(0) if handle is None else handle, code,
            [fm.make_desc(p.a.extents, p.a.strides, p.la) for p in probs],
            [fm.make_desc(p.b.extents, p.b.strides, p.lb) for p in probs],
            [fm.make_desc(p.c.extents, p.c.strides, p.lc) for p in probs])

    def execute(self, alpha, beta, stream=None):
        s = stream or self.torch.cuda.current_stream()
        self.fm.famlies_batch_execute(self.plan, alpha, beta, self.pa.data_ptr(), self.pb.data_ptr(),
                                      self.pc.data_ptr(), s.cuda_stream)

    def results(self):
        self.torch.cuda.synchronize()
        return [c.cpu().numpy().astype(np.float64) for _, _, c in self.bufs]

    def reset_c(self):
        for p, (_, _, c) in zip(self.probs, self.bufs):
            c.copy_(self.torch.from_numpy(p.cbuf.astype(c.cpu().numpy().dtype)))

    def close(self):
        self.fm.famlies_plan_destroy(self.plan)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_integer_exact(dtype):
    probs = synth.batched(80, seed=71, with_data=True, dist="int")
    note("batched int-exact %s: %d problems" % (dtype, len(probs)))
    bt = Batch(probs, dtype)
    bt.execute(1.0, 0.5)
    got = bt.results()
    for i, (p, g) in enumerate(zip(probs, got)):
        want = oracle.contract(1.0, *p.oracle_args()[:4], 0.5, *p.oracle_args()[4:])
        np.testing.assert_array_equal(g, want, err_msg="problem %d" % i)
    bt.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_real(dtype):
    probs = [round_inputs(p, dtype) for p in synth.batched(60, seed=72, with_data=True)]
    note("batched real %s: %d problems" % (dtype, len(probs)))
    bt = Batch(probs, dtype)
    bt.execute(1.0, 0.5)
    got = bt.results()
    for i, (p, g) in enumerate(zip(probs, got)):
        want, d = oracle.contract(1.0, *p.oracle_args()[:4], 0.5, *p.oracle_args()[4:],
                                  want_cond=True)
        used = np.zeros(p.cbuf.size, dtype=bool)
        used[used_offsets(p.c)] = True
        np.testing.assert_array_equal(g[~used], p.cbuf[~used])
        K = synth.sizes(p)[2]
        (check_fp64 if dtype == "f64" else check_fp32)(g, want, d, K, where=used)
    bt.close()


def test_batched_few_large_problems():
    """Two large problems and a small one: each large one costs more than a
    quarter of an XCD's share, so its tiles are cut into runs spread over the
    XCD queues; the result is still exact on integer data."""
    rng = np.random.default_rng(78)
    probs = []
    for m, n, k in ((300, 280, 40), (260, 330, 24), (20, 30, 10)):
        a, b, c = synth.layout([m, k], order=[1, 0]), synth.layout([k, n], order=[1, 0]), synth.layout([m, n])
        p = synth.Problem("big", "ik", "kj", "ij", a, b, c, 1.0, 0.5)
        p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "int") for t in (a, b, c))
        probs.append(p)
    for dtype in ("f32", "f64"):
        bt = Batch(probs, dtype)
        bt.execute(1.0, 0.5)
        for i, (p, g) in enumerate(zip(probs, bt.results())):
            want = oracle.contract(1.0, *p.oracle_args()[:4], 0.5, *p.oracle_args()[4:])
            np.testing.assert_array_equal(g, want, err_msg="%s problem %d" % (dtype, i))
        bt.close()


def test_batched_degenerate_and_alpha0():
    """Problems with K == 0 and with alpha == 0 reduce to C = beta*C."""
    rng = np.random.default_rng(73)
    probs = synth.batched(10, seed=74, with_data=True, dist="int")
    k0 = synth.Problem("k0", "ik", "kj", "ij", synth.layout([9, 0]), synth.layout([0, 6]),
                       synth.layout([9, 6]), 1.0, 0.5)
    k0.abuf, k0.bbuf, k0.cbuf = np.zeros(1), np.zeros(1), synth.fill(rng, k0.c, "int")
    probs.append(k0)
    bt = Batch(probs, "f32")
    bt.execute(1.0, 0.5)
    got = bt.results()
    for p, g in zip(probs, got):
        want = oracle.contract(1.0, *p.oracle_args()[:4], 0.5, *p.oracle_args()[4:])
        np.testing.assert_array_equal(g, want)
    bt.reset_c()
    bt.execute(0.0, 2.0)
    got = bt.results()
    for p, g in zip(probs, got):
        want = p.cbuf.copy()                   # padding of C stays untouched
        used = used_offsets(p.c)
        want[used] = 2.0 * p.cbuf[used]
        np.testing.assert_array_equal(g, want)
    bt.close()


def test_batched_graph_replay():
    """Capture one batched launch in a graph; every replay (with eager work
    and synchronisations in between) reproduces the eager result bit for
    bit."""
    import torch
    probs = [round_inputs(p, "f32") for p in synth.batched(40, seed=75, with_data=True)]
    bt = Batch(probs, "f32")
    bt.execute(1.0, 0.5)
    eager = bt.results()
    bt.reset_c()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bt.execute(1.0, 0.5, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        bt.reset_c()
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        g.replay()
        torch.cuda.synchronize()
        got = bt.results()
        for e, r in zip(eager, got):
            np.testing.assert_array_equal(r, e)
        note("replay %d ok" % rep)
    del g
    bt.close()


def _class_table(path, dtype_code, bm, bn):
    """A tile table whose batch entries give every size class the tile
    bm x bn."""
    bk = 16  # the batched kernel's K slice (recorded, not used to pick the class)
    with open(path, "w") as f:
        f.write("# every batched size class: %d x %d\n" % (bm, bn))
        for lm in range(14):
            for ln in range(14):
                for lk in range(14):
                    f.write("batch %d 0 %d %d %d %d %d %d 1\n" % (dtype_code, lm, ln, lk, bm, bn, bk))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_tile_classes_agree(dtype, tmp_path):
    """Each of the four tile classes (64/128 along M and N), forced through a
    tile table, is the class every problem gets, and all four give the same
    bits (a C entry is one tile's sum over K, in the same order whatever the
    tile), within the bound of the oracle."""
    import paper_2604_07311_amd as fm
    probs = [round_inputs(p, dtype) for p in synth.batched(48, seed=76, with_data=True)]
    code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
    results = {}
    for bm in (64, 128):
        for bn in (64, 128):
            path = str(tmp_path / ("t%d_%d.txt" % (bm, bn)))
            _class_table(path, code, bm, bn)
            h = fm.famlies_create(0)
            fm.famlies_load_tune_table(h, path)
            bt = Batch(probs, dtype, handle=h)
            tiles = fm.famlies_batch_plan_tiles(bt.plan, len(probs))
            for p, t in zip(probs, tiles):
                M, N, K = synth.sizes(p)
                assert t == ((bm, bn) if M and N and K else (0, 0))
            bt.execute(1.0, 0.5)
            results[(bm, bn)] = bt.results()
            bt.close()
            fm.famlies_destroy(h)
            note("batched %s class %dx%d done" % (dtype, bm, bn))
    ref = results[(64, 64)]
    for key, got in results.items():
        for i, (g, r) in enumerate(zip(got, ref)):
            np.testing.assert_array_equal(g, r, err_msg="class %s problem %d" % (key, i))
    for p, g in zip(probs, ref):
        want, d = oracle.contract(1.0, *p.oracle_args()[:4], 0.5, *p.oracle_args()[4:], want_cond=True)
        used = np.zeros(p.cbuf.size, dtype=bool)
        used[used_offsets(p.c)] = True
        (check_fp64 if dtype == "f64" else check_fp32)(g, want, d, synth.sizes(p)[2], where=used)


def test_autotuner_writes_and_uses_table(tmp_path):
    """famlies_tune (quick grid) measures the candidate tiles on the device,
    writes a text table, and plans then take their tiles from it: plain
    entries from the single-contraction kernels, batch entries from timed
    launches of the batched kernel."""
    import paper_2604_07311_amd as fm
    h = fm.famlies_create(0)
    path = str(tmp_path / "tiles.txt")
    fm.famlies_tune(h, path, fm.FAMLIES_TUNE_QUICK)
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert rows and all(r[0] in ("plain", "batch") and len(r) == 10 for r in rows)
    brows = [r for r in rows if r[0] == "batch"]
    assert {r[1] for r in brows} == {"1", "2"}
    for r in brows:
        assert int(r[6]) in (64, 128) and int(r[7]) in (64, 128)
        assert int(r[8]) == 16 and int(r[9]) == 1  # the batched kernel's K slice, no split
    note("tuned %d entries (%d batched)" % (len(rows), len(brows)))
    # a batched plan in a tuned size class takes the table's tile
    r = next(r for r in brows if r[1] == "2")
    M, N, K = 1 << int(r[3]), 1 << int(r[4]), 1 << int(r[5])
    plan = fm.famlies_batch_plan(h, fm.FAMLIES_F32, [fm.make_desc([M, K], [K, 1], "mk")],
                                 [fm.make_desc([K, N], [N, 1], "kn")], [fm.make_desc([M, N], [N, 1], "mn")])
    assert fm.famlies_batch_plan_tiles(plan, 1) == [(int(r[6]), int(r[7]))]
    fm.famlies_plan_destroy(plan)
    # a plan in a tuned size class takes the table's tile and split
    r = next(r for r in rows if r[0] == "plain" and r[1] == "2" and r[2] == "0")
    lm, ln, lk, bm, split = int(r[3]), int(r[4]), int(r[5]), int(r[6]), int(r[9])
    M, N, K = 1 << lm, 1 << ln, 1 << lk
    p = fm.famlies_plan_contract(h, fm.FAMLIES_F32, 0, fm.make_desc([M, K], [K, 1], "mk"),
                                 fm.make_desc([K, N], [1, K], "kn"), fm.make_desc([M, N], [N, 1], "mn"))
    info = fm.famlies_plan_get_info(p)
    assert info["swapped"] == 0
    assert info["tile_m"] == bm and info["split_k"] == split
    fm.famlies_plan_destroy(p)
    h2 = fm.famlies_create(0)
    fm.famlies_load_tune_table(h2, path)
    fm.famlies_destroy(h2)
    # one kind of entry only; asking for neither is an error
    only = str(tmp_path / "batch_only.txt")
    fm.famlies_tune(h, only, fm.FAMLIES_TUNE_QUICK | fm.FAMLIES_TUNE_BATCH_ONLY)
    kinds = {l.split()[0] for l in open(only) if l.strip() and not l.startswith("#")}
    assert kinds == {"batch"}
    with pytest.raises(fm.FamliesError) as e:
        fm.famlies_tune(h, str(tmp_path / "none.txt"), fm.FAMLIES_TUNE_BATCH_ONLY | fm.FAMLIES_TUNE_PLAIN_ONLY)
    assert e.value.code == fm.FAMLIES_ERR_INVALID_ARG
    fm.famlies_destroy(h)
