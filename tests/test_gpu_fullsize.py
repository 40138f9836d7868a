"""Parity at the full sizes the benchmark times, in the same launch
configuration (the default handle's plan): sampled C entries against the
oracle computed one by one (FP64, compensated), with the same bounds as the
small-problem tests.  Workloads: the ladder v=128 o=32 in FP64, FP32 and
bf16x3; the ring o=48 v=192 in FP32, bf16x3, bf16x6 and FP64 (the FP32 data,
exact in FP64); the ladder v=192 o=48, whose operands span more than 4 GiB
(element offsets), in FP32, bf16x3, bf16x6 and FP64; and the 20,000-problem
batch."""
import numpy as np
import pytest

import oracle
import synth
from tests.famlies_testutil import U32, U64, gamma

_CACHE = {}


def _problem(name):
    """Each full-size input is generated once per test session."""
    if name not in _CACHE:
        _CACHE.clear()  # keep one large problem in host memory at a time
        if name == "ladder128_f64":
            _CACHE[name] = synth.ladder(128, 32, seed=2, dtype=np.float64)
        elif name == "ladder128_f32":
            _CACHE[name] = synth.ladder(128, 32, seed=2, dtype=np.float32)
        elif name == "ring":
            _CACHE[name] = synth.ring(48, 192, seed=4, dtype=np.float32)
        elif name == "ladder192":
            _CACHE[name] = synth.ladder(192, 48, seed=3, dist="outliers", dtype=np.float32)
    return _CACHE[name]


def _check(compute, dtype, K, g, want, d, dp):
    """The bound of each path (the same as the small-problem tests)."""
    err = np.abs(g - want)
    if dtype == "f64":
        assert np.linalg.norm(g - want) <= 1e-12 * np.linalg.norm(want)
        assert np.all(err <= gamma(K + 2, U64) * d)
    elif compute == "native":
        assert np.all(err <= gamma(K + 4, U32) * d)
    elif compute == "bf16x3":
        assert np.all(err <= (3.0 * 2.0 ** -16 * (1 + 2.0 ** -8) + gamma(K, 2.0 ** -23) * (1 + 2.0 ** -7)) * dp
                      + 2.0 ** -23 * d)
    else:
        assert np.all(err <= (2.0 ** -22 + gamma(3 * K, 2.0 ** -23) * (1 + 2.0 ** -7)) * dp + 2.0 ** -23 * d)

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)


def _run_single(p, dtype, compute="native"):
    """Plan with the default handle, execute once from C0; returns (info,
    C storage as float64 numpy)."""
    import torch
    import paper_2604_07311_amd as fm
    code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
    comp = {"native": 0, "bf16x3": fm.FAMLIES_BF16X3, "bf16x6": fm.FAMLIES_BF16X6}[compute]
    plan = fm.famlies_plan_contract(fm.handle(0), code, comp, fm.make_desc(p.a.extents, p.a.strides, p.la),
                                    fm.make_desc(p.b.extents, p.b.strides, p.lb),
                                    fm.make_desc(p.c.extents, p.c.strides, p.lc))
    info = fm.famlies_plan_get_info(plan)
    npdt = np.float64 if dtype == "f64" else np.float32
    dev = [torch.from_numpy(np.ascontiguousarray(b, dtype=npdt)).cuda() for b in (p.abuf, p.bbuf, p.cbuf)]
    es = dev[0].element_size()
    fm.famlies_execute(plan, p.alpha, dev[0].data_ptr() + es * p.a.base, dev[1].data_ptr() + es * p.b.base,
                       p.beta, dev[2].data_ptr() + es * p.c.base, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    out = dev[2].cpu().numpy().astype(np.float64)
    fm.famlies_plan_destroy(plan)
    del dev
    torch.cuda.empty_cache()
    return info, out


def _sampled(p, got, n, seed, split=0):
    """Oracle values and D at n random C entries, and the GPU's values there.
    The oracle sees the exact FP32 values the GPU saw (buffers are FP32 or
    FP64 already)."""
    rng = np.random.default_rng(seed)
    idx = np.stack([rng.integers(0, e, size=n) for e in p.c.extents], axis=1)
    f64 = lambda b: np.ascontiguousarray(b, dtype=np.float64)
    a = (f64(p.abuf), p.a.base, p.a.extents, p.a.strides)
    b = (f64(p.bbuf), p.b.base, p.b.extents, p.b.strides)
    c = (f64(p.cbuf), p.c.base, p.c.extents, p.c.strides)
    want, d = oracle.contract_entries(p.alpha, a, p.la, b, p.lb, p.beta, c, p.lc, idx, want_cond=True,
                                      split=split)
    _, dp = oracle.contract_entries(p.alpha, a, p.la, b, p.lb, 0.0, c, p.lc, idx, want_cond=True)
    offs = p.c.base + idx @ np.array(p.c.strides, dtype=np.int64)
    return want, d, dp, got[offs]


@pytest.mark.parametrize("dtype,compute", [("f64", "native"), ("f32", "native"), ("f32", "bf16x3")])
def test_ladder_v128_o32(dtype, compute):
    p = _problem("ladder128_" + dtype)
    info, got = _run_single(p, dtype, compute)
    note("ladder v128 o32 %s %s: tile %dx%d split %d kernel %d bits %d" % (
        dtype, compute, info["tile_m"], info["tile_n"], info["split_k"], info["kernel"], info["index_bits"]))
    want, d, dp, g = _sampled(p, got, 4096, 501)
    _check(compute, dtype, 128 * 128, g, want, d, dp)
    note("ladder v128 o32 %s %s normwise %.3e" % (dtype, compute,
                                                  np.linalg.norm(g - want) / np.linalg.norm(want)))


@pytest.mark.parametrize("dtype,compute", [("f32", "native"), ("f32", "bf16x3"), ("f32", "bf16x6"),
                                           ("f64", "native")])
def test_ring_o48_v192(dtype, compute):
    p = _problem("ring")
    info, got = _run_single(p, dtype, compute)
    note("ring %s %s: tile %dx%d split %d kernel %d" % (dtype, compute, info["tile_m"], info["tile_n"],
                                                       info["split_k"], info["kernel"]))
    want, d, dp, g = _sampled(p, got, 2048, 502)
    _check(compute, dtype, 48 * 192, g, want, d, dp)
    note("ring %s %s normwise %.3e" % (dtype, compute, np.linalg.norm(g - want) / np.linalg.norm(want)))


@pytest.mark.parametrize("dtype,compute", [("f32", "native"), ("f32", "bf16x3"), ("f32", "bf16x6"),
                                           ("f64", "native")])
def test_ladder_v192_o48_past_4gib(dtype, compute):
    """W is 192^4 elements (5.4 GB in FP32, 10.9 GB in FP64): past the byte
    offsets' 4 GiB, so the plan counts its offsets in elements."""
    p = _problem("ladder192")
    info, got = _run_single(p, dtype, compute)
    note("ladder v192 o48 %s %s: bits %d elements %d kernel %d" % (dtype, compute, info["index_bits"],
                                                                  info["index_elements"], info["kernel"]))
    # 1.36e9 elements: past 4 GiB, under 2^31 elements -> 32-bit element offsets
    assert info["index_bits"] == 32 and info["index_elements"] == 1
    want, d, dp, g = _sampled(p, got, 1024, 503)
    _check(compute, dtype, 192 * 192, g, want, d, dp)
    note("ladder v192 o48 %s %s normwise %.3e" % (dtype, compute,
                                                  np.linalg.norm(g - want) / np.linalg.norm(want)))


def test_batched_20000():
    """The benchmark's batch: read-only operands in one shared pool, disjoint
    outputs, one launch, tile classes from the package's measured table (as
    bench.py runs it).  Every problem is checked on 8 sampled entries, 20
    problems in full."""
    import os
    import torch
    import paper_2604_07311_amd as fm
    h = fm.famlies_create(0)
    fm.famlies_load_tune_table(h, os.path.join(os.path.dirname(fm.__file__), "tables", "batch_mi355x.txt"))
    n = 20000
    probs = synth.batched(n, seed=5)
    pool_n = max(max(p.a.size for p in probs), max(p.b.size for p in probs)) * 8
    gen = torch.Generator(device="cuda").manual_seed(5)
    pool = torch.rand(pool_n, generator=gen, device="cuda", dtype=torch.float32) * 2 - 1
    rng = np.random.default_rng(55)
    aoff = [int(rng.integers(0, pool_n - p.a.size + 1)) for p in probs]
    boff = [int(rng.integers(0, pool_n - p.b.size + 1)) for p in probs]
    coff = np.concatenate([[0], np.cumsum([p.c.size for p in probs])]).astype(np.int64)
    C0 = torch.rand(int(coff[-1]), generator=gen, device="cuda", dtype=torch.float32) * 2 - 1
    C = C0.clone()
    ptr = lambda base, offs, lays: torch.tensor([base + 4 * (o + t.base) for o, t in zip(offs, lays)],
                                                dtype=torch.int64, device="cuda")
    pa = ptr(pool.data_ptr(), aoff, [p.a for p in probs])
    pb = ptr(pool.data_ptr(), boff, [p.b for p in probs])
    pc = ptr(C.data_ptr(), coff[:-1], [p.c for p in probs])
    plan = fm.famlies_batch_plan(h, fm.FAMLIES_F32,
                                 [fm.make_desc(p.a.extents, p.a.strides, p.la) for p in probs],
                                 [fm.make_desc(p.b.extents, p.b.strides, p.lb) for p in probs],
                                 [fm.make_desc(p.c.extents, p.c.strides, p.lc) for p in probs])
    classes = {t for t in fm.famlies_batch_plan_tiles(plan, n) if t != (0, 0)}
    print("tile classes in use: %s" % sorted(classes), flush=True)
    fm.famlies_batch_execute(plan, 1.0, 0.5, pa.data_ptr(), pb.data_ptr(), pc.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    fm.famlies_plan_destroy(plan)
    fm.famlies_destroy(h)
    pool_h = pool.cpu().numpy().astype(np.float64)
    C_h, C0_h = C.cpu().numpy().astype(np.float64), C0.cpu().numpy().astype(np.float64)
    worst = 0.0
    full = set(rng.choice(n, size=20, replace=False).tolist())
    for i, p in enumerate(probs):
        a = (pool_h[aoff[i]:aoff[i] + p.a.size], p.a.base, p.a.extents, p.a.strides)
        b = (pool_h[boff[i]:boff[i] + p.b.size], p.b.base, p.b.extents, p.b.strides)
        c = (C0_h[coff[i]:coff[i + 1]], p.c.base, p.c.extents, p.c.strides)
        got = C_h[coff[i]:coff[i + 1]]
        K = synth.sizes(p)[2]
        if i in full:  # every entry
            idx = np.stack(np.unravel_index(np.arange(int(np.prod(p.c.extents))), p.c.extents), axis=1)
        else:
            idx = np.stack([rng.integers(0, e, size=8) for e in p.c.extents], axis=1)
        w, d = oracle.contract_entries(1.0, a, p.la, b, p.lb, 0.5, c, p.lc, idx, want_cond=True, nthreads=1)
        g = got[p.c.base + idx @ np.array(p.c.strides, dtype=np.int64)]
        ratio = np.abs(g - w) / np.maximum(gamma(K + 4, U32) * d, 1e-300)
        worst = max(worst, float(ratio.max()))
    note("batched 20000: worst |err| / bound = %.3f" % worst)
    assert worst <= 1.0
