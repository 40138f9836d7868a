"""CPU tests of the C ABI library: it loads, exports every declared symbol,
and its host planner (label classification, grouping, orientation,
block-scatter indexing vectors, error codes) is right.  No compute call
reaches a device here."""
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "famlies.h")


@pytest.fixture(scope="module")
def fm():
    import paper_2604_07311_amd as fm
    if not os.path.exists(fm.LIB_PATH):
        from paper_2604_07311_amd import build
        build.build()
    fm.load_library()
    return fm


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(famlies_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(fm):
    lib = fm.load_library()
    names = declared_symbols()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(fm.EXPORTS)


def test_version_and_last_error(fm):
    assert "gfx950" in fm.famlies_version()
    assert isinstance(fm.famlies_last_error(), str)


def desc(fm, lay, labels):
    return fm.make_desc(lay.extents, lay.strides, labels)


def analyze(fm, p, dtype=None, compute=0, offsets=False):
    dtype = dtype or fm.FAMLIES_F64
    return fm.famlies_analyze(dtype, compute, desc(fm, p.a, p.la), desc(fm, p.b, p.lb),
                              desc(fm, p.c, p.lc), want_offsets=offsets)


def test_plain16_classification(fm):
    p = synth.plain16(with_data=False)
    info, _ = analyze(fm, p)
    assert (info["m"], info["n"], info["k"]) == (256, 256, 256)
    # C[a,b,i,j]: a has C stride 1 and is an I mode -> swapped so it lies in N
    assert info["swapped"] == 1
    # nothing fuses in A[a,e,i,f] or B[e,b,f,j]: two modes per group
    assert (info["n_i"], info["n_j"], info["n_p"]) == (2, 2, 2)
    assert info["flops"] == 2.0 * 256 ** 3


def test_ladder_grouping(fm):
    p = synth.ladder(128, 32, with_data=False)
    info, _ = analyze(fm, p)
    # kernel view after the swap: X = T (rows ij, fused), Y = W (columns ab)
    assert info["swapped"] == 1
    assert (info["m"], info["n"], info["k"]) == (1024, 16384, 16384)
    assert info["n_i"] == 1          # i,j fuse in T and C
    assert info["n_j"] == 2          # a,b do not fuse in W (stored e,a,f,b)
    assert info["n_p"] == 2          # e,f do not fuse in W
    assert info["x_kfast"] == 1 and info["y_kfast"] == 1  # T and W both have stride 1 on e


def test_ring_grouping(fm):
    p = synth.ring(48, 192, with_data=False)
    info, _ = analyze(fm, p, dtype=fm.FAMLIES_F32, compute=fm.FAMLIES_BF16X3)
    assert (info["m"], info["n"], info["k"]) == (9216, 9216, 9216)


def _check_offsets(fm, p):
    info, off = analyze(fm, p, offsets=True)
    # Every (m,k) / (k,n) / (m,n) maps to a distinct element of the tensor and
    # the union is exactly the tensor's element set.
    swapped = info["swapped"]
    X, Y = (p.b, p.a) if swapped else (p.a, p.b)
    def elems(r, c):
        return (r[:, None] + c[None, :]).ravel()
    from tests.famlies_testutil import used_offsets
    for lay, r, c in ((X, off["xrow"], off["xk"]), (Y, off["yk"], off["ycol"]),
                      (p.c, off["crow"], off["ccol"])):
        got = np.sort(elems(r, c) + lay.base)
        want = np.sort(used_offsets(lay))
        if all(s != 0 for s in lay.strides):
            np.testing.assert_array_equal(got, want)
        else:
            assert got.size == want.size
    return info, off


@pytest.mark.parametrize("seed", range(25))
def test_block_scatter_vectors_cover_tensors(fm, seed):
    rng = np.random.default_rng(500 + seed)
    p = synth.random_problem(rng, lo=1, hi=6, pad_hi=2)
    _check_offsets(fm, p)


def _kernel_view_numpy(fm, p):
    """The kernel view's batched GEMM run with numpy through the planner's
    indexing vectors: C(l,m,n) = alpha sum_k X(l,m,k) Y(l,k,n) + beta C."""
    info, off = analyze(fm, p, offsets=True)
    Xb, Xl, Yb, Yl = (p.bbuf, p.b, p.abuf, p.a) if info["swapped"] else (p.abuf, p.a, p.bbuf, p.b)
    out = p.cbuf.copy()
    for l in range(info["batch"]):
        Xm = Xb[Xl.base + off["xbatch"][l] + off["xrow"][:, None] + off["xk"][None, :]]
        Ym = Yb[Yl.base + off["ybatch"][l] + off["yk"][:, None] + off["ycol"][None, :]]
        cidx = p.c.base + off["cbatch"][l] + off["crow"][:, None] + off["ccol"][None, :]
        out[cidx] = p.alpha * (Xm @ Ym) + p.beta * p.cbuf[cidx]
    return info, out


@pytest.mark.parametrize("seed", range(10))
def test_block_scatter_gemm_equals_oracle(fm, oracle_lib, seed):
    """Running the kernel view's GEMM with numpy through the planner's
    indexing vectors reproduces the oracle (integer data: exact)."""
    import oracle
    rng = np.random.default_rng(600 + seed)
    p = synth.random_problem(rng, lo=1, hi=6, pad_hi=2)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "int") for t in (p.a, p.b, p.c))
    _, out = _kernel_view_numpy(fm, p)
    want = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:])
    np.testing.assert_array_equal(out, want)


@pytest.mark.parametrize("seed", range(40))
def test_general_labels_kernel_view_equals_oracle(fm, oracle_lib, seed):
    """Batch labels (in A, B and C), labels summed inside one input and
    repeated labels (diagonals): the planner's kernel view, run with numpy,
    equals the oracle's einsum semantics exactly on integer data."""
    import oracle
    from tests.test_oracle import _random_roles_problem
    rng = np.random.default_rng(700 + seed)
    la, a, lb, b, lc, c = _random_roles_problem(rng, allow_general=True, max_ext=3)
    p = synth.Problem("gen", la, lb, lc, a, b, c, 1.5, -0.5)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "int") for t in (p.a, p.b, p.c))
    try:
        info, out = _kernel_view_numpy(fm, p)
    except fm.FamliesError as e:   # only C-side problems may be rejected here
        assert e.code in (fm.FAMLIES_ERR_ALIAS,), e
        return
    want = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:])
    np.testing.assert_array_equal(out, want)


def test_general_label_classification(fm):
    # batch label b in all three, trace label t only in A, diagonal ii in B
    A = fm.make_desc([4, 3, 5, 2], [1, 4, 12, 60], "bikt")
    B = fm.make_desc([4, 5, 6, 6], [1, 4, 20, 21], "bkjj")
    C = fm.make_desc([4, 3, 6], [1, 4, 12], "bij")
    info, _ = fm.famlies_analyze(fm.FAMLIES_F64, 0, A, B, C)
    assert info["batch"] == 4 and info["n_batch"] == 1
    assert info["n_trace"] == 1 and info["n_diag"] == 1
    assert sorted((info["m"], info["n"])) == [3, 6] and info["k"] == 10   # k = 5 (k) * 2 (t)


def test_cost_model_orders_rows_by_the_gathered_operand(fm, oracle_lib):
    """C[j,i1,i2] is unit-stride along j, so the rows i1, i2 would follow C's
    order (i1 first); A stores i2 fastest.  Ordering the rows by C would make
    every row gather of A stride e2 elements; the planner orders them by A
    instead (C's column writes do not depend on the row order)."""
    e = {"i": 20, "k": 24, "j": 30, "p": 40}
    a = synth.layout([e["i"], e["k"], e["p"]], order=[1, 0, 2])      # A[i,k,p]: k fastest
    b = synth.layout([e["p"], e["j"]])                                 # B[p,j]: p fastest
    c = synth.layout([e["j"], e["i"], e["k"]])                         # C[j,i,k]: j fastest
    p = synth.Problem("rows_by_x", "ikp", "pj", "jik", a, b, c, 1.0, 0.0)
    info, off = analyze(fm, p, offsets=True)
    assert info["swapped"] == 0 and info["x_kfast"] == 0 and info["y_kfast"] == 1
    steps = np.diff(off["xrow"][: e["k"]])
    assert np.all(steps == 1)                      # coalesced row gather of A
    assert np.all(np.diff(off["yk"][: e["p"]]) == 1)
    assert np.all(np.diff(off["ccol"][: e["j"]]) == 1)
    # the reordered rows still address C consistently: kernel view == oracle
    import oracle
    rng = np.random.default_rng(7)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "int") for t in (p.a, p.b, p.c))
    _, out = _kernel_view_numpy(fm, p)
    want = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:])
    np.testing.assert_array_equal(out, want)


def _mk(labels, ext, orders, pads=(None, None, None)):
    lays = [synth.layout([ext[ch] for ch in lab], order=o, pad=pd) for lab, o, pd in zip(labels, orders, pads)]
    return synth.Problem("affine", *labels, *lays, 1.0, 0.5)


def test_affine_block_flags(fm):
    """Block strides: the plan reads an operand with 16-byte loads (kernel id
    +16 for X, +32 for Y) exactly when it is K-gathered, the K slice (8 FP64
    / 32 FP32 elements) divides K, each K-slice of its indexing vector steps
    by one element, and every run start is a multiple of the 16-byte vector
    (2 FP64 or 4 FP32 elements)."""
    F64, F32 = fm.FAMLIES_F64, fm.FAMLIES_F32
    lad = synth.ladder(32, 4, seed=1)           # W stored (e,a,f,b): K blocks inside e
    for dt in (F64, F32):
        info, _ = analyze(fm, lad, dt)
        assert info["kernel"] == 1 + 16 + 32
    # rows 34 elements apart (k extent 32, 2 padding): 34 % 2 == 0, 34 % 4 != 0
    rows34 = _mk(("ki", "kj", "ji"), {"k": 32, "i": 20, "j": 6}, (None, None, None), ([2, 0], [2, 0], None))
    assert analyze(fm, rows34, F64)[0]["kernel"] == 49
    assert analyze(fm, rows34, F32)[0]["kernel"] == 1
    # K = 30: unit stride and aligned rows (30 % 2 == 0), but the last slice
    # would be partial, so both operands are gathered element by element
    rows30 = _mk(("ki", "kj", "ji"), {"k": 30, "i": 20, "j": 6}, (None, None, None))
    assert analyze(fm, rows30, F64)[0]["kernel"] == 1
    assert analyze(fm, rows30, F32)[0]["kernel"] == 1
    # K modes that do not fuse and a K extent that splits the slices
    split = _mk(("kil", "klj", "ij"), {"k": 36, "l": 3, "i": 20, "j": 8}, ([0, 1, 2], [0, 2, 1], [0, 1]))
    info, _ = analyze(fm, split, F32)                       # 32-wide slices: 36 = 32+4
    assert info["kernel"] & 48 == 0
    info, _ = analyze(fm, split, F64)                       # 8-wide slices: 36 = 4*8+4 still splits
    assert info["kernel"] & 48 == 0
    k40 = _mk(("kil", "klj", "ij"), {"k": 40, "l": 3, "i": 20, "j": 8}, ([0, 1, 2], [0, 2, 1], [0, 1]))
    assert analyze(fm, k40, F64)[0]["kernel"] & 48 == 48    # 40 = 5*8: every 8-wide slice inside one run
    # a row-gathered operand never takes the flag; the split precisions do
    ring = synth.ring(4, 8, seed=1)
    info, _ = analyze(fm, ring, F32)
    assert info["y_kfast"] == 0 and not info["kernel"] & 32
    assert analyze(fm, lad, F32, compute=1)[0]["kernel"] == 3 + 48
    assert analyze(fm, lad, F32, compute=2)[0]["kernel"] == 4 + 48


def test_blocked_k_enumeration(fm):
    """A is fastest along p, B along q, both contracted: K is enumerated in
    8 x 4 (FP32) or 4 x 2 (FP64) blocks of (p, q), so every K slice (32 deep,
    8 deep) holds runs of consecutive elements of both operands; the kernel
    view still reproduces the oracle exactly."""
    import oracle
    ext = {"i": 20, "p": 12, "q": 10, "j": 18}
    a = synth.layout([ext["i"], ext["p"], ext["q"]], order=[1, 0, 2])   # A[i,p,q]: p fastest
    b = synth.layout([ext["q"], ext["p"], ext["j"]])                     # B[q,p,j]: q fastest
    c = synth.layout([ext["j"], ext["i"]])
    p = synth.Problem("blocked", "ipq", "qpj", "ji", a, b, c, 1.0, 0.5)
    rng = np.random.default_rng(9)
    p.abuf, p.bbuf, p.cbuf = (synth.fill(rng, t, "int") for t in (p.a, p.b, p.c))
    for dt, (bu, bw) in ((fm.FAMLIES_F32, (8, 4)), (fm.FAMLIES_F64, (4, 2))):
        info, off = analyze(fm, p, dt, offsets=True)
        assert info["x_kfast"] == 1 and info["y_kfast"] == 1
        X, Y = (p.b, p.a) if info["swapped"] else (p.a, p.b)
        lx, ly = ("qpj", "ipq") if info["swapped"] else ("ipq", "qpj")
        sx = dict(zip(lx, X.strides))
        sy = dict(zip(ly, Y.strides))
        u = "p" if sx["p"] == 1 else "q"          # X's fastest contracted mode
        w = "q" if u == "p" else "p"
        want = []
        for w0 in range(0, ext[w], bw):
            for u0 in range(0, ext[u], bu):
                for bb in range(w0, min(ext[w], w0 + bw)):
                    for aa in range(u0, min(ext[u], u0 + bu)):
                        want.append((aa, bb))
        xk = [aa * sx[u] + bb * sx[w] for aa, bb in want]
        yk = [aa * sy[u] + bb * sy[w] for aa, bb in want]
        np.testing.assert_array_equal(off["xk"], xk)
        np.testing.assert_array_equal(off["yk"], yk)
        if dt == fm.FAMLIES_F32:
            _, out = _kernel_view_numpy(fm, p)
            ref = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:])
            np.testing.assert_array_equal(out, ref)


def test_negative_and_zero_strides_offsets(fm):
    a = synth.layout([3, 4], negate=[True, False])
    b = synth.layout([4, 5], zero=[False, True])
    c = synth.layout([3, 5], order=[1, 0])
    p = synth.Problem("t", "ik", "kj", "ij", a, b, c, 1.0, 0.0)
    _check_offsets(fm, p)


def _err(fm, la, lb, lc, ea, eb, ec, sa=None, sb=None, sc=None, dtype=None, compute=0):
    sa = sa or [1] * len(ea)
    sb = sb or [1] * len(eb)
    sc = sc or list(np.cumprod([1] + list(ec[:-1]))) if ec else []
    with pytest.raises(fm.FamliesError) as e:
        fm.famlies_analyze(dtype or fm.FAMLIES_F64, compute, fm.make_desc(ea, sa, la),
                           fm.make_desc(eb, sb, lb), fm.make_desc(ec, sc, lc))
    return e.value.code


def test_error_codes(fm):
    assert _err(fm, "ik", "kj", "ij", [2, 3], [4, 5], [2, 5]) == fm.FAMLIES_ERR_SHAPE_MISMATCH
    assert _err(fm, "ik", "kj", "iz", [2, 3], [3, 5], [2, 5]) == fm.FAMLIES_ERR_LABEL
    assert _err(fm, "ik", "kj", "ii", [2, 3], [3, 2], [2, 2]) == fm.FAMLIES_ERR_LABEL
    assert _err(fm, "iik", "kj", "ij", [2, 3, 3], [3, 2], [2, 2]) == fm.FAMLIES_ERR_SHAPE_MISMATCH
    assert _err(fm, "ik", "kj", "ij", [2, 3], [3, 2], [2, 2], sc=[1, 1]) == fm.FAMLIES_ERR_ALIAS
    assert _err(fm, "ik", "kj", "ij", [2, 3], [3, 2], [2, 2], dtype=7) == fm.FAMLIES_ERR_INVALID_ARG
    assert _err(fm, "ik", "kj", "ij", [2, 3], [3, 2], [2, 2],
                compute=fm.FAMLIES_BF16X3) == fm.FAMLIES_ERR_UNSUPPORTED
    assert _err(fm, "ik", "kj", "ij", [2, -3], [3, 2], [2, 2]) == fm.FAMLIES_ERR_INVALID_ARG
    big = list("abcdefghi")
    assert _err(fm, "".join(big), "j", "j", [1] * 9, [2], [2]) == fm.FAMLIES_ERR_INVALID_ARG


def test_degenerate_shapes(fm):
    # scalar output (dot product), empty K, empty C
    info, _ = fm.famlies_analyze(fm.FAMLIES_F32, 0, fm.make_desc([5], [1], "k"),
                                 fm.make_desc([5], [2], "k"), fm.make_desc([], [], ""))
    assert (info["m"], info["n"], info["k"]) == (1, 1, 5)
    info, _ = fm.famlies_analyze(fm.FAMLIES_F32, 0, fm.make_desc([3, 0], [1, 3], "ik"),
                                 fm.make_desc([0, 2], [1, 1], "kj"), fm.make_desc([3, 2], [1, 3], "ij"))
    assert info["k"] == 0
    info, _ = fm.famlies_analyze(fm.FAMLIES_F32, 0, fm.make_desc([0, 4], [1, 1], "ik"),
                                 fm.make_desc([4, 2], [1, 4], "kj"), fm.make_desc([0, 2], [1, 1], "ij"))
    assert info["m"] == 0


def test_index_forms(fm):
    """Indexing-vector form by operand span: uint32 byte offsets below 4 GiB,
    int32 element offsets from 4 GiB up to 2^31 elements (not for the INT8
    modes), int64 element offsets beyond."""
    def form(dtype, compute, m, k):
        info, _ = fm.famlies_analyze(dtype, compute, fm.make_desc([m, k], [k, 1], "ik"),
                                     fm.make_desc([k, 8], [1, k], "kj"), fm.make_desc([m, 8], [8, 1], "ij"))
        return info["index_bits"], info["index_elements"]
    assert form(fm.FAMLIES_F32, 0, 1 << 14, 1 << 14) == (32, 0)              # 1 GiB
    assert form(fm.FAMLIES_F32, 0, 40000, 40000) == (32, 1)                  # 6.4 GB, 1.6e9 elements
    assert form(fm.FAMLIES_F64, 0, 40000, 40000) == (32, 1)                  # 12.8 GB
    assert form(fm.FAMLIES_F32, fm.FAMLIES_BF16X3, 40000, 40000) == (32, 1)
    assert form(fm.FAMLIES_F64, fm.FAMLIES_INT8X6, 40000, 40000) == (64, 1)  # INT8: bytes or int64
    assert form(fm.FAMLIES_F32, 0, 50000, 50000) == (64, 1)                  # 2.5e9 elements


def test_no_gpu_means_loud_failure(fm):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(fm.FamliesError):
        fm.famlies_create(0)


def test_tail_split_choice(fm):
    """Default tile choice (256 CUs, two workgroups each): when the tiles fill
    whole rounds plus part of one more, only the last round's tiles are split
    along K; a grid of exactly whole rounds is not split, and the bf16 kernels
    (which split every tile or none) get no split."""
    def analyze(p, dtype, compute=0, swap_c_a=False):
        d = [fm.make_desc(t.extents, t.strides, lab) for t, lab in ((p.a, p.la), (p.b, p.lb), (p.c, p.lc))]
        if swap_c_a:  # dA = G . B, written in A's layout
            d = [d[2], d[1], d[0]]
        return fm.famlies_analyze(dtype, compute, *d)[0]
    ag = synth.autograd_case(24, 96, with_data=False)
    info = analyze(ag, fm.FAMLIES_F32, swap_c_a=True)
    tiles = -(-info["m"] // info["tile_m"]) * -(-info["n"] // info["tile_n"])
    assert (info["m"], info["n"], info["k"]) in ((9216, 2304, 2304), (2304, 9216, 2304))
    assert info["split_k"] > 1 and info["split_tiles"] == tiles % 512 and 0 < info["split_tiles"] < tiles
    lad = synth.ladder(128, 32, with_data=False)
    for dt in (fm.FAMLIES_F64, fm.FAMLIES_F32):
        info = analyze(lad, dt)
        assert info["split_k"] == 1 and info["split_tiles"] == 0  # 1024 tiles: two whole rounds
    ring = synth.ring(48, 192, with_data=False)
    info = analyze(ring, fm.FAMLIES_F32)
    assert info["split_k"] > 1 and info["split_tiles"] == 72 * 72 % 512
    for comp in (1, 2):
        assert analyze(ring, fm.FAMLIES_F32, comp)["split_k"] == 1
    # fewer tiles than one round: every tile split (classic split-K)
    p16 = synth.plain16(with_data=False)
    info = analyze(p16, fm.FAMLIES_F64)
    assert info["split_k"] > 1 and info["split_tiles"] == (256 // info["tile_m"]) ** 2


def test_plan_log(tmp_path):
    """FAMLIES_LOG=1 writes one line per planning decision to stderr."""
    import subprocess
    import sys
    code = ("import paper_2604_07311_amd as fm, synth\n"
            "p = synth.ladder(128, 32, with_data=False)\n"
            "fm.famlies_analyze(fm.FAMLIES_F64, 0, fm.make_desc(p.a.extents, p.a.strides, p.la),\n"
            "                   fm.make_desc(p.b.extents, p.b.strides, p.lb),\n"
            "                   fm.make_desc(p.c.extents, p.c.strides, p.lc))\n")
    env = dict(os.environ, FAMLIES_LOG="1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    lines = [l for l in r.stderr.splitlines() if l.startswith("[famlies]")]
    assert len(lines) == 1, r.stderr
    assert "analyze f64/native M=1024 N=16384 K=16384" in lines[0] and "tile=128x128x8" in lines[0], lines[0]
    env["FAMLIES_LOG"] = "0"
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT)
    assert "[famlies]" not in r.stderr


def test_bad_tokens_rejected(fm):
    """Opaque pointers are generation-counted tokens: made-up values, null
    and pointers of another kind are rejected with INVALID_ARG, not used."""
    for bad in (0, 1, 0x1234, 0x7fff0000, (5 << 32) | (3 << 4) | 2):
        with pytest.raises(fm.FamliesError) as e:
            fm.famlies_plan_destroy(bad)
        assert e.value.code == fm.FAMLIES_ERR_INVALID_ARG
        with pytest.raises(fm.FamliesError) as e:
            fm.famlies_plan_get_info(bad)
        assert e.value.code == fm.FAMLIES_ERR_INVALID_ARG
        with pytest.raises(fm.FamliesError) as e:
            fm.famlies_destroy(bad)
        assert e.value.code == fm.FAMLIES_ERR_INVALID_ARG
