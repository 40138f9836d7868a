"""The entry point that allocates nothing on the device
(famlies_contract_noalloc): its indexing vectors and split-K partial sums
live in the library's static device array.  Checked through the C ABI
against famlies_plan_contract + famlies_execute on the same inputs (the same
plan decisions and kernels, so equal bits) and against the oracle, on two
calls in a row, the second with a smaller input; and the size limit."""
import numpy as np
import pytest

import oracle
import synth
from tests.famlies_testutil import check_fp32, check_fp64

pytestmark = pytest.mark.gpu


def _descs(fm, p):
    return [fm.make_desc(t.extents, t.strides, lab) for t, lab in ((p.a, p.la), (p.b, p.lb), (p.c, p.lc))]


def _run(fm, torch, p, dtype, noalloc, stream):
    npdt = np.float64 if dtype == "f64" else np.float32
    code = fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32
    dev = [torch.from_numpy(np.ascontiguousarray(b, dtype=npdt)).cuda() for b in (p.abuf, p.bbuf, p.cbuf)]
    es = dev[0].element_size()
    ptrs = [dev[0].data_ptr() + es * p.a.base, dev[1].data_ptr() + es * p.b.base, dev[2].data_ptr() + es * p.c.base]
    A, B, C = _descs(fm, p)
    info = None
    if noalloc:
        fm.famlies_contract_noalloc(fm.handle(0), code, 0, p.alpha, A, ptrs[0], B, ptrs[1], p.beta, C, ptrs[2],
                                    stream)
    else:
        plan = fm.famlies_plan_contract(fm.handle(0), code, 0, A, B, C)
        info = fm.famlies_plan_get_info(plan)
        fm.famlies_execute(plan, p.alpha, ptrs[0], ptrs[1], p.beta, ptrs[2], stream)
        torch.cuda.synchronize()
        fm.famlies_plan_destroy(plan)
    torch.cuda.synchronize()
    return info, dev[2].cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_execute_two_calls(dtype):
    import torch
    import paper_2604_07311_amd as fm
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(31)
    big = synth.plain16(seed=32, n=20)                 # split-K: partial sums in the scratch array
    small = synth.random_problem(rng, 3, 11)           # smaller, strided, different layout
    small.abuf, small.bbuf, small.cbuf = (synth.fill(rng, lay, "uniform") for lay in (small.a, small.b, small.c))
    if dtype == "f32":
        for p in (big, small):
            for name in ("abuf", "bbuf", "cbuf"):
                setattr(p, name, getattr(p, name).astype(np.float32).astype(np.float64))
    for p in (big, small):
        print("noalloc %s: %s %s %s" % (dtype, p.la, p.lb, p.lc), flush=True)
        info, want_exec = _run(fm, torch, p, dtype, False, stream)
        _, got = _run(fm, torch, p, dtype, True, stream)
        np.testing.assert_array_equal(got, want_exec)
        want, d = oracle.contract(p.alpha, *p.oracle_args()[:4], p.beta, *p.oracle_args()[4:], want_cond=True)
        K = synth.sizes(p)[2]
        (check_fp64 if dtype == "f64" else check_fp32)(got, want, d, K)
        if p is big:
            assert info["split_k"] > 1


def test_noalloc_size_limit():
    """Indexing vectors beyond the array's 64 MiB are refused before any
    device access (the pointers here are never dereferenced)."""
    import paper_2604_07311_amd as fm
    m, k, n = 1 << 22, 1 << 22, 128   # about 134 MB of 64-bit indexing vectors, 32768 tiles
    A = fm.make_desc([m, k], [1, m], "ik")
    B = fm.make_desc([k, n], [1, k], "kj")
    C = fm.make_desc([m, n], [1, m], "ij")
    with pytest.raises(fm.FamliesError) as e:
        fm.famlies_contract_noalloc(fm.handle(0), fm.FAMLIES_F32, 0, 1.0, A, 1 << 20, B, 1 << 40, 0.0, C,
                                    1 << 44, 0)
    assert e.value.code == fm.FAMLIES_ERR_UNSUPPORTED
    assert "bytes of scratch" in fm.famlies_last_error()
