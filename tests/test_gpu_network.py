"""Contraction networks: a coupled-cluster-like sequence with an intermediate,
a batch-mode reduction, and a constant operand kept pre-packed, in FP64,
FP32 and bf16x3.  Each step is checked against the oracle run on the inputs
that step actually read (the intermediates read back from the device), at
the componentwise bound of its precision: gamma_{K+2}(2^-53) D (FP64),
gamma_{K+4}(2^-24) D (FP32) and the bf16x3 bound."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from tests.famlies_testutil import U32, U64, bf16x3_bound, gamma

pytestmark = pytest.mark.gpu


def _dense_layout(ext):
    return synth.layout(ext)


def _read_device(ptr, n, npdt):
    """Copy n elements from a raw device pointer (an intermediate owned by the
    network) to the host with hipMemcpy."""
    import torch
    torch.cuda.synchronize()
    # the HIP runtime already in the process (torch's), never a second copy
    path = next(l.split()[-1] for l in open("/proc/self/maps") if "libamdhip64" in l)
    hip = ctypes.CDLL(path)
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    out = np.empty(n, dtype=npdt)
    assert hip.hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2) == 0  # 2 = device to host
    return out


def _check_step(got, want, d, dp, K, dtype, compute, what):
    err = np.abs(got - want)
    if dtype == "f64":
        bound = gamma(K + 2, U64) * d
    elif compute == "native":
        bound = gamma(K + 4, U32) * d
    else:
        bound = bf16x3_bound(K, dp, d)
    bad = err > bound
    assert not bad.any(), "%s: bound violated at %d entries (max ratio %.3g)" % (
        what, bad.sum(), np.max(err / np.maximum(bound, 1e-300)))
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300))


@pytest.mark.parametrize("dtype,compute", [("f64", "native"), ("f32", "native"), ("f32", "bf16x3")])
def test_network_chain(dtype, compute):
    import torch
    import paper_2604_07311_amd as fm
    v, o = 40, 10
    npdt = np.float64 if dtype == "f64" else np.float32
    rng = np.random.default_rng(111)
    W = synth.layout([v, v, v, v], order=[2, 0, 3, 1])   # W[a,b,e,f] stored (e,a,f,b)
    T = _dense_layout([v, v, o, o])                     # T[e,f,i,j]
    V = _dense_layout([o, o, o, o])                     # V[k,l,i,j]
    I1 = _dense_layout([v, v, o, o])                    # I[a,b,k,l] (intermediate)
    R = _dense_layout([v, v, o, o])                     # R[a,b,i,j]
    Q = _dense_layout([v, v, o, o])                     # Q[a,b,i,j]
    Z = _dense_layout([o, o])                           # Z[i,j] = sum_ab R Q (i,j batch)
    bufs = {name: synth.fill(rng, lay, "uniform").astype(npdt) for name, lay in
            (("W", W), ("T", T), ("V", V), ("R", R), ("Q", Q), ("Z", Z))}
    dev = {k: torch.from_numpy(b).cuda() for k, b in bufs.items()}
    f64 = {k: b.astype(np.float64) for k, b in bufs.items()}

    net = fm.Network(fm.FAMLIES_F64 if dtype == "f64" else fm.FAMLIES_F32,
                     fm.FAMLIES_BF16X3 if compute == "bf16x3" else fm.FAMLIES_NATIVE)
    ids = {}
    for name, lay, lab, inter in (("W", W, "abef", False), ("T", T, "efkl", False),
                                  ("V", V, "klij", False), ("I1", I1, "abkl", True),
                                  ("R", R, "abij", False), ("Q", Q, "abij", False),
                                  ("Z", Z, "ij", False)):
        ids[name] = net.tensor(lay.extents, lay.strides, lab, intermediate=inter)
    net.contract(1.0, ids["W"], ids["T"], 0.0, ids["I1"], pack_a=True)      # ladder, W kept packed
    net.contract(1.0, ids["I1"], ids["V"], 0.5, ids["R"])                    # R = I.V + R/2
    net.contract(2.0, ids["R"], ids["Q"], 0.0, ids["Z"])                     # batch (i,j) reduction
    net.compile()
    for name in ("W", "T", "V", "R", "Q", "Z"):
        net.bind(ids[name], dev[name].data_ptr())
    net.execute(torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got_i1 = _read_device(net.tensor_ptr(ids["I1"]), I1.size, npdt).astype(np.float64)
    got_r = dev["R"].cpu().numpy().astype(np.float64)
    got_z = dev["Z"].cpu().numpy().astype(np.float64)

    def orc(alpha, a, la, alay, b, lb, blay, beta, c, lc, clay):
        want, d = oracle.contract(alpha, (a, 0, alay.extents, alay.strides), la,
                                  (b, 0, blay.extents, blay.strides), lb, beta,
                                  (c, 0, clay.extents, clay.strides), lc, want_cond=True)
        _, dp = oracle.contract(alpha, (a, 0, alay.extents, alay.strides), la,
                                (b, 0, blay.extents, blay.strides), lb, 0.0,
                                (c, 0, clay.extents, clay.strides), lc, want_cond=True)
        return want, d, dp

    # step 1 on the bound inputs; steps 2 and 3 on what the device computed
    w, d, dp = orc(1.0, f64["W"], "abef", W, f64["T"], "efkl", T, 0.0, np.zeros(I1.size), "abkl", I1)
    e1 = _check_step(got_i1, w, d, dp, v * v, dtype, compute, "I1 = W.T")
    w, d, dp = orc(1.0, got_i1, "abkl", I1, f64["V"], "klij", V, 0.5, f64["R"], "abij", R)
    e2 = _check_step(got_r, w, d, dp, o * o, dtype, compute, "R = I1.V + R/2")
    w, d, dp = orc(2.0, got_r, "abij", R, f64["Q"], "abij", Q, 0.0, f64["Z"], "ij", Z)
    e3 = _check_step(got_z, w, d, dp, v * v, dtype, compute, "Z = 2 R.Q")
    print("network %s %s normwise per step %.2e %.2e %.2e" % (dtype, compute, e1, e2, e3), flush=True)

    # a second run with rebound W (repacked) gives the same values for the same data
    dev["R"].copy_(torch.from_numpy(bufs["R"]))
    w2 = dev["W"].clone()
    net.bind(ids["W"], w2.data_ptr())
    net.execute(torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dev["R"].cpu().numpy().astype(np.float64), got_r)
    net.close()
