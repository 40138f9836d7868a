"""Contraction networks: a coupled-cluster-like sequence with an intermediate,
a batch-mode reduction, and a constant operand kept pre-packed, checked step
by step against the oracle (FP64)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _dense_layout(ext):
    return synth.layout(ext)


def test_network_chain_fp64():
    import torch
    import paper_2604_07311_amd as fm
    v, o = 40, 10
    rng = np.random.default_rng(111)
    W = synth.layout([v, v, v, v], order=[2, 0, 3, 1])   # W[a,b,e,f] stored (e,a,f,b)
    T = _dense_layout([v, v, o, o])                     # T[e,f,i,j]
    V = _dense_layout([o, o, o, o])                     # V[k,l,i,j]
    I1 = _dense_layout([v, v, o, o])                    # I[a,b,k,l] (intermediate)
    R = _dense_layout([v, v, o, o])                     # R[a,b,i,j]
    Q = _dense_layout([v, v, o, o])                     # Q[a,b,i,j]
    Z = _dense_layout([o, o])                           # Z[i,j] = sum_ab R Q (i,j batch)
    bufs = {name: synth.fill(rng, lay, "uniform") for name, lay in
            (("W", W), ("T", T), ("V", V), ("R", R), ("Q", Q), ("Z", Z))}
    dev = {k: torch.from_numpy(b).cuda() for k, b in bufs.items()}

    net = fm.Network(fm.FAMLIES_F64)
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

    # oracle, step by step (FP64)
    i1 = oracle.contract(1.0, (bufs["W"], 0, W.extents, W.strides), "abef",
                         (bufs["T"], 0, T.extents, T.strides), "efkl", 0.0,
                         (np.zeros(I1.size), 0, I1.extents, I1.strides), "abkl")
    r = oracle.contract(1.0, (i1, 0, I1.extents, I1.strides), "abkl",
                        (bufs["V"], 0, V.extents, V.strides), "klij", 0.5,
                        (bufs["R"], 0, R.extents, R.strides), "abij")
    z = oracle.contract(2.0, (r, 0, R.extents, R.strides), "abij",
                        (bufs["Q"], 0, Q.extents, Q.strides), "abij", 0.0,
                        (bufs["Z"], 0, Z.extents, Z.strides), "ij")
    got_r = dev["R"].cpu().numpy()
    got_z = dev["Z"].cpu().numpy()
    np.testing.assert_allclose(got_r, r, rtol=0, atol=1e-12 * np.abs(r).max())
    np.testing.assert_allclose(got_z, z, rtol=0, atol=1e-11 * np.abs(z).max())
    # the intermediate is readable through its pointer
    ptr = net.tensor_ptr(ids["I1"])
    assert ptr != 0
    # a second run with rebound W (repacked) gives the same values for the same data
    dev["R"].copy_(torch.from_numpy(bufs["R"]))
    w2 = dev["W"].clone()
    net.bind(ids["W"], w2.data_ptr())
    net.execute(torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dev["R"].cpu().numpy(), got_r)
    net.close()
