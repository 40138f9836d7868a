"""Host logic of the hand-written backward, without a GPU: the engine call
is replaced by a CPU stand-in (torch.einsum written into the output's own
layout), so these tests check only the backward's bookkeeping -- which
contractions it asks for, the diagonal views of zero-filled gradients, the
broadcast along labels summed inside one input, batch labels and dC0 --
against torch's own gradients of the same einsum."""
import pytest
import torch

import paper_2604_07311_amd as fm
import paper_2604_07311_amd.autograd as ad


def _cpu_contract(alpha, A, la, B, lb, beta=0.0, C=None, lc=None, *, compute="native", stream=None):
    la, lb, lc = fm._labels(la), fm._labels(lb), fm._labels(lc)
    names = {c: chr(ord("a") + i) for i, c in enumerate(sorted(set(la) | set(lb) | set(lc)))}
    eq = "%s,%s->%s" % ("".join(names[c] for c in la), "".join(names[c] for c in lb),
                        "".join(names[c] for c in lc))
    prod = torch.einsum(eq, A, B)
    if C is None:
        assert beta == 0.0
        return (alpha * prod).contiguous()
    with torch.no_grad():
        new = alpha * prod if alpha != 0.0 else torch.zeros_like(C)
        if beta != 0.0:
            new = new + beta * C
        C.copy_(new)
    return C


@pytest.fixture
def cpu_engine(monkeypatch):
    monkeypatch.setattr(ad, "_contract", _cpu_contract)


@pytest.mark.parametrize("la,lb,lc", [
    ("aeif", "ebfj", "abij"),   # plain
    ("aeei", "ebj", "abij"),    # A diagonal over a contracted label
    ("aaei", "ebj", "aij"),     # A diagonal over a row label
    ("aeit", "ebj", "abij"),    # t summed inside A
    ("aei", "ebjs", "abij"),    # s summed inside B
    ("ttei", "eb", "bi"),       # t repeated and summed inside A
    ("aei", "ebi", "abi"),      # i in all three (batch)
    ([7, 9, 9, 3], [9, 5], [7, 5, 3]),  # integer labels
])
def test_backward_bookkeeping(cpu_engine, la, lb, lc):
    ext = {}
    g = torch.Generator().manual_seed(5)
    for c, e in zip(fm._labels(la) + fm._labels(lb), [3, 2, 4, 3, 2, 3, 2, 3, 4]):
        ext.setdefault(c, e)
    A = torch.rand([ext[c] for c in fm._labels(la)], generator=g, dtype=torch.float64, requires_grad=True)
    B = torch.rand([ext[c] for c in fm._labels(lb)], generator=g, dtype=torch.float64, requires_grad=True)
    C0 = torch.rand([ext[c] for c in fm._labels(lc)], generator=g, dtype=torch.float64, requires_grad=True)
    G = torch.randn(C0.shape, generator=g, dtype=torch.float64)
    C = ad.ContractFn.apply(1.3, A, la, B, lb, 0.6, C0, lc, "native")
    C.backward(G)
    A2, B2, C02 = (t.detach().clone().requires_grad_() for t in (A, B, C0))
    (1.3 * _cpu_contract(1.0, A2, la, B2, lb, 0.0, None, lc) + 0.6 * C02).backward(G)
    torch.testing.assert_close(A.grad, A2.grad, rtol=0, atol=1e-12)
    torch.testing.assert_close(B.grad, B2.grad, rtol=0, atol=1e-12)
    torch.testing.assert_close(C0.grad, C02.grad, rtol=0, atol=0)


def test_gradient_layout_follows_input(cpu_engine):
    """Gradients take their input's strides (a permuted dense input)."""
    A = torch.rand(4, 3, dtype=torch.float64).t().requires_grad_()   # strides (1, 3)
    B = torch.rand(4, 5, dtype=torch.float64, requires_grad=True)
    C = ad.ContractFn.apply(1.0, A, "ik", B, "kj", 0.0, None, "ij", "native")
    C.backward(torch.ones_like(C))
    assert A.grad.stride() == A.stride()
