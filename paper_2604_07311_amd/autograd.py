"""Hand-written backward for the contraction.

For  C = alpha * sum_P A[I,P] B[P,J] + beta * C0  and upstream gradient G[I,J]:

    dA[I,P] = alpha * sum_J G[I,J] B[P,J]      (a contraction over J)
    dB[P,J] = alpha * sum_I A[I,P] G[I,J]      (a contraction over I)
    dC0     = beta * G

Both gradients are themselves labelled contractions, so they run on the
same planner and kernels as the forward (the paper's aim of one engine
reused across operations, Section "Building on important advances", BLIS
2.0 building blocks; ML use of tensor operations, "Project Motivation").
The Function is functional: it never writes into C0.  Gradients take their
input's strides when that input is dense (torch's preserve_format), so the
engine accumulates them without a layout copy.
"""
from __future__ import annotations

import torch

from . import contract as _contract


class ContractFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha, A, la, B, lb, beta, C0, lc, compute="native"):
        if C0 is not None:
            C = C0.detach().clone()
            _contract(alpha, A.detach(), la, B.detach(), lb, beta, C, lc, compute=compute)
        else:
            C = _contract(alpha, A.detach(), la, B.detach(), lb, 0.0, None, lc, compute=compute)
        ctx.save_for_backward(A, B)
        ctx.cfg = (alpha, la, lb, beta, lc, compute, C0 is not None)
        return C

    @staticmethod
    def backward(ctx, G):
        A, B = ctx.saved_tensors
        alpha, la, lb, beta, lc, compute, has_c0 = ctx.cfg
        dA = dB = dC0 = None
        if ctx.needs_input_grad[1]:
            dA = torch.empty_like(A, memory_format=torch.preserve_format)
            _contract(alpha, G, lc, B.detach(), lb, 0.0, dA, la, compute=compute)
        if ctx.needs_input_grad[3]:
            dB = torch.empty_like(B, memory_format=torch.preserve_format)
            _contract(alpha, A.detach(), la, G, lc, 0.0, dB, lb, compute=compute)
        if has_c0 and ctx.needs_input_grad[6]:
            dC0 = G * beta
        return None, dA, None, dB, None, None, dC0, None, None


def contract_ad(alpha, A, la, B, lb, beta=0.0, C0=None, lc=None, compute="native"):
    """Differentiable contraction: returns a new C (C0 is not modified)."""
    return ContractFn.apply(alpha, A, la, B, lb, beta, C0, lc, compute)
