"""Hand-written backward for the contraction.

For  C = alpha * sum_P A[I,P] B[P,J] + beta * C0  and upstream gradient G[I,J]:

    dA[I,P] = alpha * sum_J G[I,J] B[P,J]      (a contraction over J)
    dB[P,J] = alpha * sum_I A[I,P] G[I,J]      (a contraction over I)
    dC0     = beta * G

Both gradients are themselves labelled contractions, so they run on the
same planner and kernels as the forward (the paper's aim of one engine
reused across operations, Section "Building on important advances", BLIS
2.0 building blocks; ML use of tensor operations, "Project Motivation").
dC0 is G copied into C0's layout and scaled by the engine's own C update
(a contraction with alpha = 0).

Labels that the forward folds into the GEMM view need one more step on the
way back:

* a label repeated within an input (a diagonal): the gradient is zero off
  the diagonal, so the gradient tensor is zero-filled and the contraction
  writes into its diagonal view (one mode per distinct label, strides of
  the repeats summed -- injective whenever the input's layout is);
* a label only in that input (summed inside it): the gradient does not
  depend on it, so the contraction runs without it and its result is
  broadcast along it.

The Function is functional: it never writes into C0.  Gradients take their
input's strides when that input is dense (torch's preserve_format), so the
engine accumulates them without a layout copy.

dA and dB do not depend on each other, so when both are needed dB runs on a
second stream of the same device beside dA (each contraction's last round
of tiles then overlaps the other's): every tensor is allocated on the
caller's stream, the second stream waits for the caller's work before it
starts and the caller's stream waits for it before the gradients are used.
"""
from __future__ import annotations

import torch

from . import _labels
from . import contract as _contract


_side_streams = {}


def _side_stream(device):
    """One extra stream per device (default priority) for dB."""
    s = _side_streams.get(device)
    if s is None:
        s = torch.cuda.Stream(device=device)
        _side_streams[device] = s
    return s


def _operand_grad(alpha, G, lc, other, lo, target, lt, compute, g_first, stream=None):
    """Gradient with respect to `target` (labels lt): alpha times the
    contraction of G (labels lc) with the other operand (labels lo) onto
    target's labels, in a tensor laid out like target.  Labels are taken as
    integer codes (a string's characters or a sequence of ints)."""
    lc, lo, lt = _labels(lc), _labels(lo), list(_labels(lt))
    uniq = []
    for ch in lt:
        if ch not in uniq:
            uniq.append(ch)
    kept = [ch for ch in uniq if ch in lc or ch in lo]

    def run(out, labels):
        if g_first:
            return _contract(alpha, G, lc, other, lo, 0.0, out, labels, compute=compute, stream=stream)
        return _contract(alpha, other, lo, G, lc, 0.0, out, labels, compute=compute, stream=stream)

    if len(uniq) == len(lt) and len(kept) == len(uniq):
        grad = torch.empty_like(target, memory_format=torch.preserve_format)
        run(grad, lt)
        return grad
    grad = torch.empty_like(target, memory_format=torch.preserve_format)
    if stream is not None:  # the fill belongs to the stream that writes the gradient
        with torch.cuda.stream(stream):
            grad.zero_()
    else:
        grad.zero_()
    ext = {ch: target.shape[i] for i, ch in enumerate(lt)}
    stride = {ch: 0 for ch in uniq}
    for i, ch in enumerate(lt):
        stride[ch] += grad.stride(i)
    view = grad.as_strided([ext[ch] for ch in uniq], [stride[ch] for ch in uniq], grad.storage_offset())
    if len(kept) == len(uniq):
        run(view, uniq)
    else:
        red = torch.empty([ext[ch] for ch in kept], dtype=target.dtype, device=target.device)
        run(red, kept)  # modes in `kept` order (a subsequence of `uniq`)
        shape = [ext[ch] if ch in kept else 1 for ch in uniq]
        if stream is not None:
            with torch.cuda.stream(stream):
                view.copy_(red.reshape(shape).expand(view.shape))
        else:
            view.copy_(red.reshape(shape).expand(view.shape))
    return grad


class ContractFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha, A, la, B, lb, beta, C0, lc, compute="native"):
        if C0 is not None:
            C = C0.detach().clone()
            _contract(alpha, A.detach(), la, B.detach(), lb, beta, C, lc, compute=compute)
        else:
            C = _contract(alpha, A.detach(), la, B.detach(), lb, 0.0, None, lc, compute=compute)
        ctx.save_for_backward(A, B, C0 if C0 is not None else None)
        ctx.cfg = (alpha, la, lb, beta, lc, compute, C0 is not None)
        return C

    @staticmethod
    def backward(ctx, G):
        A, B, C0 = ctx.saved_tensors
        alpha, la, lb, beta, lc, compute, has_c0 = ctx.cfg
        dA = dB = dC0 = None
        both = ctx.needs_input_grad[1] and ctx.needs_input_grad[3] and G.is_cuda
        if both:
            cur = torch.cuda.current_stream(G.device)
            side = _side_stream(G.device)
            side.wait_stream(cur)  # G, A, B and the new gradients' memory are ready
            dB = _operand_grad(alpha, G, lc, A.detach(), la, B, lb, compute, False, stream=side)
            dA = _operand_grad(alpha, G, lc, B.detach(), lb, A, la, compute, True)
            cur.wait_stream(side)
        else:
            if ctx.needs_input_grad[1]:
                dA = _operand_grad(alpha, G, lc, B.detach(), lb, A, la, compute, True)
            if ctx.needs_input_grad[3]:
                dB = _operand_grad(alpha, G, lc, A.detach(), la, B, lb, compute, False)
        if has_c0 and ctx.needs_input_grad[6]:
            dC0 = torch.empty_like(C0, memory_format=torch.preserve_format)
            if beta != 0.0:
                dC0.copy_(G)
            # alpha = 0: the engine's C update alone, dC0 = beta * dC0 (zeros
            # when beta == 0, without reading dC0)
            _contract(0.0, A.detach(), la, B.detach(), lb, beta, dC0, lc, compute=compute)
        return None, dA, None, dB, None, None, dC0, None, None


def contract_ad(alpha, A, la, B, lb, beta=0.0, C0=None, lc=None, compute="native"):
    """Differentiable contraction: returns a new C (C0 is not modified)."""
    return ContractFn.apply(alpha, A, la, B, lb, beta, C0, lc, compute)
