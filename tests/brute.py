"""Pure-Python enumerator of a labelled contraction (einsum semantics over
strided storage), written independently of the oracle to pin it on tiny
inputs.  Every distinct label is enumerated with itertools.product; for each
full assignment the product A*B is added to the C entry it addresses."""
import itertools


def enumerate_contraction(alpha, a, la, b, lb, beta, c, lc):
    abuf, abase, aext, astr = a
    bbuf, bbase, bext, bstr = b
    cbuf, cbase, cext, cstr = c
    ext = {}
    for labs, exts in ((lc, cext), (la, aext), (lb, bext)):
        for ch, e in zip(labs, exts):
            assert ext.setdefault(ch, e) == e
    labels = sorted(ext)
    acc = {}
    for vals in itertools.product(*[range(ext[ch]) for ch in labels]):
        v = dict(zip(labels, vals))
        ia = abase + sum(v[ch] * s for ch, s in zip(la, astr))
        ib = bbase + sum(v[ch] * s for ch, s in zip(lb, bstr))
        ic = cbase + sum(v[ch] * s for ch, s in zip(lc, cstr))
        acc[ic] = acc.get(ic, 0.0) + float(abuf[ia]) * float(bbuf[ib])
    out = [float(x) for x in cbuf]
    for cvals in itertools.product(*[range(ext[ch]) for ch in lc]):
        ic = cbase + sum(x * s for x, s in zip(cvals, cstr))
        r = alpha * acc.get(ic, 0.0) if alpha != 0 else 0.0
        if beta != 0:
            r = r + beta * float(cbuf[ic])
        out[ic] = r
    return out
