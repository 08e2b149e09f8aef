"""Oracle pin: transposition with no sort at all.  TEST INFRASTRUCTURE ONLY.

The sigma order of Sec. 2 can be produced by walking the whole (dense)
coordinate space with nested loops, the outermost loop over mode sigma_1 and
the innermost over sigma_r, and emitting at each coordinate every nonzero that
carries it, in input order (the stability contract for ties).  This needs no
comparison or counting sort, so it is an independent check of
``oracle.transpose`` on tiny tensors (a few modes, extents of a few units).
"""
import itertools

import numpy as np


def brute_transpose(crd, val, sigma, extents):
    r = len(crd)
    n = len(val)
    where = {}
    for j in range(n):
        key = tuple(int(crd[m][j]) for m in range(r))
        where.setdefault(key, []).append(j)
    order = []
    # itertools.product varies its LAST factor fastest: give it the modes in
    # sigma order so that sigma_1 is the outermost loop.
    for c in itertools.product(*[range(int(extents[m])) for m in sigma]):
        key = [0] * r
        for pos, m in enumerate(sigma):
            key[m] = c[pos]
        order.extend(where.get(tuple(key), ()))
    assert len(order) == n, "some nonzero lies outside the stated extents"
    p = np.asarray(order, dtype=np.int64)
    out_crd = [np.asarray(c)[p] for c in crd]
    out_val = np.asarray(val)[p]
    return out_crd, out_val
