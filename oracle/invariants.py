"""Properties every correct transposition has.  TEST INFRASTRUCTURE ONLY.

They hold at any size, so tests use them where a full oracle run is too slow:

* sorted:      adjacent output nonzeros are non-decreasing under sigma (Sec. 2);
* permutation: the output is a rearrangement of the input nonzeros, values
               included (transposition only changes storage order, Sec. 2.2);
* stable:      nonzeros whose coordinates tie keep their input order.
"""
import numpy as np


def lex_le_adjacent(crd, sigma):
    """Boolean array: element j <= element j+1 under sigma, for every j."""
    n = len(crd[0])
    if n < 2:
        return np.ones(0, dtype=bool)
    lt = np.zeros(n - 1, dtype=bool)
    eq = np.ones(n - 1, dtype=bool)
    for m in sigma:
        a = np.asarray(crd[m][:-1])
        b = np.asarray(crd[m][1:])
        lt |= eq & (a < b)
        eq &= a == b
    return lt | eq


def is_sorted(crd, sigma):
    return bool(np.all(lex_le_adjacent(crd, sigma)))


def _records(crd, val):
    v = np.asarray(val)
    bits = v.view(np.uint64 if v.dtype.itemsize == 8 else np.uint32).astype(np.uint64)
    cols = [np.asarray(c).astype(np.int64) for c in crd] + [bits.astype(np.int64)]
    return np.stack(cols, axis=1) if len(bits) else np.zeros((0, len(cols)), np.int64)


def same_multiset(crd_a, val_a, crd_b, val_b):
    """True when both lists hold the same (coordinates, value bits) multiset."""
    ra = _records(crd_a, val_a)
    rb = _records(crd_b, val_b)
    if ra.shape != rb.shape:
        return False
    if len(ra) == 0:
        return True
    ka = ra[np.lexsort(ra.T[::-1])]
    kb = rb[np.lexsort(rb.T[::-1])]
    return bool(np.array_equal(ka, kb))


def is_stable(out_crd, tags):
    """tags[j] = input position of output element j.  Ties must keep input order."""
    n = len(tags)
    if n < 2:
        return True
    eq = np.ones(n - 1, dtype=bool)
    for c in out_crd:
        c = np.asarray(c)
        eq &= c[:-1] == c[1:]
    t = np.asarray(tags)
    return bool(np.all(t[:-1][eq] < t[1:][eq]))
