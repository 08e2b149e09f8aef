"""Oracle: transposition by its definition.  TEST INFRASTRUCTURE ONLY.

A tensor in COO is a list of nonzeros (coordinate tuple, value) kept in a
lexicographic order of its modes (Sec. 2, Sec. 2.1).  Transposition is a change
of that storage order (Sec. 2.2): the same nonzeros, re-listed so that they are
sorted under the requested complete order sigma.  Coordinate i precedes i' under
sigma when i[sigma_1] < i'[sigma_1], or they tie there and i precedes i' under
(sigma_2, ...); all tuples tie under the empty order (Sec. 2).

The paper assumes distinct coordinates.  Its primitives (Alg. 1, Alg. 2) are
stable, so nonzeros whose coordinates tie keep the order they had in the input.
This oracle adopts that as the contract for duplicates: the output is the
STABLE sort of the input under sigma, which is unique, so results can be
compared bit for bit.  Values are an opaque payload moved without arithmetic.

Implementation: ``numpy.lexsort`` (an indirect stable sort over several keys,
last key primary) serves as the stable-sort step; the gather then copies bits.
Modes are 0-based here (the paper counts from 1).
"""
import numpy as np


def _check_sigma(sigma, r):
    sigma = tuple(int(m) for m in sigma)
    if sorted(sigma) != list(range(r)):
        raise ValueError(f"sigma={sigma} is not a complete order of {r} modes")
    return sigma


def sort_permutation(crd, sigma):
    """Positions of the input nonzeros listed in sigma order (stable).

    crd   : sequence of r 1-D integer arrays (structure of arrays), length N each
    sigma : complete order of the r modes, most significant first
    Returns an int64 array p with output[j] = input[p[j]].
    """
    r = len(crd)
    sigma = _check_sigma(sigma, r)
    n = len(crd[0]) if r else 0
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    # lexsort sorts by its LAST key first, so pass the modes least significant first.
    keys = [np.asarray(crd[m]) for m in reversed(sigma)]
    return np.lexsort(keys).astype(np.int64)


def transpose(crd, val, sigma):
    """Return (out_crd, out_val): the nonzeros stably re-sorted under sigma.

    The arrays keep their dtypes; values are gathered as raw bits so that
    signed zeros and NaN payloads survive.
    """
    p = sort_permutation(crd, sigma)
    out_crd = [np.ascontiguousarray(np.asarray(c)[p]) for c in crd]
    v = np.asarray(val)
    bits = v.view(np.uint64 if v.dtype.itemsize == 8 else np.uint32)
    out_val = np.ascontiguousarray(bits[p]).view(v.dtype)
    return out_crd, out_val
