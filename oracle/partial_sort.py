"""Oracle: the two PartialSort primitives, step by step.  TEST INFRASTRUCTURE ONLY.

A tensor here is a Python list of entries (coordinate tuple, value); the
coordinate tuple is indexed by mode (0-based).  Positions are 0-based, so the
paper's "count[1] <- 1" and "pos[1] <- 1" (1-based starting positions) become
starting positions of 0.  Pure Python loops: meant for small inputs.

* histogram_partial_sort (Alg. 1): count the keys of the sorted mode, prefix-sum
  the counts into starting positions, move every entry to its position in input
  order.  Stable, so the mode moves to the front of the order (Sec. 3.1).
* bucketed_partial_sort (Alg. 2): one scan records the buckets (runs of equal
  prefix coordinates: bucket id per entry and the start of every bucket) and the
  key counts; a stable counting sort on the mode builds perm; a final pass walks
  perm and drops every entry into the next free slot of its own bucket, which
  restores the prefix order (Sec. 3.2).
* run_calls: a list of calls (prefix, mode) executed with the primitives above.
* run_topk: Quesadilla towards the Top-K target, then every bucket of equal
  (sigma_1..sigma_K) sorted completely (Sec. 3.6) with a stable comparison sort.
"""
from . import planner


def histogram_partial_sort(A, mode, extent):
    """Alg. 1: stable counting sort of A on one mode.  Returns B."""
    count = [0] * (extent + 1)
    for crd, _ in A:  # count loop
        count[crd[mode] + 1] += 1
    for i in range(1, extent + 1):  # prefix sum: count[v] = first slot of key v
        count[i] += count[i - 1]
    B = [None] * len(A)
    for entry in A:  # move loop, input order
        i = entry[0][mode]
        B[count[i]] = entry
        count[i] += 1
    return B


def bucketed_partial_sort(A, prefix, mode, extent, trace=None):
    """Alg. 2: stable sort of A on `mode` that keeps the order on `prefix`.

    A must already be sorted on the prefix modes.  When `trace` is a dict it
    receives the bucket, pos and perm arrays (0-based) for inspection.
    """
    n = len(A)
    if n == 0:
        return []
    count = [0] * (extent + 1)
    bucket = [0] * n
    pos = [0] * n
    perm = [0] * n
    nb = 0  # id of the current bucket
    pos[0] = 0
    count[A[0][0][mode] + 1] += 1
    for j in range(1, n):  # bucket discovery + count loop
        cur = tuple(A[j][0][m] for m in prefix)
        prev = tuple(A[j - 1][0][m] for m in prefix)
        if cur != prev:
            nb += 1
            pos[nb] = j
        bucket[j] = nb
        count[A[j][0][mode] + 1] += 1
    for i in range(1, extent + 1):  # prefix sum
        count[i] += count[i - 1]
    for j in range(n):  # stable counting sort on the mode: perm
        i = A[j][0][mode]
        perm[count[i]] = j
        count[i] += 1
    if trace is not None:
        trace["bucket"] = list(bucket)
        trace["pos"] = list(pos[: nb + 1])
        trace["perm"] = list(perm)
    B = [None] * n
    for j in range(n):  # re-impose the prefix order: stable sort on bucket
        b = bucket[perm[j]]
        B[pos[b]] = A[perm[j]]
        pos[b] += 1
    return B


def partial_sort(A, prefix, mode, extents):
    """PartialSort: Alg. 1 when the prefix is empty, Alg. 2 otherwise."""
    if len(prefix) == 0:
        return histogram_partial_sort(A, mode, extents[mode])
    return bucketed_partial_sort(A, prefix, mode, extents[mode])


def run_calls(A, calls, extents):
    for prefix, mode in calls:
        A = partial_sort(A, prefix, mode, extents)
    return A


def run_quesadilla(A, tau_in, sigma, extents):
    return run_calls(A, planner.plan(tau_in, sigma), extents)


def run_topk(A, tau_in, sigma, K, extents):
    calls, K = planner.topk_plan(tau_in, sigma, K)
    A = run_calls(A, calls, extents)
    head = tuple(sigma[:K])
    out, j, n = [], 0, len(A)
    while j < n:  # walk the buckets of equal (sigma_1..sigma_K)
        e = j
        key = tuple(A[j][0][m] for m in head)
        while e < n and tuple(A[e][0][m] for m in head) == key:
            e += 1
        # Python's sort is stable: ties keep their current (input) order
        out.extend(sorted(A[j:e], key=lambda ent: tuple(ent[0][m] for m in sigma)))
        j = e
    return out


def run_lsd(A, sigma, extents):
    return run_calls(A, planner.lsd_plan(sigma), extents)


def to_entries(crd, val):
    r = len(crd)
    return [(tuple(int(crd[m][j]) for m in range(r)), val[j]) for j in range(len(val))]
