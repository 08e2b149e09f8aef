"""Pins for the CPU oracle: values printed in the paper, brute force, closed
forms, library routines and invariants.  CPU only."""
import itertools
import math

import numpy as np
import pytest

from conftest import golden_lines, read_golden
from oracle import brute, csf, invariants, partial_sort, planner
from oracle.transpose import sort_permutation, transpose


def _digits(x, r):
    return tuple(int(ch) for ch in str(x).zfill(r))


def _tiny(rng, r, n, ext_hi=4):
    """Tiny tensor with duplicates, sorted under a random input order, values tagged."""
    extents = tuple(int(e) for e in rng.integers(1, ext_hi + 1, size=r))
    cols = [rng.integers(0, e, size=n) for e in extents]
    tau = tuple(int(x) for x in rng.permutation(r))
    p = np.lexsort([cols[m] for m in reversed(tau)]) if n else np.zeros(0, np.int64)
    cols = [c[p].astype(np.int32) for c in cols]
    tags = np.arange(n, dtype=np.float64)  # value = input position
    return cols, tags, extents, tau


# ---------------------------------------------------------------- worked example (Sec. 3.3)

def test_worked_example_alg2_traces():
    g = read_golden("worked_example.txt")
    A = [(tuple(d - 1 for d in _digits(x, 4)), j) for j, x in enumerate(g["A.crd"])]
    prefix = tuple(int(m) - 1 for m in g["prefix"])
    mode = int(g["mode"][0]) - 1
    trace = {}
    B = partial_sort.bucketed_partial_sort(A, prefix, mode, 10, trace=trace)
    assert [b + 1 for b in trace["bucket"]] == [int(x) for x in g["bucket"]]
    assert [p + 1 for p in trace["pos"]] == [int(x) for x in g["pos"]]
    assert [p + 1 for p in trace["perm"]] == [int(x) for x in g["perm"]]
    got = ["".join(str(d + 1) for d in crd) for crd, _ in B]
    assert got == g["B.crd"]


def test_worked_example_definition():
    g = read_golden("worked_example.txt")
    digits = [_digits(x, 4) for x in g["A.crd"]]
    crd = [np.array([d[m] for d in digits], dtype=np.int32) for m in range(4)]
    val = np.arange(len(digits), dtype=np.float64)
    sigma = tuple(int(m) - 1 for m in g["sigma"])
    out_crd, out_val = transpose(crd, val, sigma)
    got = ["".join(str(int(out_crd[m][j])) for m in range(4)) for j in range(len(val))]
    assert got == g["B.crd"]
    # and the same through the plan the planner derives for it
    assert planner.plan((0, 1, 2, 3), sigma) == [((0, 1), 3)]


# ---------------------------------------------------------------- definition vs brute force

@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_transpose_matches_brute_force(r):
    rng = np.random.default_rng(100 + r)
    for trial in range(30):
        n = int(rng.integers(0, 65))
        cols, tags, ext, tau = _tiny(rng, r, n)
        for sigma in itertools.permutations(range(r)):
            a_crd, a_val = transpose(cols, tags, sigma)
            b_crd, b_val = brute.brute_transpose(cols, tags, sigma, ext)
            for m in range(r):
                assert np.array_equal(a_crd[m], b_crd[m])
            assert np.array_equal(a_val, b_val)


def test_transpose_invariants_and_round_trip():
    rng = np.random.default_rng(7)
    for trial in range(40):
        r = int(rng.integers(1, 6))
        n = int(rng.integers(0, 200))
        cols, tags, ext, tau = _tiny(rng, r, n, ext_hi=5)
        for sigma in itertools.permutations(range(r)):
            out_crd, out_val = transpose(cols, tags, sigma)
            assert invariants.is_sorted(out_crd, sigma)
            assert invariants.same_multiset(cols, tags, out_crd, out_val)
            assert invariants.is_stable(out_crd, out_val)
            back_crd, back_val = transpose(out_crd, out_val, tau)
            # ties are equal coordinates, so going back restores the input exactly
            for m in range(r):
                assert np.array_equal(back_crd[m], cols[m])
            if sigma == tau:
                assert np.array_equal(out_val, tags)


def test_transpose_moves_value_bits():
    vals = np.array([0.0, -0.0, np.nan, -np.inf, 1e-310], dtype=np.float64)
    bits = vals.view(np.uint64).copy()
    bits[2] = 0x7FF8_0000_DEAD_BEEF  # NaN with a payload
    vals = bits.view(np.float64)
    crd = [np.array([4, 3, 2, 1, 0], dtype=np.int32), np.zeros(5, dtype=np.int32)]
    out_crd, out_val = transpose(crd, vals, (0, 1))
    assert np.array_equal(out_val.view(np.uint64), bits[::-1])


def test_empty_and_single():
    for n in (0, 1):
        crd = [np.zeros(n, np.int32), np.zeros(n, np.int32)]
        val = np.ones(n)
        out_crd, out_val = transpose(crd, val, (1, 0))
        assert len(out_val) == n


def test_csr_to_csc_matches_scipy():
    """A matrix stored row-major transposed to column-major is CSR -> CSC (Sec. 1)."""
    sp = pytest.importorskip("scipy.sparse")
    rng = np.random.default_rng(3)
    n_r, n_c, nnz = 37, 53, 400
    flat = rng.choice(n_r * n_c, size=nnz, replace=False)
    flat.sort()
    rows, cols = (flat // n_c).astype(np.int32), (flat % n_c).astype(np.int32)
    vals = rng.standard_normal(nnz)
    csc = sp.coo_matrix((vals, (rows, cols)), shape=(n_r, n_c)).tocsc()
    csc.sort_indices()
    out_crd, out_val = transpose([rows, cols], vals, (1, 0))
    assert np.array_equal(out_crd[0], csc.indices)
    assert np.array_equal(out_val, csc.data)
    assert np.array_equal(np.bincount(out_crd[1], minlength=n_c), np.diff(csc.indptr))


# ---------------------------------------------------------------- primitives vs their output orders

def test_primitives_reach_their_output_orders():
    """Alg. 1 / Alg. 2 executed on data give a list sorted under the order the
    output equations state, stably."""
    rng = np.random.default_rng(11)
    for trial in range(60):
        r = int(rng.integers(2, 6))
        n = int(rng.integers(1, 120))
        cols, tags, ext, tau = _tiny(rng, r, n)
        A = partial_sort.to_entries(cols, tags)
        for l in range(r):
            for k in range(l, r):
                B = partial_sort.partial_sort(A, tau[:l], tau[k], ext)
                want = planner.partial_sort_order(tau, l, tau[k])
                b_crd = [np.array([e[0][m] for e in B]) for m in range(r)]
                b_tag = np.array([e[1] for e in B])
                ref_crd, ref_tag = transpose(cols, tags, want)
                assert np.array_equal(b_tag, ref_tag), (tau, l, k)


# ---------------------------------------------------------------- planner (Sec. 3.4 - 3.6)

def _parse_order(s):
    return tuple(int(x) for x in s.split())


def test_planner_examples_from_paper():
    for line in golden_lines("planner_examples.txt"):
        kind, args, want = [p.strip() for p in line.split("|")]
        if kind == "calls":
            sigma = _parse_order(args)
            got = planner.quesadilla(sigma)
            assert " ".join(f"({''.join(map(str, pre))}){m}" for pre, m in got) == want
        elif kind == "passes":
            assert len(planner.quesadilla(_parse_order(args))) == int(want)
        elif kind == "follow":
            tau, p = args.split(";")
            assert planner.follow(_parse_order(tau), int(p)) == set(_parse_order(want))
        elif kind == "lower_bound":
            tau, sigma = args.split(";")
            assert planner.lower_bound(_parse_order(tau), _parse_order(sigma)) == int(want)
        else:
            raise AssertionError(kind)


def test_pass_count_histogram_of_fig_eliminated_passes():
    for line in golden_lines("pass_counts.txt"):
        vals = [int(x) for x in line.split()]
        r, counts = vals[0], vals[1:]
        hist = [0] * (r + 1)
        for sigma in itertools.permutations(range(1, r + 1)):
            hist[len(planner.quesadilla(sigma))] += 1
        assert hist[: len(counts)] == counts and sum(hist[len(counts):]) == 0


def _stirling_first_unsigned(n, k):
    # c(n, k) = c(n-1, k-1) + (n-1) c(n-1, k): permutations of n with k cycles
    table = [[0] * (n + 1) for _ in range(n + 1)]
    table[0][0] = 1
    for i in range(1, n + 1):
        for j in range(1, i + 1):
            table[i][j] = table[i - 1][j - 1] + (i - 1) * table[i - 1][j]
    return table[n][k]


@pytest.mark.parametrize("r", [3, 4, 5, 6])
def test_pass_count_closed_form(r):
    """Passes = r - (number of right-to-left minima); the count of permutations
    with j right-to-left minima is the unsigned Stirling number c(r, j)."""
    hist = [0] * (r + 1)
    for sigma in itertools.permutations(range(1, r + 1)):
        calls = planner.quesadilla(sigma)
        rl = sum(1 for i in range(r) if all(sigma[i] < x for x in sigma[i + 1:]))
        assert len(calls) == r - rl
        hist[len(calls)] += 1
    for p in range(r + 1):
        want = _stirling_first_unsigned(r, r - p) if r - p >= 1 else 0
        assert hist[p] == want


def _all_orders(r):
    return list(itertools.permutations(range(r)))


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5])
def test_plan_reaches_sigma_and_meets_lower_bound(r):
    """Thm 3.3 (the plan reaches sigma) and Thm 3.4 (its length is b(tau, sigma))."""
    for tau in _all_orders(r):
        for sigma in _all_orders(r):
            calls = planner.plan(tau, sigma)
            seen = planner.apply_plan_orders(tau, calls)
            assert seen[-1] == sigma
            assert len(calls) == planner.lower_bound(tau, sigma)


@pytest.mark.parametrize("r", [2, 3, 4])
def test_plan_minimal_by_exhaustive_search(r):
    """BFS over every PartialSort sequence: the plan has minimum length, and the
    fewest bucketed calls among minimum-length sequences (Thm 3.4, Thm 3.5)."""
    start = tuple(range(r))
    best = {start: (0, 0)}  # order -> (calls, bucketed calls), lexicographically minimal
    frontier = [start]
    while frontier:
        nxt = []
        for psi in frontier:
            c, b = best[psi]
            for l in range(r):
                for k in range(l, r):
                    new = planner.partial_sort_order(psi, l, psi[k])
                    cand = (c + 1, b + (1 if l > 0 else 0))
                    if new not in best:
                        best[new] = cand
                        nxt.append(new)
                    elif cand[0] == best[new][0] and cand[1] < best[new][1]:
                        best[new] = cand
        frontier = nxt
    for sigma in _all_orders(r):
        calls = planner.plan(start, sigma)
        want_len, want_bucketed = best[sigma] if sigma != start else (0, 0)
        assert len(calls) == want_len
        assert sum(1 for pre, _ in calls if pre) == want_bucketed


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_plans_execute_to_the_definition(r):
    """Quesadilla, Top-K-sadilla and LSD radix, executed with Alg. 1/2 on tiny
    tensors with duplicates, all equal the stable sort under sigma."""
    rng = np.random.default_rng(50 + r)
    for trial in range(12):
        n = int(rng.integers(0, 80))
        cols, tags, ext, tau = _tiny(rng, r, n)
        A = partial_sort.to_entries(cols, tags)
        for sigma in _all_orders(r):
            _, ref = transpose(cols, tags, sigma)
            q = partial_sort.run_quesadilla(A, tau, sigma, ext)
            assert np.array_equal(np.array([e[1] for e in q]), ref)
            for K in range(0, r + 1):
                t = partial_sort.run_topk(A, tau, sigma, K, ext)
                assert np.array_equal(np.array([e[1] for e in t]), ref)
            s = partial_sort.run_lsd(A, sigma, ext)
            assert np.array_equal(np.array([e[1] for e in s]), ref)


def test_rl_minima_helper_matches_follow_sets():
    for r in range(1, 6):
        for tau in _all_orders(r):
            for sigma in _all_orders(r):
                rl = set(planner.rl_minima(tau, sigma))
                fs = {m for m in sigma if planner.follow(sigma, m) <= planner.follow(tau, m)}
                assert rl == fs


# ---------------------------------------------------------------- CSF

def test_csf_round_trip_and_counts():
    rng = np.random.default_rng(5)
    for trial in range(40):
        r = int(rng.integers(1, 5))
        n = int(rng.integers(0, 100))
        cols, tags, ext, tau = _tiny(rng, r, n)
        sigma = tuple(int(x) for x in rng.permutation(r))
        s_crd, _ = transpose(cols, tags, sigma)
        pos, lev = csf.pack_csf(s_crd, sigma)
        back = csf.unpack_csf(pos, lev, sigma)
        for m in range(r):
            assert list(back[m]) == list(s_crd[m])
        assert len(pos[0]) == 2 and pos[0][0] == 0
        for d in range(1, r + 1):
            assert pos[d - 1][-1] == len(lev[d - 1])
            assert all(a <= b for a, b in zip(pos[d - 1], pos[d - 1][1:]))
            if d > 1:
                assert len(pos[d - 1]) == len(lev[d - 2]) + 1
            # fibers at level d = distinct prefixes (sigma_1..sigma_d), leaves = nnz
            if d < r:
                pref = {tuple(int(s_crd[m][j]) for m in sigma[:d]) for j in range(n)}
                assert len(lev[d - 1]) == len(pref)
        if r:
            assert len(lev[r - 1]) == n


def test_csf_two_modes_is_doubly_compressed_csr():
    sp = pytest.importorskip("scipy.sparse")
    rng = np.random.default_rng(9)
    n_r, n_c, nnz = 40, 30, 150
    flat = np.sort(rng.choice(n_r * n_c, size=nnz, replace=False))
    rows, cols = (flat // n_c).astype(np.int32), (flat % n_c).astype(np.int32)
    m = sp.csr_matrix((np.ones(nnz), (rows, cols)), shape=(n_r, n_c))
    pos, lev = csf.pack_csf([rows, cols], (0, 1))
    nonempty = np.nonzero(np.diff(m.indptr))[0]
    assert lev[0] == list(nonempty)
    assert pos[1] == list(np.unique(m.indptr))  # row pointers with empty rows dropped
    assert lev[1] == list(m.indices)
