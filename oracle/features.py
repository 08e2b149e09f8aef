"""Oracle: the 40 features the schedule selector reads.  TEST INFRASTRUCTURE ONLY.

The features describe what the paper identifies as the drivers of run time: how many
passes a plan makes and how many of them are bucketed (Sec. 3.4-3.6, Sec. 5), the bit widths
of the sorted modes (large extents make the count arrays large, Sec. 4.2), and the structure
of the data (how many distinct values a mode takes, how skewed it is, and how often it
changes between neighbouring nonzeros of the input, which sets the bucket sizes of
Alg. 2).

Candidates (the schedules the selector chooses between; every one gives the same output):
  0  MINIMAL (Alg. 3), bucketed groups run as one global sort where that is cheaper
  1  MINIMAL with every bucketed group kept as bucket sorts        (valid when it differs from 0)
  2  Top-K-sadilla with K = 1 (Sec. 3.6)                            (valid when K <= r - 2)
  3  Top-K-sadilla with K = 2                                       (valid when K <= r - 2)
  4  Top-K-sadilla with K = 3                                       (valid when K <= r - 2)
  5  full LSD radix sort over all modes                             (valid when r >= 2)
(K = r - 1 plans exactly what MINIMAL plans, so it is not a candidate of its own.)

Sample.  With N nonzeros and S = min(N, 16384), the sampled positions are
j_k = floor(k N / S), k = 0..S-1.  A sampled pair is (j_k, j_k + 1) when j_k + 1 < N.

Per mode m, three exact integer counts over the sample:
  zero_m    zero bits of a 65536-bit map after setting bit (h(x) mod 2^16) for every
            sampled coordinate x, where h is the SplitMix64 output function applied to
            the coordinate as a 64-bit integer (Steele, Lea and Flood, OOPSLA 2014);
  top_m     the largest count of one bucket ((h(x) >> 16) mod 1024) over the sample;
  change_m  sampled pairs whose coordinates in mode m differ.
For a set of modes Q: change_Q = sampled pairs that differ in at least one mode of Q.  The
sets: Q0 = the kept prefix of the minimal plan's first bucketed call (empty when it has none),
Q1, Q2, Q3 = (sigma_1..sigma_K) for K = 1, 2, 3 (empty when K > r - 2).

Distinct values are estimated by linear counting (Whang, Vander-Zanden and Taylor, ACM TODS
1990): D = -M ln(zero / M) with M = 65536 (D = M ln M when no bit is zero).

Plan terms of a candidate: its groups (consecutive partial sorts that keep the same prefix,
as the library runs them), with modes of extent 1 dropped from the keys; a bucketed group is
run as one global sort on (prefix, keys) when its key is wider than 52 bits, or (candidate 0
and the Top-K candidates) when every nonzero packs into 64 bits, the flattened key is at most
64 bits and it needs at most one digit pass more than the key alone.  A key of B bits is
cut into 64-bit sub-keys and each into ceil(b / 8) digit passes.
  gp  digit passes of the global groups;   sb  key bits of the bucketed groups.

Feature vector (bits(n) = ceil(log2 n), 0 for n = 1; slot i is mode sigma_{i+1}; slots past
the order are zero):
  0           log2(N) / 32
  1           r / 8
  2 + 4i      bits(n_sigma_i) / 32                        (i = 0..4)
  3 + 4i      log2(1 + D_sigma_i) / 24
  4 + 4i      change_sigma_i / pairs
  5 + 4i      top_sigma_i / S
  22, 23      coordinate bytes / 8, value bytes / 8
  24 + 2c     candidate c: gp / 16                         (c = 0..5; 0 when not valid)
  25 + 2c     candidate c: sb / 64
  36 + q      change_Qq / pairs                            (q = 0..3; 0 for an empty set)
Parity: the counts are pinned by brute-force recounting in the tests and by closed forms
(constant modes, all-distinct modes); the plan terms by the planner's own pins and by hand
on small cases; the whole vector by a hand-derived golden example.
"""
import math

import numpy as np

from . import planner

NFEAT = 40
NCAND = 6
SAMPLE = 16384
BITMAP_BITS = 1 << 16
BUCKETS = 1024
SLOTS = 5
RADIX = 8
MASK64 = (1 << 64) - 1


def bits_for_extent(n):
    return (int(n) - 1).bit_length() if n > 1 else 0


def mix64(x):
    """SplitMix64's output function on uint64 arrays."""
    z = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def sample_positions(n):
    s = min(int(n), SAMPLE)
    k = np.arange(s, dtype=np.int64)
    return (k * int(n)) // s if s else k


def counts(crd, masks=()):
    """Integer counts: per mode (zero, top, change); per mode set in `masks` its change count;
    and (S, pairs)."""
    n = len(crd[0]) if crd else 0
    j = sample_positions(n)
    S = len(j)
    pj = j[j + 1 < n]
    pairs = len(pj)
    per_mode = []
    for c in crd:
        x = np.asarray(c).astype(np.int64).astype(np.uint64)[j]
        h = mix64(x)
        seen = np.zeros(BITMAP_BITS, dtype=bool)
        seen[(h & np.uint64(BITMAP_BITS - 1)).astype(np.int64)] = True
        zero = int(BITMAP_BITS - seen.sum())
        b = ((h >> np.uint64(16)) & np.uint64(BUCKETS - 1)).astype(np.int64)
        top = int(np.bincount(b, minlength=BUCKETS).max()) if S else 0
        cc = np.asarray(c)
        change = int(np.count_nonzero(cc[pj] != cc[pj + 1]))
        per_mode.append((zero, top, change))
    mask_changes = []
    for P in masks:
        diff = np.zeros(pairs, dtype=bool)
        for m in P:
            cc = np.asarray(crd[m])
            diff |= cc[pj] != cc[pj + 1]
        mask_changes.append(int(np.count_nonzero(diff)))
    return per_mode, mask_changes, S, pairs


def linear_count(zero):
    M = float(BITMAP_BITS)
    return M * math.log(M) if zero == 0 else -M * math.log(zero / M)


def _passes(key_bits):
    """Digit passes of a key: 64-bit sub-keys, each cut into ceil(b / 8) digits."""
    d, left = 0, key_bits
    while left > 0:
        b = min(64, left)
        d += -(-b // RADIX)
        left -= b
    return d


def _groups(calls):
    """Consecutive calls with the same kept prefix -> (prefix, keys most significant first)."""
    out = []
    for pre, m in calls:
        if out and out[-1][0] == tuple(pre):
            out[-1][1].insert(0, m)
        else:
            out.append((tuple(pre), [m]))
    return out


def _run_groups(groups, bits, keep_buckets):
    """(global digit passes, bucketed key bits) of groups as the library runs them."""
    total = sum(bits)
    gp = sb = 0
    for pre, keys in groups:
        keys = [m for m in keys if bits[m] > 0]
        if not keys:
            continue
        kb = sum(bits[m] for m in keys)
        if not pre:
            gp += _passes(kb)
            continue
        pb = sum(bits[m] for m in pre)
        flat = kb > 52 or (not keep_buckets and total <= 64 and pb + kb <= 64 and
                           -(-(pb + kb) // RADIX) <= -(-kb // RADIX) + 1)
        if flat:
            gp += _passes(pb + kb)
        else:
            sb += kb
    return gp, sb


def candidate_groups(tau_in, sigma, c):
    """Groups of candidate c (None when the candidate is not valid for this request)."""
    r = len(sigma)
    if c in (0, 1):
        return _groups(planner.plan(tau_in, sigma))
    if c in (2, 3, 4):
        K = c - 1
        if K > r - 2:
            return None
        calls, _ = planner.topk_plan(tau_in, sigma, K)
        g = _groups(calls)
        pos = {m: i for i, m in enumerate(tau_in)}
        q = r - 1
        while q - 1 >= K and pos[sigma[q - 1]] < pos[sigma[q]]:
            q -= 1
        tail = list(sigma[K:q])
        if tail:
            g.append((tuple(sigma[:K]), tail))
        return g
    if c == 5:
        return [((), list(sigma))] if r >= 2 else None
    raise ValueError(c)


def plan_terms(extents, tau_in, sigma):
    """Per candidate (gp, sb) or None, and the four mode sets Q0..Q3."""
    r = len(sigma)
    bits = [bits_for_extent(n) for n in extents]
    terms = []
    for c in range(NCAND):
        g = candidate_groups(tau_in, sigma, c)
        terms.append(None if g is None else _run_groups(g, bits, keep_buckets=(c == 1)))
    if _same_execution(tau_in, sigma, bits):
        terms[1] = None
    s1 = planner.plan(tau_in, sigma)
    buck = [pre for pre, _ in s1 if pre]
    Q = [tuple(buck[0]) if buck else ()]
    for K in (1, 2, 3):
        Q.append(tuple(sigma[:K]) if K <= r - 2 else ())
    return terms, Q


def _same_execution(tau_in, sigma, bits):
    """Candidate 1 runs differently from candidate 0 exactly when some bucketed group of the
    minimal plan is flattened without the flag (and kept with it)."""
    total = sum(bits)
    for pre, keys in _groups(planner.plan(tau_in, sigma)):
        keys = [m for m in keys if bits[m] > 0]
        if not pre or not keys:
            continue
        kb = sum(bits[m] for m in keys)
        pb = sum(bits[m] for m in pre)
        if kb <= 52 and total <= 64 and pb + kb <= 64 and -(-(pb + kb) // RADIX) <= -(-kb // RADIX) + 1:
            return False
    return True


def valid_candidates(extents, tau_in, sigma):
    terms, _ = plan_terms(extents, tau_in, sigma)
    return [t is not None for t in terms]


def features(crd, extents, tau_in, sigma, crd_bytes=4, val_bytes=8):
    """The 40 features (float64) of transposing (crd, sorted under tau_in) to sigma."""
    r = len(sigma)
    n = len(crd[0])
    terms, Q = plan_terms(extents, tau_in, sigma)
    per_mode, mch, S, pairs = counts(crd, Q)
    f = np.zeros(NFEAT)
    f[0] = math.log2(n) / 32 if n > 0 else 0.0
    f[1] = r / 8
    for i in range(min(r, SLOTS)):
        m = sigma[i]
        zero, top, change = per_mode[m]
        f[2 + 4 * i] = bits_for_extent(extents[m]) / 32
        f[3 + 4 * i] = math.log2(1.0 + linear_count(zero)) / 24 if S else 0.0
        f[4 + 4 * i] = change / pairs if pairs else 0.0
        f[5 + 4 * i] = top / S if S else 0.0
    f[22] = crd_bytes / 8
    f[23] = val_bytes / 8
    for c, t in enumerate(terms):
        if t is not None:
            f[24 + 2 * c] = t[0] / 16
            f[25 + 2 * c] = t[1] / 64
    for q in range(4):
        f[36 + q] = mch[q] / pairs if (pairs and Q[q]) else 0.0
    return f
