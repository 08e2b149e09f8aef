"""Oracle: the 32 features the schedule selector reads.  TEST INFRASTRUCTURE ONLY.

The features describe what the paper identifies as the drivers of run time: how many
passes a plan makes and how many of them are bucketed (Sec. 3.4-3.6, Sec. 5), the bit widths
of the sorted modes (large extents make the count arrays large, Sec. 4.2), and the structure
of the data (how many distinct values a mode takes, how skewed it is, and how often it
changes between neighbouring nonzeros of the input, which sets the bucket sizes of
Alg. 2).

Sample.  With N nonzeros and S = min(N, 16384), the sampled positions are
j_k = floor(k N / S), k = 0..S-1.  A sampled pair is (j_k, j_k + 1) when j_k + 1 < N.

Per mode m, three exact integer counts over the sample:
  zero_m    zero bits of a 65536-bit map after setting bit (h(x) mod 2^16) for every
            sampled coordinate x, where h is the SplitMix64 output function applied to
            the coordinate as a 64-bit integer (Steele, Lea and Flood, OOPSLA 2014);
  top_m     the largest count of one bucket ((h(x) >> 16) mod 1024) over the sample;
  change_m  sampled pairs whose coordinates in mode m differ.
For a set of modes P: change_P = sampled pairs that differ in at least one mode of P.

Distinct values are estimated by linear counting (Whang, Vander-Zanden and Taylor, ACM TODS
1990): D = -M ln(zero / M) with M = 65536 (D = M ln M when no bit is zero).

Feature vector (bits(n) = ceil(log2 n), 0 for n = 1; slot i is mode sigma_{i+1}; slots past
the order are zero; K = min(2, r - 2) as for the Top-K schedule):
  0           log2(N) / 32
  1           r / 8
  2 + 4i      bits(n_sigma_i) / 32                        (i = 0..4)
  3 + 4i      log2(1 + D_sigma_i) / 24
  4 + 4i      change_sigma_i / pairs
  5 + 4i      top_sigma_i / S
  22, 23      minimal plan (Alg. 3): plain calls / 8, bucketed calls / 8
  24, 25      minimal plan: key bits of plain calls / 64, of bucketed calls / 64
  26, 27      Top-K plan: key bits of plain calls / 64; key bits of bucketed calls plus the
              bits of sigma_{K+1..r} when K > 0 (the per-bucket complete sort) / 64
  28          full LSD plan: key bits of all modes / 64
  29          change_P / pairs for P = the prefix of the minimal plan's first bucketed call
              (0 when it has none)
  30          change_P / pairs for P = (sigma_1..sigma_K) (0 when K = 0)
  31          log2(1 + feature29 * N) / 32
Parity: the counts are pinned by brute-force recounting in the tests and by closed forms
(constant modes, all-distinct modes); the plan terms by the planner's own pins.
"""
import math

import numpy as np

from . import planner

NFEAT = 32
SAMPLE = 16384
BITMAP_BITS = 1 << 16
BUCKETS = 1024
SLOTS = 5
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


def plan_terms(extents, tau_in, sigma):
    """Call and key-bit counts of the three schedules, and the two bucket prefixes."""
    r = len(sigma)
    bits = [bits_for_extent(n) for n in extents]
    s1 = planner.plan(tau_in, sigma)
    K = max(0, min(2, r - 2))
    s2, _ = planner.topk_plan(tau_in, sigma, K)
    plain1 = [m for pre, m in s1 if not pre]
    buck1 = [(pre, m) for pre, m in s1 if pre]
    plain2 = [m for pre, m in s2 if not pre]
    buck2 = [m for pre, m in s2 if pre]
    tail2 = sum(bits[m] for m in sigma[K:]) if K > 0 else 0
    return dict(
        s1_plain_calls=len(plain1), s1_bucket_calls=len(buck1),
        s1_plain_bits=sum(bits[m] for m in plain1), s1_bucket_bits=sum(bits[m] for _, m in buck1),
        s2_plain_bits=sum(bits[m] for m in plain2), s2_bucket_bits=sum(bits[m] for m in buck2) + tail2,
        s3_bits=sum(bits), prefix1=tuple(buck1[0][0]) if buck1 else (), prefix2=tuple(sigma[:K]))


def features(crd, extents, tau_in, sigma):
    """The 32 features (float64) of transposing (crd, sorted under tau_in) to sigma."""
    r = len(sigma)
    n = len(crd[0])
    pt = plan_terms(extents, tau_in, sigma)
    masks = [pt["prefix1"], pt["prefix2"]]
    per_mode, mch, S, pairs = counts(crd, masks)
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
    f[22] = pt["s1_plain_calls"] / 8
    f[23] = pt["s1_bucket_calls"] / 8
    f[24] = pt["s1_plain_bits"] / 64
    f[25] = pt["s1_bucket_bits"] / 64
    f[26] = pt["s2_plain_bits"] / 64
    f[27] = pt["s2_bucket_bits"] / 64
    f[28] = pt["s3_bits"] / 64
    f[29] = mch[0] / pairs if (pairs and pt["prefix1"]) else 0.0
    f[30] = mch[1] / pairs if (pairs and pt["prefix2"]) else 0.0
    f[31] = math.log2(1.0 + f[29] * n) / 32
    return f
