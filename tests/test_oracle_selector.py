"""Pins of the selector's oracle parts (CPU): the MLP's gradient against central finite
differences, closed forms of the network and of Adam, the published SplitMix64 outputs, and
the feature counts against brute-force recounting and closed forms."""
import itertools
import math

import numpy as np
import pytest

from oracle import features as F
from oracle import mlp


def test_splitmix64_published_outputs():
    # first outputs of SplitMix64 seeded with 1234567, as published with the generator
    r = mlp.SplitMix64(1234567)
    assert [r.next() for _ in range(5)] == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                            4593380528125082431, 16408922859458223821]
    # the feature hash is the generator's output function on the incremented state
    assert int(F.mix64(np.uint64((1234567 + 0x9E3779B97F4A7C15) & mlp.MASK64))) == 6457827717110365317


def test_parameter_count():
    assert mlp.NPARAM == 40 * 64 + 64 + 64 * 64 + 64 + 64 * 6 + 6 == 7174


def _rand_theta(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, mlp.NPARAM)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(5, 40))
    T = rng.normal(size=(5, 6))
    T[rng.uniform(size=T.shape) < 0.3] = np.nan  # missing targets are part of the loss' definition
    theta = _rand_theta(2)
    L, g = mlp.backward(theta, X, T)
    assert abs(L - mlp.loss(theta, X, T)) < 1e-12
    h = 1e-6
    idx = list(range(0, mlp.NPARAM, 7)) + [mlp.NPARAM - 1, mlp.NPARAM - 2, mlp.NPARAM - 3]
    for k in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (mlp.loss(tp, X, T) - mlp.loss(tm, X, T)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), k


def test_zero_weights_output_last_bias():
    theta = np.zeros(mlp.NPARAM)
    p = mlp.unpack(theta)
    p["b3"][:] = [1.5, -2.0, 0.25, 7.0, 0.0, -0.5]
    theta = mlp.pack(p)
    X = np.random.default_rng(3).normal(size=(4, 40))
    _, _, y = mlp.forward(theta, X)
    assert np.array_equal(y, np.tile([1.5, -2.0, 0.25, 7.0, 0.0, -0.5], (4, 1)))


def test_single_path_network_by_hand():
    # one unit per hidden layer: y_0 = 2 * relu(3 * relu(x_0 - 1) + 0.5) - 1
    p = mlp.unpack(np.zeros(mlp.NPARAM))
    p["W1"][0, 0] = 1.0
    p["b1"][0] = -1.0
    p["W2"][0, 0] = 3.0
    p["b2"][0] = 0.5
    p["W3"][0, 0] = 2.0
    p["b3"][0] = -1.0
    theta = mlp.pack(p)
    X = np.zeros((3, 40))
    X[:, 0] = [0.0, 2.0, 4.0]
    _, _, y = mlp.forward(theta, X)
    assert np.allclose(y[:, 0], [2 * 0.5 - 1, 2 * (3 * 1 + 0.5) - 1, 2 * (3 * 3 + 0.5) - 1])


def test_adam_first_step_moves_by_learning_rate():
    g = np.array([3.0, -0.5, 1e-3, -40.0])
    theta, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(theta, -0.01 * np.sign(g), rtol=1e-4)


def test_training_at_zero_loss_leaves_parameters():
    # W3 = 0: the output is exactly b3 whatever the hidden layers compute, so targets equal
    # to b3 give zero error, zero gradient everywhere, and Adam must not move
    p = mlp.unpack(_rand_theta(4))
    p["W3"][:] = 0.0
    p["b3"][:] = [0.5, -1.0, 2.0, 0.0, 1.0, 3.0]
    theta = mlp.pack(p)
    X = np.random.default_rng(5).normal(size=(10, 40))
    y = np.tile([0.5, -1.0, 2.0, 0.0, 1.0, 3.0], (10, 1))
    y[::3, 4] = np.nan  # a missing target adds nothing
    out, last = mlp.train(theta, X, y, epochs=3, batch=4, lr=0.1, seed=9)
    assert last == 0.0 and np.array_equal(out, theta)


def test_training_reduces_loss_on_a_learnable_target():
    rng = np.random.default_rng(6)
    X = rng.uniform(0, 1, size=(64, 40))
    T = np.stack([X[:, 0] + X[:, 1], 2 * X[:, 2], -X[:, 3], X[:, 4], X[:, 5] * 0.5, -X[:, 6]], axis=1)
    theta = mlp.init_params(11)
    before = mlp.loss(theta, X, T)
    theta2, _ = mlp.train(theta, X, T, epochs=60, batch=16, lr=3e-3, seed=12)
    assert mlp.loss(theta2, X, T) < 0.05 * before


def test_missing_targets_contribute_nothing():
    # a NaN target is equivalent to a target equal to the prediction: same loss, same gradient
    rng = np.random.default_rng(13)
    X = rng.normal(size=(6, 40))
    theta = _rand_theta(14)
    _, _, y = mlp.forward(theta, X)
    T = rng.normal(size=(6, 6))
    miss = rng.uniform(size=T.shape) < 0.4
    Tn = np.where(miss, np.nan, T)
    Ty = np.where(miss, y, T)
    Ln, gn = mlp.backward(theta, X, Tn)
    Ly, gy = mlp.backward(theta, X, Ty)
    assert abs(Ln - Ly) < 1e-12 and np.allclose(gn, gy, rtol=0, atol=1e-12)
    # and the mean still divides by all rows x outputs
    assert abs(Ln - np.sum(np.where(miss, 0, (y - T) ** 2)) / 36) < 1e-12


def test_epoch_order_is_a_permutation_and_uniformish():
    r = mlp.SplitMix64(3)
    firsts = np.zeros(5)
    for _ in range(5000):
        o = mlp.epoch_order(r, 5)
        assert sorted(o) == list(range(5))
        firsts[o[0]] += 1
    assert np.all(np.abs(firsts / 5000 - 0.2) < 0.03)


def test_init_params_bounds_and_biases():
    theta = mlp.init_params(7)
    p = mlp.unpack(theta)
    for li in (1, 2, 3):
        W = p[f"W{li}"]
        a = math.sqrt(6.0 / W.shape[1])
        assert np.all(np.abs(W) <= a) and abs(W.mean()) < 0.1 * a
        assert np.all(p[f"b{li}"] == 0)
    assert np.array_equal(theta, theta.astype(np.float32).astype(np.float64))


# ------------------------------------------------------------------------------ features

def _brute_counts(crd):
    """Recount with Python integers: a set for the bit map, a dict for the buckets."""
    M64 = (1 << 64) - 1

    def h(x):
        z = x & M64
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        return z ^ (z >> 31)

    n = len(crd[0])
    S = min(n, F.SAMPLE)
    pos = [k * n // S for k in range(S)]
    out = []
    for c in crd:
        bits, buckets, change = set(), {}, 0
        for j in pos:
            z = h(int(c[j]))
            bits.add(z % 65536)
            b = (z >> 16) % 1024
            buckets[b] = buckets.get(b, 0) + 1
            if j + 1 < n and c[j] != c[j + 1]:
                change += 1
        out.append((65536 - len(bits), max(buckets.values()), change))
    return out


@pytest.mark.parametrize("n", [1, 2, 7, 1000, 16384, 16385, 50001])
def test_feature_counts_match_brute_force(n):
    rng = np.random.default_rng(n)
    crd = [np.sort(rng.integers(0, 50, n)).astype(np.int32), rng.integers(0, 1 << 20, n).astype(np.int32),
           rng.integers(0, 3, n).astype(np.int64)]
    per_mode, mch, S, pairs = F.counts(crd, masks=[(0,), (0, 2)])
    assert S == min(n, F.SAMPLE)
    assert per_mode == _brute_counts(crd)
    assert mch[0] == per_mode[0][2]
    pos = [k * n // S for k in range(S)]
    assert pairs == sum(1 for j in pos if j + 1 < n)
    want = sum(1 for j in pos if j + 1 < n and (crd[0][j] != crd[0][j + 1] or crd[2][j] != crd[2][j + 1]))
    assert mch[1] == want


def test_feature_counts_closed_forms():
    n = 40000
    const = np.full(n, 17, dtype=np.int32)
    inc = np.arange(n, dtype=np.int32)
    per_mode, _, S, pairs = F.counts([const, inc])
    assert per_mode[0] == (65535, S, 0)          # one value: one bit, one bucket, no change
    assert per_mode[1][2] == pairs               # strictly increasing: every pair changes
    D = F.linear_count(per_mode[1][0])           # S distinct values, well below the map size
    assert abs(D - S) < 0.03 * S


def test_plan_terms_on_the_paper_examples():
    # (4,1,2,3) needs one plain pass on mode 4 (Sec. 3.4): one global group of 3 bits -> 1 digit
    # pass; Top-1 and Top-2 plan the same (their targets are sigma itself and no tail is left to
    # sort); Top-3 is not a candidate for 4 modes; LSD sorts all 12 bits in 2 passes
    terms, Q = F.plan_terms([8, 8, 8, 8], (0, 1, 2, 3), (3, 0, 1, 2))
    assert terms == [(1, 0), None, (1, 0), (1, 0), None, (2, 0)]
    assert Q == [(), (3,), (3, 0), ()]
    # (4,3,2,1): three plain calls, one group of 9 key bits -> 2 passes
    terms, _ = F.plan_terms([8, 8, 8, 8], (0, 1, 2, 3), (3, 2, 1, 0))
    assert terms[0] == (2, 0) and terms[1] is None and terms[5] == (2, 0)
    # (0,2,1) from (0,1,2) with 2/4/8-bit modes: one bucketed call on mode 2 keeping mode 0.  It
    # packs, and flattened to (0,2) it needs 2 passes against 1, so candidate 0 runs it as a global
    # sort; candidate 1 keeps its 8-bit bucket sort; Top-1's target is the input order and its
    # tail group is the same bucketed sort
    terms, Q = F.plan_terms([4, 16, 256], (0, 1, 2), (0, 2, 1))
    assert terms == [(2, 0), (0, 8), (2, 0), None, None, (2, 0)]
    assert Q == [(0,), (0,), (), ()]
    # a prefix too wide to flatten (3 more passes) keeps the bucket sort in candidate 0 too, and
    # candidate 1 then plans nothing different
    terms, _ = F.plan_terms([1 << 20, 1 << 17, 1 << 10, 64], (0, 1, 2, 3), (0, 1, 3, 2))
    assert terms[0] == (0, 6) and terms[1] is None


def test_features_identity_and_ranges():
    rng = np.random.default_rng(8)
    n = 5000
    crd = [np.sort(rng.integers(0, 100, n)).astype(np.int32), rng.integers(0, 9, n).astype(np.int32),
           rng.integers(0, 1000, n).astype(np.int32)]
    for sigma in itertools.permutations(range(3)):
        f = F.features(crd, (100, 9, 1000), (0, 1, 2), sigma)
        assert f.shape == (40,) and np.all(np.isfinite(f)) and np.all(f >= 0) and np.all(f <= 4)
        if sigma == (0, 1, 2):
            assert f[24] == f[25] == 0  # the minimal plan sorts nothing


def _mix64_int(z):
    """SplitMix64's output function with Python integers (independent of the numpy oracle)."""
    m = (1 << 64) - 1
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def test_features_against_hand_derived_golden():
    """All 40 features of a 6-nonzero 3-mode tensor with sigma = (0, 2, 1), whose slots are not
    in mode order, against values derived by hand from the feature definitions."""
    from conftest import read_golden
    g = read_golden("features_3mode.txt")
    want = np.array([float(g[str(i)][0]) for i in range(40)])
    nz = [(0, 1, 1), (0, 1, 4), (1, 1, 0), (1, 1, 3), (1, 2, 0), (3, 2, 2)]
    crd = [np.array([t[m] for t in nz], dtype=np.int32) for m in range(3)]
    # the derivation's premise: values 0..4 share no bitmap bit and no bucket
    h = [_mix64_int(v) for v in range(5)]
    assert len({x & 0xFFFF for x in h}) == 5 and len({(x >> 16) & 1023 for x in h}) == 5
    f = F.features(crd, (9, 3, 20), (0, 1, 2), (0, 2, 1), crd_bytes=4, val_bytes=8)
    np.testing.assert_allclose(f, want, rtol=1e-12, atol=0)
