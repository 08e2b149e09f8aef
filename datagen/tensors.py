"""Seeded synthetic COO tensors with the shapes of the paper's workloads.

Recipe (every step draws from one numpy Philox stream seeded by ``seed``):

1. For every mode m with Zipf exponent s_m > 0, a random relabelling of
   [0, n_m) (a uniform permutation).  Rank k (1-based) of a Zipf(s) law over n
   values has probability proportional to k^-s; ranks are drawn with Walker's
   alias method (Vose's construction) and mapped through the relabelling, so
   the hot coordinates are scattered over the extent.  s = 0 is uniform.
2. Coordinates of every mode are drawn independently.
3. ``distinct=True``: duplicated coordinate tuples are removed (sort-unique);
   if fewer than nnz remain, more are drawn and merged until there are enough;
   a seeded uniform subset of exactly nnz distinct tuples is then kept.
4. The nonzeros are listed in lexicographic order of ``in_order`` (ties, which
   exist only when duplicates are allowed, keep their draw order).
5. Values: uniform in (-1, 1), cast to the value dtype.
"""
import dataclasses
import math

import numpy as np

BASE_SEED = 20050427

# name -> dict(extents, nnz, zipf, crd, val, in_order, sigmas, seed)
CONFIGS = {
    # 3-mode, 1e6 distinct uniform nonzeros, the small case the oracle finishes in seconds
    "small": dict(extents=(1000, 800, 600), nnz=1_000_000, zipf=(0.0, 0.0, 0.0),
                  crd=np.int32, val=np.float64, in_order=(0, 1, 2),
                  sigmas=[(1, 0, 2), (2, 1, 0)], seed=BASE_SEED + 0),
    # 3-mode, 1e8 distinct nonzeros, every mode Zipf(1.1) over a relabelled extent
    "plain": dict(extents=(500_000, 20_000, 2_000_000), nnz=100_000_000, zipf=(1.1, 1.1, 1.1),
                  crd=np.int32, val=np.float64, in_order=(0, 1, 2),
                  sigmas=[(0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)],
                  seed=BASE_SEED + 1),
    # 4-mode, 2e8 distinct nonzeros, modes 0-1 Zipf(1.3), modes 2-3 uniform, fp32 values
    "wide": dict(extents=(1_000_000, 100_000, 1_000, 50), nnz=200_000_000,
                 zipf=(1.3, 1.3, 0.0, 0.0), crd=np.int32, val=np.float32,
                 in_order=(0, 1, 2, 3), sigmas=None, seed=BASE_SEED + 2),
}


def all_non_identity(r):
    import itertools
    ident = tuple(range(r))
    return [p for p in itertools.permutations(range(r)) if p != ident]


CONFIGS["wide"]["sigmas"] = all_non_identity(4)


@dataclasses.dataclass
class SynthTensor:
    crd: list            # r numpy arrays (structure of arrays)
    val: np.ndarray
    extents: tuple
    in_order: tuple

    @property
    def nnz(self):
        return int(self.val.shape[0])

    @property
    def order(self):
        return len(self.crd)


_ALIAS_CACHE = {}


def zipf_alias(n, s):
    """Alias tables (prob, alias) for ranks 0..n-1 with weight (rank+1)^-s."""
    key = (int(n), float(s))
    if key in _ALIAS_CACHE:
        return _ALIAS_CACHE[key]
    w = np.arange(1, n + 1, dtype=np.float64) ** (-float(s))
    p = w * (n / w.sum())
    prob = np.ones(n, dtype=np.float64)
    alias = np.arange(n, dtype=np.int64)
    small = list(np.nonzero(p < 1.0)[0][::-1])
    large = list(np.nonzero(p >= 1.0)[0][::-1])
    pl = p.tolist()
    while small and large:
        lo = small.pop()
        hi = large.pop()
        prob[lo] = pl[lo]
        alias[lo] = hi
        pl[hi] = pl[hi] + pl[lo] - 1.0
        if pl[hi] < 1.0:
            small.append(hi)
        else:
            large.append(hi)
    if len(_ALIAS_CACHE) > 8:
        _ALIAS_CACHE.clear()
    _ALIAS_CACHE[key] = (prob, alias)
    return prob, alias


def _bits(n):
    return (int(n) - 1).bit_length()


def _draw_mode(rng, n, s, size, relabel):
    if s == 0.0:
        return rng.integers(0, n, size=size, dtype=np.int64)
    prob, alias = zipf_alias(n, s)
    u = rng.random(size)
    idx = np.minimum((u * n).astype(np.int64), n - 1)
    take = rng.random(size) < prob[idx]
    rank = np.where(take, idx, alias[idx])
    return relabel[rank]


def _draw(rng, extents, zipf, size, relabels):
    return [_draw_mode(rng, n, s, size, rl) for n, s, rl in zip(extents, zipf, relabels)]


def _pack(cols, extents, in_order):
    """uint64 key whose numeric order is the lexicographic order of in_order."""
    key = np.zeros(len(cols[0]), dtype=np.uint64)
    shift = 0
    for m in reversed(in_order):
        key |= cols[m].astype(np.uint64) << np.uint64(shift)
        shift += _bits(extents[m])
    return key


def _unpack(key, extents, in_order):
    cols = [None] * len(extents)
    shift = 0
    for m in reversed(in_order):
        b = _bits(extents[m])
        cols[m] = ((key >> np.uint64(shift)) & np.uint64((1 << b) - 1)).astype(np.int64)
        shift += b
    return cols


def make_tensor(extents, nnz, zipf=None, in_order=None, crd_dtype=np.int32,
                val_dtype=np.float64, seed=BASE_SEED, distinct=True):
    extents = tuple(int(n) for n in extents)
    r = len(extents)
    zipf = tuple(float(s) for s in (zipf or (0.0,) * r))
    in_order = tuple(in_order) if in_order is not None else tuple(range(r))
    nnz = int(nnz)
    rng = np.random.Generator(np.random.Philox(seed))
    relabels = [rng.permutation(n) if s > 0 else None for n, s in zip(extents, zipf)]
    total_bits = sum(_bits(n) for n in extents)

    if distinct:
        cells = math.prod(extents)
        if nnz > cells:
            raise ValueError("more distinct nonzeros requested than cells")
        if total_bits > 64:
            raise ValueError("distinct generation packs coordinates into 64 bits")
        keys = np.zeros(0, dtype=np.uint64)
        want = nnz
        while True:
            draw = max(int(want * 1.3) + 1024, 1024)
            new = _pack(_draw(rng, extents, zipf, draw, relabels), extents, in_order)
            keys = np.unique(np.concatenate([keys, new]))
            if len(keys) >= nnz:
                break
            want = nnz - len(keys)
        if len(keys) > nnz:  # keep a uniform subset of exactly nnz distinct tuples
            drop = rng.choice(len(keys), size=len(keys) - nnz, replace=False)
            keep = np.ones(len(keys), dtype=bool)
            keep[drop] = False
            keys = keys[keep]
        cols = _unpack(keys, extents, in_order)
        del keys
    else:
        cols = _draw(rng, extents, zipf, nnz, relabels)
        if nnz:
            if total_bits <= 64:
                p = np.argsort(_pack(cols, extents, in_order), kind="stable")
            else:
                p = np.lexsort([cols[m] for m in reversed(in_order)])
            cols = [c[p] for c in cols]
    val = rng.uniform(-1.0, 1.0, size=nnz).astype(val_dtype)
    crd = [np.ascontiguousarray(c.astype(crd_dtype)) for c in cols]
    return SynthTensor(crd=crd, val=val, extents=extents, in_order=in_order)


def config_tensor(name, nnz=None, seed=None):
    """The named workload; ``nnz`` shrinks it (same extents and laws) for tests."""
    c = CONFIGS[name]
    return make_tensor(c["extents"], c["nnz"] if nnz is None else nnz, c["zipf"],
                       c["in_order"], c["crd"], c["val"],
                       c["seed"] if seed is None else seed, distinct=True)


def random_orders(rng, r):
    """A random complete input order and a random requested order."""
    return tuple(int(x) for x in rng.permutation(r)), tuple(int(x) for x in rng.permutation(r))
