"""Seeded batches of independent synthetic COO tensors, drawn with torch on any device.

A batch mixes tensors of uneven size, order and mode orders.  Recipe (all per-tensor
parameters come from one numpy Philox stream seeded by ``seed``; the coordinates of
tensor i come from a torch generator on the target device seeded from that stream):

1. order r drawn from ``orders``; nnz log-uniform in ``nnz_range``; every extent
   log-uniform in ``ext_range`` (rounded down, at least 1); one Zipf exponent s uniform in
   [0, ``zipf_max``]; a random input order tau and a random requested order sigma.
2. Every mode's coordinate is an exact Zipf(s) rank over its extent (rank k has probability
   proportional to k^-s), drawn by rejection-inversion (Hoermann and Derflinger, "Rejection-
   inversion to generate variates from monotone discrete distributions", ACM TOMACS 1996),
   then relabelled by a seeded affine bijection k -> (a k + b) mod n so that the hot values
   are spread over the extent.  s = 0 is uniform.
3. Values uniform in [-1, 1).  Duplicated coordinate tuples are kept.
4. The nonzeros are listed in lexicographic order of tau (ties keep their draw order).

None of the transposition's arithmetic lives here.
"""
import dataclasses
import math

import numpy as np

BATCH_SEED = 20050427 + 3


@dataclasses.dataclass
class BatchTensor:
    crd: list           # r coordinate tensors
    val: object         # value tensor
    extents: tuple
    in_order: tuple
    out_order: tuple
    zipf: float

    @property
    def nnz(self):
        return int(self.val.shape[0])

    @property
    def order(self):
        return len(self.crd)

    def as_dict(self):
        return dict(crd=self.crd, val=self.val, extents=self.extents, in_order=self.in_order,
                    out_order=self.out_order)


def _h1(t, torch):
    """log1p(t)/t, continuous at t = 0."""
    small = t.abs() < 1e-8
    safe = torch.where(small, torch.ones_like(t), t)
    return torch.where(small, 1.0 - 0.5 * t + t * t / 3.0, torch.log1p(safe) / safe)


def _h2(x, torch):
    """expm1(x)/x, continuous at x = 0."""
    small = x.abs() < 1e-8
    safe = torch.where(small, torch.ones_like(x), x)
    return torch.where(small, 1.0 + 0.5 * x + x * x / 6.0, torch.expm1(safe) / safe)


def zipf_ranks(n, s, size, gen, device, torch):
    """`size` ranks in [0, n) with P(k) proportional to (k+1)^-s, by rejection-inversion."""
    if n <= 1 or size == 0:
        return torch.zeros(size, dtype=torch.int64, device=device)
    if s <= 0.0:
        return torch.randint(0, n, (size,), generator=gen, device=device)
    f64 = torch.float64

    def H(x):  # integral of x^-s from 1 to x (in the numerically stable form)
        lx = torch.log(x)
        return _h2((1.0 - s) * lx, torch) * lx

    def Hinv(y):
        return torch.exp(_h1(y * (1.0 - s), torch) * y)

    def h(x):
        return torch.exp(-s * torch.log(x))

    one = torch.ones(1, dtype=f64, device=device)
    hx1 = H(1.5 * one) - 1.0
    hn = H((n + 0.5) * one)
    thr = 2.0 - Hinv(H(2.5 * one) - h(2.0 * one))
    out = torch.empty(size, dtype=torch.int64, device=device)
    todo = torch.arange(size, device=device)
    while todo.numel():
        u = torch.rand(todo.numel(), generator=gen, dtype=f64, device=device)
        y = hn + u * (hx1 - hn)
        x = Hinv(y)
        k = torch.clamp(torch.round(x), 1.0, float(n))
        ok = (k - x <= thr) | (y >= H(k + 0.5) - h(k))
        out[todo[ok]] = k[ok].to(torch.int64) - 1
        todo = todo[~ok]
    return out


def _draw_params(rng, count, orders, nnz_range, ext_range, zipf_max):
    specs = []
    for _ in range(count):
        r = int(rng.choice(orders))
        nnz = int(math.exp(rng.uniform(math.log(nnz_range[0]), math.log(nnz_range[1]))))
        ext = tuple(max(1, int(math.exp(rng.uniform(math.log(ext_range[0]), math.log(ext_range[1])))))
                    for _ in range(r))
        s = float(rng.uniform(0.0, zipf_max))
        tau = tuple(int(x) for x in rng.permutation(r))
        sigma = tuple(int(x) for x in rng.permutation(r))
        affine = []
        for n in ext:
            a = int(rng.integers(1, max(n, 2)))
            while math.gcd(a, n) != 1:
                a = int(rng.integers(1, max(n, 2)))
            affine.append((a, int(rng.integers(0, n))))
        specs.append(dict(r=r, nnz=nnz, ext=ext, s=s, tau=tau, sigma=sigma, affine=affine,
                          seed=int(rng.integers(0, 2 ** 62))))
    return specs


def _tensor(spec, device, crd_dtype, val_dtype, torch):
    gen = torch.Generator(device=device)
    gen.manual_seed(spec["seed"])
    n = spec["nnz"]
    cols = []
    for m in range(spec["r"]):
        ext = spec["ext"][m]
        k = zipf_ranks(ext, spec["s"], n, gen, device, torch)
        a, b = spec["affine"][m]
        cols.append((k * a + b) % ext)
    val = (torch.rand(n, generator=gen, dtype=torch.float64, device=device) * 2.0 - 1.0).to(val_dtype)
    idx = torch.arange(n, device=device)
    for m in reversed(spec["tau"]):  # stable passes, least significant first
        idx = idx[torch.argsort(cols[m][idx], stable=True)]
    crd = [c[idx].to(crd_dtype).contiguous() for c in cols]
    return BatchTensor(crd=crd, val=val[idx].contiguous(), extents=spec["ext"], in_order=spec["tau"],
                       out_order=spec["sigma"], zipf=spec["s"])


def iter_batch(count, seed=BATCH_SEED, orders=(3, 4), nnz_range=(1e3, 1e6), ext_range=(10, 1e6), zipf_max=1.5,
               device="cpu", crd_dtype="int32", val_dtype="float64", start=0):
    """The tensors of make_batch(count, seed, ...) one at a time (index, tensor), from `start`
    on, so that large collections never sit in memory together."""
    import torch
    rng = np.random.Generator(np.random.Philox(seed))
    specs = _draw_params(rng, count, orders, nnz_range, ext_range, zipf_max)
    cd = getattr(torch, crd_dtype)
    vd = getattr(torch, val_dtype)
    for i in range(start, count):
        yield i, _tensor(specs[i], device, cd, vd, torch)


def make_batch(count, seed=BATCH_SEED, orders=(3, 4), nnz_range=(1e3, 1e6), ext_range=(10, 1e6),
               zipf_max=1.5, device="cpu", crd_dtype="int32", val_dtype="float64", extra=()):
    """`count` tensors drawn as in the module recipe, then the fixed tensors in `extra`
    (dicts with r, nnz, ext, s, tau, sigma; each gets an identity relabelling and a seed)."""
    import torch
    rng = np.random.Generator(np.random.Philox(seed))
    specs = _draw_params(rng, count, orders, nnz_range, ext_range, zipf_max)
    for e in extra:
        specs.append(dict(r=len(e["ext"]), nnz=int(e["nnz"]), ext=tuple(e["ext"]), s=float(e.get("s", 0.0)),
                          tau=tuple(e["tau"]), sigma=tuple(e["sigma"]), affine=[(1, 0)] * len(e["ext"]),
                          seed=int(rng.integers(0, 2 ** 62))))
    cd = getattr(torch, crd_dtype)
    vd = getattr(torch, val_dtype)
    return [_tensor(sp, device, cd, vd, torch) for sp in specs]


# The batched workload: 4,096 tensors of order 3 or 4 (even odds), nnz log-uniform in
# [1e3, 1e6], extents log-uniform in [10, 1e6], Zipf exponent uniform in [0, 1.5], fp64.
BATCHED = dict(count=4096, seed=BATCH_SEED, orders=(3, 4), nnz_range=(1e3, 1e6), ext_range=(10, 1e6),
               zipf_max=1.5, crd_dtype="int32", val_dtype="float64")
