"""Batched transposition through the C ABI: every tensor of a mixed batch bit-exact against
the oracle, under several tunings, after the autotuner, and on repeated HIP-graph replays."""
import sys

import numpy as np
import pytest

from datagen.batched import make_batch
from oracle.transpose import transpose as oracle_transpose

pytestmark = pytest.mark.gpu

# fixed members of every test batch: the degenerate cases and the wide keys
EXTRA = [
    dict(ext=(1, 1, 1), nnz=5000, tau=(0, 1, 2), sigma=(2, 1, 0)),           # nothing to sort
    dict(ext=(50, 60, 70), nnz=20000, tau=(0, 1, 2), sigma=(0, 1, 2)),       # identity, large
    dict(ext=(50, 60, 70), nnz=3000, tau=(1, 2, 0), sigma=(1, 2, 0)),        # identity, small
    dict(ext=(1 << 22,) * 4, nnz=30000, tau=(0, 1, 2, 3), sigma=(3, 2, 1, 0)),  # 66-bit key
    dict(ext=(3, 5), nnz=0, tau=(0, 1), sigma=(1, 0)),                       # empty
    dict(ext=(7, 9, 11), nnz=1, tau=(0, 1, 2), sigma=(2, 0, 1)),             # single
    dict(ext=(4, 4, 4), nnz=9000, tau=(2, 0, 1), sigma=(1, 2, 0)),           # heavy duplicates
    dict(ext=(4097, 3, 300), nnz=4097, tau=(0, 1, 2), sigma=(2, 1, 0), s=1.2),  # one past small
    dict(ext=(4096, 3, 300), nnz=4096, tau=(0, 1, 2), sigma=(1, 0, 2), s=0.8),  # exactly small
]


def note(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _batch(count=40, seed=5, crd="int32", val="float64", extra=EXTRA, **kw):
    args = dict(orders=(2, 3, 4, 5), nnz_range=(1, 4e4), ext_range=(1, 3e5))
    args.update(kw)
    return make_batch(count, seed=seed, device="cuda", crd_dtype=crd, val_dtype=val, extra=extra, **args)


def _check_all(tensors, out_crd, out_val):
    import torch
    torch.cuda.synchronize()
    for i, t in enumerate(tensors):
        crd = [c.cpu().numpy() for c in t.crd]
        val = t.val.cpu().numpy()
        w_crd, w_val = oracle_transpose(crd, val, t.out_order)
        for m in range(len(crd)):
            assert np.array_equal(out_crd[i][m].cpu().numpy(), w_crd[m]), (i, t.extents, t.in_order, t.out_order, m)
        u = np.uint64 if w_val.dtype.itemsize == 8 else np.uint32
        assert np.array_equal(out_val[i].cpu().numpy().view(u), w_val.view(u)), (i, "values")


def test_batch_mixed_default_tuning(gpu_lib):
    T = _batch()
    note(f"batch of {len(T)} tensors, {sum(t.nnz for t in T)} nnz")
    B = gpu_lib.Batch([t.as_dict() for t in T])
    out_crd, out_val = B.transpose()
    assert B.device_status() == 0
    _check_all(T, out_crd, out_val)


@pytest.mark.parametrize("items,radix,cap", [(8, 6, 0), (16, 7, 1024), (8, 8, 4096), (16, 5, 0), (16, 8, 0)])
def test_batch_tunings(gpu_lib, items, radix, cap):
    T = _batch(seed=6)
    B = gpu_lib.Batch([t.as_dict() for t in T])
    note(f"tuning items={items} radix={radix} small_cap={cap}")
    B.set_tuning(items, radix, cap)
    out_crd, out_val = B.transpose()
    assert B.device_status() == 0
    _check_all(T, out_crd, out_val)


def test_batch_wide_types(gpu_lib):
    T = _batch(count=24, seed=7, crd="int64", val="float32",
               extra=[dict(ext=(1 << 40, 1 << 30, 5), nnz=20000, tau=(2, 0, 1), sigma=(1, 0, 2))])
    note("int64 coordinates, fp32 values, 70-bit key")
    B = gpu_lib.Batch([t.as_dict() for t in T])
    out_crd, out_val = B.transpose()
    assert B.device_status() == 0
    _check_all(T, out_crd, out_val)


def test_batch_many_small_tensors(gpu_lib):
    T = _batch(count=600, seed=8, nnz_range=(1, 3e3), extra=())
    note("600 small tensors")
    B = gpu_lib.Batch([t.as_dict() for t in T])
    out_crd, out_val = B.transpose()
    assert B.device_status() == 0
    _check_all(T, out_crd, out_val)


def test_batch_autotune_then_transpose(gpu_lib):
    T = _batch(count=16, seed=9)
    B = gpu_lib.Batch([t.as_dict() for t in T])
    best, ms = B.tune(reps=1)
    note(f"tuned {best} {ms:.3f} ms")
    assert best[0] in (8, 16) and 6 <= best[1] <= 8 and best[2] in (0, 1024, 4096) and ms > 0
    assert B.tuning() == best
    for c in B.out_val:
        c.zero_()
    out_crd, out_val = B.transpose()
    assert B.device_status() == 0
    _check_all(T, out_crd, out_val)


def test_batch_autotune_cache(gpu_lib, tmp_path):
    """First call: a miss that tunes and appends one line; a second batch of the same key: a
    hit that applies the recorded tuning without timing; both transpose correctly.  Lines that
    do not parse and other keys are skipped."""
    cache = tmp_path / "tune.txt"
    cache.write_text("not a cache line\ngfx0/c4/v8/r9/n1/t1 8 6 0 1.0\n")
    T = _batch(count=16, seed=11)
    B = gpu_lib.Batch([t.as_dict() for t in T])
    key = B.tune_key()
    note(f"key {key}")
    assert key.split("/")[0].startswith("gfx") and "/c4/v8/" in key
    best, ms, hit = B.tune(reps=1, cache=cache)
    assert not hit and ms > 0
    lines = cache.read_text().splitlines()
    assert len(lines) == 3 and lines[-1].split()[0] == key
    assert tuple(int(x) for x in lines[-1].split()[1:4]) == best
    B2 = gpu_lib.Batch([t.as_dict() for t in T])
    assert B2.tune_key() == key
    best2, ms2, hit2 = B2.tune(reps=1, cache=cache)
    assert hit2 and best2 == best and B2.tuning() == best and ms2 == pytest.approx(float(lines[-1].split()[4]))
    assert len(cache.read_text().splitlines()) == 3  # a hit appends nothing
    for c in B2.out_val:
        c.zero_()
    out_crd, out_val = B2.transpose()
    assert B2.device_status() == 0
    _check_all(T, out_crd, out_val)


def test_batch_graph_replays_match_eager(gpu_lib):
    import torch
    T = _batch(count=24, seed=10)
    B = gpu_lib.Batch([t.as_dict() for t in T])
    out_crd, out_val = B.transpose()
    torch.cuda.synchronize()
    eager = ([[c.clone() for c in oc] for oc in out_crd], [v.clone() for v in out_val])
    _check_all(T, *eager)
    B.capture()
    for rep in range(4):
        note(f"graph replay {rep}")
        for oc, ov in zip(B.out_crd, B.out_val):  # eager work between replays
            for c in oc:
                c.fill_(-1)
            ov.fill_(7.0)
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        B.replay()
        torch.cuda.synchronize()
        assert B.device_status() == 0
        for i in range(len(T)):
            for m in range(len(T[i].crd)):
                assert torch.equal(B.out_crd[i][m], eager[0][i][m]), (rep, i, m)
            assert torch.equal(B.out_val[i].view(torch.int64), eager[1][i].view(torch.int64)), (rep, i)
        del junk
