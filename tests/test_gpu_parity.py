"""Parity of the HIP path (through the C ABI) with the CPU oracle: bit-exact outputs on the
same seeded inputs, at sizes the oracle finishes in seconds, spanning many tiles and ragged
tails, plus the edge cases (empty, single, duplicates, extent-1 modes, wide keys)."""
import itertools
import sys

import numpy as np
import pytest

from datagen import CONFIGS, config_tensor, make_tensor
from oracle.transpose import transpose as oracle_transpose

pytestmark = pytest.mark.gpu

SCHEDS = ("minimal", "top2", "lsd")


def note(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def dev(T):
    import torch
    crd = [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in T.crd]
    val = torch.from_numpy(np.ascontiguousarray(T.val)).cuda()
    return crd, val


def gpu_transpose(qsd, T, sigma, sched="minimal", crd_val=None, flags=0):
    import torch
    crd, val = crd_val if crd_val is not None else dev(T)
    P = qsd.Plan(T.extents, T.in_order, sigma, max(T.nnz, 1), str(T.crd[0].dtype), str(T.val.dtype), sched,
                 flags)
    out_crd, out_val = P.transpose(crd, val)
    torch.cuda.synchronize()
    assert P.device_status() == 0
    return [c.cpu().numpy() for c in out_crd], out_val.cpu().numpy()


def assert_bits_equal(got, want):
    g_crd, g_val = got
    w_crd, w_val = want
    for m in range(len(w_crd)):
        assert np.array_equal(g_crd[m], w_crd[m]), f"mode {m} differs"
    u = np.uint64 if w_val.dtype.itemsize == 8 else np.uint32
    assert np.array_equal(g_val.view(u), w_val.view(u)), "values differ"


def check(qsd, T, sigma, sched="minimal", crd_val=None, flags=(0, 2)):
    """Both ways of running bucketed groups: flattened where cheaper (0) and always as
    segment sorts (QSD_KEEP_BUCKETS = 2)."""
    want = oracle_transpose(T.crd, T.val, sigma)
    for fl in ((flags,) if isinstance(flags, int) else flags):
        note(f"r={T.order} n={T.nnz} ext={T.extents} tau={T.in_order} sigma={sigma} sched={sched} flags={fl}")
        got = gpu_transpose(qsd, T, sigma, sched, crd_val, fl)
        assert_bits_equal(got, want)


def test_small_config_full_size(gpu_lib):
    c = CONFIGS["small"]
    T = config_tensor("small")
    cv = dev(T)
    for sigma in c["sigmas"]:
        for sched in SCHEDS:
            check(gpu_lib, T, sigma, sched, cv)


def test_plain_config_shrunk_all_orders(gpu_lib):
    T = config_tensor("plain", nnz=300_000)
    cv = dev(T)
    for sigma in CONFIGS["plain"]["sigmas"]:
        for sched in SCHEDS:
            check(gpu_lib, T, sigma, sched, cv)


def test_wide_config_shrunk_all_orders(gpu_lib):
    T = config_tensor("wide", nnz=400_000)
    cv = dev(T)
    for sigma in CONFIGS["wide"]["sigmas"]:
        check(gpu_lib, T, sigma, "minimal", cv)
    for sigma in CONFIGS["wide"]["sigmas"][::5]:
        for sched in ("top2", "lsd"):
            check(gpu_lib, T, sigma, sched, cv)


@pytest.mark.parametrize("r", [2, 3, 4, 5])
def test_every_topk_schedule(gpu_lib, r):
    """Top-K-sadilla for every K = 1..r-1 (Sec. 3.6) on tensors with duplicates, both ways of
    running bucketed groups."""
    rng = np.random.default_rng(40 + r)
    ext = tuple(int(x) for x in rng.integers(3, 3000, size=r))
    tau = tuple(int(x) for x in rng.permutation(r))
    T = make_tensor(ext, 60000, zipf=[1.0] * r, in_order=tau, seed=77 + r, distinct=False)
    cv = dev(T)
    sigmas = list(itertools.permutations(range(r)))
    for sigma in (sigmas if r <= 4 else sigmas[::3]):
        for K in range(1, r):
            check(gpu_lib, T, sigma, f"topk{K}", cv)


def test_bucket_reuse_between_segmented_groups(gpu_lib):
    """A segmented group right after one whose kept prefix it extends takes its segment starts
    from the previous group's plus the added prefix modes (Sec. 5's reuse of buckets): 5-mode
    minimal plans and Top-K plans with such group pairs, buckets kept."""
    import torch
    ext = (40, 300, 50, 2000, 30)
    T = make_tensor(ext, 50000, zipf=[1.1] * 5, in_order=(0, 1, 2, 3, 4), seed=5, distinct=False)
    cv = dev(T)
    cases = [((0, 2, 1, 4, 3), "minimal"), ((0, 3, 1, 4, 2), "minimal"), ((0, 4, 1, 3, 2), "minimal")]
    for sigma in itertools.permutations(range(5)):
        for K in (2, 3):
            P = gpu_lib.Plan(ext, T.in_order, sigma, T.nnz, "int32", "float64", f"topk{K}", gpu_lib.QSD_KEEP_BUCKETS)
            if "reuse=0" not in P.describe() and len(cases) < 12:
                cases.append((sigma, f"topk{K}"))
    for sigma, sched in cases:
        P = gpu_lib.Plan(ext, T.in_order, sigma, T.nnz, "int32", "float64", sched, gpu_lib.QSD_KEEP_BUCKETS)
        assert "reuse=0" not in P.describe(), (sigma, sched)
        check(gpu_lib, T, sigma, sched, cv, flags=gpu_lib.QSD_KEEP_BUCKETS)
    del torch


def test_topk_on_the_wide_workload(gpu_lib):
    T = config_tensor("wide", nnz=200_000)
    cv = dev(T)
    for sigma in CONFIGS["wide"]["sigmas"][1::3]:
        for K in (1, 2):
            check(gpu_lib, T, sigma, f"topk{K}", cv)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 2047, 2048, 2049, 4095, 4096, 4097, 8193, 3 * 4096 - 1, 20000])
def test_ragged_sizes_with_duplicates(gpu_lib, n):
    rng = np.random.default_rng(n)
    for trial in range(3):
        r = int(rng.integers(2, 5))
        ext = tuple(int(x) for x in rng.integers(1, 40, size=r))
        tau = tuple(int(x) for x in rng.permutation(r))
        T = make_tensor(ext, n, zipf=[float(rng.uniform(0, 1.5)) for _ in range(r)], in_order=tau,
                        seed=int(rng.integers(1 << 30)), distinct=False)
        for sigma in itertools.permutations(range(r)):
            for sched in SCHEDS:
                check(gpu_lib, T, sigma, sched)


@pytest.mark.parametrize("crd,val", [("int32", "float32"), ("int64", "float64"), ("int64", "float32")])
def test_types_and_orders_up_to_five(gpu_lib, crd, val):
    rng = np.random.default_rng({"int32": 1, "int64": 2}[crd] * 10 + {"float32": 1, "float64": 2}[val])
    for r in (1, 2, 3, 4, 5):
        ext = tuple(int(x) for x in rng.integers(2, 300, size=r))
        tau = tuple(int(x) for x in rng.permutation(r))
        T = make_tensor(ext, 30000, zipf=[1.2] * r, in_order=tau, crd_dtype=np.dtype(crd),
                        val_dtype=np.dtype(val), seed=17 + r, distinct=False)
        cv = dev(T)
        sigmas = list(itertools.permutations(range(r)))
        for sigma in (sigmas if r <= 3 else sigmas[::4]):
            for sched in SCHEDS:
                check(gpu_lib, T, sigma, sched, cv)


def test_int64_wide_keys(gpu_lib):
    """Extents beyond 2^32 (int64 coordinates): composite keys wider than 64 bits are cut
    into sub-keys; bucketed groups with wide keys sort globally on (prefix, keys)."""
    rng = np.random.default_rng(5)
    ext = (3_000_000_000, 5_000_000_000, 70_000, 9)
    n = 50_000
    cols = [rng.integers(0, e, size=n, dtype=np.int64) for e in ext]
    # a few heavy coordinates so that segments of every size class appear
    cols[0][: n // 3] = 123_456_789
    cols[1][: n // 5] = 42
    tau = (0, 1, 2, 3)
    p = np.lexsort([cols[m] for m in reversed(tau)])
    from datagen import SynthTensor
    T = SynthTensor(crd=[c[p] for c in cols], val=rng.standard_normal(n), extents=ext, in_order=tau)
    cv = dev(T)
    for sigma in itertools.permutations(range(4)):
        for sched in SCHEDS:
            check(gpu_lib, T, sigma, sched, cv)


def test_extent_one_and_identity(gpu_lib):
    T = make_tensor((1, 50, 1, 7), 3000, in_order=(0, 1, 2, 3), seed=3, distinct=False)
    for sigma in [(0, 1, 2, 3), (2, 0, 3, 1), (3, 1, 0, 2), (1, 3, 2, 0)]:
        for sched in SCHEDS:
            check(gpu_lib, T, sigma, sched)


def test_value_bits_survive(gpu_lib):
    rng = np.random.default_rng(1)
    T = make_tensor((30, 30), 5000, in_order=(0, 1), seed=4, distinct=False)
    bits = T.val.view(np.uint64)
    bits[::7] = 0x7FF8_0000_DEAD_BEEF  # NaN payloads
    bits[3::11] = 0x8000_0000_0000_0000  # -0.0
    check(gpu_lib, T, (1, 0))


def test_empty(gpu_lib):
    import torch
    P = gpu_lib.Plan((5, 6), (0, 1), (1, 0), 10)
    crd = [torch.zeros(1, dtype=torch.int32, device="cuda") for _ in range(2)]
    val = torch.zeros(1, dtype=torch.float64, device="cuda")
    P.transpose(crd, val, nnz=0)
    torch.cuda.synchronize()


def test_deterministic_repeats(gpu_lib):
    import torch
    T = config_tensor("plain", nnz=200_000, seed=99)
    cv = dev(T)
    P = gpu_lib.Plan(T.extents, T.in_order, (0, 2, 1), T.nnz)
    ref = None
    for rep in range(5):
        oc, ov = P.transpose(*cv)
        torch.cuda.synchronize()
        h = [c.cpu().numpy().tobytes() for c in oc] + [ov.cpu().numpy().tobytes()]
        if ref is None:
            ref = h
        assert h == ref


def test_validation_errors(gpu_lib):
    import torch
    T = make_tensor((10, 10, 10), 500, in_order=(0, 1, 2), seed=8)
    crd, val = dev(T)
    P = gpu_lib.Plan(T.extents, (0, 1, 2), (2, 1, 0), T.nnz, flags=gpu_lib.QSD_VALIDATE)
    P.transpose(crd, val)  # valid input passes
    bad = [c.clone() for c in crd]
    bad[1][7] = 10  # out of range
    with pytest.raises(gpu_lib.QsdError) as e:
        P.transpose(bad, val)
    assert e.value.code == 6
    uns = [c.flip(0).contiguous() for c in crd]
    with pytest.raises(gpu_lib.QsdError) as e:
        P.transpose(uns, val)
    assert e.value.code == 5
    torch.cuda.synchronize()


@pytest.mark.parametrize("crd_dtype", ["int32", "int64"])
def test_csf_pack_matches_oracle(gpu_lib, crd_dtype):
    """The pack against the oracle's CSF for every order r = 1..8, with duplicates (separate
    leaves), sizes spanning several 2048-record tiles with ragged tails and exact multiples."""
    import torch
    from oracle import csf
    rng = np.random.default_rng(12 if crd_dtype == "int32" else 13)
    sizes = [1, 2047, 2048, 2049, 4096, 6145, 20000, 40000]
    for trial, r in enumerate(list(range(1, 9)) + [int(x) for x in rng.integers(1, 9, size=4)]):
        ext = tuple(int(x) for x in rng.integers(1, 12, size=r))
        sigma = tuple(int(x) for x in rng.permutation(r))
        n = sizes[trial % len(sizes)]
        T = make_tensor(ext, n, in_order=sigma, seed=trial, distinct=False,
                        crd_dtype=np.dtype(crd_dtype))  # already sigma-sorted
        note(f"csf r={r} n={n} ext={ext} sigma={sigma} {crd_dtype}")
        P = gpu_lib.Plan(ext, sigma, sigma, n, crd_dtype, "float64")
        crd, _ = dev(T)
        pos, lev, counts = P.pack_csf(crd)
        torch.cuda.synchronize()
        assert P.device_status() == 0
        want_pos, want_lev = csf.pack_csf([c.tolist() for c in T.crd], sigma)
        assert counts == [1] + [len(lv) for lv in want_lev]
        for d in range(r):
            assert pos[d].cpu().tolist() == want_pos[d], f"pos level {d + 1}"
            assert lev[d].cpu().tolist() == want_lev[d], f"crd level {d + 1}"


@pytest.mark.parametrize("crd_dtype", ["int32", "int64"])
def test_csf_to_csf_matches_oracle(gpu_lib, crd_dtype):
    """CSF (levels in tau) -> CSF (levels in sigma) against the oracle's unpack -> transpose ->
    pack, on tensors with duplicate coordinates (separate leaves), r = 1..5, ragged sizes."""
    import torch
    from oracle import csf
    rng = np.random.default_rng(31 if crd_dtype == "int32" else 32)
    cases = [(3, 1, (1, 1, 1)), (2, 1, (5, 7))]
    for _ in range(10):
        r = int(rng.integers(1, 6))
        cases.append((r, int(rng.integers(1, 30000)), tuple(int(x) for x in rng.integers(1, 40, size=r))))
    for r, n, ext in cases:
        tau = tuple(int(x) for x in rng.permutation(r))
        sigma = tuple(int(x) for x in rng.permutation(r))
        T = make_tensor(ext, n, zipf=[1.0] * r, in_order=tau, seed=n + r, distinct=False,
                        crd_dtype=np.dtype(crd_dtype))
        note(f"csf->csf r={r} n={n} ext={ext} tau={tau} sigma={sigma} {crd_dtype}")
        in_pos, in_lev = csf.pack_csf([c.tolist() for c in T.crd], tau)
        td = torch.int64 if crd_dtype == "int64" else torch.int32
        ip = [torch.tensor(p, dtype=td, device="cuda") for p in in_pos]
        ic = [torch.tensor(lv if lv else [0], dtype=td, device="cuda") for lv in in_lev]
        iv = torch.from_numpy(T.val).cuda()
        P = gpu_lib.Plan(ext, tau, sigma, n, crd_dtype, "float64")
        pos, lev, val, counts = P.transpose_csf(ip, ic, iv)
        torch.cuda.synchronize()
        assert P.device_status() == 0
        # the oracle: expand the input tree, transpose, pack under sigma
        coo = csf.unpack_csf(in_pos, in_lev, tau)
        for m in range(r):
            assert coo[m] == T.crd[m].tolist()  # (the oracle round trip itself)
        w_crd, w_val = oracle_transpose([np.asarray(c, dtype=T.crd[0].dtype) for c in coo], T.val, sigma)
        want_pos, want_lev = csf.pack_csf([c.tolist() for c in w_crd], sigma)
        assert counts == [1] + [len(lv) for lv in want_lev]
        for d in range(r):
            assert pos[d].cpu().tolist() == want_pos[d], f"pos level {d + 1}"
            assert lev[d].cpu().tolist() == want_lev[d], f"crd level {d + 1}"
        assert np.array_equal(val.cpu().numpy().view(np.uint64), w_val.view(np.uint64)), "values"


def test_csf_to_csf_plain_workload(gpu_lib):
    """The 3-mode workload shrunk to 1.5e5 nonzeros, its CSF in the input order transposed to the
    CSF of every other order."""
    import torch
    from oracle import csf
    T = config_tensor("plain", nnz=150_000)
    in_pos, in_lev = csf.pack_csf([c.tolist() for c in T.crd], T.in_order)
    ip = [torch.tensor(p, dtype=torch.int32, device="cuda") for p in in_pos]
    ic = [torch.tensor(lv, dtype=torch.int32, device="cuda") for lv in in_lev]
    iv = torch.from_numpy(T.val).cuda()
    for sigma in CONFIGS["plain"]["sigmas"]:
        note(f"csf->csf plain sigma={sigma}")
        P = gpu_lib.Plan(T.extents, T.in_order, sigma, T.nnz)
        pos, lev, val, counts = P.transpose_csf(ip, ic, iv)
        torch.cuda.synchronize()
        assert P.device_status() == 0
        w_crd, w_val = oracle_transpose(T.crd, T.val, sigma)
        want_pos, want_lev = csf.pack_csf([c.tolist() for c in w_crd], sigma)
        for d in range(3):
            assert pos[d].cpu().tolist() == want_pos[d] and lev[d].cpu().tolist() == want_lev[d], (sigma, d)
        assert np.array_equal(val.cpu().numpy().view(np.uint64), w_val.view(np.uint64))
