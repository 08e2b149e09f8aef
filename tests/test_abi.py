"""Host-side checks of libqsd: it loads, exports every declared entry point, plans like the
oracle planner, and rejects bad arguments before launching anything.  CPU only."""
import itertools
import os
import re

import pytest

from conftest import ROOT
from oracle import planner

qsd = pytest.importorskip("paper_2005_10427_amd.qsd")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(qsd.LIB_PATH):
        pytest.fail("libqsd.so is not built (run __graft_entry__.build())")
    return qsd.load()


def _declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(qsd_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert "qsd_transpose" in names and "qsd_plan" in names
    for name in names:
        assert hasattr(lib, name), name


def _parse(desc):
    calls, groups, head = [], [], None
    for line in desc.strip().splitlines():
        kv = dict(tok.split("=", 1) for tok in line.split()[1:]) if " " in line else {}
        if line.startswith("sched="):
            head = dict(tok.split("=") for tok in line.split())
        elif line.startswith("call "):
            pre = tuple(int(x) for x in kv["prefix"].split(",") if x != "")
            calls.append((pre, int(kv["mode"])))
        elif line.startswith("group "):
            groups.append(kv)
    return head, calls, groups


def _plan(r, tau, sigma, sched, extents=None, nnz=1000, flags=None):
    """Plan structure; by default bucketed groups are kept as such (Alg. 3's grouping)."""
    extents = extents or [7] * r
    flags = qsd.QSD_KEEP_BUCKETS if flags is None else flags
    h = qsd.qsd_plan(r, nnz, extents, qsd.QSD_I32, qsd.QSD_F64, tau, sigma, sched, flags)
    try:
        return _parse(qsd.qsd_plan_describe(h))
    finally:
        qsd.qsd_plan_destroy(h)


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5])
def test_minimal_plan_equals_oracle_alg3(lib, r):
    for tau in itertools.permutations(range(r)):
        for sigma in itertools.permutations(range(r)):
            head, calls, groups = _plan(r, tau, sigma, "minimal")
            assert head["sched"] == "MINIMAL"
            want = planner.plan(tau, sigma)
            assert calls == want, (tau, sigma)
            # groups: maximal runs of calls sharing a prefix; keys most significant first
            exp = []
            for pre, m in want:
                if exp and exp[-1][0] == pre:
                    exp[-1][1].insert(0, m)
                else:
                    exp.append((pre, [m]))
            got = [(tuple(int(x) for x in g["prefix"].split(",") if x), [int(x) for x in g["keys"].split(",")])
                   for g in groups]
            assert got == [(p, k) for p, k in exp]


@pytest.mark.parametrize("r", [2, 3, 4, 5])
def test_top2_and_lsd_plans(lib, r):
    K = max(0, min(2, r - 2))
    for tau in itertools.permutations(range(r)):
        for sigma in itertools.permutations(range(r)):
            head, calls, groups = _plan(r, tau, sigma, "top2")
            assert int(head["K"]) == K
            want, _ = planner.topk_plan(tau, sigma, K)
            assert calls == want
            head, calls, groups = _plan(r, tau, sigma, "lsd")
            assert calls == planner.lsd_plan(sigma)
            assert len(groups) == 1 and groups[0]["prefix"] == ""


@pytest.mark.parametrize("r", [2, 3, 4, 5])
def test_every_topk_plan_equals_oracle(lib, r):
    """Top-K-sadilla for every K = 1..r-1 (Sec. 3.6): the Quesadilla calls towards sigma^K equal
    the oracle's, the last group sorts each (sigma_1..sigma_K) bucket on the rest of sigma
    that is not already in input order, and K = r-1 plans what MINIMAL plans."""
    for K in range(1, r):
        for tau in itertools.permutations(range(r)):
            for sigma in itertools.permutations(range(r)):
                head, calls, groups = _plan(r, tau, sigma, f"topk{K}")
                assert head["sched"] == "TOPK" and int(head["K"]) == K
                want, _ = planner.topk_plan(tau, sigma, K)
                assert calls == want, (K, tau, sigma)
                pos = {m: i for i, m in enumerate(tau)}
                q = r - 1
                while q - 1 >= K and pos[sigma[q - 1]] < pos[sigma[q]]:
                    q -= 1
                tail = list(sigma[K:q])
                if tail:
                    assert groups[-1]["prefix"] == ",".join(str(m) for m in sigma[:K])
                    assert groups[-1]["keys"] == ",".join(str(m) for m in tail)
                if K == r - 1:
                    _, mcalls, mgroups = _plan(r, tau, sigma, "minimal")
                    assert calls == mcalls and groups == mgroups
    for bad in (0, r):
        with pytest.raises(qsd.QsdError):
            qsd.qsd_plan(r, 10, [7] * r, qsd.QSD_I32, qsd.QSD_F64, tuple(range(r)), tuple(range(r)), f"topk{bad}")


def test_bucket_reuse_is_planned_between_nested_segmented_groups(lib):
    # (0,2,1,4,3): groups (0)[2] and (0,2,1)[4], both kept as bucket sorts; the second extends
    # the first's prefix, so it reuses its segment starts
    h = qsd.qsd_plan(5, 1000, [40, 300, 50, 2000, 30], qsd.QSD_I32, qsd.QSD_F64, (0, 1, 2, 3, 4), (0, 2, 1, 4, 3),
                     "minimal", qsd.QSD_KEEP_BUCKETS)
    try:
        d = qsd.qsd_plan_describe(h)
    finally:
        qsd.qsd_plan_destroy(h)
    _, calls, groups = _parse(d.split("layout")[0])
    assert [g["prefix"] for g in groups] == ["0", "0,2,1"]
    assert "reuse=1" in d
    # a plain group in between (or none before) gives nothing to reuse
    h = qsd.qsd_plan(4, 1000, [40, 300, 50, 2000], qsd.QSD_I32, qsd.QSD_F64, (0, 1, 2, 3), (1, 0, 3, 2),
                     "minimal", qsd.QSD_KEEP_BUCKETS)
    try:
        assert "reuse=0" in qsd.qsd_plan_describe(h)
    finally:
        qsd.qsd_plan_destroy(h)


def test_digit_split_covers_key_bits(lib):
    # 3-mode workload with 19/15/21-bit modes: (2,1,0) sorts modes 1 then 2 -> 36 key bits
    head, calls, groups = _plan(3, (0, 1, 2), (2, 1, 0), "minimal", extents=[500000, 20000, 2000000])
    assert calls == [((), 1), ((), 2)]
    assert groups[0]["keys"] == "2,1" and int(groups[0]["bits"]) == 36 and int(groups[0]["passes"]) == 5
    head, calls, groups = _plan(3, (0, 1, 2), (0, 2, 1), "minimal", extents=[500000, 20000, 2000000])
    assert groups[0]["prefix"] == "0" and groups[0]["segmented"] == "1" and int(groups[0]["bits"]) == 21


def test_bucketed_group_flattening_rule(lib):
    ext = [500000, 20000, 2000000]  # 19/15/21 bits: every nonzero packs into 55 bits
    # (0,2,1): bucket prefix 0 (19 bits) over key 2 (21 bits): 3 key passes, 5 flattened, so
    # the buckets are kept
    _, calls, groups = _plan(3, (0, 1, 2), (0, 2, 1), "minimal", extents=ext, flags=0)
    assert calls == [((0,), 2)]  # the PartialSort calls are Alg. 3's either way
    assert groups == [dict(prefix="0", keys="2", bits="21", passes="3", segmented="1")]
    # a 3-mode case where the prefix adds one pass (10 + 10 bits: 2 key passes, 3 flattened)
    _, _, groups = _plan(3, (0, 1, 2), (0, 2, 1), "minimal", extents=[1000, 800, 600], flags=0)
    assert groups == [dict(prefix="", keys="0,2", bits="20", passes="3", segmented="0")]
    # a 4-mode case where the prefix would add three passes keeps its buckets
    ext4 = [1000000, 100000, 1000, 50]  # 20/17/10/6 bits
    _, _, groups = _plan(4, (0, 1, 2, 3), (0, 1, 3, 2), "minimal", extents=ext4, flags=0)
    assert groups[0]["segmented"] == "1" and groups[0]["prefix"] == "0,1"
    # a 4-mode case where it adds two: buckets kept too
    _, _, groups = _plan(4, (0, 1, 2, 3), (0, 2, 1, 3), "minimal", extents=ext4, flags=0)
    assert groups[0]["segmented"] == "1" and groups[0]["prefix"] == "0"
    # too wide to pack (int32 extents summing past 64 bits): buckets kept
    _, _, groups = _plan(4, (0, 1, 2, 3), (0, 2, 1, 3), "minimal", extents=[1 << 20, 1 << 20, 1 << 20, 1 << 10],
                         flags=0)
    assert groups[0]["segmented"] == "1"


def test_extent_one_modes_need_no_pass(lib):
    head, calls, groups = _plan(3, (0, 1, 2), (2, 1, 0), "minimal", extents=[5, 1, 1])
    assert groups == []


def test_bad_arguments_are_rejected_before_launch(lib):
    with pytest.raises(qsd.QsdError) as e:
        qsd.qsd_plan(3, 10, [4, 4, 4], qsd.QSD_I32, qsd.QSD_F64, (0, 1, 2), (0, 0, 1))
    assert e.value.code == 2
    with pytest.raises(qsd.QsdError) as e:
        qsd.qsd_plan(3, 10, [4, 0, 4], qsd.QSD_I32, qsd.QSD_F64, (0, 1, 2), (0, 2, 1))
    assert e.value.code == 3
    with pytest.raises(qsd.QsdError) as e:
        qsd.qsd_plan(3, 1 << 30, [4, 4, 4], qsd.QSD_I32, qsd.QSD_F64, (0, 1, 2), (0, 2, 1))
    assert e.value.code == 4
    with pytest.raises(qsd.QsdError) as e:
        qsd.qsd_plan(9, 10, [4] * 9, qsd.QSD_I32, qsd.QSD_F64, tuple(range(9)), tuple(range(9)))
    assert e.value.code == 2
    with pytest.raises(qsd.QsdError) as e:
        qsd.qsd_plan(2, 10, [1 << 32, 4], qsd.QSD_I32, qsd.QSD_F64, (0, 1), (1, 0))
    assert e.value.code == 3
    h = qsd.qsd_plan(3, 100, [4, 4, 4], qsd.QSD_I32, qsd.QSD_F64, (0, 1, 2), (2, 1, 0))
    try:
        ws = qsd.qsd_plan_workspace(h)
        assert ws > 0
        fake = [0x1000] * 3
        with pytest.raises(qsd.QsdError) as e:  # workspace too small
            qsd.qsd_transpose(h, 100, fake, 0x1000, fake, 0x1000, 0x1000, ws - 1, None)
        assert e.value.code == 7
        with pytest.raises(qsd.QsdError) as e:  # more nonzeros than planned
            qsd.qsd_transpose(h, 101, fake, 0x1000, fake, 0x1000, 0x1000, ws, None)
        assert e.value.code == 4
        with pytest.raises(qsd.QsdError) as e:  # null coordinate pointer
            qsd.qsd_transpose(h, 100, [0x1000, 0, 0x1000], 0x1000, fake, 0x1000, 0x1000, ws, None)
        assert e.value.code == 1
        qsd.qsd_transpose(h, 0, fake, 0x1000, fake, 0x1000, 0x1000, ws, None)  # nnz = 0: no-op
    finally:
        qsd.qsd_plan_destroy(h)
    assert qsd.qsd_status_str(7).startswith("workspace")


def test_selector_host_parts(lib):
    import numpy as np
    from oracle import features as OF
    from oracle import mlp as OM
    # initial weights: same SplitMix64 stream and rounding as the oracle's
    for seed in (0, 7, 2 ** 63 + 5):
        assert np.array_equal(np.array(qsd.qsd_mlp_init(seed), dtype=np.float64), OM.init_params(seed))
    # the candidates' plan terms (host planner) equal the oracle's restatement of the library's
    # grouping, flattening and digit rules, for every order pair up to 5 modes and extents that
    # make flattening go either way
    import itertools
    for r, ext in [(2, (300, 9)), (3, (4, 16, 256)), (3, (500000, 20000, 2000000)), (4, (1 << 20, 1 << 17, 1 << 10, 64)),
                   (4, (9, 1, 40, 3000)), (5, (40, 300, 50, 2000, 30)), (5, (2000000, 300000, 50000, 2000, 100))]:
        perms = list(itertools.permutations(range(r)))
        for tau in perms[:: max(1, len(perms) // 6)]:
            for sigma in perms:
                got = qsd.qsd_candidate_terms((r, 1000, ext, qsd.QSD_I32, qsd.QSD_F64, tau, sigma))
                want, _ = OF.plan_terms(ext, tau, sigma)
                assert [g[0] for g in got] == [w is not None for w in want], (ext, tau, sigma)
                assert [g[1:] for g in got if g[0]] == [w for w in want if w is not None], (ext, tau, sigma)
    for c in range(qsd.NCAND):
        sc, fl = qsd.qsd_candidate(c)
        name, sched, flags = qsd.CANDIDATES[c]
        assert sc == qsd.sched_code(sched) and fl == flags
    with pytest.raises(qsd.QsdError) as e:  # workspace too small for a real request
        qsd.qsd_features((3, 10, (4, 4, 4), qsd.QSD_I32, qsd.QSD_F64, (0, 1, 2), (2, 1, 0)), [0x1000] * 3, 0x1000,
                         16, None)
    assert e.value.code == 7
    with pytest.raises(qsd.QsdError) as e:  # bad order
        qsd.qsd_features((3, 10, (4, 4, 4), qsd.QSD_I32, qsd.QSD_F64, (0, 1, 1), (2, 1, 0)), [0x1000] * 3, 0x1000,
                         4096, None)
    assert e.value.code == 2
    assert qsd.qsd_mlp_train_workspace(1000, 128) > 1000 * 4
    with pytest.raises(qsd.QsdError):
        qsd.qsd_mlp_train_workspace(10, 0)


def test_batch_workspace_max_covers_every_tuning(lib):
    # a 6-bit key is one pass at digit widths 6-8 but two (and packed records) at 4-5
    h = qsd.qsd_batch_plan([(2, 100000, [64, 64], 0, 1, (0, 1), (1, 0)),
                            (3, 50000, [100, 2000, 30], 0, 1, (0, 1, 2), (2, 1, 0)),
                            (4, 3000, [9, 9, 9, 9], 0, 1, (3, 2, 1, 0), (0, 1, 2, 3))])
    try:
        mx = qsd.qsd_batch_workspace_max(h)
        for rb in (4, 5, 6, 7, 8):
            for items in (0, 8, 16):
                for cap in (0, 100, 1024, 4096):
                    qsd.qsd_batch_set_tuning(h, items, rb, cap)
                    assert qsd.qsd_batch_workspace(h) <= mx, (items, rb, cap)
        with pytest.raises(qsd.QsdError):
            qsd.qsd_batch_set_tuning(h, 12, 8, 0)
    finally:
        qsd.qsd_batch_destroy(h)
