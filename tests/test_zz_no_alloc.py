"""The entry point that allocates nothing (qsd_transpose_noalloc) through the C ABI: its output
equals qsd_transpose's on a caller workspace, bit for bit, on two calls in a row (the second
smaller, on another plan), and a plan needing more than the fixed workspace is rejected."""
import sys

import numpy as np
import pytest

from datagen import config_tensor

pytestmark = pytest.mark.gpu


def note(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _bits(t):
    import torch
    return t.view(torch.int64) if t.dtype == torch.float64 else t.view(torch.int32)


def _compare(qsd, name, nnz, sigma, max_ws):
    import torch
    T = config_tensor(name, nnz=nnz)
    dev = torch.device("cuda:0")
    crd = [torch.from_numpy(c).to(dev) for c in T.crd]
    val = torch.from_numpy(T.val).to(dev)
    vd = "float64" if T.val.dtype == np.float64 else "float32"
    P = qsd.Plan(T.extents, T.in_order, sigma, T.nnz, "int32", vd, "minimal")
    assert P.ws_bytes <= max_ws
    note(f"{name} nnz={nnz} sigma={sigma} workspace={P.ws_bytes}")
    want_crd, want_val = P.transpose(crd, val)
    torch.cuda.synchronize()
    assert P.device_status() == 0
    got_crd = [torch.full_like(c, -1) for c in crd]
    got_val = torch.full_like(val, 7.0)
    s = torch.cuda.current_stream(dev)
    qsd.qsd_transpose_noalloc(P.handle, T.nnz, [c.data_ptr() for c in crd], val.data_ptr(),
                              [c.data_ptr() for c in got_crd], got_val.data_ptr(), s.cuda_stream)
    torch.cuda.synchronize()
    for m in range(len(crd)):
        assert torch.equal(got_crd[m], want_crd[m]), (name, sigma, m)
    assert torch.equal(_bits(got_val), _bits(want_val)), (name, sigma, "values")


def test_noalloc_matches_the_workspace_entry_point(gpu_lib):
    max_ws = gpu_lib.QSD_NOALLOC_MAX_WORKSPACE
    # first call: 1e6 nonzeros of the 3-mode workload (packed passes); second, smaller, on
    # another plan: 4-mode tensor with a bucketed group
    _compare(gpu_lib, "plain", 1_000_000, (2, 1, 0), max_ws)
    _compare(gpu_lib, "wide", 150_000, (0, 3, 2, 1), max_ws)


def test_noalloc_rejects_a_plan_beyond_the_maximum(gpu_lib):
    import torch
    P = gpu_lib.Plan((500000, 20000, 2000000), (0, 1, 2), (2, 1, 0), 50_000_000, "int32", "float64")
    assert P.ws_bytes > gpu_lib.QSD_NOALLOC_MAX_WORKSPACE
    dummy = torch.empty(8, dtype=torch.int32, device="cuda")
    with pytest.raises(gpu_lib.QsdError) as e:
        gpu_lib.qsd_transpose_noalloc(P.handle, 10, [dummy.data_ptr()] * 3, dummy.data_ptr(),
                                      [dummy.data_ptr()] * 3, dummy.data_ptr(),
                                      torch.cuda.current_stream().cuda_stream)
    assert e.value.code == gpu_lib.QSD_ERR_WORKSPACE
