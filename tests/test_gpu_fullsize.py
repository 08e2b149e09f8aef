"""Full-size transpositions (the 1e8-nonzero 3-mode and 2e8-nonzero 4-mode workloads, in the
launch configuration the benchmark times) checked through properties that fix the output:
the nonzeros are distinct, so the stable sort under sigma is the unique sorted arrangement.
  * sorted: the composite sigma key strictly increases along the output;
  * same nonzeros: an order-independent hash of every (coordinates, value bits) record is
    equal on both sides;
  * positions: at sampled output positions j the record has exactly j input keys below its
    key (its rank by definition), computed one position at a time."""
import sys

import numpy as np
import pytest

from datagen import CONFIGS, config_tensor

pytestmark = pytest.mark.gpu


def note(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _mix(x, torch):
    """SplitMix64's output function on int64 tensors (arithmetic wraps modulo 2^64)."""
    def shr(v, k):  # logical shift right
        return (v >> k) & ((1 << (64 - k)) - 1)
    z = x
    z = (z ^ shr(z, 30)) * torch.tensor(-4658895280553007687, dtype=torch.int64, device=x.device)  # 0xBF58476D1CE4E5B9
    z = (z ^ shr(z, 27)) * torch.tensor(-7723592293110705685, dtype=torch.int64, device=x.device)  # 0x94D049BB133111EB
    return z ^ shr(z, 31)


def _record_hash(crd, val, torch):
    h = torch.zeros_like(crd[0], dtype=torch.int64)
    for m, c in enumerate(crd):
        salt = ((m + 1) * 0x9E3779B97F4A7C15) % (1 << 64)  # a different offset per mode, as int64
        salt -= (1 << 64) if salt >= (1 << 63) else 0
        h = _mix(h + c.to(torch.int64) + salt, torch)
    vb = val.view(torch.int64) if val.dtype == torch.float64 else val.view(torch.int32).to(torch.int64)
    h = _mix(h ^ vb, torch)
    return int(h.sum().item())


def _key(crd, sigma, extents, torch):
    key = torch.zeros_like(crd[0], dtype=torch.int64)
    for m in sigma:
        b = (int(extents[m]) - 1).bit_length() if extents[m] > 1 else 0
        key = (key << b) | crd[m].to(torch.int64)
    return key


def _check_full(qsd, name, sigmas, samples=512):
    import torch
    note(f"generating {name} at full size")
    T = config_tensor(name)
    dev = torch.device("cuda:0")
    crd = [torch.from_numpy(c).to(dev) for c in T.crd]
    val = torch.from_numpy(T.val).to(dev)
    del T.crd[:]
    h_in = _record_hash(crd, val, torch)
    plans = [qsd.Plan(T.extents, T.in_order, s, val.shape[0], str(crd[0].dtype).replace("torch.", ""),
                      str(val.dtype).replace("torch.", ""), "minimal") for s in sigmas]
    ws = torch.empty(max(p.ws_bytes for p in plans), dtype=torch.uint8, device=dev)
    out_crd = [torch.empty_like(c) for c in crd]
    out_val = torch.empty_like(val)
    g = torch.Generator(device=dev)
    g.manual_seed(20050427)
    n = val.shape[0]
    for P, sigma in zip(plans, sigmas):
        note(f"{name} sigma={sigma}")
        P.transpose(crd, val, out_crd, out_val, ws=ws)
        torch.cuda.synchronize()
        assert P.device_status() == 0
        k_out = _key(out_crd, sigma, P.extents, torch)
        assert bool((k_out[1:] > k_out[:-1]).all()), "output not strictly sorted under sigma"
        assert _record_hash(out_crd, out_val, torch) == h_in, "records differ"
        k_in = _key(crd, sigma, P.extents, torch)
        pos = torch.randint(0, n, (samples,), generator=g, device=dev)
        pos[0], pos[1] = 0, n - 1
        for j in pos.tolist():
            assert int((k_in < k_out[j]).sum().item()) == j, (sigma, j)
        del k_in, k_out


def test_plain_full_size(gpu_lib):
    _check_full(gpu_lib, "plain", CONFIGS["plain"]["sigmas"], samples=256)


def test_wide_full_size(gpu_lib):
    # the orders whose plans differ most: bucketed groups kept or flattened, two-pass groups,
    # packed and unpacked paths
    sig = CONFIGS["wide"]["sigmas"]
    _check_full(gpu_lib, "wide", sig[::4], samples=64)
