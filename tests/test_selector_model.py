"""The committed selector: its weights reproduce the fit recorded at training time (oracle
forward pass on the committed training features), the policy in the weights file is the
recorded one, and the held-out evaluation report is consistent with its measurements.
These are measured timings: parity unpinned; the report states what the network gains over
the minimal-pass schedule alone."""
import json
import os
import struct

import numpy as np
import pytest

from conftest import ROOT
from oracle import mlp

SEL = os.path.join(ROOT, "paper_2005_10427_amd", "selector")


def _model():
    with open(os.path.join(SEL, "selector_model.bin"), "rb") as f:
        b = f.read()
    assert b[:8] == b"QSDMLP2\0"
    n, margin, min_nnz = struct.unpack("<ifq", b[8:24])
    assert n == mlp.NPARAM and len(b) == 24 + 4 * n
    return np.frombuffer(b[24:], dtype="<f4").astype(np.float64), margin, min_nnz


def test_weights_reproduce_the_recorded_fit():
    theta, margin, min_nnz = _model()
    rep = json.load(open(os.path.join(SEL, "report.json")))["train"]
    assert (margin, min_nnz) == (pytest.approx(rep["margin"]), rep["min_nnz"])
    with np.load(os.path.join(SEL, "train.npz")) as z:
        X, ms = z["X"].astype(np.float64), z["ms"]
    _, _, y = mlp.forward(theta, X)
    valid = np.isfinite(ms)  # candidates that exist for a row; the others carry no target
    mse = float(np.mean(np.where(valid, y - np.log2(np.where(valid, ms, 1.0)), 0.0) ** 2))
    assert mse == pytest.approx(rep["train_mse_log2"], rel=1e-3)
    assert rep["rows"] == len(X)


def test_heldout_report_matches_its_measurements():
    rep = json.load(open(os.path.join(SEL, "report.json")))["eval"]
    with np.load(os.path.join(SEL, "eval.npz")) as z:
        ms, chosen, sel = z["ms"], z["chosen"], z["sel_ms"]
    n = len(ms)
    assert rep["tensors"] == n
    assert np.all(np.isfinite(ms[:, 0]))  # the minimal-pass plan exists for every request
    t_auto = ms[np.arange(n), chosen]
    assert np.all(np.isfinite(t_auto))    # AUTO only ever chooses a candidate that exists
    best = np.nanmin(ms, axis=1)
    assert rep["total_ms"]["minimal"] == pytest.approx(ms[:, 0].sum())
    assert rep["total_ms"]["auto_without_selection"] == pytest.approx(t_auto.sum())
    assert rep["total_ms"]["auto_with_selection"] == pytest.approx((t_auto + sel).sum())
    assert rep["regret_auto"]["mean"] == pytest.approx((t_auto / best - 1).mean())
    # what the network gains: amortised speed-up over always taking the minimal-pass plan,
    # bounded by the gain of a perfect per-request choice
    gain = ms[:, 0].sum() / t_auto.sum()
    assert gain == pytest.approx(rep["speedup_auto_over_minimal_amortised"])
    assert gain <= ms[:, 0].sum() / best.sum() + 1e-12
    print(f"held-out: AUTO amortised x{gain:.4f} over minimal (perfect choice x{ms[:, 0].sum() / best.sum():.4f}); "
          f"one-shot x{rep['speedup_auto_over_minimal_one_shot']:.3f}")
