"""The schedule selector's HIP kernels through the C ABI against the oracle: feature counts
bit-exact, features, forward and backward passes, Adam and minibatch training within float32
tolerances, and the AUTO choice agreeing with the oracle's prediction."""
import sys

import numpy as np
import pytest

from datagen import make_tensor
from oracle import features as OF
from oracle import mlp as OM
from oracle.transpose import transpose as oracle_transpose

pytestmark = pytest.mark.gpu


def note(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _dev(T):
    import torch
    crd = [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in T.crd]
    val = torch.from_numpy(np.ascontiguousarray(T.val)).cuda()
    return crd, val


def _desc(qsd, T, sigma):
    ct = qsd.QSD_I64 if T.crd[0].dtype == np.int64 else qsd.QSD_I32
    vt = qsd.QSD_F64 if T.val.dtype == np.float64 else qsd.QSD_F32
    return (T.order, T.nnz, T.extents, ct, vt, T.in_order, sigma)


CASES = [  # extents, nnz, zipf, in_order, sigma, crd dtype
    ((1000, 800, 600), 100_000, (0, 0, 0), (0, 1, 2), (0, 2, 1), np.int32),
    ((5000, 40, 300_000), 250_000, (1.1, 1.1, 1.1), (0, 1, 2), (2, 1, 0), np.int32),
    ((300, 20, 50, 7), 60_000, (1.3, 1.3, 0, 0), (2, 0, 1, 3), (1, 3, 0, 2), np.int32),
    ((50, 60, 70, 80, 9), 16_385, (0.5,) * 5, (0, 1, 2, 3, 4), (4, 2, 0, 3, 1), np.int64),
    ((7, 9), 5, (0, 0), (1, 0), (0, 1), np.int32),
    ((1, 1, 1), 1, (0, 0, 0), (0, 1, 2), (2, 1, 0), np.int32),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_feature_counts_and_features_match_oracle(gpu_lib, case):
    import torch
    qsd = gpu_lib
    ext, nnz, z, tau, sigma, cd = CASES[case]
    T = make_tensor(ext, nnz, z, tau, cd, np.float64, seed=900 + case)
    note(f"features ext={ext} nnz={nnz} tau={tau} sigma={sigma}")
    crd, _ = _dev(T)
    wsb = qsd.qsd_select_workspace()
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    counts, S, pairs = qsd.qsd_feature_counts(_desc(qsd, T, sigma), [c.data_ptr() for c in crd], ws.data_ptr(),
                                              wsb, s)
    terms, Q = OF.plan_terms(ext, tau, sigma)
    per_mode, mch, S0, P0 = OF.counts(T.crd, masks=Q)
    assert (S, pairs) == (S0, P0)
    r = len(ext)
    if nnz:
        for m in range(r):
            assert tuple(counts[3 * m:3 * m + 3]) == per_mode[m], m
        for q in range(4):
            assert counts[3 * (r + q)] == (mch[q] if Q[q] else 0), q
    assert qsd.qsd_candidates_valid(_desc(qsd, T, sigma)) == [t is not None for t in terms]
    f = np.array(qsd.qsd_features(_desc(qsd, T, sigma), [c.data_ptr() for c in crd], ws.data_ptr(), wsb, s))
    want = OF.features(T.crd, ext, tau, sigma, T.crd[0].dtype.itemsize, 8)
    assert np.allclose(f, want, rtol=1e-6, atol=1e-6)


def _theta(seed):
    return np.random.default_rng(seed).normal(0, 0.25, OM.NPARAM).astype(np.float32).astype(np.float64)


def _t(a):
    import torch
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda").contiguous()


@pytest.mark.parametrize("n", [1, 255, 1000])
def test_forward_and_backward_match_oracle(gpu_lib, n):
    import torch
    qsd = gpu_lib
    rng = np.random.default_rng(n)
    X = rng.uniform(0, 1, size=(n, OM.SIZES[0])).astype(np.float32).astype(np.float64)
    T = rng.normal(0, 2, size=(n, OM.SIZES[3])).astype(np.float32).astype(np.float64)
    T[rng.uniform(size=T.shape) < 0.3] = np.nan  # candidates that do not exist for a row
    theta = _theta(n)
    P, Xd, Td = _t(theta), _t(X), _t(T)
    H1 = torch.empty(n, 64, device="cuda")
    H2 = torch.empty(n, 64, device="cuda")
    Y = torch.empty(n, OM.SIZES[3], device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    qsd.qsd_mlp_forward(P.data_ptr(), Xd.data_ptr(), n, H1.data_ptr(), H2.data_ptr(), Y.data_ptr(), s)
    h1, h2, y = OM.forward(theta, X)
    torch.cuda.synchronize()
    assert np.allclose(Y.cpu().numpy(), y, rtol=1e-4, atol=1e-4)
    assert np.allclose(H1.cpu().numpy(), h1, rtol=1e-4, atol=1e-4)
    G = torch.empty(OM.NPARAM, device="cuda")
    L = torch.empty(1, device="cuda")
    wsb = qsd.qsd_mlp_backward_workspace(n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    qsd.qsd_mlp_backward(P.data_ptr(), Xd.data_ptr(), H1.data_ptr(), H2.data_ptr(), Y.data_ptr(), Td.data_ptr(), n,
                         G.data_ptr(), L.data_ptr(), ws.data_ptr(), wsb, s)
    loss, g = OM.backward(theta, X, T)
    torch.cuda.synchronize()
    assert abs(float(L.item()) - loss) <= 1e-4 * max(1.0, loss)
    gd = G.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(gd - g)) <= 1e-4 * max(1e-3, np.max(np.abs(g)))


def test_adam_step_matches_oracle(gpu_lib):
    import torch
    qsd = gpu_lib
    rng = np.random.default_rng(3)
    theta = _theta(3)
    g = rng.normal(0, 1e-2, OM.NPARAM).astype(np.float32).astype(np.float64)
    m = rng.normal(0, 1e-3, OM.NPARAM).astype(np.float32).astype(np.float64)
    v = np.abs(rng.normal(0, 1e-4, OM.NPARAM)).astype(np.float32).astype(np.float64)
    P, Gd, Md, Vd = _t(theta), _t(g), _t(m), _t(v)
    qsd.qsd_mlp_adam(P.data_ptr(), Gd.data_ptr(), Md.data_ptr(), Vd.data_ptr(), 5, 1e-3, 0.9, 0.999, 1e-8,
                     torch.cuda.current_stream().cuda_stream)
    t2, m2, v2 = OM.adam_step(theta, g, m, v, 5, 1e-3)
    torch.cuda.synchronize()
    assert np.allclose(P.cpu().numpy(), t2, rtol=0, atol=1e-6)
    assert np.allclose(Md.cpu().numpy(), m2, rtol=1e-5, atol=1e-9)
    assert np.allclose(Vd.cpu().numpy(), v2, rtol=1e-5, atol=1e-12)


def test_minibatch_training_matches_oracle(gpu_lib):
    import torch
    qsd = gpu_lib
    rng = np.random.default_rng(4)
    n, epochs, batch, lr = 100, 3, 32, 1e-3
    X = rng.uniform(0, 1, size=(n, OM.SIZES[0])).astype(np.float32).astype(np.float64)
    T = np.stack([X[:, 0] + X[:, 1], 2 * X[:, 2], -X[:, 3], X[:, 4] * X[:, 5], X[:, 6], X[:, 7] - X[:, 8]],
                 axis=1).astype(np.float32).astype(np.float64)
    T[:, 4][X[:, 9] < 0.5] = np.nan
    theta0 = np.array(qsd.qsd_mlp_init(21), dtype=np.float64)
    assert np.array_equal(theta0, OM.init_params(21))
    P, Xd, Td = _t(theta0), _t(X), _t(T)
    wsb = qsd.qsd_mlp_train_workspace(n, batch)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    last = qsd.qsd_mlp_train(P.data_ptr(), Xd.data_ptr(), Td.data_ptr(), n, epochs, batch, lr, 99, ws.data_ptr(),
                             wsb, torch.cuda.current_stream().cuda_stream)
    theta, last0 = OM.train(theta0, X, T, epochs, batch, lr, 99)
    diff = np.abs(P.cpu().numpy().astype(np.float64) - theta)
    steps = epochs * -(-n // batch)
    note(f"training: max |dtheta| {diff.max():.2e}, loss {last:.5f} vs {last0:.5f}")
    assert abs(last - last0) <= 1e-3 * max(1.0, last0)
    assert np.quantile(diff, 0.99) < 1e-4 and diff.max() <= 2 * lr * steps


def test_select_follows_the_prediction_and_auto_is_bit_exact(gpu_lib, tmp_path):
    import torch
    qsd = gpu_lib
    theta = _theta(11)
    path = tmp_path / "model.bin"
    qsd.write_model_file(str(path), theta.astype(np.float32), 0.0)
    model = qsd.qsd_model_load(str(path))
    try:
        wsb = qsd.qsd_select_workspace()
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        s = torch.cuda.current_stream().cuda_stream
        for case in range(4):
            ext, nnz, z, tau, sigma, cd = CASES[case]
            T = make_tensor(ext, nnz, z, tau, cd, np.float64, seed=950 + case)
            crd, val = _dev(T)
            ch, pred = qsd.qsd_select(model, _desc(qsd, T, sigma), [c.data_ptr() for c in crd], ws.data_ptr(),
                                      wsb, s)
            feat = OF.features(T.crd, ext, tau, sigma, T.crd[0].dtype.itemsize, 8)
            _, _, y = OM.forward(theta, feat[None, :])
            assert np.allclose(pred, y[0], rtol=1e-4, atol=1e-4)
            valid = OF.valid_candidates(ext, tau, sigma)
            yv = np.where(valid, y[0], np.inf)
            order = np.argsort(yv)
            in_range = bool(np.all((feat >= 0) & (feat <= 4)))
            if in_range and yv[order[1]] - yv[order[0]] > 1e-3:  # a clear winner: both sides agree
                assert ch == int(order[0]), (pred, y, valid)
            h, ch2 = qsd.qsd_plan_auto(model, _desc(qsd, T, sigma), [c.data_ptr() for c in crd], ws.data_ptr(),
                                       wsb, s)
            assert ch2 == ch
            try:
                pws = torch.empty(max(qsd.qsd_plan_workspace(h), 1), dtype=torch.uint8, device="cuda")
                oc = [torch.empty_like(c) for c in crd]
                ov = torch.empty_like(val)
                qsd.qsd_transpose(h, T.nnz, [c.data_ptr() for c in crd], val.data_ptr(),
                                  [c.data_ptr() for c in oc], ov.data_ptr(), pws.data_ptr(), pws.numel(), s)
                torch.cuda.synchronize()
                w_crd, w_val = oracle_transpose(T.crd, T.val, sigma)
                for m in range(T.order):
                    assert np.array_equal(oc[m].cpu().numpy(), w_crd[m])
                assert np.array_equal(ov.cpu().numpy().view(np.uint64), w_val.view(np.uint64))
            finally:
                qsd.qsd_plan_destroy(h)
    finally:
        qsd.qsd_model_destroy(model)
