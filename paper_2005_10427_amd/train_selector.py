"""Training tool of the schedule selector.

    python -m paper_2005_10427_amd.train_selector all --dir OUT [--count 20000 --eval-count 200]

1. collect: generate seeded synthetic tensors (orders 3-5, extents log-uniform in
   [10, 1e7], nnz log-uniform in [1e4, 1e7], Zipf exponents uniform in [0, 1.5], random input
   and requested orders; identity requests skipped), compute each request's features with the
   library and time every valid candidate schedule (HIP events on the launch stream, best of 3
   after a warm-up; NaN for a candidate that does not exist for the request).  Rows are
   appended to an .npz file, so an interrupted collection resumes.
2. train: fit the perceptron on the GPU with the library's own kernels (qsd_mlp_train) to the
   log2 of the measured times, then choose the margin and the size cutoff that minimise the
   total time of the selected schedules on the training rows.  A plan is chosen once and
   reused, so the stored policy minimises the amortised time; the policy that would minimise
   one-shot time (the selection paid by every call) is reported beside it.
3. evaluate: on held-out tensors (a different seed, plus one 5-mode tensor of 1.5e8
   nonzeros), time every valid candidate and AUTO (the selection's wall time plus the chosen
   candidate), and report the regret t(chosen)/min_c t(c) - 1 and the speed-up over always
   using the minimal-pass schedule.

The weights file (qsd_model_load's format) and a JSON report are written to OUT.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2005_10427_amd import qsd  # noqa: E402

TRAIN_SEED = 20050427 + 4
EVAL_SEED = 20050427 + 5
GEN = dict(orders=(3, 4, 5), nnz_range=(1e4, 1e7), ext_range=(10, 1e7), zipf_max=1.5)
BIG = dict(ext=(2_000_000, 300_000, 50_000, 2_000, 100), nnz=150_000_000, s=0.8, tau=(0, 1, 2, 3, 4),
           sigma=(3, 0, 4, 1, 2))
CANDS = qsd.CANDIDATES  # (name, schedule, extra plan flags)
NC = len(CANDS)


def log(*a):
    print("[selector]", *a, file=sys.stderr, flush=True)


class Timer:
    """Plans, workspace and output buffers for timing transpositions on one stream."""

    def __init__(self, torch):
        self.torch = torch
        self.ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
        self.sel_ws = torch.empty(qsd.qsd_select_workspace(), dtype=torch.uint8, device="cuda")
        self.stream = torch.cuda.current_stream()
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def desc(self, T):
        ct = qsd.QSD_I64 if T.crd[0].dtype == self.torch.int64 else qsd.QSD_I32
        vt = qsd.QSD_F64 if T.val.dtype == self.torch.float64 else qsd.QSD_F32
        return (T.order, T.nnz, T.extents, ct, vt, T.in_order, T.out_order)

    def features(self, T):
        return qsd.qsd_features(self.desc(T), [c.data_ptr() for c in T.crd], self.sel_ws.data_ptr(),
                                self.sel_ws.numel(), self.stream.cuda_stream)

    def time(self, T, cand, reps=3):
        d = self.desc(T)
        _, sched, flags = CANDS[cand]
        h = qsd.qsd_plan(*d, sched=sched, flags=flags)
        try:
            need = qsd.qsd_plan_workspace(h)
            if need > self.ws.numel():
                self.ws = self.torch.empty(need, dtype=self.torch.uint8, device="cuda")
            oc = [self.torch.empty_like(c) for c in T.crd]
            ov = self.torch.empty_like(T.val)
            args = (h, T.nnz, [c.data_ptr() for c in T.crd], T.val.data_ptr(), [c.data_ptr() for c in oc],
                    ov.data_ptr(), self.ws.data_ptr(), self.ws.numel(), self.stream.cuda_stream)
            qsd.qsd_transpose(*args)
            best = math.inf
            for _ in range(reps):
                self.e0.record(self.stream)
                qsd.qsd_transpose(*args)
                self.e1.record(self.stream)
                self.e1.synchronize()
                best = min(best, self.e0.elapsed_time(self.e1))
            return best
        finally:
            qsd.qsd_plan_destroy(h)

    def select(self, model, T, reps=3):
        """(chosen schedule, predictions, best wall time of the selection in ms)."""
        d = self.desc(T)
        ptrs = [c.data_ptr() for c in T.crd]
        best, out = math.inf, None
        for _ in range(reps):
            self.torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = qsd.qsd_select(model, d, ptrs, self.sel_ws.data_ptr(), self.sel_ws.numel(), self.stream.cuda_stream)
            best = min(best, (time.perf_counter() - t0) * 1e3)
        return out[0], out[1], best


def collect(path, count, seed, big=False, budget_s=None):
    import torch
    from datagen.batched import iter_batch, make_batch
    rows = {}
    if os.path.exists(path):
        with np.load(path) as z:
            rows = {k: list(z[k]) for k in z.files}
    done = set(int(i) for i in rows.get("index", []))
    start = (max(done) + 1) if done else 0
    keys = ("index", "X", "ms", "nnz", "r", "zipf", "sel_ms")
    for k in keys:
        rows.setdefault(k, [])
    tm = Timer(torch)
    probe = qsd.qsd_model_create(qsd.qsd_mlp_init(0), 0.0, 0)  # an untrained model: selection cost only
    t_start = time.time()

    def add(i, T):
        feats = tm.features(T)
        valid = qsd.qsd_candidates_valid(tm.desc(T))
        ms = [tm.time(T, c) if valid[c] else math.nan for c in range(NC)]
        _, _, sel = tm.select(probe, T)
        rows["index"].append(i)
        rows["X"].append(np.asarray(feats, dtype=np.float32))
        rows["ms"].append(np.asarray(ms, dtype=np.float64))
        rows["nnz"].append(T.nnz)
        rows["r"].append(T.order)
        rows["zipf"].append(T.zipf)
        rows["sel_ms"].append(sel)

    def save():
        np.savez_compressed(path, **{k: np.asarray(v) for k, v in rows.items()})

    try:
        for i, T in iter_batch(count, seed=seed, device="cuda", start=start, **GEN):
            if T.in_order != T.out_order:
                add(i, T)
            del T
            if (i + 1) % 100 == 0:
                save()
                log(f"collected {len(rows['index'])} rows ({i + 1}/{count} tensors, {time.time() - t_start:.0f} s)")
                if budget_s is not None and time.time() - t_start > budget_s:
                    log(f"time budget of {budget_s:.0f} s used: stopping after tensor {i} (run again to resume)")
                    return None
        if big and count not in done:
            log("generating the 1.5e8-nonzero 5-mode tensor ...")
            T = make_batch(0, seed=seed, device="cuda", extra=[BIG])[0]
            add(count, T)
            del T
            torch.cuda.empty_cache()
        save()
    finally:
        qsd.qsd_model_destroy(probe)
    log(f"collection done: {len(rows['index'])} rows in {path}")
    return path


def _choose(pred, margin, valid):
    """The library's rule: candidate 0 unless a valid candidate is predicted faster by more than
    the margin (the fastest such one)."""
    best = np.zeros(len(pred), dtype=int)
    for s in range(1, NC):
        better = valid[:, s] & (pred[:, s] < pred[:, 0] - margin) & (pred[:, s] < pred[np.arange(len(pred)), best])
        best[better] = s
    return best


def train(paths, out_model, epochs=300, batch=128, lr=2e-3, seed=7):
    import torch
    X, ms, nnz, sel = [], [], [], []
    for p in paths:
        with np.load(p) as z:
            X.append(z["X"])
            ms.append(z["ms"])
            nnz.append(z["nnz"])
            sel.append(z["sel_ms"])
    X = np.concatenate(X).astype(np.float32)
    ms = np.concatenate(ms)
    nnz = np.concatenate(nnz)
    sel = np.concatenate(sel)
    Y = np.log2(ms).astype(np.float32)  # NaN where a candidate does not exist: no target
    valid = np.isfinite(ms)
    n = len(X)
    log(f"training on {n} rows")
    P = torch.tensor(np.asarray(qsd.qsd_mlp_init(seed), dtype=np.float32), device="cuda")
    Xd = torch.tensor(X, device="cuda")
    Yd = torch.tensor(Y, device="cuda")
    wsb = qsd.qsd_mlp_train_workspace(n, batch)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    t0 = time.time()
    last = qsd.qsd_mlp_train(P.data_ptr(), Xd.data_ptr(), Yd.data_ptr(), n, epochs, batch, lr, seed + 1,
                             ws.data_ptr(), wsb, s)
    train_s = time.time() - t0
    Yp = torch.empty(n, NC, device="cuda")
    qsd.qsd_mlp_forward(P.data_ptr(), Xd.data_ptr(), n, 0, 0, Yp.data_ptr(), s)
    pred = Yp.cpu().numpy().astype(np.float64)
    mse = float(np.mean(np.where(valid, pred - Y, 0.0) ** 2))  # the training loss' definition
    log(f"trained {epochs} epochs in {train_s:.1f} s: last batch loss {last:.4f}, training mse {mse:.4f}")
    # Margin and size cutoff.  A plan is built once and reused for every transposition of the
    # same request, so the choice is made for the amortised cost (selection excluded); the
    # one-shot optimum (selection paid by every call) is reported beside it.
    def fit(with_selection):
        best = None
        for margin in (0.0, 0.05, 0.1, 0.2, 0.3, 0.5):
            choice = _choose(pred, margin, valid)
            for min_nnz in (0, 1 << 16, 1 << 18, 1 << 20, 1 << 22, 1 << 24, 1 << 62):
                on = nnz >= min_nnz
                t = np.where(on, (sel if with_selection else 0.0) + ms[np.arange(n), choice], ms[:, 0])
                tot = float(t.sum())
                if best is None or tot < best[0] - 1e-9:
                    best = (tot, margin, min_nnz)
        return best
    total, margin, min_nnz = fit(False)
    one_shot = fit(True)
    log(f"amortised: margin {margin}, min_nnz {min_nnz}: training total {total:.1f} ms vs minimal "
        f"{ms[:, 0].sum():.1f} ms (best possible {np.nanmin(ms, axis=1).sum():.1f}); one-shot optimum: margin "
        f"{one_shot[1]}, min_nnz {one_shot[2]}, {one_shot[0]:.1f} ms")
    params = P.cpu().numpy()
    qsd.write_model_file(out_model, params, margin, min_nnz)
    return dict(rows=n, epochs=epochs, batch=batch, lr=lr, seed=seed, train_seconds=train_s,
                last_batch_loss=last, train_mse_log2=mse, margin=margin, min_nnz=int(min_nnz),
                train_total_ms_auto_amortised=total, train_total_ms_minimal=float(ms[:, 0].sum()),
                train_total_ms_best=float(np.nanmin(ms, axis=1).sum()),
                best_counts={CANDS[c][0]: int((np.nanargmin(ms, axis=1) == c).sum()) for c in range(NC)},
                one_shot_policy=dict(margin=one_shot[1], min_nnz=int(one_shot[2]), total_ms=one_shot[0]),
                selection_ms_median=float(np.median(sel)))


def evaluate(model_path, count, seed, out_npz, big=True, one_shot_min_nnz=None):
    import torch
    from datagen.batched import iter_batch, make_batch
    tm = Timer(torch)
    model = qsd.qsd_model_load(model_path)
    recs = []

    def one(T):
        valid = qsd.qsd_candidates_valid(tm.desc(T))
        ms = [tm.time(T, c) if valid[c] else math.nan for c in range(NC)]
        chosen, pred, sel = tm.select(model, T)
        recs.append(dict(nnz=T.nnz, r=T.order, ms=ms, chosen=int(chosen), sel_ms=sel, pred=list(pred)))

    try:
        for i, T in iter_batch(count, seed=seed, device="cuda", **GEN):
            if T.in_order != T.out_order:
                one(T)
            del T
            if (i + 1) % 50 == 0:
                log(f"evaluated {i + 1}/{count}")
        if big:
            log("generating the 1.5e8-nonzero 5-mode tensor ...")
            T = make_batch(0, seed=seed, device="cuda", extra=[BIG])[0]
            one(T)
            log(f"big tensor: ms {recs[-1]['ms']}, chosen {recs[-1]['chosen']}, selection {recs[-1]['sel_ms']:.3f} ms")
            del T
            torch.cuda.empty_cache()
    finally:
        qsd.qsd_model_destroy(model)
    ms = np.array([r["ms"] for r in recs])
    ch = np.array([r["chosen"] for r in recs])
    sel = np.array([r["sel_ms"] for r in recs])
    nnz = np.array([r["nnz"] for r in recs])
    np.savez(out_npz, ms=ms, chosen=ch, sel_ms=sel, nnz=nnz, r=np.array([r["r"] for r in recs]))
    best = np.nanmin(ms, axis=1)
    n = len(ms)

    def stats(t):
        reg = t / best - 1.0
        return dict(mean=float(reg.mean()), median=float(np.median(reg)), p95=float(np.quantile(reg, 0.95)),
                    max=float(reg.max()))

    t_auto = ms[np.arange(n), ch]
    auto_total = float((t_auto + sel).sum())
    # the one-shot policy fitted on the training rows: requests below its size cutoff take the
    # minimal plan without sampling, the others pay the selection
    once = None
    if one_shot_min_nnz is not None:
        on = nnz >= one_shot_min_nnz
        t_once = np.where(on, t_auto + sel, ms[:, 0])
        once = dict(min_nnz=int(one_shot_min_nnz), requests_selected=int(on.sum()), total_ms=float(t_once.sum()),
                    speedup_over_minimal=float(ms[:, 0].sum() / t_once.sum()))
    names = [c[0] for c in CANDS]
    with_cand = {names[c]: ms[np.isfinite(ms[:, c]), c] for c in range(NC)}
    rep = dict(
        tensors=n,
        candidates=names,
        valid_counts={names[c]: int(np.isfinite(ms[:, c]).sum()) for c in range(NC)},
        best_counts={names[c]: int((np.nanargmin(ms, axis=1) == c).sum()) for c in range(NC)},
        chosen_counts={names[c]: int((ch == c).sum()) for c in range(NC)},
        regret_auto=stats(t_auto), regret_minimal=stats(ms[:, 0]),
        regret_per_candidate={names[c]: stats(np.where(np.isfinite(ms[:, c]), ms[:, c], best)) for c in range(NC)},
        total_ms=dict(minimal=float(ms[:, 0].sum()), auto_with_selection=auto_total,
                      auto_without_selection=float(t_auto.sum()), oracle_best=float(best.sum()),
                      lsd=float(np.nansum(ms[:, 5]))),
        speedup_auto_over_minimal_amortised=float(ms[:, 0].sum() / t_auto.sum()),
        speedup_auto_over_minimal_one_shot=float(ms[:, 0].sum() / auto_total),
        one_shot_policy=once,
        speedup_best_over_minimal=float(ms[:, 0].sum() / best.sum()),
        choice_accuracy=float((ch == np.nanargmin(ms, axis=1)).mean()),
        selection_ms=dict(median=float(np.median(sel)), max=float(sel.max())),
        rows_with_candidate={k: int(len(v)) for k, v in with_cand.items()},
    )
    if big:
        r = recs[-1]
        rep["big_tensor"] = dict(extents=BIG["ext"], nnz=BIG["nnz"], ms=dict(zip(names, r["ms"])),
                                 chosen=names[r["chosen"]], selection_ms=r["sel_ms"])
    return rep


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["collect", "train", "evaluate", "all"])
    ap.add_argument("--dir", default="selector_runs", help="where collected timings, the trained model and the report are written")
    ap.add_argument("--count", type=int, default=20000)
    ap.add_argument("--eval-count", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--no-big", action="store_true")
    ap.add_argument("--budget-s", type=float, default=None,
                    help="collect: stop (after a save) once this many seconds are spent; a later run resumes")
    ap.add_argument("--train-data", default=None, help="an existing collection to train on (skips collect)")
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        log("no GPU visible")
        return 1
    qsd.load()
    os.makedirs(args.dir, exist_ok=True)
    data = args.train_data or os.path.join(args.dir, "train.npz")
    model = os.path.join(args.dir, "selector_model.bin")
    report = {}
    if args.cmd in ("collect", "all") and not args.train_data:
        if collect(data, args.count, TRAIN_SEED, budget_s=args.budget_s) is None:
            return 3  # unfinished: run again to resume
    if args.cmd in ("train", "all"):
        report["train"] = train([data], model, epochs=args.epochs)
    if args.cmd in ("evaluate", "all"):
        once = None
        if "train" in report:
            once = report["train"]["one_shot_policy"]["min_nnz"]
        elif os.path.exists(os.path.join(args.dir, "report.json")):
            with open(os.path.join(args.dir, "report.json")) as f:
                once = json.load(f)["train"]["one_shot_policy"]["min_nnz"]
        report["eval"] = evaluate(model, args.eval_count, EVAL_SEED, os.path.join(args.dir, "eval.npz"),
                                  big=not args.no_big, one_shot_min_nnz=once)
        log(json.dumps(report["eval"]))
    report["generator"] = dict(GEN, train_seed=TRAIN_SEED, eval_seed=EVAL_SEED, train_count=args.count,
                               eval_count=args.eval_count)
    with open(os.path.join(args.dir, f"report_{args.cmd}.json"), "w") as f:
        json.dump(report, f, indent=1, default=float)
    return 0


if __name__ == "__main__":
    sys.exit(main())
