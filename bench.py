"""Benchmark: transposed nonzeros per second on one MI355X.

Default workload ("plain"; one step): the 3-mode tensor with extents 500000 x 20000 x 2000000, 1e8 distinct
nonzeros whose coordinates are Zipf(1.1) over a relabelled extent, int32 coordinates, fp64
values, input order (0,1,2), transposed to all five other orders.  Inputs are resident in
device memory before the timed region; value = 5e8 * steps / seconds.

Also reported: the roofline of the dominant kernel (the digit pass), timed with HIP events
recorded by the library on the stream each launch runs on, and the CPU oracle timed on a
bounded sample of the same workload.

``--workload wide``: the 4-mode tensor with extents 1000000 x 100000 x 1000 x 50, 2e8
distinct nonzeros (modes 0-1 Zipf(1.3), modes 2-3 uniform), int32 coordinates, fp32 values,
input order (0,1,2,3), transposed to all 23 other orders per step (the plans with bucketed
groups run the segment sorts).

``--workload batched``: 4,096 independent tensors (order 3 or 4, nnz log-uniform in
[1e3, 1e6], extents log-uniform in [10, 1e6], Zipf exponents uniform in [0, 1.5], fp64
values, random input and requested orders); one step is one replay of the autotuned,
graph-captured batched transposition, compared with the same transpositions issued one by
one with the minimal-pass plan.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "transposed nnz/s & HBM GB/s (% of peak); learned+batched vs plain schedule"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_digit_plain_traffic.json")
CSRC = os.path.join(ROOT, "paper_2005_10427_amd", "csrc")
KERNEL_SRCS = ["kernels_impl.h", "kernels.h", "kernels.hip"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_sha():
    """Hash of the device-code sources (the counters are valid for exactly this code)."""
    h = hashlib.sha256()
    for name in KERNEL_SRCS:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per digit-pass launch from rocprofv3 counters, if taken on this kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha256") != kernel_sha():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(T, sigmas, budget_s=20.0):
    """The oracle (numpy stable sort + gather), single-threaded, on a prefix sample of the
    tensor (still sorted in the input order), all requested orders."""
    import numpy as np
    from oracle.transpose import transpose as oracle_transpose
    n = 1_000_000
    t_one = None
    while True:
        crd = [c[:n] for c in T.crd]
        val = T.val[:n]
        t0 = time.perf_counter()
        for s in sigmas:
            oracle_transpose(crd, val, s)
        dt = time.perf_counter() - t0
        if dt > budget_s / 4 or n * 4 > T.nnz:
            t_one = dt
            break
        n *= 4
    rate = n * len(sigmas) / t_one
    # a comparison sort costs about N log N: the rate at the full size is lower by log n / log N
    full = rate * math.log(n) / math.log(T.nnz) if n < T.nnz else rate
    return {"value": rate, "unit": "nnz/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} nonzeros of the {T.nnz}-nonzero workload tensor (a prefix, still "
                      f"sorted in the input order), all {len(sigmas)} orders, {t_one:.1f} s "
                      f"single-threaded numpy (lexsort + gather)",
            "full_size_estimate": {"value": full, "rule": "sample rate x log(sample) / log(nnz)"},
            "host": host_cpu()}


def host_cpu():
    """The host's CPU model and thread count, as the oracle's rate depends on them."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sched", default="minimal", choices=["minimal", "top2", "lsd", "auto"])
    ap.add_argument("--keep-buckets", action="store_true",
                    help="run bucketed groups as segment sorts (QSD_KEEP_BUCKETS) instead of flattening")
    ap.add_argument("--nnz", type=int, default=None, help="shrink the workload (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="plain", choices=["plain", "wide", "batched"])
    ap.add_argument("--count", type=int, default=None, help="tensors of the batched workload (testing only)")
    ap.add_argument("--no-sequence", action="store_true",
                    help="batched workload: skip timing the one-by-one comparison (for profiler runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="K",
                    help="after timing, run K identity transpositions (plain copies of every array) "
                         "that calibrate hardware byte counters against a known size")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU path is "
              f"not built", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from datagen import CONFIGS, config_tensor
    from paper_2005_10427_amd import qsd

    qsd.load()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    if args.workload == "batched":
        return bench_batched(args)
    name = args.workload
    cfg = CONFIGS[name]
    sigmas = cfg["sigmas"]
    log(f"generating the {name} workload ...")
    t0 = time.time()
    T = config_tensor(name, nnz=args.nnz)
    N = T.nnz
    log(f"generated {N} nonzeros in {time.time() - t0:.1f} s")
    ct, vt = str(T.crd[0].dtype), str(T.val.dtype)

    dev = torch.device("cuda:0")
    crd = [torch.from_numpy(c).to(dev) for c in T.crd]
    val = torch.from_numpy(T.val).to(dev)
    model = qsd.qsd_model_load(qsd.MODEL_PATH) if args.sched == "auto" else None
    flags = qsd.QSD_KEEP_BUCKETS if args.keep_buckets else 0
    plans = [qsd.Plan(T.extents, T.in_order, s, N, ct, vt, args.sched, flags, model=model, crd=crd)
             for s in sigmas]
    if model is not None:
        log("selector chose " + ", ".join(f"{s}: {qsd.CAND_NAMES[p.chosen]}" for s, p in zip(sigmas, plans)))
    ws = torch.empty(max(p.ws_bytes for p in plans), dtype=torch.uint8, device=dev)
    if name == "plain":
        outs = [([torch.empty_like(c) for c in crd], torch.empty_like(val)) for _ in sigmas]
    else:  # 23 orders: one output set, overwritten by every order in turn
        outs = [([torch.empty_like(c) for c in crd], torch.empty_like(val))] * len(sigmas)
    stream = torch.cuda.current_stream(dev)

    def step():
        for p, (oc, ov) in zip(plans, outs):
            p.transpose(crd, val, oc, ov, stream=stream, ws=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    status = qsd.qsd_device_status(ws.data_ptr(), stream.cuda_stream)
    if status:
        log(f"device status {status}")
        return 1
    log("warm-up done; timing")

    qsd.qsd_profile_start()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = qsd.qsd_profile_stop()
    # the status bits accumulate over calls: this covers every timed transposition
    status = qsd.qsd_device_status(ws.data_ptr(), stream.cuda_stream)
    if status:
        log(f"device status {status} after the timed steps")
        return 1
    sec = t1 - t0
    ms_per_step = 1e3 * sec / args.steps
    value = N * len(sigmas) * args.steps / sec
    log(f"{ms_per_step:.3f} ms/step, {value / 1e9:.2f} G nnz/s")
    for k, (n_l, ms, b) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        log(f"  {k:10s} launches={n_l:6d} total={ms:9.3f} ms avg={ms / max(n_l, 1) * 1e3:8.1f} us"
            + (f"  {b / ms / 1e6:8.1f} GB/s" if b and ms else ""))

    # roofline of the dominant kernel: algorithmic bytes per launch / mean launch time
    n_l, ms, b = prof["digit"]
    avg_s = ms / n_l / 1e3
    bytes_per_launch = b / n_l
    achieved = bytes_per_launch / avg_s / 1e9
    traffic = measured_traffic() if name == "plain" else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_digit (global digit pass)", "launches": n_l,
                "avg_launch_us": round(avg_s * 1e6, 2),
                "algorithmic_bytes_per_launch": bytes_per_launch}
    whole_bytes = sum(v[2] for v in prof.values())
    out = {
        "metric": METRIC, "value": value, "unit": "nnz/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": ("plain: 3-mode COO 500000x20000x2000000, 1e8 distinct nonzeros, "
                                "Zipf(1.1) coordinates, int32 coordinates, fp64 values, input order "
                                "(0,1,2) -> all 5 other orders per step") if name == "plain" else
                               ("wide: 4-mode COO 1000000x100000x1000x50, 2e8 distinct nonzeros, "
                                "Zipf(1.3) on modes 0-1, uniform modes 2-3, int32 coordinates, fp32 "
                                "values, input order (0,1,2,3) -> all 23 other orders per step"),
                   "nnz": N, "orders": [list(s) for s in sigmas], "schedule": args.sched,
                   "bucketed_groups": "segment sorts" if args.keep_buckets else "flattened where cheaper"},
        "roofline": roofline,
        "modelled_bytes_per_step": whole_bytes / args.steps,
    }
    # CSF pack of the last order's output (reported beside the metric, not part of it)
    csf = None
    if outs and name == "plain":
        P = plans[-1]
        oc = outs[-1][0]
        P.pack_csf(oc)  # warm-up (allocates its outputs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            _, _, counts = P.pack_csf(oc)
        sec = (time.perf_counter() - t0) / reps
        csf = {"order": list(sigmas[-1]), "ms": sec * 1e3, "fiber_counts": counts,
               "note": "wall time of qsd_pack_csf incl. its output allocation and count read-back"}
        log(f"CSF pack of sigma={sigmas[-1]}: {sec * 1e3:.3f} ms, fibers {counts}")
    out["csf_pack"] = csf
    if args.copy_probe:
        ident = qsd.Plan(T.extents, T.in_order, T.in_order, N, ct, vt, args.sched)
        oc, ov = outs[0]
        for _ in range(args.copy_probe):
            ident.transpose(crd, val, oc, ov, stream=stream, ws=ws)
        torch.cuda.synchronize()
        out["copy_probe"] = {"launches_per_call": T.order + 1,
                             "bytes_per_crd_copy": 2 * N * T.crd[0].itemsize, "bytes_per_val_copy": 2 * N * T.val.itemsize}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample ...")
        out["cpu_baseline"] = cpu_baseline(T, sigmas)
    print(json.dumps(out), flush=True)
    return 0


def cpu_baseline_batched(T, budget_s=20.0):
    """The oracle on the first tensors of the batch (copied to the host), single-threaded."""
    from oracle.transpose import transpose as oracle_transpose
    done, k, sec = 0, 0, 0.0
    while k < len(T) and sec < budget_s / 2:
        crd = [c.cpu().numpy() for c in T[k].crd]
        val = T[k].val.cpu().numpy()
        t0 = time.perf_counter()
        oracle_transpose(crd, val, T[k].out_order)
        sec += time.perf_counter() - t0
        done += T[k].nnz
        k += 1
    return {"value": done / sec, "unit": "nnz/s", "cores": 1, "kind": "oracle",
            "sample": f"first {k} tensors of the batch ({done} nonzeros), {sec:.1f} s single-threaded "
                      f"numpy (lexsort + gather)", "host": host_cpu()}


def bench_batched(args):
    import torch
    from datagen.batched import BATCHED, make_batch
    from paper_2005_10427_amd import qsd

    cfg = dict(BATCHED)
    if args.count:
        cfg["count"] = args.count
    log(f"generating {cfg['count']} tensors on the GPU ...")
    t0 = time.time()
    T = make_batch(device="cuda", **cfg)
    torch.cuda.synchronize()
    N = sum(t.nnz for t in T)
    log(f"generated {N} nonzeros in {time.time() - t0:.1f} s")
    stream = torch.cuda.current_stream()

    B = qsd.Batch([t.as_dict() for t in T])
    best, best_ms = B.tune(reps=2)
    log(f"autotuned items/radix/small_cap = {best}: {best_ms:.3f} ms")
    B.capture()

    # the same transpositions one by one with the minimal-pass plan (shared workspace)
    plans = [qsd.Plan(t.extents, t.in_order, t.out_order, max(t.nnz, 1), "int32", "float64", "minimal")
             for t in T]
    ws = torch.empty(max(p.ws_bytes for p in plans), dtype=torch.uint8, device="cuda")
    out = (B.out_crd, B.out_val)

    def plain_step():
        for i, (p, t) in enumerate(zip(plans, T)):
            if t.nnz:
                p.transpose(t.crd, t.val, out[0][i], out[1][i], stream=stream, ws=ws)

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    plain_sec = plain_graph_sec = None
    if not args.no_sequence:
        plain_sec = timed(plain_step, max(1, args.steps // 4))
        log(f"plain sequence: {plain_sec * 1e3:.3f} ms/step, {N / plain_sec / 1e9:.2f} G nnz/s")
        # the stronger baseline: the same one-by-one sequence captured into one HIP graph, so
        # that host launch overhead is gone and only the per-tensor kernels remain
        cap = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=cap):
            for i, (p, t) in enumerate(zip(plans, T)):
                if t.nnz:
                    p.transpose(t.crd, t.val, out[0][i], out[1][i], stream=cap, ws=ws)
        plain_graph_sec = timed(graph.replay, max(1, args.steps // 4))
        log(f"plain sequence as one graph: {plain_graph_sec * 1e3:.3f} ms/step, "
            f"{N / plain_graph_sec / 1e9:.2f} G nnz/s")
        del graph
    eager_sec = timed(lambda: B.transpose(stream), args.steps)
    log(f"batched eager: {eager_sec * 1e3:.3f} ms/step")
    sec = timed(lambda: B.replay(stream), args.steps)
    value = N / sec
    log(f"batched graph: {sec * 1e3:.3f} ms/step, {value / 1e9:.2f} G nnz/s")
    if B.device_status():
        log("device status nonzero")
        return 1

    # roofline of the dominant kernel, from library-recorded events over eager batched steps
    qsd.qsd_profile_start()
    for _ in range(args.steps):
        B.transpose(stream)
    torch.cuda.synchronize()
    prof = qsd.qsd_profile_stop()
    if B.device_status():
        log("device status nonzero after the profiled steps")
        return 1
    for k, (n_l, ms, b) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        log(f"  {k:12s} launches={n_l:6d} total={ms:9.3f} ms avg={ms / max(n_l, 1) * 1e3:8.1f} us"
            + (f"  {b / ms / 1e6:8.1f} GB/s" if b and ms else ""))
    n_l, ms, b = prof["digit_batch"]
    avg_s = ms / n_l / 1e3
    achieved = b / n_l / avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_digit (batched digit pass)", "launches": n_l,
                "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": b / n_l}
    res = {
        "metric": METRIC, "value": value, "unit": "nnz/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "batched: 4096 tensors of order 3 or 4, nnz log-uniform in [1e3, 1e6], "
                               "extents log-uniform in [10, 1e6], Zipf s uniform in [0, 1.5], int32 "
                               "coordinates, fp64 values, random input and output orders; one graph "
                               "replay per step",
                   "tensors": len(T), "nnz": N, "tuning": {"items": best[0], "radix_bits": best[1],
                                                           "small_cap": best[2]}},
        "plain_sequence": None if plain_sec is None else
        {"value": N / plain_sec, "ms_per_step": plain_sec * 1e3, "schedule": "minimal",
         "launch": "one qsd_transpose per tensor"},
        "plain_sequence_graph": None if plain_graph_sec is None else
        {"value": N / plain_graph_sec, "ms_per_step": plain_graph_sec * 1e3, "schedule": "minimal",
         "launch": "one qsd_transpose per tensor, the whole sequence captured into one HIP graph"},
        "batched_eager_ms_per_step": eager_sec * 1e3,
        "speedup_vs_plain_sequence": None if plain_sec is None else plain_sec / sec,
        "speedup_vs_plain_sequence_graph": None if plain_graph_sec is None else plain_graph_sec / sec,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample ...")
        res["cpu_baseline"] = cpu_baseline_batched(T)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
