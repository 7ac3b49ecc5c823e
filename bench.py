"""Benchmark: log-det estimates per second on one MI355X.

A step is one pass of the whole hot path over one problem instance:
materialize M = K + noise I from the points (the stored-matrix workload
keeps M in HBM), build the randomized truncated-SVD preconditioner, and run
the estimator for each requested order r_k (Section 2, Algorithm 1 with the
solves run to tolerance), each with its own probe stream.  The default
workload is Matern-5/2 on 50,000 points from an 8-component Gaussian mixture
in [0,1]^3, l = 0.15, noise 1e-3, FP32 with M stored (10 GB), rank 500, 64
Rademacher probes, r_1, r_3 and r_5.

Prints one JSON line (see the design doc for every field).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402

METRIC = "log-det estimates/s at ≤1e-3 rel err vs FP64; mixed/batched vs plain FP32"
PEAKS = {"fp32": 157.3e12, "fp64": 78.6e12, "hbm": 8.0e12}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_exact(name):
    p = os.path.join(ROOT, "tests", "golden", "exact_logdet.json")
    if not os.path.exists(p):
        return None
    return json.load(open(p)).get(name, {}).get("logdet")


def cpu_baseline(cfg, sample_n: int, orders, precision_f32: bool):
    """The oracle on a bounded sample: the same workload recipe at sample_n
    points, timed on this host; the rate is scaled to the full n by the
    oracle's O(n^3) dense-factorization cost."""
    from oracle import estimate as oest
    from oracle import gp, precond
    sub = cfg.with_n(sample_n)
    t0 = time.perf_counter()
    X = sub.X()
    M = gp.dense_matrix(sub.kind, X, sub.lengthscale, sub.variance, sub.noise)
    P = precond.rsvd(M, sub.rank, sub.oversample, sub.power_iters, sub.precond_seed,
                     precond.d_floor(sub.noise, sub.variance))
    Pd = P.dense()
    for k in orders:
        Z = oest.probes(sub.probe_seed + k, sub.n, sub.probes)
        oest.estimate_dense(M, Pd, P.logdet, k, Z)
    dt = time.perf_counter() - t0
    scale = (cfg.n / sample_n) ** 3
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": len(orders) / (dt * scale),
        "unit": "log-det estimates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle (FP64 numpy/scipy, dense Cholesky shifted solves) on the same recipe at "
                   f"n={sample_n}: {len(orders)} estimates in {dt:.2f} s; scaled to n={cfg.n} by "
                   f"(n/{sample_n})^3"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2_matern_gm50k", choices=["c2_matern_gm50k", "c1_rbf_2k"])
    ap.add_argument("--n", type=int, default=0, help="override n (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=8000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2405_03474_amd as L

    cfg = {"c2_matern_gm50k": workloads.C2, "c1_rbf_2k": workloads.C1}[args.workload]
    if args.n:
        cfg = cfg.with_n(args.n, rank=min(cfg.rank, args.n // 10))
    f32 = cfg.name.startswith("c2")
    prec = L.LD_F32 if f32 else L.LD_F64
    tol = 1e-6 if f32 else 1e-12
    stored = f32
    log(f"[bench] workload {cfg.name} n={cfg.n} rank={cfg.rank} probes={cfg.probes} "
        f"orders={cfg.orders} precision={'f32' if f32 else 'f64'} stored={stored}")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream(0)
    ctx = L.Context(0, stream)
    X = torch.as_tensor(cfg.X(), dtype=torch.float64, device=dev).contiguous()
    op = L.GPOperator(X=X, kind=cfg.kind, lengthscale=cfg.lengthscale, variance=cfg.variance,
                      noise=cfg.noise, precision=prec,
                      layout=L.LD_TILED if stored else L.LD_ROW_MAJOR)
    Mbuf = torch.empty((L.stored_elements(cfg.n, op.layout),),
                       dtype=torch.float32 if f32 else torch.float64, device=dev) if stored else None

    def step():
        out = {}
        if stored:
            op.M = None
            L.kernel_materialize(ctx, op, out=Mbuf)
            op.M = Mbuf
        P = L.Precond(ctx, op, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed)
        for k in cfg.orders:
            res, _ = L.logdet_estimate(ctx, op, P, k, cfg.probes, cfg.probe_seed + k, tol, 5000)
            out[k] = res
        P.close()
        return out

    for w in range(args.warmup):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w} {time.perf_counter() - t0:.3f} s")

    ctx.set_timing(True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(step())
        log(f"[bench] step {i} done {time.perf_counter() - t0:.3f} s")
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(stop)
    mm_ms, mm_calls, mm_flops, mm_bytes = ctx.read_timing()
    ctx.set_timing(False)

    n_est = args.steps * len(cfg.orders)
    value = n_est / (ms_total / 1e3)
    iters = {f"r{k}": results[-1][k]["iterations"] for k in cfg.orders}
    probe_solves = sum(results[-1][k]["num_probes"] for k in cfg.orders) * args.steps / (ms_total / 1e3)

    exact = load_exact(cfg.name) if not args.n else None
    accuracy = {}
    for k in cfg.orders:
        r = results[-1][k]
        acc = {"logdet": r["logdet"], "logdet_P": r["logdet_P"], "stderr": r["std_err"],
               "iterations": r["iterations"], "rel_resid": r["rel_resid"]}
        if exact is not None:
            acc["exact_logdet"] = exact
            acc["rel_err_vs_exact"] = abs(r["logdet"] - exact) / abs(exact)
            acc["within_1e-3"] = acc["rel_err_vs_exact"] <= 1e-3
        accuracy[f"r{k}"] = acc

    avg_ms = mm_ms / max(mm_calls, 1)
    achieved = (mm_flops / max(mm_calls, 1)) / (avg_ms / 1e3)
    peak = PEAKS["fp32"] if f32 else PEAKS["fp64"]
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None,
                "kernel": "k_mm32_st<2,tiled> (FP32 MFMA 32x32x2)" if f32 else "k_mm64<on the fly> (FP64 MFMA)",
                "avg_launch_ms": avg_ms, "launches": mm_calls,
                "hbm_GBps_algorithmic": (mm_bytes / max(mm_calls, 1)) / (avg_ms / 1e3) / 1e9}

    line = {
        "metric": METRIC, "value": value, "unit": "log-det estimates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_total / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if f32 else "f64", "data": "synthetic",
        "config": {"workload": cfg.name, "n": cfg.n, "d": cfg.d,
                   "kernel": "matern52" if cfg.kind == 1 else "rbf",
                   "points": cfg.points, "lengthscale": cfg.lengthscale, "variance": cfg.variance,
                   "noise": cfg.noise,
                   "storage": "stored_fp32_tiled" if stored else "on_the_fly",
                   "orders": list(cfg.orders), "probes": cfg.probes, "rank": cfg.rank,
                   "oversample": cfg.oversample, "power_iters": cfg.power_iters, "tol": tol},
        "probe_solves_per_s": probe_solves, "iterations": iters, "wall_s": wall,
        "accuracy": accuracy, "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(cfg, min(args.cpu_sample_n, cfg.n), cfg.orders, f32)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
