"""Benchmark: log-det estimates per second on one MI355X.

A step is one pass of the whole hot path over one problem instance: (for
the stored workload) materialize M = K + noise I from the points, build the
randomized truncated-SVD preconditioner, and run the estimator for each
requested order r_k (Section 2, Algorithm 1 with its shifted solves run to a
tolerance), each order with its own probe stream.

Workloads (all synthetic, inputs from workloads/):
  c2_matern_gm50k  (default) Matern-5/2, 50,000 points from an 8-component
                   Gaussian mixture in [0,1]^3, l = 0.15, noise 1e-3; FP64
                   (the paper's arithmetic) with M stored in HBM (tiled
                   layout, 20 GB), solves to 1e-10; rank 500; 64 Rademacher
                   probes; r_1, r_3, r_5.  After the timed FP64 steps the
                   plain FP32 path (10 GB M, solves to 1e-6) and the
                   split-BF16 precision form are timed on the same problem
                   and probes (`forms`, `speedup_vs_plain_fp32`, each with
                   its difference from the FP64 estimates); --precision
                   f32|bf16 makes either the timed path.
  c1_rbf_2k        RBF, 2,000 uniform points, FP64 on the fly, rank 100, 32
                   probes, r_3.
  c3_matern_200k   precision form: Matern-5/2, 200,000 uniform points,
                   l = 0.05, noise 1e-3, split-BF16 matrix-core products on
                   the fly, rank 1,000, 64 probes, r_3.  --compare-fp32 times
                   the plain FP32 on-the-fly path on the same problem;
                   --check-fp64 runs the FP64 path on the same probes.
  c4_batch256      batched form: 256 independent GP problems, n log-uniform
                   in [500, 20000], d in {2,3,8}, RBF or Matern-5/2, random
                   hyperparameters, rank min(200, n/10), 16 probes, r_3, FP32
                   on the fly, all instances in one pass (solver iterations
                   replayed from a HIP graph).  A step estimates all 256.
                   --compare-plain times the same 256 problems as sequential
                   single-instance plain FP32 calls.
  c5_surrogate     learned surrogate: training targets from the batched r_5
                   estimator (64 probes) on problems with the c4
                   hyperparameter distribution at --c5-train-n, ensemble
                   training, then a 32 x 32 (lengthscale, noise) Matern-5/2
                   sweep at --c5-eval-n: preconditioners + BF16 ensemble
                   prediction + fallback to the estimator where the members
                   disagree, timed against the plain estimator on every grid
                   point (which is also the error reference).  A step is one
                   sweep over the grid.  --c5-train-family grid trains on the
                   grid's own family; --c5-calibrate scales the spread by a
                   factor from held-out training problems.

Other modes on the single-problem workloads:
  --union-shifts       all orders from one solve over the union of their
                       poles (one shared probe block), reported separately
  --lanczos-steps T    Algorithm 1 as printed with T Lanczos steps
  --precond, --scaled  the Appendix's preconditioners
  --probes             Gaussian or normal orthogonal probes
  --gradient           d log det / d(lengthscale, variance, noise)
  --graphs             solver iterations replayed from captured HIP graphs
  --plain-fp32         c3 on the plain FP32 path (fused FP32 product)
  --kernel-kind        another covariance kernel on the same points
  --sensitivity axes|dims  the Appendix's sweeps against exact log det
                       (n = 20,000; prints its own JSON record)

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from dataclasses import replace

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "log-det estimates/s at ≤1e-3 rel err vs FP64; mixed/batched vs plain FP32"
PEAK = {"fp32": 157.3e12, "fp64": 78.6e12, "bf16": 2.5e15}
DTYPE_NAME = {0: "f64", 1: "f32", 2: "bf16x3+f32"}  # by ld_precision (on the fly)


def dtype_name(precision, stored):
    """BF16 products take three terms on the fly and four from stored FP32 tiles."""
    return "bf16x4+f32" if (precision == 2 and stored) else DTYPE_NAME[precision]
WORKLOADS = {"c2_matern_gm50k": workloads.C2, "c1_rbf_2k": workloads.C1,
             "c3_matern_200k": workloads.C3, "c4_batch256": None, "c5_surrogate": None}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Measured HBM traffic per launch of the dominant kernel, from the committed
# rocprofv3 counter summaries; valid only while the kernel's source file is
# byte-identical to the one profiled.
PROFILED_TRAFFIC = {
    "c2_matern_gm50k/f64": ("profiles/c2_matern_gm50k_k_mm64_tf.md",
                            "paper_2405_03474_amd/csrc/matmat.hip"),
    "c2_matern_gm50k/f32": ("profiles/c2_matern_gm50k_k_mm32_tf.md",
                            "paper_2405_03474_amd/csrc/matmat.hip"),
    "c2_matern_gm50k/bf16x4+f32": ("profiles/c2_matern_gm50k_k_mm16_tf.md",
                                   "paper_2405_03474_amd/csrc/matmat.hip"),
}


def profiled_traffic(workload):
    import hashlib
    entry = PROFILED_TRAFFIC.get(workload)
    if not entry:
        return None
    summary, source = (os.path.join(ROOT, x) for x in entry)
    if not (os.path.exists(summary) and os.path.exists(source)):
        return None
    fields = {}
    for line in open(summary):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_source_sha256"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    digest = hashlib.sha256(open(source, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != digest or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def load_exact(name):
    p = os.path.join(ROOT, "tests", "golden", "exact_logdet.json")
    if not os.path.exists(p):
        return None
    return json.load(open(p)).get(name, {}).get("logdet")


def cpu_baseline(cfg, sample_n: int, lanczos_steps: int = 0, pkind: str = "rsvd",
                 scaled: bool = False, probes: str = "rademacher"):
    """The oracle on a bounded sample: the same workload recipe at sample_n
    points (same preconditioner rank), timed on this host phase by phase and
    each phase scaled to the full n by its own cost: the dense matrix and the
    randomized SVD (products of M with rank + oversample columns) as n^2, the
    estimates (a dense Cholesky factorization per shift, O(n^3)) as n^3.
    With lanczos_steps the oracle of Algorithm 1 as printed (t Lanczos steps
    per probe, O(n^2) per step with a factored P) is timed and scaled as n^2."""
    from oracle import estimate as oest
    from oracle import gp, lanczos as olz
    sub = cfg.with_n(sample_n, rank=min(cfg.rank, sample_n // 10))
    t0 = time.perf_counter()
    X = sub.X()
    M = gp.dense_matrix(sub.kind, X, sub.lengthscale, sub.variance, sub.noise)
    t1 = time.perf_counter()
    P = oracle_precond(sub, M, pkind, scaled)
    Pd = P.dense()
    t2 = time.perf_counter()
    for k in cfg.orders:
        Z = oest.probe_block(probes, sub.probe_seed + k, sub.n, sub.probes)
        if lanczos_steps:
            olz.estimate_lanczos(M, Pd, P.logdet, k, Z, lanczos_steps)
        else:
            oest.estimate_dense(M, Pd, P.logdet, k, Z)
    t3 = time.perf_counter()
    r = cfg.n / sample_n
    est_scale = r ** 2 if lanczos_steps else r ** 3
    full = (t1 - t0) * r ** 2 + (t2 - t1) * r ** 2 + (t3 - t2) * est_scale
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": len(cfg.orders) / full,
        "unit": "log-det estimates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle (FP64 numpy/scipy, "
                   + (f"{lanczos_steps} Lanczos steps per probe with dense P^-1 solves"
                      if lanczos_steps else "dense Cholesky shifted solves")
                   + ") on the same recipe at "
                   f"n={sample_n}, rank {sub.rank}: matrix {t1 - t0:.2f} s, preconditioner "
                   f"{t2 - t1:.2f} s, {len(cfg.orders)} estimates {t3 - t2:.2f} s; scaled to "
                   f"n={cfg.n} by (n/{sample_n})^2 for the matrix and preconditioner and "
                   f"(n/{sample_n})^{2 if lanczos_steps else 3} for the estimates: "
                   f"{full:.0f} s per step"),
    }


PRECOND_KINDS = {"rsvd": 0, "identity": 1, "diagonal": 2, "rank_one": 3, "pchol": 4}


def oracle_precond(cfg, M, pkind: str, scaled: bool):
    """The oracle's preconditioner of the given kind (Appendix list)."""
    from oracle import precond
    floor = precond.d_floor(cfg.noise, cfg.variance)
    if pkind == "identity":
        P = precond.identity(M.shape[0])
    elif pkind == "diagonal":
        P = precond.diagonal(M)
    elif pkind == "rank_one":
        P = precond.rank_one(M, cfg.oversample, cfg.power_iters, cfg.precond_seed, floor)
    elif pkind == "pchol":
        P = precond.partial_cholesky(M, cfg.rank, floor)
    else:
        P = precond.rsvd(M, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed, floor)
    return precond.scaled(P, cfg.noise) if scaled else P


class Runner:
    """One problem instance on the GPU in a given arithmetic."""

    def __init__(self, L, torch, ctx, cfg, precision, stored, lanczos_steps=0, pkind="rsvd",
                 scaled=False, union=False, tol=0.0):
        self.L, self.torch, self.ctx, self.cfg = L, torch, ctx, cfg
        self.lanczos_steps = lanczos_steps
        self.union = union
        self.pkind = PRECOND_KINDS[pkind]
        self.scaled = scaled
        dev = torch.device("cuda:0")
        X = torch.as_tensor(cfg.X(), dtype=torch.float64, device=dev).contiguous()
        self.stored = stored
        self.op = L.GPOperator(X=X, kind=cfg.kind, lengthscale=cfg.lengthscale,
                               variance=cfg.variance, noise=cfg.noise, precision=precision,
                               layout=L.LD_TILED if stored else L.LD_ROW_MAJOR)
        self.Mbuf = None
        if stored:
            self.Mbuf = torch.empty((L.stored_elements(cfg.n, self.op.layout),),
                                    dtype=torch.float32 if precision != L.LD_F64 else torch.float64,
                                    device=dev)
        self.tol = tol or (1e-12 if precision == L.LD_F64 else 1e-6)

    def release(self):
        self.op.M = None
        self.Mbuf = None

    def step(self):
        L, cfg, op = self.L, self.cfg, self.op
        out = {}
        if self.stored:
            op.M = None
            L.kernel_materialize(self.ctx, op, out=self.Mbuf)
            op.M = self.Mbuf
        P = L.Precond(self.ctx, op, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed,
                      kind=self.pkind, scaled=self.scaled)
        if self.union:
            # every order from one solve (CG over the union of the poles, or
            # one Lanczos recurrence), one shared probe block
            if self.lanczos_steps:
                res, _ = L.logdet_estimate_lanczos_orders(self.ctx, op, P, list(cfg.orders),
                                                          cfg.probes, cfg.probe_seed,
                                                          self.lanczos_steps)
            else:
                res, _ = L.logdet_estimate_orders(self.ctx, op, P, list(cfg.orders), cfg.probes,
                                                  cfg.probe_seed, self.tol, 5000)
            P.close()
            return dict(zip(cfg.orders, res))
        for k in cfg.orders:
            if self.lanczos_steps:
                res, per = L.logdet_estimate_lanczos(self.ctx, op, P, k, cfg.probes,
                                                     cfg.probe_seed + k, self.lanczos_steps)
            else:
                res, per = L.logdet_estimate(self.ctx, op, P, k, cfg.probes, cfg.probe_seed + k,
                                             self.tol, 5000)
            out[k] = res
        P.close()
        return out


class GradRunner(Runner):
    """d log det M / d(lengthscale, variance, noise) on one problem."""

    def step(self):
        L, cfg, op = self.L, self.cfg, self.op
        if self.stored:
            op.M = None
            L.kernel_materialize(self.ctx, op, out=self.Mbuf)
            op.M = self.Mbuf
        P = L.Precond(self.ctx, op, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed,
                      kind=self.pkind, scaled=self.scaled)
        grad, se, _, res = L.logdet_gradient(self.ctx, op, P, cfg.probes, cfg.probe_seed,
                                             self.tol, 5000)
        P.close()
        return {"grad": grad.tolist(), "std_err": se.tolist(), "iterations": res["iterations"]}


def gradient_main(args, torch, L, cfg, precision, stored):
    stream = torch.cuda.current_stream(0)
    ctx = L.Context(0, stream)
    runner = GradRunner(L, torch, ctx, cfg, precision, stored, 0, args.precond, args.scaled)
    results, ms_total, wall, _ = timed_steps(runner, args.steps, args.warmup, stream, torch)
    last = results[-1]
    line = {
        "metric": "log-det gradients/s (lengthscale, variance, noise)",
        "value": args.steps / (ms_total / 1e3), "unit": "gradients/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_total / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE_NAME[precision],
        "data": "synthetic",
        "config": {"workload": cfg.name, "n": cfg.n, "probes": cfg.probes, "rank": cfg.rank,
                   "precond": {"kind": args.precond, "scaled": args.scaled},
                   "solver": {"kind": "pcg", "tol": runner.tol}},
        "gradient": last, "wall_s": wall,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


class BatchRunner:
    """The heterogeneous batch through logdet_estimate_batched."""

    K, S, OVER, POWER = 3, 16, 10, 2

    def __init__(self, L, torch, ctx, insts, graph=True, symmetric=False):
        self.L, self.ctx, self.insts, self.graph = L, ctx, insts, graph
        self.symmetric = symmetric
        dev = torch.device("cuda:0")
        self.items = [L.BatchItem(X=torch.as_tensor(g.X(), dtype=torch.float64, device=dev),
                                  kind=g.kind, lengthscale=g.lengthscale, variance=g.variance,
                                  noise=g.noise, rank=g.rank, precond_seed=g.precond_seed,
                                  probe_seed=g.probe_seed) for g in insts]
        self.tol = 1e-6

    def step(self):
        res, per, status = self.L.logdet_estimate_batched(
            self.ctx, self.items, self.K, self.S, self.OVER, self.POWER, tol=self.tol,
            max_iters=5000, graph=self.graph, symmetric=self.symmetric)
        return {self.K: res}


class PlainSequential:
    """The same problems as one plain FP32 on-the-fly call each (own
    preconditioner build, same seeds), one after another."""

    def __init__(self, L, torch, ctx, batch):
        self.L, self.ctx, self.b = L, ctx, batch

    def step(self):
        L, b = self.L, self.b
        out = []
        for g, it in zip(b.insts, b.items):
            op = L.GPOperator(X=it.X, kind=g.kind, lengthscale=g.lengthscale,
                              variance=g.variance, noise=g.noise, precision=L.LD_F32)
            P = L.Precond(self.ctx, op, g.rank, b.OVER, b.POWER, g.precond_seed)
            res, _ = L.logdet_estimate(self.ctx, op, P, b.K, b.S, g.probe_seed, b.tol, 5000)
            P.close()
            out.append(res)
        return {b.K: out}


def copy_calibration(torch, mib):
    """One plain device-to-device copy of `mib` MiB, so that a counter run can
    scale FETCH_SIZE / WRITE_SIZE by what they read for known traffic."""
    if mib <= 0:
        return
    src = torch.ones(mib * 262144, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: {mib} MiB read + {mib} MiB written")
    del src, dst


def r11_error(got, exact, n):
    """Relative error where |log det| >= 0.01 n, else |error| / n."""
    e = abs(got - exact)
    return e / abs(exact) if abs(exact) >= 0.01 * n else e / n


def batch_main(args, torch, L):
    insts = workloads.batch_instances()
    log(f"[bench] workload c4_batch256: {len(insts)} instances, sum n = {sum(g.n for g in insts)}")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream(0)
    ctx = L.Context(0, stream)
    runner = BatchRunner(L, torch, ctx, insts, graph=not args.no_graph,
                         symmetric=args.batch_form == "symmetric")
    results, ms_total, wall, (mm_ms, mm_calls, mm_flops, mm_bytes) = timed_steps(
        runner, args.steps, args.warmup, stream, torch)
    count = len(insts)
    value = args.steps * count / (ms_total / 1e3)
    eager_value = None
    if runner.graph:
        # kernel events cannot sit inside the replayed graph: the product
        # kernel is timed over a second timed region of eager steps
        log("[bench] eager steps (kernel timing)")
        eager = BatchRunner(L, torch, ctx, insts, graph=False,
                            symmetric=args.batch_form == "symmetric")
        eager.items = runner.items
        _, ems, _, (mm_ms, mm_calls, mm_flops, mm_bytes) = timed_steps(eager, args.steps, 0,
                                                                      stream, torch)
        eager_value = args.steps * count / (ems / 1e3)
    last = results[-1][BatchRunner.K]
    exact_all = json.load(open(os.path.join(ROOT, "tests", "golden", "exact_logdet.json"))).get(
        "c4_batch256", {}).get("logdet") if os.path.exists(
        os.path.join(ROOT, "tests", "golden", "exact_logdet.json")) else None
    if args.dump:
        json.dump([{"n": g.n, **r} for g, r in zip(insts, last)], open(args.dump, "w"))
    accuracy = {"iterations": last[0]["iterations"],
                "converged": sum(r["converged_cols"] == BatchRunner.S for r in last)}
    if exact_all:
        errs = [r11_error(r["logdet"], e, g.n) for r, e, g in zip(last, exact_all, insts)]
        accuracy.update({"max_err_vs_exact": max(errs), "median_err_vs_exact": float(
            sorted(errs)[len(errs) // 2]), "within_1e-3": sum(e <= 1e-3 for e in errs),
            "error_rule": "relative where |log det| >= 0.01 n, else abs/n"})
        worst = sorted(range(count), key=lambda i: -errs[i])[:6]
        accuracy["worst"] = [{"i": i, "n": insts[i].n, "d": insts[i].d, "kind": insts[i].kind,
                              "lengthscale": insts[i].lengthscale, "noise": insts[i].noise,
                              "err": errs[i], "logdet": last[i]["logdet"], "exact": exact_all[i],
                              "logdet_P": last[i]["logdet_P"], "std_err": last[i]["std_err"]}
                             for i in worst]
    avg_ms = mm_ms / max(mm_calls, 1)
    achieved = (mm_flops / max(mm_calls, 1)) / (avg_ms / 1e3) if mm_calls else 0.0
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK["fp32"] / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK["fp32"], "traffic": None,
                "kernel": ("k_bmm_sym + k_bsym_reduce (FP32 MFMA, blocks on and above the "
                           "diagonal generated once, feeding both rows)"
                           if args.batch_form == "symmetric" else
                           "k_bmm (FP32 MFMA 32x32x2, kernel entries generated on the fly, "
                           "one workgroup per instance row block)"),
                "avg_launch_ms": avg_ms, "launches": mm_calls,
                "algorithmic_GBps": (mm_bytes / max(mm_calls, 1)) / (avg_ms / 1e3) / 1e9
                if mm_calls else 0.0,
                "timed_over": "eager steps" if runner.graph else "the timed steps"}
    line = {
        "metric": METRIC, "value": value, "unit": "log-det estimates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_total / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c4_batch256", "instances": count,
                   "sum_n": sum(g.n for g in insts), "max_n": max(g.n for g in insts),
                   "orders": [BatchRunner.K], "probes": BatchRunner.S,
                   "rank": "min(200, n/10)", "oversample": BatchRunner.OVER,
                   "power_iters": BatchRunner.POWER, "tol": runner.tol,
                   "graph": not args.no_graph, "batch_form": args.batch_form},
        "probe_solves_per_s": BatchRunner.S * value,
        "eager_value": eager_value,
        "wall_s": wall, "accuracy": accuracy, "roofline": roofline,
    }
    if args.compare_plain:
        log("[bench] plain FP32 single-instance calls, same 256 problems")
        plain = PlainSequential(L, torch, ctx, runner)
        pres, pms, _, _ = timed_steps(plain, 1, 0, stream, torch)
        pv = count / (pms / 1e3)
        pl = pres[-1][BatchRunner.K]
        line["plain_fp32_sequential"] = {
            "value": pv, "ms_per_step": pms,
            "max_rel_diff_vs_batched": max(abs(a["logdet"] - b["logdet"]) / max(abs(b["logdet"]), 1e-300)
                                           for a, b in zip(last, pl))}
        line["speedup_vs_plain_fp32"] = value / pv
    if args.no_cpu_baseline:
        line["cpu_baseline"] = None
    else:
        log("[bench] cpu baseline (oracle) ...")
        line["cpu_baseline"] = batch_cpu_baseline(insts, args.cpu_sample_count)
    print(json.dumps(line), flush=True)
    ctx.close()


def batch_cpu_baseline(insts, sample_count):
    """The oracle on a bounded sample of the batch: the first sample_count
    instances in order, timed on this host, scaled to the whole batch by
    sum n^3 (the oracle's dense factorizations)."""
    from oracle import estimate as oest
    from oracle import gp, precond
    order = sorted(range(len(insts)), key=lambda i: insts[i].n)
    pick = [insts[i] for i in order[::max(1, len(order) // sample_count)]][:sample_count]
    pick = [g for g in pick if g.n <= 6000]
    t0 = time.perf_counter()
    for g in pick:
        M = gp.dense_matrix(g.kind, g.X(), g.lengthscale, g.variance, g.noise)
        P = precond.rsvd(M, g.rank, BatchRunner.OVER, BatchRunner.POWER, g.precond_seed,
                         precond.d_floor(g.noise, g.variance))
        Z = oest.probes(g.probe_seed, g.n, BatchRunner.S)
        oest.estimate_dense(M, P.dense(), P.logdet, BatchRunner.K, Z)
    dt = time.perf_counter() - t0
    scale = sum(g.n ** 3 for g in insts) / sum(g.n ** 3 for g in pick)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": len(insts) / (dt * scale), "unit": "log-det estimates/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"oracle (FP64 numpy/scipy, dense Cholesky shifted solves) on {len(pick)} "
                       f"instances of the batch spread over its n range (n = "
                       f"{min(g.n for g in pick)}..{max(g.n for g in pick)}): {dt:.2f} s; "
                       f"scaled to all {len(insts)} instances by sum n^3")}


def surrogate_main(args, torch, L):
    from paper_2405_03474_amd import sweep
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream(0)
    ctx = L.Context(0, stream)
    cfg = sweep.Config()
    if args.c5_chunk:
        cfg.chunk = args.c5_chunk
    rank = args.c5_rank or None

    def training_set(start, count):
        if args.c5_train_family == "grid":
            assert start == 0, "--c5-train-start needs the batched family"
            return workloads.surrogate_family_instances(count, args.c5_train_n)
        return workloads.surrogate_training_instances(count, args.c5_train_n, rank=rank,
                                                      start=start)

    grid = workloads.surrogate_grid(args.c5_eval_n, side=args.c5_side, rank=rank)
    t0 = time.perf_counter()
    if args.c5_data_in:
        # training targets generated earlier by --c5-data-out runs (the same
        # estimator on the same seeded problems)
        train_used, lams, y, t_gen = [], [], [], 0.0
        for path in args.c5_data_in.split(","):
            z = np.load(path)
            part = training_set(int(z["start"]), len(z["y"]))
            keep = z["converged"].astype(bool)
            train_used += [g for g, k in zip(part, keep) if k]
            lams += [row[:g.rank].astype(np.float64) for row, g, k in zip(z["lam"], part, keep) if k]
            y += [v for v, k in zip(z["y"], keep) if k]
            t_gen += float(z["seconds"])
        y = np.array(y)
        train_count = len(y)
        log(f"[bench] c5: {train_count} converged training problems loaded")
    else:
        train_insts = training_set(args.c5_train_start, args.c5_train_count)
        train_count = len(train_insts)
        log(f"[bench] c5: {len(train_insts)} training problems at n={args.c5_train_n}, "
            f"{len(grid)} grid points at n={args.c5_eval_n}")
        def save(res, lams, seconds):
            # the problems done so far (rewritten after every chunk, so that
            # an interrupted run keeps what it finished)
            done = train_insts[:len(res)]
            lam_rows = np.zeros((len(res), max(g.rank for g in done)), dtype=np.float32)
            for i, l in enumerate(lams):
                lam_rows[i, :len(l)] = l
            conv = np.array([r["converged_cols"] == cfg.probes for r in res])
            y_done = np.array([(r["logdet"] - r["logdet_P"]) / g.n for r, g in zip(res, done)])
            np.savez(args.c5_data_out, start=args.c5_train_start, y=y_done, lam=lam_rows,
                     converged=conv, seconds=seconds)
            return conv

        if args.c5_data_out:
            res, lams = [], []
            for c0 in range(0, len(train_insts), cfg.chunk):
                r, lm, _ = sweep.estimate_all(ctx, train_insts[c0:c0 + cfg.chunk], cfg, torch)
                res += r
                lams += lm
                conv = save(res, lams, time.perf_counter() - t0)
                log(f"[bench] c5 training data: {len(res)}/{len(train_insts)} problems "
                    f"{time.perf_counter() - t0:.1f} s")
            t_gen = time.perf_counter() - t0
            conv = save(res, lams, t_gen)
            print(json.dumps({"c5_training_data": args.c5_data_out, "start": args.c5_train_start,
                              "count": len(res), "converged": int(conv.sum()),
                              "train_n": args.c5_train_n, "seconds": t_gen}), flush=True)
            ctx.close()
            return
        res, lams, _ = sweep.estimate_all(ctx, train_insts, cfg, torch, log=log)
        t_gen = time.perf_counter() - t0
        ok = [i for i, r in enumerate(res) if r["converged_cols"] == cfg.probes]
        yall = np.array([(r["logdet"] - r["logdet_P"]) / g.n for r, g in zip(res, train_insts)])
        train_used = [train_insts[i] for i in ok]
        lams = [lams[i] for i in ok]
        y = yall[ok]
    edges = sweep.feature_edges(lams, train_used)
    F = sweep.features(lams, train_used, edges)
    log(f"[bench] training data {t_gen:.2f} s")
    t0 = time.perf_counter()
    if args.c5_calibrate:
        # hold out a tenth of the problems to calibrate the spread multiplier
        tr, ho = sweep.split_holdout(len(y), 0.1)
        S, hist = sweep.train(ctx, F[tr], y[tr], torch, epochs=args.c5_epochs)
        cfg.kappa = sweep.calibrate(S, F[ho], y[ho], torch)
        log(f"[bench] spread multiplier from {len(ho)} held-out problems: {cfg.kappa:.2f}")
    else:
        S, hist = sweep.train(ctx, F, y, torch, epochs=args.c5_epochs)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"[bench] training {t_train:.2f} s, loss {hist[0]:.3e} -> {hist[-1]:.3e}")

    if args.c5_split_timing:
        # one surrogate sweep, then the plain estimator on the points that did
        # not fall back: the fallback estimates are the plain estimator's own
        # values on those points, so every point is estimated once and the
        # plain sweep's time is the fallback time plus the rest (two batched
        # calls instead of one); kernel events over the whole give the roofline
        ctx.set_timing(True)
        torch.cuda.synchronize()
        logdet, fb, stages, items = sweep.sweep(ctx, S, grid, edges, cfg, torch,
                                                score_rest=True, log=log)
        torch.cuda.synchronize()
        mm_ms, mm_calls, mm_flops, mm_bytes = ctx.read_timing()
        ctx.set_timing(False)
        predicted, spread = stages.pop("predicted"), stages.pop("spread")
        plain = stages.pop("rest_plain")
        t_plain = stages["fallback"] + stages["rest_seconds"]
        times = [stages]
        log(f"[bench] surrogate sweep: {stages}")
    else:
        # plain estimator on every grid point (error reference and the
        # comparison); kernel events around its products give the roofline
        ctx.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain, _, items = sweep.estimate_all(ctx, grid, cfg, torch, log=log)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        mm_ms, mm_calls, mm_flops, mm_bytes = ctx.read_timing()
        ctx.set_timing(False)
        log(f"[bench] plain sweep {t_plain:.2f} s")
        for w in range(args.warmup):
            sweep.sweep(ctx, S, grid, edges, cfg, torch, items=items)
        times = []
        for i in range(args.steps):
            torch.cuda.synchronize()
            logdet, fb, stages, _ = sweep.sweep(ctx, S, grid, edges, cfg, torch, items=items)
            torch.cuda.synchronize()
            predicted, spread = stages.pop("predicted"), stages.pop("spread")
            times.append(stages)
            log(f"[bench] surrogate sweep {i}: {stages}")
    t_sur = float(np.mean([st["total"] for st in times]))
    ref = np.array([r["logdet"] for r in plain])
    # points where the plain FP32 estimator itself did not converge (a solver
    # breakdown: smooth kernels with tiny noise are not numerically positive
    # definite in FP32 products) cannot score a prediction
    valid = np.array([r["converged_cols"] == cfg.probes for r in plain])
    plain_unconverged = int((~valid).sum())
    if args.dump:
        Fg = sweep.features(sweep.estimate_all(ctx, grid, cfg, torch, precond_only=True,
                                               items=items)[1], grid, edges)
        np.savez(args.dump, F_train=F, y_train=y, F_grid=Fg, predicted=predicted, spread=spread,
                 ref=ref, logdet_P=np.array([r["logdet_P"] for r in plain]),
                 n_grid=np.array([g.n for g in grid]), edges=edges,
                 n_train=np.array([g.n for g in train_used]))
    rel = (np.abs(logdet - ref) / np.abs(ref))[valid]
    rel_pred = (np.abs(predicted - ref) / np.abs(ref))[valid]
    fbv = fb[valid]
    spread = spread[valid]
    ref_v = ref[valid]
    avg_ms = mm_ms / max(mm_calls, 1)
    achieved = (mm_flops / max(mm_calls, 1)) / (avg_ms / 1e3) if mm_calls else 0.0
    line = {
        "metric": METRIC, "value": len(grid) / t_sur, "unit": "log-det estimates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_sur * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {"workload": "c5_surrogate", "train_n": args.c5_train_n,
                   "train_count": train_count, "train_converged": len(y),
                   "train_family": args.c5_train_family,
                   "eval_n": args.c5_eval_n,
                   "grid": f"{args.c5_side}x{args.c5_side}", "order": cfg.k, "probes": cfg.probes,
                   "rank": args.c5_rank or "n/40", "members": 5, "epochs": args.c5_epochs,
                   "fallback_rel_tol": cfg.rel_tol, "spread_multiplier": cfg.kappa},
        "plain_estimator": {"value": len(grid) / t_plain, "seconds": t_plain,
                            "unconverged": plain_unconverged},
        "speedup_vs_plain": t_plain / t_sur,
        "stages_s": times[-1],
        "fallbacks": int(fb.sum()),
        "error_vs_plain": {"scored_points": int(valid.sum()),
                           "max_rel": float(rel.max()), "median_rel": float(np.median(rel)),
                           "within_1e-3": int((rel <= 1e-3).sum()),
                           "max_rel_predicted": float(rel[~fbv].max()) if (~fbv).any() else None},
        "ensemble_only_error_vs_plain": {
            "median_rel": float(np.median(rel_pred)), "p90_rel": float(np.quantile(rel_pred, 0.9)),
            "within_1e-3": int((rel_pred <= 1e-3).sum()), "within_1e-2": int((rel_pred <= 1e-2).sum()),
            "median_rel_spread": float(np.median(spread / np.abs(ref_v)))},
        "training": {"data_seconds": t_gen, "train_seconds": t_train, "loss_first": hist[0],
                     "loss_last": hist[-1]},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK["fp32"] / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK["fp32"], "traffic": None,
                     "kernel": "k_bmm (batched FP32 product of the plain estimator on the grid)",
                     "avg_launch_ms": avg_ms, "launches": mm_calls},
    }
    if args.no_cpu_baseline:
        line["cpu_baseline"] = None
    else:
        log("[bench] cpu baseline (oracle) ...")
        line["cpu_baseline"] = surrogate_cpu_baseline(grid, cfg, args.cpu_sample_count)
    print(json.dumps(line), flush=True)
    S.close()
    ctx.close()


def surrogate_cpu_baseline(grid, cfg, count, max_n=4000):
    """The oracle estimator on a few grid points, scaled to the whole grid;
    grid points larger than max_n are sampled at max_n (same recipe, rank
    scaled with n) and the time scaled by (n / max_n)^3."""
    from oracle import estimate as oest
    from oracle import gp, precond
    pick = grid[:: max(1, len(grid) // max(1, min(count, 3)))][:3]
    n_full = pick[0].n
    scale = 1.0
    if n_full > max_n:
        pick = [g.with_n(max_n, rank=max(1, g.rank * max_n // n_full)) for g in pick]
        scale = (n_full / max_n) ** 3
    t0 = time.perf_counter()
    for g in pick:
        M = gp.dense_matrix(g.kind, g.X(), g.lengthscale, g.variance, g.noise)
        P = precond.rsvd(M, g.rank, cfg.oversample, cfg.power_iters, g.precond_seed,
                         precond.d_floor(g.noise, g.variance))
        oest.estimate_dense(M, P.dense(), P.logdet, cfg.k, oest.probes(g.probe_seed, g.n, cfg.probes))
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": len(pick) / (dt * scale), "unit": "log-det estimates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"oracle (FP64, dense Cholesky shifted solves) on {len(pick)} grid points "
                      f"at n={pick[0].n} (rank {pick[0].rank}): {dt:.2f} s"
                      + (f", scaled to n={n_full} by (n/{max_n})^3" if scale != 1.0 else "")}


def exact_logdet_stored(ctx, op):
    """The sweeps' yardstick: log det M = 2 sum log diag(L), M = L L^T, from
    a Cholesky factorisation of the stored FP64 matrix (torch's linear
    algebra, outside the library: a measurement, not part of the method)."""
    import torch
    ctx.synchronize()
    Lf = torch.linalg.cholesky(op.M)
    v = float(2.0 * torch.log(torch.diagonal(Lf)).sum())
    del Lf
    return v


def sensitivity_main(args, torch, L):
    """The Appendix's sensitivity sweeps (one parameter at a time around the
    paper's choice, Matern-5/2 in d = 5) or the Section 3 sweep over d;
    errors against the exact log det of each stored FP64 matrix."""
    from paper_2405_03474_amd import sensitivity as S
    torch.cuda.set_device(0)
    ctx = L.Context(0)
    n, count = args.sens_n, args.sens_count
    base = S.Setting()
    t0 = time.perf_counter()
    if args.sensitivity == "axes":
        axes = dict(S.AXES, solver=["lanczos", "cg"])
        settings = S.axis_settings(base, axes, orders=(1, 3, 5))
        insts = workloads.sensitivity_instances(workloads.MATERN52, 5, count, n=n)
        cells, exacts = S.sweep(ctx, insts, settings, torch, exact_logdet_stored, log=log)
        rows = [{"axis": a, "value": v, "k": k, **cells[(a, v, k)].summary()}
                for (a, v, k) in settings]
    else:
        ds = [int(x) for x in args.sens_dims.split(",")]
        settings = {("lanczos", k): replace(base, k=k) for k in (1, 3, 5)}
        settings[("cg", 3)] = replace(base, k=3, solver="cg")
        rows, exacts = [], []
        for kind in (workloads.RBF, workloads.MATERN52):
            for d in ds:
                insts = workloads.sensitivity_instances(kind, d, count, n=n)
                cells, ex = S.sweep(ctx, insts, settings, torch, exact_logdet_stored, log=log)
                exacts += ex
                rows += [{"kernel": "rbf" if kind == workloads.RBF else "matern52", "d": d,
                          "solver": sv, "k": k, **cells[(sv, k)].summary()}
                         for (sv, k) in settings]
    wall = time.perf_counter() - t0
    line = {"metric": "sensitivity_" + args.sensitivity, "n": n, "instances_per_point": count,
            "noise": workloads.sensitivity_instances(1, 1, 1, n=2)[0].noise,
            "base": {"probes": base.probes, "steps": base.steps, "rank": base.rank,
                     "power_iters": base.power_iters, "oversample": base.oversample},
            "dtype": "f64", "data": "synthetic", "seconds": wall, "rows": rows,
            "mean_abs_exact_logdet": float(np.mean(np.abs(exacts)))}
    if args.dump:
        with open(args.dump, "w") as f:
            json.dump(line, f, indent=1)
    print(json.dumps(line))


def timed_steps(runner, steps, warmup, stream, torch, instrument=True):
    for w in range(warmup):
        t0 = time.perf_counter()
        runner.step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w} {time.perf_counter() - t0:.3f} s")
    if instrument:
        runner.ctx.set_timing(True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    t0 = time.perf_counter()
    results = []
    for i in range(steps):
        results.append(runner.step())
        log(f"[bench] step {i} done {time.perf_counter() - t0:.3f} s")
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    timing = runner.ctx.read_timing() if instrument else None
    runner.ctx.set_timing(False)
    return results, ms, time.perf_counter() - t0, timing


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2_matern_gm50k", choices=sorted(WORKLOADS))
    ap.add_argument("--n", type=int, default=0, help="override n (smaller test runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=8000)
    ap.add_argument("--graphs", action="store_true",
                    help="replay the solver's iterations from captured HIP graphs")
    ap.add_argument("--batch-form", default="symmetric", choices=["symmetric", "tiled"],
                    help="batched product: the symmetric form, or the tile shape the autotuner "
                         "times fastest")
    ap.add_argument("--symmetric", default="", choices=["", "none", "f32", "bf16", "both"],
                    help="on-the-fly forms that generate each off-diagonal block once "
                         "(default: the library's, FP32 only)")
    ap.add_argument("--kernel-kind", default="", choices=["", "rbf", "matern52"],
                    help="override the workload's covariance kernel (same points and sizes)")
    ap.add_argument("--plain-fp32", action="store_true",
                    help="c3: time the plain FP32 on-the-fly path as the main path (its "
                         "product kernel's FP32 matrix-core fraction)")
    ap.add_argument("--precision", default="", choices=["", "f64", "f32", "bf16"],
                    help="arithmetic of the products and vectors (default: c1 and c2 f64, "
                         "c3 bf16)")
    ap.add_argument("--tol", type=float, default=0.0,
                    help="solver tolerance (default 1e-10 for c2 in FP64, 1e-12 for other "
                         "FP64 runs, 1e-6 otherwise)")
    ap.add_argument("--no-forms", action="store_true",
                    help="c2 in FP64: skip timing the plain FP32 and split-BF16 forms")
    ap.add_argument("--compare-fp32", action="store_true",
                    help="precision form: also time the plain FP32 path on the same problem")
    ap.add_argument("--stored-bf16", action="store_true",
                    help="stored workload in the precision form (same as --precision bf16)")
    ap.add_argument("--check-fp64", action="store_true",
                    help="precision form: also run the FP64 path on the same probes")
    ap.add_argument("--compare-plain", action="store_true",
                    help="batched form: also time 256 sequential plain FP32 calls")
    ap.add_argument("--no-graph", action="store_true", help="batched form: eager launches")
    ap.add_argument("--cpu-sample-count", type=int, default=12)
    ap.add_argument("--dump", default="", help="batched form: write per-instance results (JSON)")
    ap.add_argument("--c5-train-n", type=int, default=1000)
    ap.add_argument("--c5-train-count", type=int, default=1024)
    ap.add_argument("--c5-eval-n", type=int, default=5000)
    ap.add_argument("--c5-side", type=int, default=32)
    ap.add_argument("--c5-epochs", type=int, default=300)
    ap.add_argument("--c5-rank", type=int, default=0,
                    help="preconditioner rank of the training and grid problems (default n/40)")
    ap.add_argument("--c5-chunk", type=int, default=0, help="problems per batched call")
    ap.add_argument("--c5-train-start", type=int, default=0,
                    help="first training problem of the seeded sequence")
    ap.add_argument("--c5-data-out", default="",
                    help="only generate the training targets and eigenvalues and save them here")
    ap.add_argument("--c5-split-timing", action="store_true",
                    help="estimate every grid point once: the surrogate sweep, then the plain "
                         "estimator on the points that did not fall back (large n)")
    ap.add_argument("--c5-data-in", default="",
                    help="comma-separated files from --c5-data-out to train on")
    ap.add_argument("--c5-calibrate", action="store_true",
                    help="scale the ensemble spread by a factor calibrated on held-out "
                         "training problems before the fallback test")
    ap.add_argument("--c5-train-family", default="batched", choices=["batched", "grid"],
                    help="training problems: the batched form's hyperparameter distribution "
                         "(default) or the evaluation grid's own family")
    ap.add_argument("--lanczos-steps", type=int, default=0,
                    help="c1/c2/c3: run Algorithm 1 as printed (this many Lanczos steps per "
                         "probe, tridiagonal solves) instead of the multi-shift CG to tolerance")
    ap.add_argument("--precond", default="rsvd", choices=sorted(PRECOND_KINDS),
                    help="c1/c2/c3: preconditioner of the Appendix's list")
    ap.add_argument("--probes", default="rademacher", choices=["rademacher", "gaussian", "orthogonal"],
                    help="c1/c2/c3: probe distribution (Algorithm 1 step 1, Appendix)")
    ap.add_argument("--gradient", action="store_true",
                    help="c1/c2/c3: time d log det / d(lengthscale, variance, noise) instead")
    ap.add_argument("--scaled", action="store_true",
                    help="the preconditioner's 'plus scaling' variant (D = noise I)")
    ap.add_argument("--union-shifts", action="store_true",
                    help="all orders from one solve over the union of their poles "
                         "(shared probes; reported separately from the default)")
    ap.add_argument("--sensitivity", default="", choices=["", "axes", "dims"],
                    help="the Appendix's parameter sweeps (axes) or the sweep over d (dims)")
    ap.add_argument("--sens-n", type=int, default=20000)
    ap.add_argument("--sens-count", type=int, default=8, help="problems per sweep point")
    ap.add_argument("--sens-dims", default="1,2,3,4,5,6,8,10,12,15,20")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the workload, run one device-to-device copy of this many MiB "
                         "(the reference dispatch for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2405_03474_amd as L

    if args.sensitivity:
        return sensitivity_main(args, torch, L)
    if args.workload == "c4_batch256":
        return batch_main(args, torch, L)
    if args.workload == "c5_surrogate":
        return surrogate_main(args, torch, L)
    cfg = WORKLOADS[args.workload]
    if args.n:
        cfg = cfg.with_n(args.n, rank=min(cfg.rank, args.n // 10))
    if args.kernel_kind:
        cfg = replace(cfg, kind=workloads.RBF if args.kernel_kind == "rbf" else workloads.MATERN52,
                      name=f"{cfg.name}@{args.kernel_kind}")
    kind = args.workload.split("_")[0]
    precision = {"c1": L.LD_F64, "c2": L.LD_F64, "c3": L.LD_BF16}[kind]
    if args.precision:
        precision = {"f64": L.LD_F64, "f32": L.LD_F32, "bf16": L.LD_BF16}[args.precision]
    if kind == "c2" and args.stored_bf16:
        precision = L.LD_BF16
    if kind == "c3" and args.plain_fp32:
        precision = L.LD_F32
    stored = kind == "c2"
    dtype = dtype_name(precision, stored)
    # FP64 solves of the stored workload stop at 1e-10 (the estimate then
    # agrees with the oracle's exact solves to ~1e-12; tested at n = 20,000)
    tol = args.tol or (1e-10 if (kind == "c2" and precision == L.LD_F64) else 0.0)
    log(f"[bench] workload {cfg.name} n={cfg.n} rank={cfg.rank} probes={cfg.probes} "
        f"orders={cfg.orders} dtype={dtype} stored={stored}")

    torch.cuda.set_device(0)
    if args.gradient:
        return gradient_main(args, torch, L, cfg, precision, stored)
    stream = torch.cuda.current_stream(0)
    copy_calibration(torch, args.copy_calibration_mib)
    ctx = L.Context(0, stream)
    ctx.set_probes({"rademacher": L.LD_PROBE_RADEMACHER, "gaussian": L.LD_PROBE_GAUSSIAN,
                    "orthogonal": L.LD_PROBE_ORTHOGONAL}[args.probes])
    if args.symmetric:
        ctx.set_symmetric(f32=args.symmetric in ("f32", "both"),
                          bf16=args.symmetric in ("bf16", "both"))
    runner = Runner(L, torch, ctx, cfg, precision, stored, args.lanczos_steps, args.precond,
                    args.scaled, args.union_shifts, tol)
    if args.graphs:
        # replayed iterations carry no timing events: the timed steps run
        # uninstrumented, one more instrumented (eager) step times the product
        ctx.set_graphs(True)
        results, ms_total, wall, _ = timed_steps(runner, args.steps, args.warmup, stream, torch,
                                                 instrument=False)
        _, _, _, (mm_ms, mm_calls, mm_flops, mm_bytes) = timed_steps(runner, 1, 0, stream, torch)
    else:
        results, ms_total, wall, (mm_ms, mm_calls, mm_flops, mm_bytes) = timed_steps(
            runner, args.steps, args.warmup, stream, torch)

    n_est = args.steps * len(cfg.orders)
    value = n_est / (ms_total / 1e3)
    last = results[-1]
    exact = load_exact(cfg.name) if not args.n else None
    accuracy = {}
    for k in cfg.orders:
        r = last[k]
        acc = {"logdet": r["logdet"], "logdet_P": r["logdet_P"], "stderr": r["std_err"],
               "iterations": r["iterations"], "rel_resid": r["rel_resid"]}
        if exact is not None:
            acc["exact_logdet"] = exact
            acc["rel_err_vs_exact"] = abs(r["logdet"] - exact) / abs(exact)
            acc["within_1e-3"] = acc["rel_err_vs_exact"] <= 1e-3
        accuracy[f"r{k}"] = acc

    avg_ms = mm_ms / max(mm_calls, 1)
    achieved = (mm_flops / max(mm_calls, 1)) / (avg_ms / 1e3)
    peak = {L.LD_F32: PEAK["fp32"], L.LD_F64: PEAK["fp64"], L.LD_BF16: PEAK["bf16"]}[precision]
    kname = {"c2": "k_mm32_tf<2> (FP32 MFMA 32x32x2, stored LD_TILED fragment tiles)",
             "c1": "k_mm64<fly> (FP64 MFMA 16x16x4, on the fly)",
             "c3": "k_mm16<fly> (split-BF16 MFMA 32x32x16, 3 terms, on the fly)"}[kind]
    if kind == "c2" and precision == L.LD_F64:
        kname = "k_mm64_tf<4> (FP64 MFMA 16x16x4, stored LD_TILED fragment tiles)"
    if kind == "c3" and precision == L.LD_F32:
        kname = "k_mm32_fly (FP32 MFMA 32x32x2, kernel entries generated on the fly)"
        if cfg.n >= 16384 and 32 < cfg.probes <= 64 and args.symmetric in ("", "f32", "both"):
            kname = ("k_mm32_sym (FP32 MFMA over the symmetric split: blocks on and above the "
                     "diagonal generated once, applied directly 32x32x2 and transposed 16x16x4)")
    traffic = profiled_traffic(f"{cfg.name}/{dtype}") if not args.n and stored else None
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic, "kernel": kname,
                "avg_launch_ms": avg_ms, "launches": mm_calls,
                "algorithmic_GBps": (mm_bytes / max(mm_calls, 1)) / (avg_ms / 1e3) / 1e9}

    line = {
        "metric": METRIC, "value": value, "unit": "log-det estimates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_total / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": cfg.name, "n": cfg.n, "d": cfg.d,
                   "kernel": "matern52" if cfg.kind == 1 else "rbf", "points": cfg.points,
                   "lengthscale": cfg.lengthscale, "variance": cfg.variance, "noise": cfg.noise,
                   "storage": ("stored_tiled"
                               if stored else "on_the_fly"),
                   "orders": list(cfg.orders), "probes": cfg.probes, "rank": cfg.rank,
                   "oversample": cfg.oversample, "power_iters": cfg.power_iters,
                   "precond": {"kind": args.precond, "scaled": args.scaled},
                   "probe_kind": args.probes,
                   "solver": ({"kind": "lanczos", "steps": args.lanczos_steps}
                              if args.lanczos_steps else
                              {"kind": "multishift_pcg", "tol": runner.tol,
                               "orders_share_probes": bool(args.union_shifts),
                               "graph_replay": bool(args.graphs)}),
                   "symmetric_split": args.symmetric or "f32"},
        "probe_solves_per_s": cfg.probes * n_est / (ms_total / 1e3),
        # the same estimates without the preconditioner build and M (host wall
        # time of each solve as the library reports it)
        "solve_only_estimates_per_s": n_est / max(sum(r[k]["seconds_solve"] for r in results
                                                      for k in cfg.orders), 1e-12),
        "iterations": {f"r{k}": last[k]["iterations"] for k in cfg.orders},
        "wall_s": wall, "accuracy": accuracy, "roofline": roofline,
    }

    if kind == "c2" and precision == L.LD_BF16:
        # the FP32 tiles' bytes with under a third of the FP32 matrix-core
        # time: the product is bound by HBM
        gbps = (mm_bytes / max(mm_calls, 1)) / (avg_ms / 1e3) / 1e9
        line["roofline"].update({
            "bound": "hbm", "achieved": gbps, "peak": 8000.0, "unit": "GB/s", "frac": gbps / 8000.0,
            "traffic": traffic,
            "kernel": "k_mm16_tf<2> (BF16 MFMA 32x32x16, stored FP32 tiles split exactly into "
                      "3 bf16 parts, V into 2, 4 terms)",
            "flops_TFLOPs": achieved / 1e12})
    if kind == "c2" and precision == L.LD_F64 and not args.no_forms:
        # the metric's other forms on the same problem and probes: plain FP32
        # and the split-BF16 precision form, each against this FP64 result
        forms = {}
        for fprec in (L.LD_F32, L.LD_BF16):
            name = dtype_name(fprec, stored)
            log(f"[bench] form {name}, same problem")
            fr = Runner(L, torch, ctx, cfg, fprec, stored, args.lanczos_steps, args.precond,
                        args.scaled, args.union_shifts)
            fres, fms, _, _ = timed_steps(fr, 1, 1, stream, torch, instrument=False)
            fr.release()
            fv = len(cfg.orders) / (fms / 1e3)
            forms[name] = {
                "value": fv, "ms_per_step": fms, "tol": fr.tol,
                "rel_diff_vs_f64": {f"r{k}": abs(fres[-1][k]["logdet"] - last[k]["logdet"])
                                    / abs(last[k]["logdet"]) for k in cfg.orders},
                "iterations": {f"r{k}": fres[-1][k]["iterations"] for k in cfg.orders}}
        base = forms["f32"]["value"]
        for f in forms.values():
            f["speedup_vs_plain_fp32"] = f["value"] / base
        line["forms"] = forms
        line["speedup_vs_plain_fp32"] = {"bf16x4+f32": forms["bf16x4+f32"]["speedup_vs_plain_fp32"],
                                         "f64": value / base}
    if exact is not None:
        within = [f"r{k}" for k in cfg.orders if accuracy[f"r{k}"]["within_1e-3"]]
        line["accuracy_qualifier"] = {
            "rule": "relative error vs exact FP64 Cholesky log det <= 1e-3",
            "orders_within": within,
            "qualified_estimates_per_s": value * len(within) / len(cfg.orders),
            "note": "the error of each order is the bias of r_k on the spectrum of M P^-1 at "
                    "this preconditioner rank (a property of the method, not of the "
                    "arithmetic); the FP64 path matches the oracle's exact-solve estimate"}
    if kind in ("c2", "c3") and args.compare_fp32:
        log("[bench] plain FP32 path, same problem")
        plain = Runner(L, torch, ctx, cfg, L.LD_F32, stored, args.lanczos_steps, args.precond,
                       args.scaled)
        pres, pms, _, _ = timed_steps(plain, 1, 0, stream, torch)
        pv = len(cfg.orders) / (pms / 1e3)
        line["plain_fp32"] = {"value": pv, "ms_per_step": pms,
                              "logdet": {f"r{k}": pres[-1][k]["logdet"] for k in cfg.orders}}
        line["speedup_vs_plain_fp32"] = value / pv
    if kind == "c3" and args.check_fp64:
        log("[bench] FP64 reference run on the same probes")
        ref = Runner(L, torch, ctx, cfg, L.LD_F64, False, args.lanczos_steps, args.precond,
                     args.scaled)
        rres = ref.step()
        line["fp64_reference"] = {
            f"r{k}": {"logdet": rres[k]["logdet"],
                      "rel_err": abs(last[k]["logdet"] - rres[k]["logdet"]) / abs(rres[k]["logdet"]),
                      "iterations": rres[k]["iterations"]} for k in cfg.orders}

    if args.no_cpu_baseline:
        line["cpu_baseline"] = None
    else:
        log("[bench] cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(cfg, min(args.cpu_sample_n, cfg.n), args.lanczos_steps,
                                            args.precond, args.scaled, args.probes)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
