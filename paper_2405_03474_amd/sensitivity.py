"""Sensitivity of the r* estimators to their parameters: the Appendix's
sweeps over the preconditioner (kind, rank, power iterations), the probes
(kind, count), the Lanczos steps t of Algorithm 1 and the order k, and the
Section 3 sweep over the dimension d of the index points.

Each problem is stored once in FP64 (row-major, from the library's
kernel_materialize).  Its exact log det, the yardstick of the paper's
accuracy plots, is supplied by the caller (`exact_fn`: the benchmark and the
tests factor the stored matrix outside this package; it is a measurement of
the estimator, not part of it).  Every estimate is a library call
(preconditioner build plus Algorithm 1 or the multi-shift CG); its time
includes the preconditioner, as the paper's timings do.  Errors are
|estimate - log det M| (absolute, as in the paper's figures) and that divided
by |log det M|.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field, replace

import numpy as np

from . import _binding as B


@dataclass(frozen=True)
class Setting:
    """One estimator configuration; the defaults are the paper's parameter
    choice of Section 3 (35 Rademacher probes, t = 20 Lanczos steps, the
    randomized truncated SVD with 25 eigenvalues and 5 power iterations)."""
    k: int = 3
    probes: int = 35
    steps: int = 20
    rank: int = 25
    power_iters: int = 5
    oversample: int = 10
    precond: int = B.LD_PRECOND_RSVD
    scaled: bool = False
    probe_kind: int = B.LD_PROBE_RADEMACHER
    solver: str = "lanczos"          # "lanczos" (Algorithm 1) or "cg" (multi-shift CG)
    tol: float = 1e-10               # CG only: relative residual per probe
    max_iters: int = 5000            # CG only

    def with_value(self, axis: str, value):
        if axis == "precond":
            kind, scaled = value
            return replace(self, precond=kind, scaled=scaled)
        return replace(self, **{axis: value})


PRECOND_NAMES = {(B.LD_PRECOND_IDENTITY, False): "identity",
                 (B.LD_PRECOND_DIAGONAL, False): "diagonal",
                 (B.LD_PRECOND_RANK_ONE, False): "rank one",
                 (B.LD_PRECOND_PCHOL, False): "partial Cholesky",
                 (B.LD_PRECOND_PCHOL, True): "partial Cholesky + scaling",
                 (B.LD_PRECOND_RSVD, False): "randomized SVD",
                 (B.LD_PRECOND_RSVD, True): "randomized SVD + scaling"}
PROBE_NAMES = {B.LD_PROBE_RADEMACHER: "rademacher", B.LD_PROBE_GAUSSIAN: "gaussian",
               B.LD_PROBE_ORTHOGONAL: "normal orthogonal"}

# the Appendix's parameter axes (values around the paper's choice)
AXES = {
    "precond": list(PRECOND_NAMES),
    "rank": [5, 10, 25, 50, 100, 200],
    "power_iters": [0, 1, 2, 5, 10],
    "probe_kind": list(PROBE_NAMES),
    "probes": [5, 10, 20, 35, 70, 140],
    "steps": [5, 10, 20, 40, 80],
}


def value_name(axis: str, value) -> str:
    if axis == "precond":
        return PRECOND_NAMES[tuple(value)]
    if axis == "probe_kind":
        return PROBE_NAMES[value]
    return str(value)


@dataclass
class Cell:
    """The estimates of one (setting, problem set) cell."""
    errors: list = field(default_factory=list)      # |est - exact|
    rel: list = field(default_factory=list)         # |est - exact| / |exact|
    seconds: list = field(default_factory=list)     # preconditioner + estimator
    signed: list = field(default_factory=list)      # est - exact

    def add(self, est: float, exact: float, seconds: float):
        self.signed.append(est - exact)
        self.errors.append(abs(est - exact))
        self.rel.append(abs(est - exact) / abs(exact))
        self.seconds.append(seconds)

    def summary(self) -> dict:
        e = np.asarray(self.errors)
        m = len(e)
        return {"count": m, "mean_abs_err": float(e.mean()),
                "sem_abs_err": float(e.std(ddof=1) / math.sqrt(m)) if m > 1 else 0.0,
                "mean_signed_err": float(np.mean(self.signed)),
                "mean_rel_err": float(np.mean(self.rel)),
                "mean_seconds": float(np.mean(self.seconds))}


def stored_operator(ctx: B.Context, g, torch):
    """Problem g with its FP64 matrix stored row-major on the device."""
    X = torch.as_tensor(g.X(), dtype=torch.float64, device=f"cuda:{ctx.device}")
    op = B.GPOperator(X=X, kind=g.kind, lengthscale=g.lengthscale, variance=g.variance,
                      noise=g.noise, precision=B.LD_F64)
    op.M = B.kernel_materialize(ctx, op)
    return op


def estimate(ctx: B.Context, op, g, st: Setting):
    """One estimate of log det M with setting st; returns (value, seconds)."""
    ctx.set_probes(st.probe_kind)
    t0 = time.perf_counter()
    P = B.Precond(ctx, op, st.rank, st.oversample, st.power_iters, g.precond_seed,
                  kind=st.precond, scaled=st.scaled)
    try:
        if st.solver == "lanczos":
            res, _ = B.logdet_estimate_lanczos(ctx, op, P, st.k, st.probes, g.probe_seed, st.steps)
        else:
            res, _ = B.logdet_estimate(ctx, op, P, st.k, st.probes, g.probe_seed, st.tol,
                                       st.max_iters, allow_noconv=True)
    finally:
        P.close()
    return res["logdet"], time.perf_counter() - t0


def _print(msg: str):
    print(msg, flush=True)


def sweep(ctx: B.Context, instances, settings: dict, torch, exact_fn, log=_print):
    """Every setting of `settings` (name -> Setting) on every problem of
    `instances`; the problem's matrix and exact log det (exact_fn(ctx, op):
    the caller's yardstick for the stored FP64 matrix op.M) are computed once.
    Returns ({name: Cell}, [exact log det per problem])."""
    cells = {name: Cell() for name in settings}
    exacts = []
    for i, g in enumerate(instances):
        op = stored_operator(ctx, g, torch)
        exact = exact_fn(ctx, op)
        exacts.append(exact)
        if i == 0:      # first call on the device: library set-up outside the timings
            estimate(ctx, op, g, next(iter(settings.values())))
        done = {}       # equal settings (the base point of every axis) run once
        for name, st in settings.items():
            if st not in done:
                done[st] = estimate(ctx, op, g, st)
            est, sec = done[st]
            cells[name].add(est, exact, sec)
        log(f"[sensitivity] {g.name} n={g.n} d={g.d} exact {exact:.6e}: "
            f"{len(done)} settings done")
        del op
    return cells, exacts


def axis_settings(base: Setting, axes: dict, orders=(3,)):
    """Settings varying one parameter at a time around `base`, for each
    order k: {(axis, value, k): Setting}."""
    out = {}
    for axis, values in axes.items():
        for v in values:
            for k in orders:
                out[(axis, value_name(axis, v), k)] = replace(base.with_value(axis, v), k=k)
    return out
