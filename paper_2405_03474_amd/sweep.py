"""Hyperparameter sweeps with the learned surrogate.

Workflow (the estimator, the preconditioners, the features, training and
prediction run in the library; this module moves batches between its entry
points and, per grid point, adds log det P to n times the predicted trace
term and applies the fallback rule to those two host scalars):
  1. training data: the batched estimator (r_k, s probes) on a set of
     problems gives targets (log det - log det P) / n and, with the kept
     eigenvalues, the 38 features of each problem;
  2. training: minibatch Adam steps of the ensemble;
  3. sweep: for every grid point the batched preconditioner build alone
     (log det P and the eigenvalues), the ensemble's BF16 prediction, and
     the plain estimator only where the members disagree by more than
     rel_tol * |log det| (the fallback).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import _binding as B


def _items(insts, torch):
    dev = torch.device("cuda:0")
    return [B.BatchItem(X=torch.as_tensor(g.X(), dtype=torch.float64, device=dev), kind=g.kind,
                        lengthscale=g.lengthscale, variance=g.variance, noise=g.noise, rank=g.rank,
                        precond_seed=g.precond_seed, probe_seed=g.probe_seed) for g in insts]


@dataclass
class Config:
    k: int = 5
    probes: int = 64
    oversample: int = 10
    power_iters: int = 2
    tol: float = 1e-6
    chunk: int = 256          # instances per batched call
    rel_tol: float = 1e-3     # fallback when kappa * n * std > rel_tol * |log det|
    kappa: float = 1.0        # spread multiplier (1: the ensemble's raw spread; see calibrate)
    max_iters: int = 5000     # solver iterations per batch (unconverged results are flagged)


def estimate_all(ctx, insts, cfg: Config, torch, precond_only=False, items=None, log=None):
    """Batched estimates (or preconditioners only) of a list of problems, in
    chunks; returns (results, eigenvalue rows, items).  log(msg), if given,
    is called after every chunk."""
    items = items if items is not None else _items(insts, torch)
    res, lams = [], []
    t0 = time.perf_counter()
    for c0 in range(0, len(items), cfg.chunk):
        r, _, _, lam = B.logdet_estimate_batched(
            ctx, items[c0:c0 + cfg.chunk], cfg.k, cfg.probes, cfg.oversample, cfg.power_iters,
            tol=cfg.tol, max_iters=cfg.max_iters, precond_only=precond_only, want_lambda=True,
            allow_noconv=True, allow_breakdown=True)
        res += r
        lams += [row[:g.rank] for row, g in zip(lam, insts[c0:c0 + cfg.chunk])]
        if log:
            log(f"[sweep] {min(c0 + cfg.chunk, len(items))}/{len(items)} problems "
                f"{time.perf_counter() - t0:.1f} s")
    return res, lams, items


def feature_edges(lams, insts):
    """Histogram edges from the global range of log(lambda / n) of a set."""
    lo = min(float(np.log(l.min() / g.n)) for l, g in zip(lams, insts))
    hi = max(float(np.log(l.max() / g.n)) for l, g in zip(lams, insts))
    pad = 1e-6 * (hi - lo + 1.0)
    return np.linspace(lo - pad, hi + pad, B.LD_SUR_BINS + 1)


def features(lams, insts, edges):
    return np.stack([B.surrogate_features(l, g.kind, g.lengthscale, g.variance, g.noise, g.n, g.d,
                                          edges) for l, g in zip(lams, insts)])


def train(ctx, F, y, torch, members=5, seed=0, epochs=300, batch=256, lr=1e-3):
    """Fit the ensemble on features F (N x 38) and targets y (N); returns the
    surrogate and the per-epoch mean loss of the members."""
    F64 = np.asarray(F, dtype=np.float64)
    mean = F64.mean(0)
    sd = F64.std(0)
    # a feature that is constant over the training set (log n when every
    # training problem has the same n) is switched off: its weights would
    # never be trained, so any other value must not reach them
    sd = np.where(sd > 1e-6 * np.maximum(1.0, np.abs(mean)), sd, 1e30)
    # the histogram bins share one scale: per-bin standardisation would blow
    # a bin that is nearly empty in training up to hundreds of units
    hist = F64[:, 6:]
    mean[6:] = hist.mean()
    sd[6:] = max(float(hist.std()), 1e-6)
    S = B.Surrogate(ctx, members=members, seed=seed)
    S.set_scaling(mean, sd, float(y.mean()), float(y.std() if y.std() > 0 else 1.0))
    dev = torch.device("cuda:0")
    Fd = torch.as_tensor(F, dtype=torch.float32, device=dev)
    yd = torch.as_tensor(y, dtype=torch.float32, device=dev)
    g = np.random.default_rng(seed)
    hist = []
    N = len(y)
    for _ in range(epochs):
        perm = torch.as_tensor(g.permutation(N), device=dev)
        losses = []
        for b0 in range(0, N, batch):
            idx = perm[b0:b0 + batch]
            last = b0 + batch >= N
            l = S.train_step(Fd[idx].contiguous(), yd[idx].contiguous(), lr=lr, want_loss=last)
            if last:
                losses.append(float(np.mean(l)))
        hist.append(losses[-1])
    return S, hist


def split_holdout(N: int, frac: float, seed: int = 1):
    """Indices (train, holdout) of a random split of N problems."""
    perm = np.random.default_rng(seed).permutation(N)
    h = int(round(frac * N))
    return np.sort(perm[h:]), np.sort(perm[:h])


def calibrate(S, F_hold, y_hold, torch, quantile: float = 0.99) -> float:
    """Spread multiplier from problems the ensemble was not trained on: the
    given quantile of |mean - target| / std over them (at least 1).  The raw
    spread of members trained on the same data can sit far below their shared
    error; scaled by this factor it bounds the held-out error at that
    quantile (the targets' own probe noise is included, so it is
    conservative)."""
    mean, sd = S.predict(torch.as_tensor(F_hold, dtype=torch.float32, device="cuda:0"))
    torch.cuda.synchronize()
    mean = mean.double().cpu().numpy()
    sd = np.maximum(sd.double().cpu().numpy(), 1e-300)
    ratio = np.abs(mean - np.asarray(y_hold, dtype=np.float64)) / sd
    return float(max(1.0, np.quantile(ratio, quantile)))


def sweep(ctx, S, grid, edges, cfg: Config, torch, items=None, score_rest=False, log=None):
    """Surrogate sweep over grid problems: returns per-point log det, whether
    the point fell back to the estimator, the stage times (s) together with
    the ensemble's own log det and spread at every point, and the items.
    With score_rest the plain estimator then also runs on the points that did
    not fall back (after the timed sweep, not part of it): the stages also
    carry "rest_plain" (its results, None at fallback points) and
    "rest_seconds", so that fallback plus rest is the plain estimator on every
    point, each point computed once."""
    t0 = time.perf_counter()
    pre, lams, items = estimate_all(ctx, grid, cfg, torch, precond_only=True, items=items)
    t1 = time.perf_counter()
    F = features(lams, grid, edges)
    mean, sd = S.predict(torch.as_tensor(F, dtype=torch.float32, device="cuda:0"))
    torch.cuda.synchronize()
    mean = mean.double().cpu().numpy()
    sd = sd.double().cpu().numpy()
    n = np.array([g.n for g in grid], dtype=np.float64)
    logdet_P = np.array([r["logdet_P"] for r in pre])
    logdet = logdet_P + n * mean
    fallback = cfg.kappa * n * sd > cfg.rel_tol * np.abs(logdet)
    predicted = logdet.copy()
    t2 = time.perf_counter()
    fb = np.nonzero(fallback)[0]
    plain_at = [None] * len(grid)
    if len(fb):
        res, _, _ = estimate_all(ctx, [grid[i] for i in fb], cfg, torch,
                                 items=[items[i] for i in fb], log=log)
        logdet[fb] = [r["logdet"] for r in res]
        for i, r in zip(fb, res):
            plain_at[i] = r
    t3 = time.perf_counter()
    stages = {"precond": t1 - t0, "predict": t2 - t1, "fallback": t3 - t2, "total": t3 - t0,
              "predicted": predicted, "spread": n * sd}
    if score_rest:
        rest = np.nonzero(~fallback)[0]
        t4 = time.perf_counter()
        if len(rest):
            res, _, _ = estimate_all(ctx, [grid[i] for i in rest], cfg, torch,
                                     items=[items[i] for i in rest], log=log)
            for i, r in zip(rest, res):
                plain_at[i] = r
        torch.cuda.synchronize()
        stages["rest_seconds"] = time.perf_counter() - t4
        stages["rest_plain"] = plain_at
    return logdet, fallback, stages, items
