"""Seeded synthetic inputs for the log-determinant estimator.

This module holds only input generation (point clouds, kernel choices and
hyperparameters of each workload); it contains none of the estimator's
arithmetic.  Both the oracle-side tests and the GPU-side tests and
benchmark draw their inputs from here.

Workloads (all synthetic; the paper's experiments use synthetic GP kernels
as well, Section 3):

  c1_rbf_2k       RBF, n=2,000 points uniform in [0,1]^3, l=0.2, s2=1,
                  noise 1e-2; r_3; rank 100 (+10 oversampling, 2 power
                  iterations); 32 Rademacher probes; FP64.
  c2_matern_gm50k Matern-5/2, n=50,000 points from an 8-component Gaussian
                  mixture (std 0.1, means uniform in [0,1]^3, equal weights);
                  l=0.15, s2=1, noise 1e-3; r_1, r_3, r_5; rank 500; 64
                  probes; FP32 with the matrix stored in HBM.
  c3_matern_200k  Matern-5/2, n=200,000 uniform in [0,1]^3, l=0.05, noise
                  1e-3; r_3; rank 1,000; 64 probes; kernel generated on the fly.
  c4_batch256     256 instances: n log-uniform in [500, 20,000], d in {2,3,8},
                  RBF or Matern-5/2, l log-U[0.02,0.5], s2 log-U[0.5,2],
                  noise log-U[1e-4,1e-1], points uniform in [0,1]^d; r_3;
                  16 probes; rank min(200, n/10).
  sensitivity     the Appendix's parameter sweeps (Section 3 setting):
                  amplitude and lengthscale 1, index points standard normal
                  in R^d, noise 1e-2 (the paper does not print it), RBF or
                  Matern-5/2, n = 20,000; the paper's estimator parameters
                  (35 Rademacher probes, t = 20, rank 25, 5 iterations).
  c5_surrogate    training set: instances with the c4 hyperparameter
                  distribution at one fixed n (r_5, 64 probes, rank n/40);
                  evaluation grid: 32 x 32 log-spaced lengthscales in
                  [0.02, 0.5] x noises in [1e-4, 1e-1], variance 1,
                  Matern-5/2, d = 3, points uniform in [0,1]^3, at a larger n.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

BASE_SEED = 240503474
RBF = 0
MATERN52 = 1


@dataclass(frozen=True)
class GPInstance:
    name: str
    n: int
    d: int
    kind: int              # 0 = RBF, 1 = Matern-5/2
    lengthscale: float
    variance: float
    noise: float
    points: str            # "uniform" or "gmix8"
    seed: int
    rank: int
    oversample: int = 10
    power_iters: int = 2
    probes: int = 32
    orders: tuple = (3,)
    probe_seed: int = 0
    precond_seed: int = 0

    def X(self) -> np.ndarray:
        return make_points(self.points, self.n, self.d, self.seed)

    def with_n(self, n: int, rank: int | None = None):
        return replace(self, n=n, rank=self.rank if rank is None else rank,
                       name=f"{self.name}@n{n}")


def make_points(kind: str, n: int, d: int, seed: int) -> np.ndarray:
    """Point cloud, FP64 row-major n x d."""
    g = np.random.default_rng(seed)
    if kind == "uniform":
        return g.random((n, d))
    if kind == "normal":
        return g.standard_normal((n, d))
    if kind == "gmix8":
        means = g.random((8, d))
        labels = g.integers(0, 8, size=n)
        return means[labels] + 0.1 * g.standard_normal((n, d))
    raise ValueError(kind)


C1 = GPInstance("c1_rbf_2k", n=2000, d=3, kind=RBF, lengthscale=0.2, variance=1.0,
                noise=1e-2, points="uniform", seed=BASE_SEED + 0, rank=100,
                probes=32, orders=(3,), probe_seed=BASE_SEED + 100, precond_seed=BASE_SEED + 200)
C2 = GPInstance("c2_matern_gm50k", n=50000, d=3, kind=MATERN52, lengthscale=0.15,
                variance=1.0, noise=1e-3, points="gmix8", seed=BASE_SEED + 1, rank=500,
                probes=64, orders=(1, 3, 5), probe_seed=BASE_SEED + 101,
                precond_seed=BASE_SEED + 201)
C3 = GPInstance("c3_matern_200k", n=200000, d=3, kind=MATERN52, lengthscale=0.05,
                variance=1.0, noise=1e-3, points="uniform", seed=BASE_SEED + 2, rank=1000,
                probes=64, orders=(3,), probe_seed=BASE_SEED + 102, precond_seed=BASE_SEED + 202)


def batch_instances(count: int = 256, seed: int = BASE_SEED + 3, n_lo: int = 500,
                    n_hi: int = 20000, probes: int = 16):
    """The heterogeneous batch (reading: n = round(exp(U[ln lo, ln hi])),
    rank = floor(min(200, n/10)))."""
    g = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(np.exp(g.uniform(np.log(n_lo), np.log(n_hi)))))
        d = int(g.choice([2, 3, 8]))
        kind = int(g.integers(0, 2))
        ls = float(np.exp(g.uniform(np.log(0.02), np.log(0.5))))
        var = float(np.exp(g.uniform(np.log(0.5), np.log(2.0))))
        noise = float(np.exp(g.uniform(np.log(1e-4), np.log(1e-1))))
        rank = int(min(200, n // 10))
        out.append(GPInstance(f"c4_{i}", n=n, d=d, kind=kind, lengthscale=ls, variance=var,
                              noise=noise, points="uniform", seed=seed * 1000 + i,
                              rank=rank, probes=probes, orders=(3,),
                              probe_seed=seed + 10000 + i, precond_seed=seed + 20000 + i))
    return out


def surrogate_training_instances(count: int, n: int, seed: int = BASE_SEED + 4,
                                 probes: int = 64, rank: int | None = None, start: int = 0):
    """Training problems for the surrogate: the c4 hyperparameter distribution
    at a fixed n, rank n/40 unless given; problems start .. start + count - 1
    of the seeded sequence."""
    g = np.random.default_rng(seed)
    rank = rank or max(1, n // 40)
    out = []
    for i in range(start + count):
        d = int(g.choice([2, 3, 8]))
        kind = int(g.integers(0, 2))
        ls = float(np.exp(g.uniform(np.log(0.02), np.log(0.5))))
        var = float(np.exp(g.uniform(np.log(0.5), np.log(2.0))))
        noise = float(np.exp(g.uniform(np.log(1e-4), np.log(1e-1))))
        if i < start:
            continue
        out.append(GPInstance(f"c5t_{i}", n=n, d=d, kind=kind, lengthscale=ls, variance=var,
                              noise=noise, points="uniform", seed=seed * 1000 + i,
                              rank=rank, probes=probes, orders=(5,),
                              probe_seed=seed + 10000 + i, precond_seed=seed + 20000 + i))
    return out


def surrogate_family_instances(count: int, n: int, seed: int = BASE_SEED + 7, probes: int = 64):
    """Training problems from the evaluation grid's own family (Matern-5/2,
    d = 3, variance 1, points uniform in [0,1]^3) with lengthscale and noise
    log-uniform over the grid's ranges; each problem has its own point cloud
    (none is a grid problem)."""
    g = np.random.default_rng(seed)
    out = []
    for i in range(count):
        ls = float(np.exp(g.uniform(np.log(0.02), np.log(0.5))))
        noise = float(np.exp(g.uniform(np.log(1e-4), np.log(1e-1))))
        out.append(GPInstance(f"c5f_{i}", n=n, d=3, kind=MATERN52, lengthscale=ls, variance=1.0,
                              noise=noise, points="uniform", seed=seed * 1000 + i,
                              rank=max(1, n // 40), probes=probes, orders=(5,),
                              probe_seed=seed + 10000 + i, precond_seed=seed + 20000 + i))
    return out


def surrogate_grid(n: int, side: int = 32, seed: int = BASE_SEED + 5, probes: int = 64,
                   rank: int | None = None):
    """The evaluation sweep: side x side log-spaced (lengthscale, noise) pairs,
    variance 1, Matern-5/2, d = 3, one point cloud shared by the grid; rank
    n/40 unless given."""
    rank = rank or max(1, n // 40)
    out = []
    for a, ls in enumerate(np.exp(np.linspace(np.log(0.02), np.log(0.5), side))):
        for b, nz in enumerate(np.exp(np.linspace(np.log(1e-4), np.log(1e-1), side))):
            i = a * side + b
            out.append(GPInstance(f"c5g_{a}_{b}", n=n, d=3, kind=MATERN52, lengthscale=float(ls),
                                  variance=1.0, noise=float(nz), points="uniform", seed=seed,
                                  rank=rank, probes=probes, orders=(5,),
                                  probe_seed=seed + 10000 + i, precond_seed=seed + 20000 + i))
    return out


def sensitivity_instances(kind: int, d: int, count: int, n: int = 20000, noise: float = 1e-2,
                          seed: int = BASE_SEED + 6, probes: int = 35):
    """Problems of the Appendix's sweeps: amplitude 1, lengthscale 1, index
    points standard normal in R^d (Section 3); rank 25 and 5 power iterations
    are the paper's preconditioner parameters.  Instance i of (kind, d) has
    its own point cloud, probe seed and sketch seed."""
    out = []
    for i in range(count):
        tag = (kind * 64 + d) * 1000 + i
        out.append(GPInstance(f"sens_{'rbf' if kind == RBF else 'm52'}_d{d}_{i}", n=n, d=d,
                              kind=kind, lengthscale=1.0, variance=1.0, noise=noise,
                              points="normal", seed=seed * 1000003 + tag, rank=25,
                              power_iters=5, probes=probes, orders=(1, 3, 5),
                              probe_seed=seed + 10 ** 7 + tag, precond_seed=seed + 2 * 10 ** 7 + tag))
    return out
