"""Write tests/golden/parity_c2_n20000.json: the oracle's estimates for the
c2 recipe (Matern-5/2, 8-component Gaussian mixture in [0,1]^3, l = 0.15,
noise 1e-3, randomized SVD rank 500 with 10 oversampling and 2 power
iterations, 64 Rademacher probes, r_1 / r_3 / r_5 with probe seed + k) at
n = 20,000, with the per-probe values of Algorithm 1's output (exact
shifted solves, Section 2), log det P, and the exact log det (Cholesky,
Section 3).  The GPU parity tests at that size compare against it.

Calls only the oracle and the seeded input generators.
Usage: python tests/golden/make_parity_golden.py [n]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import estimate, gp, precond  # noqa: E402


def main(n):
    t0 = time.time()
    cfg = workloads.C2.with_n(n, rank=500)
    X = cfg.X()
    M = gp.dense_matrix(cfg.kind, X, cfg.lengthscale, cfg.variance, cfg.noise)
    P = precond.rsvd(M, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed,
                     precond.d_floor(cfg.noise, cfg.variance))
    Pd = P.dense()
    out = {"workload": "c2_matern_gm50k recipe", "n": n, "rank": cfg.rank,
           "oversample": cfg.oversample, "power_iters": cfg.power_iters, "probes": cfg.probes,
           "precond_seed": cfg.precond_seed, "logdet_P": P.logdet, "orders": {}}
    for k in cfg.orders:
        Z = estimate.probes(cfg.probe_seed + k, n, cfg.probes)
        est = estimate.estimate_dense(M, Pd, P.logdet, k, Z)
        out["orders"][str(k)] = {"probe_seed": cfg.probe_seed + k, "logdet": est.logdet,
                                 "stderr": est.stderr, "per_probe": est.per_probe.tolist()}
        print(f"r_{k}: {est.logdet:.10f} ({time.time() - t0:.0f} s)", flush=True)
    del Pd
    out["exact_logdet"] = estimate.logdet_exact_blocked(M, 2048)
    out["method"] = ("oracle.gp.dense_matrix, oracle.precond.rsvd, oracle.estimate.estimate_dense "
                     "(Cholesky shifted solves), oracle.estimate.logdet_exact_blocked")
    out["seconds"] = round(time.time() - t0, 1)
    path = os.path.join(HERE, f"parity_c2_n{n}.json")
    json.dump(out, open(path, "w"), indent=1)
    print(path, out["exact_logdet"], flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 20000)
