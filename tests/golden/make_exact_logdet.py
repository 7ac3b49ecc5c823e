"""Write tests/golden/exact_logdet.json: the exact log det (FP64 Cholesky,
the paper's accuracy reference in Section 3) of the seeded workloads whose
matrices are too large to factor inside a test or benchmark run.

Calls only the oracle and the seeded input generators.
Usage: python tests/golden/make_exact_logdet.py [workload ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import estimate, gp  # noqa: E402

OUT = os.path.join(HERE, "exact_logdet.json")


def exact(cfg):
    X = cfg.X()
    M = gp.dense_matrix(cfg.kind, X, cfg.lengthscale, cfg.variance, cfg.noise)
    return estimate.logdet_exact_blocked(M, 2048)


def main(names):
    table = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        if name == "c4_batch256":
            t0 = time.time()
            insts = workloads.batch_instances()
            vals = [exact(g) for g in insts]
            table[name] = {"n": [g.n for g in insts], "logdet": vals,
                           "method": "per instance: oracle.gp.dense_matrix + "
                                     "oracle.estimate.logdet_exact_blocked (FP64 Cholesky)",
                           "seconds": round(time.time() - t0, 1)}
            json.dump(table, open(OUT, "w"), indent=1, sort_keys=True)
            print(name, len(vals), flush=True)
            continue
        cfg = {"c1_rbf_2k": workloads.C1, "c2_matern_gm50k": workloads.C2}[name]
        t0 = time.time()
        v = exact(cfg)
        table[name] = {"n": cfg.n, "logdet": v, "method": "oracle.gp.dense_matrix + oracle.estimate.logdet_exact_blocked (FP64 Cholesky)",
                       "seconds": round(time.time() - t0, 1)}
        json.dump(table, open(OUT, "w"), indent=1, sort_keys=True)
        print(name, v, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1_rbf_2k", "c2_matern_gm50k"])
