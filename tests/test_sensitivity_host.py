"""Host logic of the sensitivity sweeps (no GPU): the problem recipe of the
Appendix's sweeps (Section 3: amplitude and lengthscale 1, standard normal
index points) and the one-parameter-at-a-time settings around the paper's
parameter choice (35 probes, t = 20, rank 25, 5 iterations)."""
import numpy as np
import pytest

import workloads
from paper_2405_03474_amd import sensitivity as S
import paper_2405_03474_amd as L


def test_instances_follow_section3_recipe():
    insts = workloads.sensitivity_instances(workloads.MATERN52, 5, 4, n=3000)
    assert [g.n for g in insts] == [3000] * 4 and all(g.d == 5 for g in insts)
    assert all(g.lengthscale == 1.0 and g.variance == 1.0 for g in insts)
    assert all((g.rank, g.power_iters, g.probes) == (25, 5, 35) for g in insts)
    X = insts[0].X()
    # standard normal points: mean ~0, variance ~1 per coordinate
    assert np.all(np.abs(X.mean(0)) < 0.1) and np.all(np.abs(X.var(0) - 1) < 0.1)
    np.testing.assert_array_equal(X, insts[0].X())            # seeded
    seeds = {(g.seed, g.probe_seed, g.precond_seed) for g in insts}
    assert len(seeds) == 4                                     # distinct problems
    other = workloads.sensitivity_instances(workloads.RBF, 5, 4, n=3000)
    assert not {g.seed for g in insts} & {g.seed for g in other}


def test_axis_settings_vary_one_parameter():
    base = S.Setting()
    assert (base.probes, base.steps, base.rank, base.power_iters) == (35, 20, 25, 5)
    st = S.axis_settings(base, {"rank": [5, 50], "precond": [(L.LD_PRECOND_PCHOL, True)]},
                         orders=(1, 3))
    assert set(st) == {("rank", "5", 1), ("rank", "5", 3), ("rank", "50", 1), ("rank", "50", 3),
                       ("precond", "partial Cholesky + scaling", 1),
                       ("precond", "partial Cholesky + scaling", 3)}
    assert st[("rank", "50", 3)] == S.Setting(rank=50, k=3)
    p = st[("precond", "partial Cholesky + scaling", 1)]
    assert (p.precond, p.scaled, p.k, p.rank) == (L.LD_PRECOND_PCHOL, True, 1, 25)


def test_every_axis_value_has_a_name():
    for axis, values in S.AXES.items():
        names = [S.value_name(axis, v) for v in values]
        assert len(set(names)) == len(names)
        for v in values:
            S.Setting().with_value(axis, v)


def test_cell_summary():
    c = S.Cell()
    for est, ex in ((10.5, 10.0), (9.0, 10.0), (10.25, 10.0)):
        c.add(est, ex, 0.1)
    s = c.summary()
    assert s["count"] == 3
    assert s["mean_abs_err"] == pytest.approx(0.5833333333333334)
    assert s["mean_signed_err"] == pytest.approx(-0.0833333333333333)
    assert s["mean_rel_err"] == pytest.approx(0.05833333333333334)
