"""Pins for oracle.estimate: the output of Algorithm 1 (Section 2) with
exact shifted solves, checked on cases whose answer is known in closed form
and by Hutchinson's identity (Section 1)."""
import numpy as np
import pytest

import workloads
from oracle import estimate, gp, precond, rational, rng


def _spd(n, seed):
    g = np.random.default_rng(seed)
    A = g.standard_normal((n, n))
    return A @ A.T / n + 0.5 * np.eye(n)


@pytest.mark.parametrize("k", [1, 3, 5])
def test_diagonal_matrices_exact_for_rademacher(k):
    # For diagonal M and P, z^T f(M P^-1) z = sum_i f(m_i / p_i) for every
    # +-1 probe, so the estimate is exact for any seed.
    g = np.random.default_rng(k)
    n = 50
    m = g.uniform(0.2, 9.0, n)
    p = g.uniform(0.5, 3.0, n)
    for seed in (1, 2, 3):
        Z = estimate.probes(seed, n, 4)
        est = estimate.estimate_dense(np.diag(m), np.diag(p), float(np.sum(np.log(p))), k, Z)
        expect = np.sum(np.log(p)) + np.sum(rational.r_eval(k, m / p))
        assert est.logdet == pytest.approx(expect, rel=1e-13)
        np.testing.assert_allclose(est.per_probe, np.sum(rational.r_eval(k, m / p)), rtol=1e-12)


@pytest.mark.parametrize("k", [1, 3, 5])
def test_scalar_multiple(k):
    # M = gamma P: every shifted solve is z / (gamma + a_j), so
    # est = log det P + n r_k(gamma) for any probes.
    n, gamma = 40, 2.7
    P = _spd(n, 10)
    ldP = np.linalg.slogdet(P)[1]
    Z = estimate.probes(4, n, 3)
    est = estimate.estimate_dense(gamma * P, P, ldP, k, Z)
    assert est.logdet == pytest.approx(ldP + n * float(rational.r_eval(k, gamma)), rel=1e-12)


def test_exact_preconditioner_gives_exact_logdet():
    # P = M: M P^-1 = I and r_k(1) = 0, so the trace term vanishes.
    M = _spd(60, 11)
    ld = np.linalg.slogdet(M)[1]
    est = estimate.estimate_dense(M, M, ld, 3, estimate.probes(9, 60, 5))
    np.testing.assert_allclose(est.per_probe, 0.0, atol=1e-10)
    assert est.logdet == pytest.approx(ld, rel=1e-12)


def test_exact_logdet_matches_slogdet():
    M = _spd(80, 12)
    assert estimate.logdet_exact(M) == pytest.approx(np.linalg.slogdet(M)[1], rel=1e-13)


def test_per_shift_cg_agrees_with_dense_solves():
    X = np.random.default_rng(13).random((300, 3))
    M = gp.dense_matrix(gp.MATERN52, X, 0.2, 1.0, 1e-3)
    P = precond.rsvd(M, 20, 10, 2, 14, 1e-3)
    Pd = P.dense()
    z = estimate.probes(15, 300, 1)[:, 0]
    _, a, _ = rational.partial_fraction(3)
    for aj in a:
        y = estimate.per_shift_cg(lambda v: M @ v, P, z, aj, tol=1e-13)
        np.testing.assert_allclose(y, np.linalg.solve(M + aj * Pd, z), rtol=1e-9, atol=1e-9)


def test_unbiased_over_seeds():
    # Hutchinson's identity: E_z[est] = log det P + sum r_k(lambda(M P^-1)).
    X = np.random.default_rng(16).random((120, 3))
    M = gp.dense_matrix(gp.RBF, X, 0.25, 1.0, 1e-2)
    P = precond.rsvd(M, 8, 4, 1, 17, 1e-2)
    Pd = P.dense()
    expect, _ = estimate.expected_estimate(M, Pd, P.logdet, 3)
    vals = np.array([estimate.estimate_dense(M, Pd, P.logdet, 3, estimate.probes(s, 120, 4)).logdet
                     for s in range(300)])
    se = vals.std(ddof=1) / np.sqrt(len(vals))
    assert abs(vals.mean() - expect) < 4.0 * se


def test_expectation_equals_exact_when_log_is_used():
    # with log in place of r_k the expectation is exactly log det M
    X = np.random.default_rng(18).random((90, 2))
    M = gp.dense_matrix(gp.MATERN52, X, 0.3, 1.0, 1e-2)
    P = precond.rsvd(M, 6, 4, 1, 19, 1e-2)
    lam = estimate.generalized_eigs(M, P.dense())
    assert P.logdet + np.sum(np.log(lam)) == pytest.approx(estimate.logdet_exact(M), rel=1e-11)


def test_small_workload_error_within_bias_plus_noise():
    cfg = workloads.C1.with_n(1000, rank=50)
    X = cfg.X()
    M = gp.dense_matrix(cfg.kind, X, cfg.lengthscale, cfg.variance, cfg.noise)
    P = precond.rsvd(M, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed,
                     precond.d_floor(cfg.noise, cfg.variance))
    Pd = P.dense()
    est = estimate.estimate_dense(M, Pd, P.logdet, 3, estimate.probes(cfg.probe_seed, cfg.n, cfg.probes))
    exact = estimate.logdet_exact(M)
    _, bias = estimate.expected_estimate(M, Pd, P.logdet, 3)
    assert abs(est.logdet - exact) <= abs(bias) + 4.0 * est.stderr


def test_blocked_cholesky_logdet_matches_lapack():
    X = np.random.default_rng(20).random((700, 3))
    M = gp.dense_matrix(gp.MATERN52, X, 0.2, 1.0, 1e-3)
    ref = oest_ref = estimate.logdet_exact(M)
    for block in (64, 100, 700):
        assert estimate.logdet_exact_blocked(M.copy(), block) == pytest.approx(ref, rel=1e-12)


def test_standard_error_hand_cases():
    # The reported standard error is the sample standard deviation of the
    # per-probe values over sqrt(s): for two values it is |t_1 - t_2| / 2;
    # for equal values it is 0; for s values that are all 0 but one 1 the
    # sample variance is 1/s, so it is 1/s.
    assert estimate.combine(0.0, [3.0, 7.5]).stderr == pytest.approx(2.25, rel=1e-15)
    assert estimate.combine(0.0, [-1.0, 1.0]).stderr == pytest.approx(1.0, rel=1e-15)
    assert estimate.combine(5.0, [2.0] * 9).stderr == 0.0
    for s in (3, 8, 50):
        t = np.zeros(s)
        t[s // 2] = 1.0
        assert estimate.combine(0.0, t).stderr == pytest.approx(1.0 / s, rel=1e-13)
    one = estimate.combine(1.5, [4.0])
    assert np.isnan(one.stderr) and one.logdet == 5.5


def test_standard_error_matches_spread_over_repeats():
    # Over many independent probe sets the standard error predicts the
    # spread of the estimate: the mean of stderr^2 over repeats equals the
    # variance of the means (both estimate Var(t) / s).
    g = np.random.default_rng(33)
    s, reps = 16, 4000
    T = g.exponential(2.0, size=(reps, s))
    se2 = np.array([estimate.combine(0.0, row).stderr ** 2 for row in T])
    means = T.mean(axis=1)
    assert np.mean(se2) == pytest.approx(4.0 / s, rel=0.05)
    assert np.mean(se2) == pytest.approx(np.var(means, ddof=1), rel=0.08)
