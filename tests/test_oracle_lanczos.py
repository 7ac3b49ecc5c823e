"""Pins for oracle.lanczos (Algorithm 1 as printed, Section 2): t Lanczos
steps on M P^-1 in the P^-1 inner product and shifted tridiagonal solves,
checked against closed forms, exact termination on low-dimensional Krylov
spaces, the exact shifted solves of oracle.estimate, and t steps of a
textbook preconditioned CG (the Galerkin solution on the same space)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import estimate, lanczos, rational


def _spd(n, seed, shift=0.5):
    g = np.random.default_rng(seed)
    A = g.standard_normal((n, n))
    return A @ A.T / n + shift * np.eye(n)


@pytest.mark.parametrize("k", [1, 3, 5])
def test_scalar_multiple_stops_after_one_step(k):
    # M = gamma P: M P^-1 = gamma I, the recurrence stops at once with
    # T = [gamma], and est = log det P + n r_k(gamma) for Rademacher probes.
    n, gamma = 40, 2.7
    P = _spd(n, 21)
    ldP = np.linalg.slogdet(P)[1]
    Z = estimate.probes(5, n, 4)
    est, steps, resid = lanczos.estimate_lanczos(gamma * P, P, ldP, k, Z, 20)
    assert np.all(steps == 1)
    assert est.logdet == pytest.approx(ldP + n * float(rational.r_eval(k, gamma)), rel=1e-12)
    assert np.all(resid < 1e-12)


@pytest.mark.parametrize("k", [3, 5])
def test_rank_two_perturbation_terminates_exactly(k):
    # M = gamma P + W W^T (W: n x 2) makes M P^-1 = gamma I + W W^T P^-1, which
    # has at most three distinct eigenvalues; in the P^-1 inner product the
    # recurrence is symmetric and stops after at most three steps with the
    # exact shifted solves (a Euclidean recurrence on the non-symmetric
    # M P^-1 would not).
    n, gamma = 60, 1.3
    P = _spd(n, 22)
    W = np.random.default_rng(23).standard_normal((n, 2))
    M = gamma * P + W @ W.T
    Z = estimate.probes(6, n, 5)
    t_l, steps, _ = lanczos.per_probe_lanczos(M, P, k, Z, 30)
    t_d = estimate.per_probe_dense(M, P, k, Z)
    assert np.all(steps <= 3)
    np.testing.assert_allclose(t_l, t_d, rtol=1e-10)


@pytest.mark.parametrize("k", [1, 3, 5])
def test_full_krylov_space_equals_exact_solves(k):
    n = 10
    M, P = _spd(n, 24, 1.0), _spd(n, 25, 1.0)
    Z = estimate.probes(7, n, 6)
    t_l, steps, _ = lanczos.per_probe_lanczos(M, P, k, Z, n)
    np.testing.assert_allclose(t_l, estimate.per_probe_dense(M, P, k, Z), rtol=1e-9)


def test_converges_to_exact_solves_as_t_grows():
    n = 300
    M, P = _spd(n, 26, 0.3), _spd(n, 27, 1.0)
    Z = estimate.probes(8, n, 3)
    exact = estimate.per_probe_dense(M, P, 3, Z)
    errs = []
    for t in (5, 10, 20, 60):
        t_l, _, _ = lanczos.per_probe_lanczos(M, P, 3, Z, t)
        errs.append(np.max(np.abs(t_l - exact) / np.abs(exact)))
    assert errs[0] > errs[1] > errs[2] and errs[3] < 1e-10, errs


def _pcg_t_steps(M, P, z, shift, t):
    """t iterations of textbook preconditioned CG for (M + shift P) y = z
    with preconditioner P (applied through P^-1), from y = 0."""
    fac = sla.cho_factor(P, lower=True)
    A = M + shift * P
    y = np.zeros_like(z)
    r = z.copy()
    u = sla.cho_solve(fac, r)
    p = u.copy()
    rho = r @ u
    for _ in range(t):
        q = A @ p
        al = rho / (p @ q)
        y = y + al * p
        r = r - al * q
        u = sla.cho_solve(fac, r)
        rho_new = r @ u
        p = u + (rho_new / rho) * p
        rho = rho_new
    return y


@pytest.mark.parametrize("t", [3, 8])
def test_equals_t_steps_of_preconditioned_cg(t):
    # With x = P y, (M P^-1 + a I) x = z is (M + a P) y = z; t steps of PCG
    # give the Galerkin solution on the same Krylov space as t Lanczos steps,
    # so v^T x_t = (P v)^T y_t shift by shift.
    n = 120
    M, P = _spd(n, 28, 0.2), _spd(n, 29, 1.0)
    Z = estimate.probes(10, n, 2)
    b, a, c = rational.partial_fraction(5)
    t_l, _, _ = lanczos.per_probe_lanczos(M, P, 5, Z, t)
    for i in range(Z.shape[1]):
        v = Z[:, i].astype(np.float64)
        want = b * (v @ v)
        for aj, cj in zip(a, c):
            want += cj * float((P @ v) @ _pcg_t_steps(M, P, v, aj, t))
        assert t_l[i] == pytest.approx(want, rel=1e-10)


@pytest.mark.parametrize("t", [2, 5, 11])
def test_residual_equals_pcg_residual_norm(t):
    # The reported residual beta_t |w_t| / |v| is the P^-1-norm of
    # v - (M P^-1 + a_1 I) x_t for the smallest shift a_1, relative to
    # |v| = sqrt(v^T P^-1 v): with x_t = P y_t from t PCG steps on
    # (M + a_1 P) y = v, that residual is v - (M + a_1 P) y_t, formed here
    # explicitly from the PCG iterate.
    n = 90
    M, P = _spd(n, 31, 0.2), _spd(n, 32, 1.0)
    Z = estimate.probes(12, n, 3)
    _, a, _ = rational.partial_fraction(3)
    _, steps, resid = lanczos.per_probe_lanczos(M, P, 3, Z, t)
    assert np.all(steps == t)
    fac = sla.cho_factor(P, lower=True)
    for i in range(Z.shape[1]):
        v = Z[:, i].astype(np.float64)
        y = _pcg_t_steps(M, P, v, a[0], t)
        r = v - (M + a[0] * P) @ y
        want = np.sqrt(r @ sla.cho_solve(fac, r)) / np.sqrt(v @ sla.cho_solve(fac, v))
        assert resid[i] == pytest.approx(want, rel=1e-8)
