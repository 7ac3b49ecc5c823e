"""Pins for oracle.gradient: the derivative matrices against central finite
differences of oracle.gp, the exact gradient against finite differences of
the exact log det, and Hutchinson's estimator of it (exact for diagonal
matrices' noise component, unbiased over seeds)."""
import numpy as np
import pytest

from oracle import estimate, gp, gradient


@pytest.mark.parametrize("kind", [gp.RBF, gp.MATERN52])
def test_derivative_matrices_match_finite_differences(kind):
    X = np.random.default_rng(1).random((40, 3))
    l, v, s2 = 0.3, 1.4, 1e-2
    dl, dv, dn = gradient.derivative_matrices(kind, X, l, v, s2)
    h = 1e-6
    fd_l = (gp.dense_matrix(kind, X, l + h, v, s2) - gp.dense_matrix(kind, X, l - h, v, s2)) / (2 * h)
    fd_v = (gp.dense_matrix(kind, X, l, v + h, s2) - gp.dense_matrix(kind, X, l, v - h, s2)) / (2 * h)
    fd_n = (gp.dense_matrix(kind, X, l, v, s2 + h) - gp.dense_matrix(kind, X, l, v, s2 - h)) / (2 * h)
    np.testing.assert_allclose(dl, fd_l, atol=1e-8)
    np.testing.assert_allclose(dv, fd_v, atol=1e-8)
    np.testing.assert_allclose(dn, fd_n, atol=1e-8)


@pytest.mark.parametrize("kind", [gp.RBF, gp.MATERN52])
def test_exact_gradient_is_the_derivative_of_log_det(kind):
    X = np.random.default_rng(2).random((120, 3))
    l, v, s2 = 0.25, 0.9, 3e-2
    M = gp.dense_matrix(kind, X, l, v, s2)
    g = gradient.gradient_exact(M, gradient.derivative_matrices(kind, X, l, v, s2))
    h = 1e-6
    ld = lambda l_, v_, s_: estimate.logdet_exact(gp.dense_matrix(kind, X, l_, v_, s_))  # noqa: E731
    fd = [(ld(l + h, v, s2) - ld(l - h, v, s2)) / (2 * h),
          (ld(l, v + h, s2) - ld(l, v - h, s2)) / (2 * h),
          (ld(l, v, s2 + h) - ld(l, v, s2 - h)) / (2 * h)]
    np.testing.assert_allclose(g, fd, rtol=1e-6)


def test_noise_component_exact_for_diagonal_matrix():
    # M diagonal: (M^-1 z)^T z = sum z_k^2 / m_k = sum 1 / m_k for +-1 probes
    m = np.random.default_rng(3).uniform(0.5, 4.0, 30)
    Z = estimate.probes(4, 30, 5)
    g = gradient.per_probe_gradient(np.diag(m), [np.eye(30)], Z)
    np.testing.assert_allclose(g[0], np.sum(1.0 / m), rtol=1e-13)


def test_unbiased_over_seeds():
    X = np.random.default_rng(5).random((60, 3))
    l, v, s2 = 0.3, 1.0, 5e-2
    M = gp.dense_matrix(gp.MATERN52, X, l, v, s2)
    dMs = gradient.derivative_matrices(gp.MATERN52, X, l, v, s2)
    exact = gradient.gradient_exact(M, dMs)
    means = np.array([gradient.gradient_estimate(M, dMs, estimate.probes(sd, 60, 4))[0]
                      for sd in range(300)])
    se = means.std(axis=0, ddof=1) / np.sqrt(len(means))
    assert np.all(np.abs(means.mean(axis=0) - exact) < 4 * se)
