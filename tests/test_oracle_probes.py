"""Pins for the probe types of oracle.estimate (Algorithm 1 step 1 with a
mean-0 variance-1 distribution D; Appendix 'normal orthogonal' probes):
moments, orthogonality, the estimator's exact per-probe form for diagonal
matrices, and unbiasedness over seeds."""
import numpy as np
import pytest

from oracle import estimate, rational


def test_gaussian_probe_moments():
    Z = estimate.probes_gaussian(3, 4000, 50)
    assert abs(Z.mean()) < 0.01 and abs(Z.var() - 1.0) < 0.01


def test_orthogonal_probes_are_orthogonal_with_chi_norms():
    n, s = 300, 40
    W = estimate.probes_orthogonal(4, n, s)
    G = estimate.probes_gaussian(4, n, s)
    Gram = W.T @ W
    np.testing.assert_allclose(Gram, np.diag(np.sum(G * G, axis=0)), atol=1e-9)
    # the unit directions are the QR factor of G with a positive R diagonal
    Q = W / np.linalg.norm(W, axis=0)
    R = Q.T @ G
    np.testing.assert_allclose(np.tril(R, -1), 0.0, atol=1e-10)
    assert np.all(np.diag(R) > 0)
    with pytest.raises(ValueError):
        estimate.probes_orthogonal(4, 10, 11)


def test_orthogonal_probe_marginals_over_seeds():
    # each column is marginally N(0, I): E[w_k^2] = 1 entrywise
    n, s = 30, 6
    acc = np.zeros((n, s))
    for seed in range(400):
        acc += estimate.probes_orthogonal(seed, n, s) ** 2
    assert abs(acc.mean() / 400 - 1.0) < 0.03


@pytest.mark.parametrize("kind", ["gaussian", "orthogonal"])
def test_diagonal_matrices_per_probe_form(kind):
    # for diagonal M and P, z^T f(M P^-1) z = sum_i f(m_i / p_i) z_i^2 for any z
    g = np.random.default_rng(7)
    n = 60
    m = g.uniform(0.2, 9.0, n)
    p = g.uniform(0.5, 3.0, n)
    Z = estimate.probe_block(kind, 5, n, 8)
    est = estimate.estimate_dense(np.diag(m), np.diag(p), float(np.sum(np.log(p))), 3, Z)
    want = rational.r_eval(3, m / p) @ (Z * Z)
    np.testing.assert_allclose(est.per_probe, want, rtol=1e-12)


@pytest.mark.parametrize("kind", ["gaussian", "orthogonal"])
def test_unbiased_over_seeds(kind):
    g = np.random.default_rng(8)
    n = 40
    A = g.standard_normal((n, n))
    M = A @ A.T / n + 0.5 * np.eye(n)
    P = np.diag(np.diag(M))
    ldP = float(np.sum(np.log(np.diag(P))))
    expect, _ = estimate.expected_estimate(M, P, ldP, 3)
    vals = [estimate.estimate_dense(M, P, ldP, 3, estimate.probe_block(kind, sd, n, 4)).logdet
            for sd in range(300)]
    se = np.std(vals, ddof=1) / np.sqrt(len(vals))
    assert abs(np.mean(vals) - expect) < 4 * se
