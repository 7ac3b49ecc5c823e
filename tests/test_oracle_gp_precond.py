"""Pins for oracle.gp (the Section 3 covariance kernels) and oracle.precond
(the randomized truncated-SVD preconditioner of Section 2 / Appendix)."""
import numpy as np
import pytest
from sklearn.gaussian_process import kernels as skk

from oracle import gp, precond, rng


def test_kernel_closed_forms():
    l, v = 0.3, 1.7
    assert gp.kernel_of_r(gp.RBF, 0.0, l, v) == pytest.approx(v, rel=1e-15)
    assert gp.kernel_of_r(gp.MATERN52, 0.0, l, v) == pytest.approx(v, rel=1e-15)
    assert gp.kernel_of_r(gp.RBF, l, l, v) == pytest.approx(v * np.exp(-0.5), rel=1e-15)
    s5 = np.sqrt(5.0)
    assert gp.kernel_of_r(gp.MATERN52, l, l, v) == pytest.approx(
        v * (1 + s5 + 5.0 / 3.0) * np.exp(-s5), rel=1e-15)


@pytest.mark.parametrize("kind", [gp.RBF, gp.MATERN52])
def test_kernel_matches_library_routine(kind):
    g = np.random.default_rng(0)
    X = g.random((40, 3))
    l, v = 0.27, 1.3
    ref = skk.RBF(length_scale=l)(X) if kind == gp.RBF else skk.Matern(length_scale=l, nu=2.5)(X)
    M = gp.dense_matrix(kind, X, l, v, 0.0)
    np.testing.assert_allclose(M, v * ref, rtol=1e-13, atol=1e-15)


def test_dense_matrix_spd_and_noise():
    g = np.random.default_rng(1)
    X = g.random((300, 3))
    M = gp.dense_matrix(gp.MATERN52, X, 0.2, 1.0, 1e-3)
    np.testing.assert_array_equal(M, M.T)
    np.testing.assert_allclose(np.diag(M), 1.0 + 1e-3, rtol=1e-15)
    np.linalg.cholesky(M)
    rows = gp.kernel_rows(gp.MATERN52, X, np.array([3, 299]), 0.2, 1.0, 1e-3)
    np.testing.assert_array_equal(rows, M[[3, 299]])


def _lowrank_plus_noise(n, rank, sigma2, seed):
    g = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(g.standard_normal((n, rank)))
    lam = np.sort(g.uniform(1.0, 50.0, rank))[::-1]
    return (Q * lam) @ Q.T + sigma2 * np.eye(n), Q, lam


def test_low_rank_plus_noise_closed_form():
    # M = Q diag(lam) Q^T + s2 I with rank(Q) = l: the range finder with power
    # iterations captures range(Q), so the kept eigenvalues are lam + s2 and
    # U spans range(Q).  Then diag(M) - diag(U (lam + s2) U^T) = s2 (1 - |Q_i|^2)
    # falls below the floor s2, so D = s2 I and P = M + s2 Q Q^T exactly.
    n, r, s2 = 300, 12, 1e-3
    M, Q, lam = _lowrank_plus_noise(n, r, s2, 2)
    P = precond.rsvd(M, rank=r, oversample=5, power_iters=2, seed=3, floor=s2)
    np.testing.assert_allclose(P.lam, lam + s2, rtol=1e-12)
    np.testing.assert_array_equal(P.D, np.full(n, s2))
    np.testing.assert_allclose(P.dense(), M + s2 * (Q @ Q.T), atol=1e-11)
    expect = np.sum(np.log(lam + 2 * s2)) + (n - r) * np.log(s2)
    assert P.logdet == pytest.approx(expect, rel=1e-12)


def test_logdet_lemma_matches_dense_and_woodbury_solve():
    g = np.random.default_rng(4)
    X = g.random((400, 3))
    M = gp.dense_matrix(gp.RBF, X, 0.2, 1.0, 1e-2)
    P = precond.rsvd(M, rank=30, oversample=10, power_iters=2, seed=5, floor=1e-2)
    Pd = P.dense()
    sign, ld = np.linalg.slogdet(Pd)
    assert sign > 0 and P.logdet == pytest.approx(ld, rel=1e-12)
    V = g.standard_normal((400, 3))
    np.testing.assert_allclose(P.solve(P.apply(V)), V, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(P.apply(V), Pd @ V, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(P.U.T @ P.U, np.eye(30), atol=1e-12)
    # unfloored entries keep diag(P) = diag(M)
    low = (P.U * P.U) @ P.lam
    keep = np.diag(M) - low > 1e-2
    np.testing.assert_allclose(np.diag(Pd)[keep], np.diag(M)[keep], rtol=1e-12)


def test_rsvd_approaches_best_rank_l():
    # For a kernel matrix with fast spectral decay the randomized SVD with
    # power iterations captures the top eigenvalues (Halko et al.).
    g = np.random.default_rng(6)
    X = g.random((500, 2))
    M = gp.dense_matrix(gp.RBF, X, 0.3, 1.0, 1e-3)
    ev = np.sort(np.linalg.eigvalsh(M))[::-1]
    P = precond.rsvd(M, rank=20, oversample=10, power_iters=2, seed=7, floor=1e-3)
    np.testing.assert_allclose(P.lam[:12], ev[:12], rtol=1e-12)
    np.testing.assert_allclose(P.lam, ev[:20], rtol=1e-4)


def test_rsvd_uses_gaussian_stream():
    # Omega must be the stream-1 Gaussian block: the rank-(l+p) projection
    # with zero power iterations spans M @ Omega exactly.
    g = np.random.default_rng(8)
    X = g.random((120, 3))
    M = gp.dense_matrix(gp.RBF, X, 0.4, 1.0, 1e-2)
    P = precond.rsvd(M, rank=15, oversample=0, power_iters=0, seed=11, floor=1e-2)
    Y = M @ rng.gaussian(11, rng.STREAM_OMEGA, 120, 15)
    proj = P.U @ (P.U.T @ Y)
    np.testing.assert_allclose(proj, Y, rtol=1e-9, atol=1e-9 * np.abs(Y).max())
