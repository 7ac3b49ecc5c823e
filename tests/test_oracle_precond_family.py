"""Pins for the Appendix's preconditioner list in oracle.precond: identity,
diagonal, rank one, greedy pivoted partial Cholesky and the "plus scaling"
variants, checked against their definitions (dense algebra, eigenvalues,
exact low-rank recovery, the Nystrom interpolation property of pivoted
Cholesky)."""
import numpy as np
import pytest

from oracle import gp, precond


def _kernel(n=300, seed=3, ls=0.3, noise=1e-2):
    X = np.random.default_rng(seed).random((n, 3))
    return gp.dense_matrix(gp.MATERN52, X, ls, 1.0, noise)


def test_identity_and_diagonal():
    M = _kernel()
    R = np.random.default_rng(1).standard_normal((M.shape[0], 4))
    I = precond.identity(M.shape[0])
    np.testing.assert_array_equal(I.solve(R), R)
    assert I.logdet == 0.0
    Dg = precond.diagonal(M)
    np.testing.assert_array_equal(Dg.dense(), np.diag(np.diag(M)))
    np.testing.assert_allclose(Dg.solve(R), R / np.diag(M)[:, None], rtol=1e-15)
    assert Dg.logdet == pytest.approx(np.sum(np.log(np.diag(M))), rel=1e-14)


def test_rank_one_is_the_top_eigenpair():
    M = _kernel()
    # with 12 power iterations the sketch's top Ritz pair is the top
    # eigenpair to rounding (lambda_2 / lambda_1 = 0.49 here)
    P = precond.rank_one(M, 10, 12, 7, 1e-2)
    w, V = np.linalg.eigh(M)
    assert P.lam.shape == (1,)
    assert P.lam[0] == pytest.approx(w[-1], rel=1e-13)
    assert abs(abs(P.U[:, 0] @ V[:, -1]) - 1.0) < 1e-13
    np.testing.assert_allclose(P.D, np.maximum(np.diag(M) - w[-1] * V[:, -1] ** 2, 1e-2),
                               rtol=1e-11)


def test_partial_cholesky_full_rank_is_a_pivoted_cholesky():
    M = _kernel(n=40, ls=0.5, noise=1e-1)
    C, piv = precond.partial_cholesky_factor(M, 40)
    np.testing.assert_allclose(C @ C.T, M, atol=1e-12)
    assert sorted(piv.tolist()) == list(range(40))
    Cp = C[piv]                       # lower triangular in pivot order
    assert np.max(np.abs(np.triu(Cp, 1))) < 1e-12


def test_partial_cholesky_recovers_low_rank_and_interpolates():
    W = np.random.default_rng(5).standard_normal((50, 3))
    M = W @ W.T
    C, piv = precond.partial_cholesky_factor(M, 3)
    np.testing.assert_allclose(C @ C.T, M, atol=1e-10)
    Mk = _kernel(n=200, seed=6)
    C, piv = precond.partial_cholesky_factor(Mk, 25)
    # C C^T reproduces M exactly on the pivot rows (Nystrom interpolation)
    np.testing.assert_allclose((C @ C.T)[piv], Mk[piv], atol=1e-12)


def test_partial_cholesky_pivot_rule():
    M = _kernel(n=120, seed=8)
    C, piv = precond.partial_cholesky_factor(M, 3)
    assert piv[0] == 0                # stationary kernel: every diagonal entry ties
    res = np.diag(M) - M[:, 0] ** 2 / M[0, 0]
    assert piv[1] == int(np.argmax(res))


@pytest.mark.parametrize("scale", [False, True])
def test_partial_cholesky_preconditioner_woodbury_and_logdet(scale):
    M = _kernel(n=250, seed=9)
    P = precond.partial_cholesky(M, 30, 1e-2)
    if scale:
        P = precond.scaled(P, 1e-2)
        np.testing.assert_array_equal(P.D, 1e-2)
    Pd = P.dense()
    R = np.random.default_rng(2).standard_normal((250, 3))
    np.testing.assert_allclose(P.solve(R), np.linalg.solve(Pd, R), rtol=1e-9, atol=1e-9)
    assert P.logdet == pytest.approx(np.linalg.slogdet(Pd)[1], rel=1e-11)
    C, _ = precond.partial_cholesky_factor(M, 30)
    if not scale:
        np.testing.assert_allclose(P.D, np.maximum(np.diag(M - C @ C.T), 1e-2), rtol=1e-12)
