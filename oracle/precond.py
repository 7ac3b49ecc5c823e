"""Preconditioners P = D + U diag(lam) U^T: the randomized truncated SVD of
Section 2 (a simplified randomized SVD after Halko et al., range finder of
their Algorithm 4.1 and the eigen-decomposition of the projected matrix of
their Algorithm 5.3; Appendix, "Truncated Randomized SVD"), and the other
members of the Appendix's list (identity, diagonal, rank one, partial
Cholesky, each "plus scaling" variant) at the end of this module.

Oracle module (test infrastructure).  Steps, in the order the method takes
them (readings of the paper in brackets):

  1. Omega = n x (rank + oversample) standard normal test matrix [drawn from
     the counter stream of oracle.rng, stream 1].
  2. Y = M Omega; Q = orth(Y)                      (range finder)
  3. power_iters times: Y = M Q; Q = orth(Y)      [subspace iteration]
  4. B = Q^T M Q, symmetrized; eigenpairs of B    (projected problem)
  5. keep the `rank` largest: lam, U = Q V        (truncated SVD; M is SPD so
                                                  singular values = eigenvalues)
  6. D = diag(M) - sum_j lam_j U_{.j}^2, floored  [the paper never defines D for
     this preconditioner; the reading follows its rank-one and partial
     Cholesky variants, D = diag(M - low-rank part), floored at the noise
     variance so that P stays positive definite]

log det P follows from the matrix determinant lemma,
    log det P = sum log D + sum log lam + log det(diag(1/lam) + U^T D^-1 U),
or, for small n, directly from the dense P (both are provided; the tests
check that they agree).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import rng


def d_floor(noise: float, variance: float) -> float:
    """Lower bound applied to the diagonal part D (a reading; see step 6)."""
    return noise if noise > 0.0 else 1e-12 * variance


@dataclass
class Precond:
    U: np.ndarray      # n x rank, orthonormal columns
    lam: np.ndarray    # rank, descending, > 0
    D: np.ndarray      # n, > 0
    logdet: float
    ritz: np.ndarray | None = None  # all rank + oversample Ritz values, descending

    def dense(self):
        return np.diag(self.D) + (self.U * self.lam) @ self.U.T

    def apply(self, V):
        """P V (V is n x s)."""
        return self.D[:, None] * V + (self.U * self.lam) @ (self.U.T @ V)

    def solve(self, R):
        """P^-1 R by the Woodbury identity (R is n x s)."""
        Dinv_R = R / self.D[:, None]
        if self.lam.size == 0:
            return Dinv_R
        C = np.diag(1.0 / self.lam) + self.U.T @ (self.U / self.D[:, None])
        t = np.linalg.solve(C, self.U.T @ Dinv_R)
        return Dinv_R - (self.U / self.D[:, None]) @ t


def orth(Y):
    Q, _ = np.linalg.qr(Y)
    return Q


def logdet_lemma(U, lam, D):
    if lam.size == 0:
        return float(np.sum(np.log(D)))
    C = np.diag(1.0 / lam) + U.T @ (U / D[:, None])
    sign, ld_c = np.linalg.slogdet(C)
    if sign <= 0:
        raise np.linalg.LinAlgError("capacitance matrix not positive definite")
    return float(np.sum(np.log(D)) + np.sum(np.log(lam)) + ld_c)


def rsvd(M, rank: int, oversample: int, power_iters: int, seed: int, floor: float):
    n = M.shape[0]
    m = rank + oversample
    if not (1 <= rank and m <= n):
        raise ValueError("need 1 <= rank and rank + oversample <= n")
    omega = rng.gaussian(seed, rng.STREAM_OMEGA, n, m)
    Q = orth(M @ omega)
    for _ in range(power_iters):
        Q = orth(M @ Q)
    B = Q.T @ (M @ Q)
    B = 0.5 * (B + B.T)
    theta, V = np.linalg.eigh(B)
    order = np.argsort(theta)[::-1][:rank]
    lam = theta[order]
    if np.any(lam <= 0):
        raise np.linalg.LinAlgError("projected matrix not positive definite")
    U = Q @ V[:, order]
    D = np.diag(M) - (U * U) @ lam
    D = np.maximum(D, floor)
    return Precond(U=U, lam=lam, D=D, logdet=logdet_lemma(U, lam, D),
                   ritz=np.sort(theta)[::-1].copy())


# ---------------------------------------------------------------------------
# The Appendix's other preconditioners.  Readings: where the Appendix takes D
# as the diagonal of M minus the low-rank part, D is floored at `floor` (the
# noise variance) as for the randomized SVD; "plus scaling" replaces D by
# a I with a = the noise variance (this build has no separate jitter); the
# rank-one preconditioner's top eigenpair is the randomized SVD's of rank 1;
# the partial Cholesky factorization is the greedy pivoted one (pivot = the
# largest remaining diagonal entry, lowest index on ties), and its D is
# diag(M - C C^T) (the printed formula is garbled).

def _with(U, lam, D):
    return Precond(U=U, lam=lam, D=D, logdet=logdet_lemma(U, lam, D))


def identity(n: int):
    """P = I."""
    return _with(np.zeros((n, 0)), np.zeros(0), np.ones(n))


def diagonal(M):
    """P = diag(M)."""
    n = M.shape[0]
    return _with(np.zeros((n, 0)), np.zeros(0), np.diag(M).copy())


def rank_one(M, oversample: int, power_iters: int, seed: int, floor: float):
    """P = D + lam v v^T, (lam, v) the top eigenpair, D = diag(M - lam v v^T)."""
    return rsvd(M, 1, oversample, power_iters, seed, floor)


def partial_cholesky_factor(M, rank: int):
    """Greedy pivoted partial Cholesky: C (n x rank) with C C^T matching M on
    the pivot rows and columns, and the pivot sequence."""
    n = M.shape[0]
    C = np.zeros((n, rank))
    res = np.diag(M).astype(np.float64).copy()
    piv = []
    for k in range(rank):
        p = int(np.argmax(res))          # first index of the largest value
        piv.append(p)
        col = (M[:, p] - C[:, :k] @ C[p, :k]) / np.sqrt(res[p])
        C[:, k] = col
        res = res - col * col
        res[p] = 0.0
    return C, np.array(piv)


def partial_cholesky(M, rank: int, floor: float):
    """P = D + C C^T with C the rank-`rank` pivoted partial Cholesky factor and
    D = diag(M - C C^T) floored."""
    C, _ = partial_cholesky_factor(M, rank)
    D = np.maximum(np.diag(M) - np.sum(C * C, axis=1), floor)
    return _with(C, np.ones(rank), D)


def scaled(P: Precond, a: float):
    """The "plus scaling" variant of P: D replaced by a I."""
    return _with(P.U, P.lam, np.full(P.D.shape, float(a)))
