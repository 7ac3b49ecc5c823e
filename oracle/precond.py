"""Randomized truncated-SVD preconditioner P = D + U diag(lam) U^T
(Section 2: a simplified randomized SVD after Halko et al., range finder of
their Algorithm 4.1 and the eigen-decomposition of the projected matrix of
their Algorithm 5.3; Appendix, "Truncated Randomized SVD").

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
        C = np.diag(1.0 / self.lam) + self.U.T @ (self.U / self.D[:, None])
        t = np.linalg.solve(C, self.U.T @ Dinv_R)
        return Dinv_R - (self.U / self.D[:, None]) @ t


def orth(Y):
    Q, _ = np.linalg.qr(Y)
    return Q


def logdet_lemma(U, lam, D):
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
