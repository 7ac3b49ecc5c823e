"""The estimator of Algorithm 1 (Section 2) with exact shifted solves.

Oracle module (test infrastructure).

The output of Algorithm 1 and its derivation (Section 2) give

    est = log det P + (1/s) sum_i t_i,
    t_i = b z_i^T z_i + sum_j c_j z_i^T (M P^-1 + a_j I)^-1 z_i ,

for r_k(x) = b + sum_j c_j / (x + a_j) (Table 1).  Algorithm 1 reaches the
inner products through t Lanczos steps and tridiagonal solves; the converged
value is the plain definition above, which is what this module computes
[reading: the normalisation is 1/s over the s probes; the derivation prints
1/n in Section 1].  Since (M P^-1 + a I)^-1 = P (M + a P)^-1 and M + a P is
SPD, each inner product is (P z)^T y with (M + a P) y = z, solved by dense
Cholesky.

Also here: the exact log det (Cholesky); the expectation of the estimator
over probes, log det P + sum_i r_k(lambda_i) over the generalized eigenvalues
lambda_i of (M, P), used to split the error into the bias of r_k and the
Hutchinson noise; and a per-shift conjugate gradient solve for sizes where
dense factorizations are too large.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import rational, rng


@dataclass
class Estimate:
    logdet: float
    logdet_P: float
    per_probe: np.ndarray   # t_i, length s
    stderr: float

    @property
    def trace_term(self):
        return float(np.mean(self.per_probe))


def probes(seed: int, n: int, s: int):
    """Rademacher probe block Z (n x s) from the counter stream (Algorithm 1 step 1)."""
    return rng.rademacher(seed, rng.STREAM_PROBES, n, s)


def probes_gaussian(seed: int, n: int, s: int):
    """Standard normal probe block (Algorithm 1 step 1 with D = N(0, 1))."""
    return rng.gaussian(seed, rng.STREAM_PROBES, n, s)


def probes_orthogonal(seed: int, n: int, s: int):
    """'Normal orthogonal' probes (Appendix; orthogonal Monte Carlo): W = Q S
    with Q the n x s orthonormal factor of a standard normal block G (the QR
    factor whose R has a positive diagonal) and S = diag of G's column norms,
    which are chi-distributed with n degrees of freedom and independent of Q
    [reading: the Appendix draws S independently; G's own column norms have
    that distribution and are independent of Q].  Needs s <= n."""
    if s > n:
        raise ValueError("orthogonal probes need s <= n")
    G = probes_gaussian(seed, n, s)
    Q, R = np.linalg.qr(G)
    Q = Q * np.sign(np.diag(R))
    return Q * np.linalg.norm(G, axis=0)


def probe_block(kind: str, seed: int, n: int, s: int):
    return {"rademacher": probes, "gaussian": probes_gaussian,
            "orthogonal": probes_orthogonal}[kind](seed, n, s)


def per_probe_dense(M, P_dense, k: int, Z):
    """t_i for every column of Z with exact (Cholesky) shifted solves."""
    b, a, c = rational.partial_fraction(k)
    t = b * np.sum(Z * Z, axis=0)
    PZ = P_dense @ Z
    for aj, cj in zip(a, c):
        fac = sla.cho_factor(M + aj * P_dense, lower=True)
        Y = sla.cho_solve(fac, Z)
        t = t + cj * np.sum(PZ * Y, axis=0)
    return t


def combine(logdet_P: float, t) -> Estimate:
    t = np.asarray(t, dtype=np.float64)
    s = t.shape[0]
    se = float(np.std(t, ddof=1) / np.sqrt(s)) if s > 1 else float("nan")
    return Estimate(logdet=float(logdet_P + np.mean(t)), logdet_P=float(logdet_P),
                    per_probe=t, stderr=se)


def estimate_dense(M, P_dense, logdet_P: float, k: int, Z) -> Estimate:
    return combine(logdet_P, per_probe_dense(M, P_dense, k, Z))


def logdet_exact(M) -> float:
    """log det M by Cholesky (the paper's accuracy reference, Section 3)."""
    L = sla.cholesky(M, lower=True, check_finite=False)
    return float(2.0 * np.sum(np.log(np.diag(L))))


def generalized_eigs(M, P_dense):
    """Eigenvalues of M P^-1 (= generalized eigenvalues of the pair (M, P))."""
    return sla.eigh(M, P_dense, eigvals_only=True)


def expected_estimate(M, P_dense, logdet_P: float, k: int):
    """E_z[est] = log det P + sum_i r_k(lambda_i): the value the estimator is
    unbiased for (Hutchinson's identity, Section 1), and the bias against
    the exact log det (sum_i log lambda_i) of using r_k in place of log."""
    lam = generalized_eigs(M, P_dense)
    expect = logdet_P + float(np.sum(rational.r_eval(k, lam)))
    bias = float(np.sum(rational.r_eval(k, lam)) - np.sum(np.log(lam)))
    return expect, bias


def per_shift_cg(matvec, precond, z, shift: float, tol: float = 1e-13, maxiter: int = 100000):
    """Preconditioned CG for (M + shift P) y = z, preconditioner P^-1
    (used where dense factorizations do not fit); returns y."""
    y = np.zeros_like(z)
    r = z.copy()
    u = precond.solve(r[:, None])[:, 0]
    p = u.copy()
    rho = float(r @ u)
    nz = np.sqrt(rho)
    for _ in range(maxiter):
        q = matvec(p) + shift * precond.apply(p[:, None])[:, 0]
        alpha = rho / float(p @ q)
        y += alpha * p
        r -= alpha * q
        u = precond.solve(r[:, None])[:, 0]
        rho_new = float(r @ u)
        if np.sqrt(max(rho_new, 0.0)) <= tol * nz:
            break
        p = u + (rho_new / rho) * p
        rho = rho_new
    return y


def logdet_exact_blocked(M, block: int = 2048) -> float:
    """log det M by a right-looking blocked Cholesky that overwrites M
    (lower triangle), for matrices too large for a single LAPACK call.  The
    same factorization as logdet_exact, organised by blocks."""
    n = M.shape[0]
    total = 0.0
    for k0 in range(0, n, block):
        k1 = min(n, k0 + block)
        Lkk = np.linalg.cholesky(M[k0:k1, k0:k1])
        total += 2.0 * float(np.sum(np.log(np.diag(Lkk))))
        if k1 == n:
            break
        # panel below the diagonal block: M[k1:, k0:k1] Lkk^-T
        panel = sla.solve_triangular(Lkk, M[k1:, k0:k1].T, lower=True, check_finite=False).T
        # trailing update of the lower triangle, one column block at a time
        for j0 in range(k1, n, block):
            j1 = min(n, j0 + block)
            M[j0:, j0:j1] -= panel[j0 - k1:, :] @ panel[j0 - k1:j1 - k1, :].T
    return total
