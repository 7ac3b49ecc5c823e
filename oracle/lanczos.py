"""Algorithm 1 as printed (Section 2): t Lanczos steps on M P^-1 for each
probe, a tridiagonal solve per pole, and the output
    log det P + (1/s) sum_i v_i^T (b v_i + sum_j c_j Q^T w_ij).

Oracle module (test infrastructure).

Readings of the paper (it prints the steps but not the inner product):
  * M P^-1 is not symmetric; it is self-adjoint in <x, y> = x^T P^-1 y, so
    the Lanczos recurrence runs in that inner product.  The Lanczos vectors
    q_1 .. q_t are P^-1-orthonormal, q_1 = v / |v| with |v| = sqrt(v^T P^-1 v),
    and T is the t x t tridiagonal matrix of the recurrence
        M P^-1 q_l = beta_{l-1} q_{l-1} + alpha_l q_l + beta_l q_{l+1}.
  * Step 3's system is (T + a_j I) w = |v| e_1 with a_j = -alpha_j of the
    partial fractions (Table 1): its right side holds the P^-1 products
    <q_l, v>, which are |v| e_1 because v starts the recurrence (the
    derivation's "Q b = |b| e_1").
  * The output's v^T Q^T w is sum_l (v^T q_l) w_l with Euclidean products
    v^T q_l, so that with t = n it equals v^T (M P^-1 + a_j I)^-1 v, the
    per-probe value of the estimator's definition (oracle.estimate).
  * The normalisation is 1/s over the probes.
  * A probe whose recurrence reaches an invariant subspace (beta_l <= 1e-12
    times the largest |alpha| so far) stops there; its T is the leading l x l
    block, which then solves the shifted systems exactly.

The shifted tridiagonal systems are solved here by a dense solve (the paper
uses the Thomas algorithm; the result is the same).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import rational
from .estimate import combine

BREAKDOWN = 1e-12


def lanczos(matvec, psolve, v, t: int):
    """t steps of Lanczos on A = matvec(psolve(.)) in the P^-1 inner product,
    started at v.  Returns (alpha, beta, g, norm_v, steps) with alpha (steps),
    beta (steps; beta[l] couples q_{l+1} and q_{l+2}, the last one is the
    residual coefficient of the final step), g[l] = v^T q_{l+1} and
    norm_v = sqrt(v^T P^-1 v)."""
    u = psolve(v)
    norm_v = float(np.sqrt(v @ u))
    q = v / norm_v
    u = u / norm_v
    q_prev = np.zeros_like(v)
    beta_prev = 0.0
    alpha, beta, g = [], [], [float(v @ q)]
    amax = 0.0
    for _ in range(t):
        y = matvec(u)                      # M P^-1 q_l
        a = float(u @ y)                   # <q_l, M P^-1 q_l>_{P^-1}
        alpha.append(a)
        amax = max(amax, abs(a))
        r = y - a * q - beta_prev * q_prev
        ur = psolve(r)
        b = float(np.sqrt(max(r @ ur, 0.0)))
        beta.append(b)
        if b <= BREAKDOWN * amax:
            break
        q_prev, q = q, r / b
        u = ur / b
        beta_prev = b
        g.append(float(v @ q))
    steps = len(alpha)
    return (np.array(alpha), np.array(beta), np.array(g[:steps]), norm_v, steps)


def tridiag(alpha, beta):
    m = len(alpha)
    T = np.diag(alpha)
    if m > 1:
        T += np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
    return T


def per_probe_lanczos(M, P_dense, k: int, Z, t: int):
    """Per-probe values b v^T v + sum_j c_j (Q v)^T w_j of Algorithm 1, with
    the number of Lanczos steps each probe took and the P^-1-norm residual
    of its smallest-shift system relative to |v| (beta_t |w_t| / |v|)."""
    b, a, c = rational.partial_fraction(k)
    fac = sla.cho_factor(P_dense, lower=True)
    psolve = lambda x: sla.cho_solve(fac, x)  # noqa: E731
    matvec = lambda x: M @ x                 # noqa: E731
    s = Z.shape[1]
    out = np.empty(s)
    steps = np.empty(s, dtype=int)
    resid = np.empty(s)
    for i in range(s):
        v = Z[:, i].astype(np.float64)
        al, be, g, nv, m = lanczos(matvec, psolve, v, t)
        T = tridiag(al, be)
        e1 = np.zeros(m)
        e1[0] = nv
        val = b * float(v @ v)
        for aj, cj in zip(a, c):
            w = np.linalg.solve(T + aj * np.eye(m), e1)
            val += cj * float(g @ w)
        w0 = np.linalg.solve(T + a[0] * np.eye(m), e1)
        resid[i] = be[m - 1] * abs(w0[-1]) / nv
        out[i] = val
        steps[i] = m
    return out, steps, resid


def estimate_lanczos(M, P_dense, logdet_P: float, k: int, Z, t: int):
    t_i, steps, resid = per_probe_lanczos(M, P_dense, k, Z, t)
    return combine(logdet_P, t_i), steps, resid
