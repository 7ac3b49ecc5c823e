"""Gradient of log det M with respect to the kernel hyperparameters by
Hutchinson's estimator over probe solves (the CG-based gradient the paper
cites as its tuning objective's derivative, Section 3).

Oracle module (test infrastructure).

    d log det M / d theta = tr(M^-1 dM/dtheta)
                          ~ (1/s) sum_i (M^-1 z_i)^T (dM/dtheta) z_i

for theta in (lengthscale, variance, noise) of M = K + noise I with the
kernels of oracle.gp:
    dM/d noise    = I
    dM/d variance = K / variance
    dM/d l:  RBF        k(r) r^2 / l^3
             Matern-5/2 variance t^2 (1 + t) e^-t / (3 l),  t = sqrt5 r / l
The solves here are dense Cholesky solves; the exact gradient is the trace
itself.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import gp

PARAMS = ("lengthscale", "variance", "noise")


def _distances(X):
    X = np.asarray(X, dtype=np.float64)
    diff = X[:, None, :] - X[None, :, :]
    return np.sqrt(np.sum(diff * diff, axis=-1))


def dK_dlengthscale(kind, X, lengthscale, variance):
    r = _distances(X)
    if kind == gp.RBF:
        return gp.kernel_of_r(kind, r, lengthscale, variance) * r * r / lengthscale ** 3
    t = np.sqrt(5.0) * r / lengthscale
    return variance * t * t * (1.0 + t) * np.exp(-t) / (3.0 * lengthscale)


def derivative_matrices(kind, X, lengthscale, variance, noise):
    """dM/dtheta for theta = lengthscale, variance, noise."""
    n = len(X)
    K = gp.dense_matrix(kind, X, lengthscale, variance, 0.0)
    return (dK_dlengthscale(kind, X, lengthscale, variance), K / variance, np.eye(n))


def gradient_exact(M, dMs):
    fac = sla.cho_factor(M, lower=True)
    return np.array([float(np.trace(sla.cho_solve(fac, A))) for A in dMs])


def per_probe_gradient(M, dMs, Z):
    """g[p, i] = (M^-1 z_i)^T (dM_p z_i) for each parameter p and probe i."""
    fac = sla.cho_factor(M, lower=True)
    Y = sla.cho_solve(fac, Z)
    return np.array([np.sum(Y * (A @ Z), axis=0) for A in dMs])


def gradient_estimate(M, dMs, Z):
    """Hutchinson mean and standard error of each component."""
    g = per_probe_gradient(M, dMs, Z)
    s = Z.shape[1]
    se = np.std(g, axis=1, ddof=1) / np.sqrt(s) if s > 1 else np.full(len(dMs), np.nan)
    return g.mean(axis=1), se, g
