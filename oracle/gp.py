"""Gaussian-process covariance matrices used in the paper's experiments
(Section 3: Matern-5/2 and RBF kernels, citing Williams & Rasmussen).

Oracle module (test infrastructure).  The paper does not print the kernel
formulas; the textbook forms are used (a reading):

    RBF:        k(r) = s2 * exp(-r^2 / (2 l^2))
    Matern-5/2: k(r) = s2 * (1 + sqrt5 r / l + 5 r^2 / (3 l^2)) * exp(-sqrt5 r / l)

with r = ||x_i - x_j|| (differences taken directly, no norm expansion),
s2 the signal variance and l the lengthscale.  The matrix whose log det is
estimated is M = K + noise * I.
"""
from __future__ import annotations

import numpy as np

RBF = 0
MATERN52 = 1


def kernel_of_r(kind: int, r, lengthscale: float, variance: float):
    r = np.asarray(r, dtype=np.float64)
    if kind == RBF:
        return variance * np.exp(-(r * r) / (2.0 * lengthscale * lengthscale))
    if kind == MATERN52:
        t = np.sqrt(5.0) * r / lengthscale
        return variance * (1.0 + t + t * t / 3.0) * np.exp(-t)
    raise ValueError(f"unknown kernel kind {kind}")


def pairwise_r(X, Y=None):
    X = np.asarray(X, dtype=np.float64)
    Y = X if Y is None else np.asarray(Y, dtype=np.float64)
    diff = X[:, None, :] - Y[None, :, :]
    return np.sqrt(np.sum(diff * diff, axis=-1))


def kernel_rows(kind, X, rows, lengthscale, variance, noise):
    """Rows `rows` of M = K + noise I, shape (len(rows), n)."""
    X = np.asarray(X, dtype=np.float64)
    rows = np.asarray(rows)
    R = pairwise_r(X[rows], X)
    out = kernel_of_r(kind, R, lengthscale, variance)
    out[np.arange(len(rows)), rows] += noise
    return out


def dense_matrix(kind, X, lengthscale, variance, noise):
    """The full M = K + noise I in FP64."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    block = max(1, (1 << 24) // (n * d))
    M = np.empty((n, n), dtype=np.float64)
    for i0 in range(0, n, block):
        rows = np.arange(i0, min(n, i0 + block))
        M[i0:i0 + len(rows)] = kernel_rows(kind, X, rows, lengthscale, variance, noise)
    return M
