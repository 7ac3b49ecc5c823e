"""Reference for the learned surrogate of the trace term (FP64, numpy).

Oracle module (test infrastructure).

The surrogate is not in the paper; its definition is the one the library
documents: an MLP 38 -> 256 -> 256 -> 256 -> 1 with GELU (erf form) after
the first three layers, inputs standardised by (x - mean) / std, target
standardised by (y - y_mean) / y_std, loss = mean squared error on the
standardised target, Adam with bias correction.  This module writes those
definitions out directly: a forward pass, the gradient by the chain rule,
one Adam step, and the feature vector (kind, log lengthscale, log variance,
log noise, log n, d, and the normalised histogram of log(lambda_j / n) in 32
equal bins between fixed edges, values outside falling in the end bins).

Parameters are handled as the flat vector the library exports: tensors W1
(38 x 256), b1, W2 (256 x 256), b2, W3, b3, w4 (256), b4, in this order, each
starting at a multiple of 64 floats.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

NF, W, BINS = 38, 256, 32


def _a64(x: int) -> int:
    return (x + 63) // 64 * 64


def layout():
    """(name, offset, shape) of each tensor in the flat parameter vector."""
    shapes = [("W1", (NF, W)), ("b1", (W,)), ("W2", (W, W)), ("b2", (W,)), ("W3", (W, W)),
              ("b3", (W,)), ("w4", (W,)), ("b4", (1,))]
    out, off = [], 0
    for name, shp in shapes:
        off = _a64(off)
        out.append((name, off, shp))
        off += int(np.prod(shp))
    return out


def param_count() -> int:
    name, off, shp = layout()[-1]
    return off + int(np.prod(shp))


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return {name: p[off:off + int(np.prod(shp))].reshape(shp) for name, off, shp in layout()}


def pack(t: dict):
    p = np.zeros(param_count())
    for name, off, shp in layout():
        p[off:off + int(np.prod(shp))] = np.asarray(t[name], dtype=np.float64).ravel()
    return p


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(p, X, x_mean, x_std, y_mean=0.0, y_std=1.0, standardised=False):
    """Prediction for rows of X (raw features); the standardised output when
    standardised=True, else de-standardised."""
    t = unpack(p)
    Xs = (np.asarray(X, dtype=np.float64) - x_mean) / x_std
    h = gelu(Xs @ t["W1"] + t["b1"])
    h = gelu(h @ t["W2"] + t["b2"])
    h = gelu(h @ t["W3"] + t["b3"])
    y = h @ t["w4"] + t["b4"][0]
    return y if standardised else y_mean + y_std * y


def loss_and_grad(p, X, target, x_mean, x_std, y_mean=0.0, y_std=1.0):
    """Mean squared error on the standardised target and its gradient with
    respect to the flat parameter vector (chain rule, layer by layer)."""
    t = unpack(p)
    Xs = (np.asarray(X, dtype=np.float64) - x_mean) / x_std
    ts = (np.asarray(target, dtype=np.float64) - y_mean) / y_std
    B = Xs.shape[0]
    z1 = Xs @ t["W1"] + t["b1"]
    h1 = gelu(z1)
    z2 = h1 @ t["W2"] + t["b2"]
    h2 = gelu(z2)
    z3 = h2 @ t["W3"] + t["b3"]
    h3 = gelu(z3)
    y = h3 @ t["w4"] + t["b4"][0]
    r = y - ts
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B
    g = {"w4": h3.T @ dy, "b4": np.array([dy.sum()])}
    dz3 = np.outer(dy, t["w4"]) * gelu_grad(z3)
    g["W3"], g["b3"] = h2.T @ dz3, dz3.sum(0)
    dz2 = (dz3 @ t["W3"].T) * gelu_grad(z2)
    g["W2"], g["b2"] = h1.T @ dz2, dz2.sum(0)
    dz1 = (dz2 @ t["W2"].T) * gelu_grad(z1)
    g["W1"], g["b1"] = Xs.T @ dz1, dz1.sum(0)
    return loss, pack(g)


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def features(lam, kind, lengthscale, variance, noise, n, d, edges):
    lam = np.asarray(lam, dtype=np.float64)
    f = np.zeros(NF)
    f[:6] = [kind, np.log(lengthscale), np.log(variance), np.log(noise), np.log(n), d]
    width = (edges[BINS] - edges[0]) / BINS
    b = np.floor((np.log(lam / n) - edges[0]) / width).astype(int)
    b = np.clip(b, 0, BINS - 1)
    f[6:] = np.bincount(b, minlength=BINS) / len(lam)
    return f
