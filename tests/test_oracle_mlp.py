"""Pins of the surrogate reference (oracle/mlp.py): the GELU identities, the
chain-rule gradient against central finite differences in FP64 for every
parameter tensor, Adam's first step in closed form, and the feature
histogram on hand-made inputs."""
import numpy as np
import pytest

from oracle import mlp


def test_layout_matches_documented_packing():
    names = [n for n, _, _ in mlp.layout()]
    assert names == ["W1", "b1", "W2", "b2", "W3", "b3", "w4", "b4"]
    assert all(off % 64 == 0 for _, off, _ in mlp.layout())
    # 38*256 + 256 + 2*(256*256 + 256) + 256 + 1 values plus alignment padding
    assert mlp.param_count() >= 38 * 256 + 256 + 2 * (65536 + 256) + 257


def test_gelu_identities():
    x = np.linspace(-6, 6, 101)
    # Phi(x) + Phi(-x) = 1  =>  gelu(x) - gelu(-x) = x
    np.testing.assert_allclose(mlp.gelu(x) - mlp.gelu(-x), x, atol=1e-14)
    assert mlp.gelu(0.0) == 0.0
    assert abs(mlp.gelu(10.0) - 10.0) < 1e-20
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h),
                               rtol=1e-8, atol=1e-9)


def _problem(seed=0, B=12):
    g = np.random.default_rng(seed)
    p = g.standard_normal(mlp.param_count()) * 0.08
    X = g.standard_normal((B, mlp.NF)) * 2 + 1
    xm, xs = X.mean(0), X.std(0) + 0.5
    t = g.standard_normal(B) * 3 + 1
    return p, X, t, xm, xs


def test_gradient_matches_central_differences():
    p, X, t, xm, xs = _problem()
    loss, grad = mlp.loss_and_grad(p, X, t, xm, xs, 1.0, 3.0)
    g = np.random.default_rng(1)
    h = 1e-6
    for name, off, shp in mlp.layout():
        size = int(np.prod(shp))
        idx = off + g.choice(size, size=min(size, 6), replace=False)
        for i in idx:
            pp, pm = p.copy(), p.copy()
            pp[i] += h
            pm[i] -= h
            fd = (mlp.loss_and_grad(pp, X, t, xm, xs, 1.0, 3.0)[0]
                  - mlp.loss_and_grad(pm, X, t, xm, xs, 1.0, 3.0)[0]) / (2 * h)
            assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, i, fd, grad[i])
    # padding entries have zero gradient
    used = np.zeros(mlp.param_count(), bool)
    for name, off, shp in mlp.layout():
        used[off:off + int(np.prod(shp))] = True
    assert np.all(grad[~used] == 0)


def test_forward_is_the_loss_model():
    p, X, t, xm, xs = _problem(3)
    y = mlp.forward(p, X, xm, xs, 1.0, 3.0, standardised=True)
    loss, _ = mlp.loss_and_grad(p, X, t, xm, xs, 1.0, 3.0)
    assert loss == pytest.approx(np.mean((y - (t - 1.0) / 3.0) ** 2), rel=1e-14)


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p0 = np.ones(4)
    p1, m, v = mlp.adam_step(p0, g, np.zeros(4), np.zeros(4), 1, 1e-3)
    # bias correction makes mhat = g, vhat = g^2 on the first step
    np.testing.assert_allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_features_histogram():
    edges = np.linspace(-10.0, 0.0, mlp.BINS + 1)
    n = 100
    lam = n * np.exp(np.array([-9.99, -9.6, -5.01, -0.01, 3.0, -20.0]))
    f = mlp.features(lam, 1, 0.5, 2.0, 1e-3, n, 3, edges)
    assert f[0] == 1 and f[5] == 3
    np.testing.assert_allclose(f[1:5], np.log([0.5, 2.0, 1e-3, 100.0]))
    h = f[6:]
    assert h.sum() == pytest.approx(1.0)
    # bin width 10/32: -9.99, -9.6 -> bin 0 and 1; -5.01 -> 15; -0.01 and 3.0
    # (above the top edge) -> 31; -20 (below) -> 0
    expect = np.zeros(mlp.BINS)
    expect[[0, 1, 15, 31]] = [2, 1, 1, 2]
    np.testing.assert_allclose(h, expect / 6)
