"""GPU parity of the learned surrogate against the FP64 reference
(oracle/mlp.py) on the same parameters and minibatches: the FP32 gradient of
every parameter tensor, the loss, one Adam step, the BF16 ensemble
prediction and the feature vector."""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # collected on CPU hosts but never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2405_03474_amd as L  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = L.Context(0)
    yield c
    c.close()


def dev32(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda:0")


def problem(seed, B, scale=0.06):
    g = np.random.default_rng(seed)
    p = (g.standard_normal(mlp.param_count()) * scale).astype(np.float32)
    X = (g.standard_normal((B, mlp.NF)) * 2 + 1).astype(np.float32)
    xm = X.mean(0).astype(np.float32)
    xs = (X.std(0) + 0.5).astype(np.float32)
    t = (g.standard_normal(B) * 3 + 1).astype(np.float32)
    return p, X, t, xm, xs


def test_param_count_matches_reference():
    assert L.surrogate_param_count() == mlp.param_count()


@pytest.mark.parametrize("B", [1, 37, 256])
def test_gradient_and_loss_match_reference(ctx, B):
    p, X, t, xm, xs = problem(B, B)
    S = L.Surrogate(ctx, members=2, seed=5)
    S.set_scaling(xm, xs, 1.0, 3.0)
    S.set_params(1, dev32(p))
    g_gpu, loss = S.gradient(1, dev32(X), dev32(t))
    g_gpu = g_gpu.double().cpu().numpy()
    want_loss, want = mlp.loss_and_grad(p.astype(np.float64), X, t, xm.astype(np.float64),
                                        xs.astype(np.float64), 1.0, 3.0)
    assert loss == pytest.approx(want_loss, rel=1e-5)
    for name, off, shp in mlp.layout():
        size = int(np.prod(shp))
        a, b = g_gpu[off:off + size], want[off:off + size]
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert err < 1e-4, (name, err)
    S.close()


def test_adam_step_matches_reference(ctx):
    p, X, t, xm, xs = problem(7, 64)
    S = L.Surrogate(ctx, members=1, seed=1)
    S.set_scaling(xm, xs, 1.0, 3.0)
    S.set_params(0, dev32(p))
    lr = 1e-3
    loss = S.train_step(dev32(X), dev32(t), lr=lr)
    after = S.get_params(0).double().cpu().numpy()
    p64 = p.astype(np.float64)
    want_loss, g = mlp.loss_and_grad(p64, X, t, xm.astype(np.float64), xs.astype(np.float64), 1.0, 3.0)
    z = np.zeros_like(p64)
    want, _, _ = mlp.adam_step(p64, g, z, z, 1, lr)
    assert loss[0] == pytest.approx(want_loss, rel=1e-5)
    # the first Adam step is lr * g / (|g| + eps): compare where |g| is not tiny
    big = np.abs(g) > 1e-5
    np.testing.assert_allclose((after - p64)[big], (want - p64)[big], rtol=1e-3, atol=1e-9)
    assert np.all(np.abs((after - p64)[~big]) <= lr * 1.0001)


def test_training_reduces_loss(ctx):
    g = np.random.default_rng(11)
    X = g.standard_normal((512, mlp.NF)).astype(np.float32)
    w = g.standard_normal(mlp.NF)
    t = (np.tanh(X @ w / 4) * 2 + 0.1 * g.standard_normal(512)).astype(np.float32)
    S = L.Surrogate(ctx, members=3, seed=2)
    S.set_scaling(X.mean(0), X.std(0), float(t.mean()), float(t.std()))
    Xd, td = dev32(X), dev32(t)
    first = S.train_step(Xd, td, lr=1e-3)
    for _ in range(150):
        last = S.train_step(Xd, td, lr=1e-3)
    assert np.all(last < 0.2 * first), (first, last)
    S.close()


def test_bf16_prediction_matches_reference_forward(ctx):
    B = 300
    S = L.Surrogate(ctx, members=5, seed=3)
    g = np.random.default_rng(4)
    X = (g.standard_normal((B, mlp.NF)) * 1.5).astype(np.float32)
    xm, xs = X.mean(0).astype(np.float32), (X.std(0) + 0.1).astype(np.float32)
    ym, ys = -0.4, 0.7
    S.set_scaling(xm, xs, ym, ys)
    outs = []
    for m in range(5):
        p = S.get_params(m).double().cpu().numpy()
        outs.append(mlp.forward(p, X, xm.astype(np.float64), xs.astype(np.float64), ym, ys))
    outs = np.array(outs)
    mean, sd = S.predict(dev32(X))
    mean, sd = mean.double().cpu().numpy(), sd.double().cpu().numpy()
    want_mean, want_sd = outs.mean(0), outs.std(0, ddof=1)
    # BF16 weights and activations: errors of a few 2^-8 relative per layer
    assert np.max(np.abs(mean - want_mean)) <= 2e-2 * ys
    assert np.max(np.abs(sd - want_sd)) <= 2e-2 * ys + 0.1 * np.max(want_sd)
    S.close()


def test_features_match_reference():
    g = np.random.default_rng(5)
    edges = np.linspace(-12.0, 1.0, mlp.BINS + 1)
    for rank in (1, 7, 200):
        n = 4000
        lam = n * np.exp(g.uniform(-14, 3, size=rank))
        got = L.surrogate_features(lam, 1, 0.3, 1.2, 2e-3, n, 3, edges)
        want = mlp.features(lam, 1, 0.3, 1.2, 2e-3, n, 3, edges)
        np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-7)


def test_errors(ctx):
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        L.Surrogate(ctx, members=0)
    S = L.Surrogate(ctx, members=1)
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        S.set_scaling(np.zeros(mlp.NF), np.zeros(mlp.NF), 0.0, 1.0)
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        S.gradient(3, dev32(np.zeros((4, mlp.NF))), dev32(np.zeros(4)))
    S.close()
