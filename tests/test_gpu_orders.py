"""GPU parity of logdet_estimate_orders (r_1, r_3 and r_5 from one
multi-shift solve over the union of their poles, one shared probe block)
against the oracle's exact shifted solves with the same probes and
preconditioner (Algorithm 1's output, Table 1's partial fractions), and
against logdet_estimate order by order."""
import numpy as np
import pytest

import workloads
from oracle import estimate as oest
from oracle import gp, lanczos as olz, precond as oprec

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


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def _pair(ctx, cfg, precision=L.LD_F64, stored=False):
    X = cfg.X()
    M = gp.dense_matrix(cfg.kind, X, cfg.lengthscale, cfg.variance, cfg.noise)
    op = L.GPOperator(X=dev(X), kind=cfg.kind, lengthscale=cfg.lengthscale,
                      variance=cfg.variance, noise=cfg.noise, precision=precision)
    if stored:
        op.layout = L.LD_TILED
        op.M = L.kernel_materialize(ctx, op)
    P = L.Precond(ctx, op, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed)
    ref = oprec.rsvd(M, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed,
                     oprec.d_floor(cfg.noise, cfg.variance))
    return M, op, P, ref


@pytest.mark.parametrize("ks", [(1, 3, 5), (5, 1), (3,)])
def test_orders_fp64_parity(ctx, ks):
    cfg = workloads.C1.with_n(700, rank=40)   # ragged: 700 rows
    M, op, P, ref = _pair(ctx, cfg)
    s, seed = 24, 91
    res, per = L.logdet_estimate_orders(ctx, op, P, list(ks), s, seed, 1e-12, 5000)
    Z = oest.probes(seed, cfg.n, s)
    for i, k in enumerate(ks):
        want = oest.estimate_dense(M, ref.dense(), ref.logdet, k, Z)
        assert res[i]["k"] == k and res[i]["status"] == "LD_OK"
        np.testing.assert_allclose(per[i], want.per_probe, rtol=1e-9)
        assert res[i]["logdet"] == pytest.approx(want.logdet, rel=1e-10)
        assert res[i]["std_err"] == pytest.approx(want.stderr, rel=1e-6)
        # the same values as the single-order estimator with the same probes
        r1, p1 = L.logdet_estimate(ctx, op, P, k, s, seed, 1e-12, 5000)
        np.testing.assert_allclose(per[i], p1, rtol=1e-9)
    # one solve, seeded at the smallest pole of the requested orders
    single, _ = L.logdet_estimate(ctx, op, P, max(ks), s, seed, 1e-12, 5000)
    assert res[0]["iterations"] == single["iterations"]


def test_orders_fp32_stored_parity(ctx):
    cfg = workloads.C2.with_n(3000, rank=150)
    M, op, P, ref = _pair(ctx, cfg, precision=L.LD_F32, stored=True)
    res, per = L.logdet_estimate_orders(ctx, op, P, [1, 3, 5], cfg.probes, cfg.probe_seed,
                                        1e-6, 5000)
    Z = oest.probes(cfg.probe_seed, cfg.n, cfg.probes)
    for i, k in enumerate((1, 3, 5)):
        want = oest.estimate_dense(M, ref.dense(), ref.logdet, k, Z)
        assert res[i]["logdet"] == pytest.approx(want.logdet, rel=1e-4)
        np.testing.assert_allclose(per[i], want.per_probe, rtol=1e-3,
                                   atol=1e-4 * np.max(np.abs(want.per_probe)))


def test_orders_errors(ctx):
    cfg = workloads.C1.with_n(200, rank=10)
    M, op, P, ref = _pair(ctx, cfg)
    for bad in ([], [1, 3, 5, 1], [3, 3], [2], [1, 4]):
        with pytest.raises(L.LogdetError, match="LD_EINVAL"):
            L.logdet_estimate_orders(ctx, op, P, bad, 4, 1, 1e-10)


@pytest.mark.parametrize("ks", [(1, 3, 5), (3, 5)])
def test_lanczos_orders_fp64_parity(ctx, ks):
    # Algorithm 1: one recurrence per probe serves every order; each order
    # equals the single-order Lanczos estimate and the oracle's
    cfg = workloads.C1.with_n(700, rank=40)
    M, op, P, ref = _pair(ctx, cfg)
    s, seed, t = 16, 17, 12
    res, per = L.logdet_estimate_lanczos_orders(ctx, op, P, list(ks), s, seed, t)
    Z = oest.probes(seed, cfg.n, s)
    for i, k in enumerate(ks):
        want, steps, resid = olz.estimate_lanczos(M, ref.dense(), ref.logdet, k, Z, t)
        assert res[i]["k"] == k and res[i]["iterations"] == t
        np.testing.assert_allclose(per[i], want.per_probe, rtol=1e-10)
        _, p1 = L.logdet_estimate_lanczos(ctx, op, P, k, s, seed, t)
        np.testing.assert_allclose(per[i], p1, rtol=1e-12)


def test_lanczos_orders_errors(ctx):
    cfg = workloads.C1.with_n(200, rank=10)
    M, op, P, ref = _pair(ctx, cfg)
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        L.logdet_estimate_lanczos_orders(ctx, op, P, [1, 1], 4, 1, 5)
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        L.logdet_estimate_lanczos_orders(ctx, op, P, [3], 4, 1, 0)
