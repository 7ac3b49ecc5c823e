"""GPU parity of the probe types (ld_ctx_set_probes: Gaussian and 'normal
orthogonal', Appendix) against oracle.estimate's probe blocks, through the
multi-shift CG and Algorithm 1's Lanczos estimators."""
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

KINDS = {"gaussian": L.LD_PROBE_GAUSSIAN, "orthogonal": L.LD_PROBE_ORTHOGONAL}


@pytest.fixture(scope="module")
def ctx():
    c = L.Context(0)
    yield c
    c.set_probes(L.LD_PROBE_RADEMACHER)
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


@pytest.mark.parametrize("kind", sorted(KINDS))
@pytest.mark.parametrize("k", [3, 5])
def test_probe_kinds_fp64_parity(ctx, kind, k):
    cfg = workloads.C1.with_n(700, rank=40)
    M, op, P, ref = _pair(ctx, cfg)
    ctx.set_probes(KINDS[kind])
    try:
        res, per = L.logdet_estimate(ctx, op, P, k, 24, 41, 1e-12, 5000)
        Z = oest.probe_block(kind, 41, cfg.n, 24)
        want = oest.estimate_dense(M, ref.dense(), ref.logdet, k, Z)
        np.testing.assert_allclose(per, want.per_probe, rtol=1e-9)
        assert res["logdet"] == pytest.approx(want.logdet, rel=1e-10)
        res_l, per_l = L.logdet_estimate_lanczos(ctx, op, P, k, 24, 41, 12)
        want_l, _, _ = olz.estimate_lanczos(M, ref.dense(), ref.logdet, k, Z, 12)
        np.testing.assert_allclose(per_l, want_l.per_probe, rtol=1e-9)
    finally:
        ctx.set_probes(L.LD_PROBE_RADEMACHER)


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_probe_kinds_fp32_stored(ctx, kind):
    cfg = workloads.C2.with_n(3000, rank=150)
    M, op, P, ref = _pair(ctx, cfg, precision=L.LD_F32, stored=True)
    ctx.set_probes(KINDS[kind])
    try:
        res, per = L.logdet_estimate(ctx, op, P, 3, cfg.probes, 5, 1e-6, 5000)
    finally:
        ctx.set_probes(L.LD_PROBE_RADEMACHER)
    want = oest.estimate_dense(M, ref.dense(), ref.logdet, 3,
                               oest.probe_block(kind, 5, cfg.n, cfg.probes))
    assert res["status"] == "LD_OK"
    assert res["logdet"] == pytest.approx(want.logdet, rel=1e-4)


def test_probe_kind_errors(ctx):
    cfg = workloads.C1.with_n(50, rank=5)
    M, op, P, ref = _pair(ctx, cfg)
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        ctx.set_probes(7)
    ctx.set_probes(L.LD_PROBE_ORTHOGONAL)
    try:
        with pytest.raises(L.LogdetError, match="LD_EINVAL"):
            L.logdet_estimate(ctx, op, P, 3, 51, 1, 1e-10, 100)   # s > n
    finally:
        ctx.set_probes(L.LD_PROBE_RADEMACHER)
