"""GPU parity of the Appendix's preconditioner list (logdet_precond_build_kind:
identity, diagonal, rank one, pivoted partial Cholesky, "plus scaling")
against oracle.precond on the same inputs: the factors, log det P, and the
estimates (multi-shift CG and Algorithm 1's Lanczos) that use them."""
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


def host(t):
    return t.detach().double().cpu().numpy()


CFG = workloads.C1.with_n(700, rank=40)   # ragged: 700 rows


def _problem(cfg=CFG):
    X = cfg.X()
    M = gp.dense_matrix(cfg.kind, X, cfg.lengthscale, cfg.variance, cfg.noise)
    op = L.GPOperator(X=dev(X), kind=cfg.kind, lengthscale=cfg.lengthscale,
                      variance=cfg.variance, noise=cfg.noise, precision=L.LD_F64)
    return M, op


def _oracle(kind, M, cfg, scaled):
    floor = oprec.d_floor(cfg.noise, cfg.variance)
    if kind == L.LD_PRECOND_IDENTITY:
        P = oprec.identity(M.shape[0])
    elif kind == L.LD_PRECOND_DIAGONAL:
        P = oprec.diagonal(M)
    elif kind == L.LD_PRECOND_RANK_ONE:
        P = oprec.rank_one(M, cfg.oversample, cfg.power_iters, cfg.precond_seed, floor)
    elif kind == L.LD_PRECOND_PCHOL:
        P = oprec.partial_cholesky(M, cfg.rank, floor)
    else:
        P = oprec.rsvd(M, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed, floor)
    return oprec.scaled(P, cfg.noise) if scaled else P


KINDS = [(L.LD_PRECOND_IDENTITY, False), (L.LD_PRECOND_DIAGONAL, False),
         (L.LD_PRECOND_RANK_ONE, False), (L.LD_PRECOND_PCHOL, False),
         (L.LD_PRECOND_PCHOL, True), (L.LD_PRECOND_RSVD, True)]


@pytest.mark.parametrize("kind,scaled", KINDS)
def test_factors_and_estimate_fp64_parity(ctx, kind, scaled):
    M, op = _problem()
    cfg = CFG
    P = L.Precond(ctx, op, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed,
                  kind=kind, scaled=scaled)
    ref = _oracle(kind, M, cfg, scaled)
    U, lam, D = (host(t) for t in P.export())
    assert P.rank == ref.lam.size
    np.testing.assert_allclose(D, ref.D, rtol=1e-9)
    if P.rank:
        np.testing.assert_allclose(lam, ref.lam, rtol=1e-9)
        np.testing.assert_allclose((U * lam) @ U.T, (ref.U * ref.lam) @ ref.U.T,
                                   atol=1e-9 * np.max(np.abs(M)))
    assert P.logdet == pytest.approx(ref.logdet, rel=1e-11)
    res, per = L.logdet_estimate(ctx, op, P, 3, 8, cfg.probe_seed, 1e-12, 5000)
    want = oest.estimate_dense(M, ref.dense(), ref.logdet, 3, oest.probes(cfg.probe_seed, cfg.n, 8))
    assert res["status"] == "LD_OK"
    np.testing.assert_allclose(per, want.per_probe, rtol=1e-9)
    assert res["logdet"] == pytest.approx(want.logdet, rel=1e-10)


def test_partial_cholesky_factor_matches_oracle(ctx):
    # C itself (pivot order and values), not only C C^T
    M, op = _problem()
    P = L.Precond(ctx, op, 60, kind=L.LD_PRECOND_PCHOL)
    C, piv = oprec.partial_cholesky_factor(M, 60)
    U, lam, D = (host(t) for t in P.export())
    np.testing.assert_allclose(U, C, atol=1e-10)
    np.testing.assert_array_equal(lam, 1.0)
    # C vanishes above the diagonal in pivot order (the pivots were the same)
    assert np.max(np.abs(np.triu(U[piv], 1))) < 1e-12


@pytest.mark.parametrize("kind", [L.LD_PRECOND_IDENTITY, L.LD_PRECOND_PCHOL])
def test_lanczos_with_family_fp64_parity(ctx, kind):
    M, op = _problem()
    cfg = CFG
    P = L.Precond(ctx, op, cfg.rank, kind=kind)
    ref = _oracle(kind, M, cfg, False)
    res, per = L.logdet_estimate_lanczos(ctx, op, P, 5, 8, 11, 15)
    want, _, _ = olz.estimate_lanczos(M, ref.dense(), ref.logdet, 5, oest.probes(11, cfg.n, 8), 15)
    np.testing.assert_allclose(per, want.per_probe, rtol=1e-9)


def test_partial_cholesky_fp32_stored(ctx):
    cfg = workloads.C2.with_n(3000, rank=150)
    X = cfg.X()
    M = gp.dense_matrix(cfg.kind, X, cfg.lengthscale, cfg.variance, cfg.noise)
    op = L.GPOperator(X=dev(X), kind=cfg.kind, lengthscale=cfg.lengthscale,
                      variance=cfg.variance, noise=cfg.noise, precision=L.LD_F32,
                      layout=L.LD_TILED)
    op.M = L.kernel_materialize(ctx, op)
    P = L.Precond(ctx, op, cfg.rank, kind=L.LD_PRECOND_PCHOL)
    # the factor is computed in FP64 from the stored FP32 entries
    M32 = M.astype(np.float32).astype(np.float64)
    ref = oprec.partial_cholesky(M32, cfg.rank, oprec.d_floor(cfg.noise, cfg.variance))
    U, lam, D = (host(t) for t in P.export())
    np.testing.assert_allclose(U, ref.U, atol=1e-9)
    assert P.logdet == pytest.approx(ref.logdet, rel=1e-10)
    res, per = L.logdet_estimate(ctx, op, P, 3, cfg.probes, cfg.probe_seed, 1e-6, 5000)
    want = oest.estimate_dense(M, ref.dense(), ref.logdet, 3,
                               oest.probes(cfg.probe_seed, cfg.n, cfg.probes))
    assert res["status"] == "LD_OK"
    assert res["logdet"] == pytest.approx(want.logdet, rel=1e-4)


def test_family_errors(ctx):
    M, op = _problem()
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        L.Precond(ctx, op, 10, kind=L.LD_PRECOND_IDENTITY, scaled=True)
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        L.Precond(ctx, op, 0, kind=L.LD_PRECOND_PCHOL)
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        L.Precond(ctx, op, 10, kind=9)
    op0 = L.GPOperator(X=op.X, kind=op.kind, lengthscale=op.lengthscale, variance=op.variance,
                       noise=0.0, precision=L.LD_F64)
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        L.Precond(ctx, op0, 10, kind=L.LD_PRECOND_PCHOL, scaled=True)
