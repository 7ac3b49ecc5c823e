"""GPU parity of Algorithm 1 as printed (logdet_estimate_lanczos: t Lanczos
steps per probe in the P^-1 inner product, Thomas solves per pole) against
oracle.lanczos on the same probes and preconditioner factors; its agreement
with t iterations of the multi-shift CG; exact termination in a two-step
Krylov space."""
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


@pytest.mark.parametrize("t", [1, 7, 20])
@pytest.mark.parametrize("k", [3, 5])
def test_lanczos_fp64_parity(ctx, k, t):
    cfg = workloads.C1.with_n(700, rank=40)   # ragged: 700 rows, 32 probes
    M, op, P, ref = _pair(ctx, cfg)
    res, per = L.logdet_estimate_lanczos(ctx, op, P, k, cfg.probes, cfg.probe_seed, t)
    Z = oest.probes(cfg.probe_seed, cfg.n, cfg.probes)
    want, steps, resid = olz.estimate_lanczos(M, ref.dense(), ref.logdet, k, Z, t)
    assert res["status"] == "LD_OK"
    assert res["iterations"] == t and np.all(steps == t)
    np.testing.assert_allclose(per, want.per_probe, rtol=1e-10)
    assert res["logdet"] == pytest.approx(want.logdet, rel=1e-10)
    assert res["rel_resid"] == pytest.approx(np.max(resid), rel=1e-6)


@pytest.mark.parametrize("t", [4, 9])
def test_lanczos_equals_t_cg_iterations(ctx, t):
    # t Lanczos steps and t iterations of the multi-shift CG give the same
    # Galerkin solutions on the same Krylov space, shift by shift.
    cfg = workloads.C1.with_n(900, rank=30)
    M, op, P, ref = _pair(ctx, cfg)
    _, per_l = L.logdet_estimate_lanczos(ctx, op, P, 5, 16, 77, t)
    _, per_c = L.logdet_estimate(ctx, op, P, 5, 16, 77, 1e-30, t, allow_noconv=True)
    np.testing.assert_allclose(per_l, per_c, rtol=1e-9)


def test_lanczos_fp32_stored_parity(ctx):
    cfg = workloads.C2.with_n(3000, rank=150)
    M, op, P, ref = _pair(ctx, cfg, precision=L.LD_F32, stored=True)
    t = 20
    res, per = L.logdet_estimate_lanczos(ctx, op, P, 3, cfg.probes, cfg.probe_seed, t)
    Z = oest.probes(cfg.probe_seed, cfg.n, cfg.probes)
    want, _, _ = olz.estimate_lanczos(M, ref.dense(), ref.logdet, 3, Z, t)
    assert res["status"] == "LD_OK"
    assert res["logdet"] == pytest.approx(want.logdet, rel=1e-4)
    np.testing.assert_allclose(per, want.per_probe, rtol=1e-3)


def test_lanczos_stops_in_two_step_krylov_space(ctx):
    # M = noise I (stored): the sketch spans range(Omega), every Ritz value is
    # the noise, D is floored at the noise, so P = noise (I + U U^T) and
    # M P^-1 has the two eigenvalues 1/2 and 1: every probe's recurrence
    # reaches an invariant subspace after two steps, and the values are the
    # exact shifted solves with the exported factors.
    n, noise = 400, 1e-2
    X = np.random.default_rng(31).random((n, 3))
    Mref = noise * np.eye(n)
    op = L.GPOperator(X=dev(X), kind=L.LD_RBF, lengthscale=0.3, variance=1.0, noise=noise,
                      precision=L.LD_F64, M=dev(Mref))
    P = L.Precond(ctx, op, 10, 10, 2, 5)
    res, per = L.logdet_estimate_lanczos(ctx, op, P, 5, 12, 3, 20)
    U, lam, D = (t.double().cpu().numpy() for t in P.export())
    Pd = np.diag(D) + (U * lam) @ U.T
    want = oest.per_probe_dense(Mref, Pd, 5, oest.probes(3, n, 12))
    assert res["iterations"] == 2 and res["converged_cols"] == 12
    np.testing.assert_allclose(per, want, rtol=1e-10)
    assert res["logdet"] == pytest.approx(P.logdet + np.mean(want), rel=1e-12)
    assert res["rel_resid"] < 1e-12


def test_lanczos_errors(ctx):
    cfg = workloads.C1.with_n(200, rank=10)
    M, op, P, ref = _pair(ctx, cfg)
    for bad in (0, L.LD_LANCZOS_MAX + 1):
        with pytest.raises(L.LogdetError, match="LD_EINVAL"):
            L.logdet_estimate_lanczos(ctx, op, P, 3, 4, 1, bad)
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        L.logdet_estimate_lanczos(ctx, op, P, 2, 4, 1, 5)
