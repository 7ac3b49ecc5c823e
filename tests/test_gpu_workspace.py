"""GPU check of the caller-owned workspace (ld_workspace_bytes,
ld_set_workspace): every single-problem entry point runs on a workspace of
the reported size with results equal to those on library scratch, allocates
no device scratch meanwhile, and a workspace that is too small fails with
LD_ENOMEM before any work."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # collected on CPU hosts but never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2405_03474_amd as L  # noqa: E402
from paper_2405_03474_amd import _binding as B  # noqa: E402


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def _op(cfg, precision, stored, ctx):
    op = L.GPOperator(X=dev(cfg.X()), kind=cfg.kind, lengthscale=cfg.lengthscale,
                      variance=cfg.variance, noise=cfg.noise, precision=precision)
    if stored:
        op.layout = L.LD_TILED
        op.M = L.kernel_materialize(ctx, op)
    return op


def _run_all(ctx, op, cfg, s, tol):
    out = {}
    P = L.Precond(ctx, op, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed)
    out["logdet_P"] = P.logdet
    _, out["est"] = L.logdet_estimate(ctx, op, P, 3, s, 5, tol, 5000)
    _, out["orders"] = L.logdet_estimate_orders(ctx, op, P, [1, 3, 5], s, 6, tol, 5000)
    _, out["lanczos"] = L.logdet_estimate_lanczos(ctx, op, P, 5, s, 7, 20)
    g, _, _, _ = L.logdet_gradient(ctx, op, P, s, 8, tol, 5000)
    out["grad"] = g
    V = L.fill_probes(ctx, 9, op.n, s, op.precision)
    out["matmat"] = L.kernel_matmat(ctx, op, V).double().cpu().numpy()
    out["pinv"] = P.apply_inverse(V, op.precision).double().cpu().numpy()
    Pc = L.Precond(ctx, op, cfg.rank, kind=L.LD_PRECOND_PCHOL)
    out["pchol_logdet"] = Pc.logdet
    ctx.set_probes(L.LD_PROBE_ORTHOGONAL)
    _, out["orth"] = L.logdet_estimate(ctx, op, Pc, 3, s, 10, tol, 5000)
    ctx.set_probes(L.LD_PROBE_RADEMACHER)
    ctx.synchronize()
    return out


@pytest.mark.parametrize("case", ["fp64_fly", "fp32_stored"])
def test_workspace_runs_every_entry_point(case):
    if case == "fp64_fly":
        cfg, precision, stored, s, tol = workloads.C1.with_n(700, rank=40), L.LD_F64, False, 24, 1e-12
    else:
        cfg, precision, stored, s, tol = workloads.C2.with_n(3000, rank=150), L.LD_F32, True, 64, 1e-6
    ref_ctx = L.Context(0)
    op = _op(cfg, precision, stored, ref_ctx)
    want = _run_all(ref_ctx, op, cfg, s, tol)

    ws = L.workspace_bytes(op, s, cfg.rank, cfg.oversample, 5)
    buf = torch.empty(ws, dtype=torch.uint8, device="cuda:0")
    ctx = L.Context(0)
    ctx.set_workspace(buf)
    _run_all(ctx, op, cfg, s, tol)          # first calls: code loading etc.
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    got = _run_all(ctx, op, cfg, s, tol)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info(0)[0]
    # the calls' scratch came from the workspace: free device memory did not
    # drop by anything like its size (the two preconditioners are allocated
    # and freed inside _run_all)
    assert free0 - free1 < min(ws // 4, 64 << 20), (free0, free1, ws)
    for key, v in want.items():
        np.testing.assert_allclose(got[key], v, rtol=1e-13, atol=0, err_msg=key)

    # too small: LD_ENOMEM before any work, with the size the call needs
    small = buf[: 1 << 20]
    ctx.set_workspace(small)
    with pytest.raises(L.LogdetError, match="LD_ENOMEM") as ei:
        L.logdet_estimate(ctx, op, None, 3, s, 5, tol, 5000)
    assert "needs" in str(ei.value)
    # back to library scratch
    ctx.set_workspace(None)
    _, per = L.logdet_estimate(ctx, op, L.Precond(ctx, op, cfg.rank, cfg.oversample,
                                                  cfg.power_iters, cfg.precond_seed),
                               3, s, 5, tol, 5000)
    np.testing.assert_allclose(per, want["est"], rtol=1e-13, atol=0)
    ctx.close()
    ref_ctx.close()


def test_workspace_argument_errors():
    ctx = L.Context(0)
    buf = torch.empty(1 << 16, dtype=torch.uint8, device="cuda:0")
    lib = B.load()
    import ctypes
    assert lib.ld_set_workspace(ctx.handle, ctypes.c_void_p(buf.data_ptr() + 1), 1024) == B.LD_EINVAL
    assert lib.ld_set_workspace(ctx.handle, ctypes.c_void_p(buf.data_ptr()), 0) == B.LD_EINVAL
    assert lib.ld_set_workspace(ctx.handle, None, 1024) == B.LD_EINVAL
    ctx.close()


def test_result_times():
    # seconds_precond: the build this call did itself (P NULL; the batched
    # form always builds), else 0
    ctx = L.Context(0)
    cfg = workloads.C1.with_n(500, rank=30)
    op = _op(cfg, L.LD_F64, False, ctx)
    res, _ = L.logdet_estimate(ctx, op, None, 3, 8, 1, 1e-10, 5000)
    assert res["seconds_precond"] > 0 and res["seconds_solve"] > 0
    P = L.Precond(ctx, op, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed)
    res, _ = L.logdet_estimate(ctx, op, P, 3, 8, 1, 1e-10, 5000)
    assert res["seconds_precond"] == 0 and res["seconds_solve"] > 0
    items = [L.BatchItem(X=dev(g.X()), kind=g.kind, lengthscale=g.lengthscale,
                         variance=g.variance, noise=g.noise, rank=g.rank,
                         precond_seed=g.precond_seed, probe_seed=g.probe_seed)
             for g in workloads.batch_instances(count=3, n_hi=1500)]
    out = L.logdet_estimate_batched(ctx, items, 3, 4, tol=1e-6, max_iters=5000)[0]
    assert all(r["seconds_precond"] > 0 and r["seconds_solve"] > 0 for r in out)
    ctx.close()
