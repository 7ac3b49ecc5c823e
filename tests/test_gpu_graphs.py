"""GPU check of the solver's HIP-graph replay (ld_ctx_set_graphs): estimates,
multi-order estimates and gradients are bitwise equal to eager launches,
repeatedly and with the program's own eager work between the calls, on the
null stream and on a torch side stream, for chunks of 8 iterations (small n),
of 1 iteration (large n) and with a last chunk shorter than the captured one."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # collected on CPU hosts but never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2405_03474_amd as L  # noqa: E402


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def _op(ctx, cfg, precision, stored):
    op = L.GPOperator(X=dev(cfg.X()), kind=cfg.kind, lengthscale=cfg.lengthscale,
                      variance=cfg.variance, noise=cfg.noise, precision=precision)
    if stored:
        op.layout = L.LD_TILED
        op.M = L.kernel_materialize(ctx, op)
    return op


def _both(ctx, fn):
    ctx.set_graphs(False)
    a = fn()
    ctx.set_graphs(True)
    b = fn()
    ctx.set_graphs(False)
    return a, b


@pytest.mark.parametrize("case", ["fp64_small", "fp32_stored_small", "fp32_stored_large"])
def test_graph_replay_equals_eager(case):
    ctx = L.Context(0)
    if case == "fp64_small":
        cfg, prec, stored, s, tol = workloads.C1.with_n(700, rank=40), L.LD_F64, False, 16, 1e-12
    elif case == "fp32_stored_small":
        cfg, prec, stored, s, tol = workloads.C2.with_n(3000, rank=150), L.LD_F32, True, 32, 1e-6
    else:   # n >= 16,384: one iteration per chunk
        cfg, prec, stored, s, tol = workloads.C2.with_n(16500, rank=100), L.LD_F32, True, 16, 1e-6
    op = _op(ctx, cfg, prec, stored)
    P = L.Precond(ctx, op, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed)
    V = L.fill_probes(ctx, 3, op.n, 8, prec)
    for rep in range(3):
        (ra, pa), (rb, pb) = _both(ctx, lambda: L.logdet_estimate(ctx, op, P, 3, s, 11 + rep, tol))
        np.testing.assert_array_equal(pa, pb)
        assert ra["iterations"] == rb["iterations"] and ra["logdet"] == rb["logdet"]
        # eager work of the program between replays
        Y = L.kernel_matmat(ctx, op, V)
        torch.cuda.synchronize()
        assert torch.isfinite(Y).all()
    (oa, qa), (ob, qb) = _both(ctx, lambda: L.logdet_estimate_orders(ctx, op, P, [1, 3, 5], s, 5,
                                                                       tol))
    np.testing.assert_array_equal(qa, qb)
    (ga, sa, pga, _), (gb, sb, pgb, _) = _both(ctx, lambda: L.logdet_gradient(ctx, op, P, s, 6, tol))
    np.testing.assert_array_equal(pga, pgb)
    # a last chunk shorter than the captured one (max_iters not a multiple of it)
    (ra, pa), (rb, pb) = _both(ctx, lambda: L.logdet_estimate(ctx, op, P, 5, s, 7, 1e-14, 21,
                                                              allow_noconv=True))
    np.testing.assert_array_equal(pa, pb)
    assert ra["iterations"] == rb["iterations"] == 21
    ctx.close()


def test_graph_replay_on_a_torch_side_stream():
    cfg = workloads.C1.with_n(700, rank=40)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = L.Context(0, stream)
        op = _op(ctx, cfg, L.LD_F64, False)
        P = L.Precond(ctx, op, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed)
        (ra, pa), (rb, pb) = _both(ctx, lambda: L.logdet_estimate(ctx, op, P, 3, 16, 4, 1e-12))
        np.testing.assert_array_equal(pa, pb)
        # work enqueued on the stream after the call sees its results
        Z = L.fill_probes(ctx, 4, op.n, 16, L.LD_F64)
        Y = L.kernel_matmat(ctx, op, Z)
    stream.synchronize()
    assert torch.isfinite(Y).all()
    ctx.close()


def test_timing_turns_replay_off():
    ctx = L.Context(0)
    cfg = workloads.C1.with_n(500, rank=30)
    op = _op(ctx, cfg, L.LD_F64, False)
    P = L.Precond(ctx, op, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed)
    ctx.set_graphs(True)
    ctx.set_timing(True)
    res, _ = L.logdet_estimate(ctx, op, P, 3, 8, 1, 1e-10)
    ms, calls, _, _ = ctx.read_timing()
    assert calls == res["iterations"] and ms > 0    # every product launch was timed
    ctx.set_timing(False)
    ctx.close()
