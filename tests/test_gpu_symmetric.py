"""GPU checks of the symmetric split of the on-the-fly FP32 and split-BF16
products (M is symmetric, Section 2: each off-diagonal block is generated
once and applied to both its row and its column block).  Products of 33..64
columns at n >= 16,384 take it when its form is on (ld_ctx_set_symmetric;
the default is FP32 only): they are compared element by element with the
plain split (the same entries and products, another summation order),
sampled rows with the FP64 oracle, and a full estimate with the plain split
and with the FP64 path on the same probes (1e-4, the FP32 contract)."""
import numpy as np
import pytest

import workloads
from oracle import gp

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


def _points(n, d, seed):
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(n, d))


def _product(ctx, op, V, symmetric):
    ctx.set_symmetric(f32=symmetric, bf16=symmetric)
    try:
        Y = L.kernel_matmat(ctx, op, V)
        ctx.synchronize()
    finally:
        ctx.set_symmetric()
    return Y


# precision, kind, d, n, s: ragged last blocks (n % 128 != 0), the generic
# and the specialised point dimensions, 64 columns and fewer
CASES = [
    (L.LD_F32, L.LD_MATERN52, 3, 20000, 64),
    (L.LD_F32, L.LD_RBF, 2, 16500, 40),
    (L.LD_F32, L.LD_MATERN52, 5, 17000, 64),
    (L.LD_F32, L.LD_RBF, 8, 16384, 33),
    (L.LD_BF16, L.LD_MATERN52, 3, 20000, 64),
    (L.LD_BF16, L.LD_RBF, 2, 16500, 40),
    (L.LD_BF16, L.LD_MATERN52, 5, 17000, 64),
    (L.LD_BF16, L.LD_RBF, 8, 40000, 33),
]
# sampled rows against the oracle: FP32 entries, and the split-BF16 terms
# (hi*hi + hi*lo + lo*hi drops lo*lo, about 2^-16 of each term)
ROW_TOL = {L.LD_F32: 1e-5, L.LD_BF16: 1e-4}


@pytest.mark.parametrize("prec,kind,d,n,s", CASES)
def test_symmetric_product_matches_plain_split_and_oracle(ctx, prec, kind, d, n, s):
    print(f"[symmetric] product precision {prec} kind {kind} d {d} n {n} s {s}", flush=True)
    X = _points(n, d, 11 * n + d)
    ls, var, noise = 0.12, 1.3, 1e-2
    op = L.GPOperator(X=torch.as_tensor(X, device="cuda:0"), kind=kind, lengthscale=ls,
                      variance=var, noise=noise, precision=prec)
    V = torch.as_tensor(np.random.default_rng(n + s).standard_normal((n, s)),
                        dtype=torch.float32, device="cuda:0")
    Ys = _product(ctx, op, V, True)
    Yp = _product(ctx, op, V, False)
    # M >= 0 entrywise, so M |V| bounds every term of a row's sum
    scale = _product(ctx, op, V.abs(), False).double()
    err = ((Ys.double() - Yp.double()).abs() / scale).max().item()
    assert err < 1e-5, err
    assert not torch.equal(Ys, Yp)  # another summation order: the split ran
    rows = np.unique(np.concatenate([
        [0, 127, 128, n - 1, n - 2, min(n - 1, (n // 128) * 128)],
        np.random.default_rng(n).choice(n, size=24, replace=False)]))
    ref = gp.kernel_rows(kind, X, rows, ls, var, noise)
    Vh = V.double().cpu().numpy()
    want = ref @ Vh
    got = Ys[rows].double().cpu().numpy()
    assert np.max(np.abs(got - want) / (np.abs(ref) @ np.abs(Vh))) < ROW_TOL[prec]


def test_noalloc_keeps_the_plain_split(ctx):
    """kernel_matmat_noalloc never takes the symmetric split: bit-identical to
    kernel_matmat with it off."""
    n, s = 20000, 64
    X = _points(n, 3, 5)
    op = L.GPOperator(X=torch.as_tensor(X, device="cuda:0"), kind=L.LD_MATERN52,
                      lengthscale=0.1, variance=1.0, noise=1e-2, precision=L.LD_F32)
    V = torch.as_tensor(np.random.default_rng(6).standard_normal((n, s)), dtype=torch.float32,
                        device="cuda:0")
    want = _product(ctx, op, V, False)
    got = L.kernel_matmat_noalloc(ctx, op, V)
    ctx.synchronize()
    assert torch.equal(got, want)


@pytest.mark.parametrize("prec", [L.LD_F32, L.LD_BF16])
def test_symmetric_estimate_matches_plain_split_and_fp64(ctx, prec):
    """A full FP32 / split-BF16 estimate on the fly (n = 20,000, Matern-5/2 in
    3-D, rank 200, 64 probes, r_3) with and without the split, and the FP64
    path on the same probes."""
    cfg = workloads.C3.with_n(20000, rank=200)
    X = torch.as_tensor(cfg.X(), device="cuda:0")
    out = {}
    for key, prec, sym, tol in (("sym", prec, True, 1e-6), ("plain", prec, False, 1e-6),
                                ("f64", L.LD_F64, True, 1e-10)):
        print(f"[symmetric] estimate {key}", flush=True)
        op = L.GPOperator(X=X, kind=cfg.kind, lengthscale=cfg.lengthscale,
                          variance=cfg.variance, noise=cfg.noise, precision=prec)
        ctx.set_symmetric(f32=sym, bf16=sym)
        try:
            P = L.Precond(ctx, op, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed)
            res, per = L.logdet_estimate(ctx, op, P, 3, cfg.probes, cfg.probe_seed, tol, 5000)
            P.close()
        finally:
            ctx.set_symmetric()
        assert res["status"] == "LD_OK" and res["converged_cols"] == cfg.probes
        out[key] = (res, per)
    (a, pa), (b, pb), (c, pc) = out["sym"], out["plain"], out["f64"]
    assert a["logdet"] == pytest.approx(b["logdet"], rel=1e-5)
    np.testing.assert_allclose(pa, pb, rtol=1e-4)
    assert a["logdet"] == pytest.approx(c["logdet"], rel=1e-4)
    assert a["logdet_P"] == pytest.approx(c["logdet_P"], rel=1e-4)


@pytest.mark.parametrize("prec", [L.LD_F32, L.LD_BF16])
def test_symmetric_product_at_c3_size_sampled_rows(ctx, prec):
    """The 200,000-point workload's solver product, split-BF16 (the precision
    form) and FP32 (the plain comparison path), in the launch configuration
    the benchmark times (symmetric split, 64 columns)."""
    cfg = workloads.C3
    X = cfg.X()
    op = L.GPOperator(X=torch.as_tensor(X, device="cuda:0"), kind=cfg.kind,
                      lengthscale=cfg.lengthscale, variance=cfg.variance, noise=cfg.noise,
                      precision=prec)
    V = torch.as_tensor(np.random.default_rng(7).standard_normal((cfg.n, cfg.probes)),
                        dtype=torch.float32, device="cuda:0")
    Y = _product(ctx, op, V, True)
    rows = np.unique(np.concatenate([[0, 128, cfg.n - 1],
                                     np.random.default_rng(8).choice(cfg.n, 24, replace=False)]))
    ref = gp.kernel_rows(cfg.kind, X, rows, cfg.lengthscale, cfg.variance, cfg.noise)
    Vh = V.double().cpu().numpy()
    err = np.max(np.abs(Y[rows].double().cpu().numpy() - ref @ Vh) / (np.abs(ref) @ np.abs(Vh)))
    assert err < ROW_TOL[prec], err
