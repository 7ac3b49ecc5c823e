"""GPU parity: every step of the HIP path against the FP64 CPU oracle on the
same seeded inputs (Section 2 method; tolerances: 1e-10 relative for FP64,
1e-4 relative for FP32 on the estimate)."""
import numpy as np
import pytest

import workloads
from oracle import estimate as oest
from oracle import gp, precond as oprec, rational, rng

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


def make_op(X, kind, ls, var, noise, precision=L.LD_F64, M=None):
    return L.GPOperator(X=dev(X), kind=kind, lengthscale=ls, variance=var, noise=noise,
                        precision=precision, M=M)


# ------------------------------------------------------------------ RNG --
def test_probes_bitwise_equal_oracle(ctx):
    for n, s, seed in [(1, 1, 0), (1037, 7, 5), (2000, 32, workloads.C1.probe_seed)]:
        Z = L.fill_probes(ctx, seed, n, s, L.LD_F64)
        Z32 = L.fill_probes(ctx, seed, n, s, L.LD_F32)
        ctx.synchronize()
        ref = rng.rademacher(seed, rng.STREAM_PROBES, n, s)
        np.testing.assert_array_equal(host(Z), ref)
        np.testing.assert_array_equal(host(Z32), ref)


def test_gaussian_matches_oracle(ctx):
    G = L.fill_gaussian(ctx, 123, rng.STREAM_OMEGA, 501, 13)
    ctx.synchronize()
    ref = rng.gaussian(123, rng.STREAM_OMEGA, 501, 13)
    np.testing.assert_allclose(host(G), ref, rtol=1e-13, atol=1e-14)


# ------------------------------------------------------------- matmat --
MM_CASES = [
    # n, d, s, kind
    (1037, 3, 64, gp.MATERN52),
    (1037, 3, 7, gp.RBF),
    (300, 2, 1, gp.RBF),
    (513, 8, 33, gp.MATERN52),
    (200, 5, 100, gp.RBF),
    (70, 3, 16, gp.MATERN52),
    (777, 3, 300, gp.MATERN52),  # 128-column tiles of the fused kernels, ragged
]


def untile64(buf, n):
    """Dense n x n view of an FP64 LD_TILED buffer (128 x 32 tiles; inside a
    tile entry (r, c) at (r/32)*1024 + (4*((r/16)%2) + (c%8)/2)*128 +
    (16*(c/8) + r%16)*2 + c%2, as documented in logdet.h)."""
    kt = -(-n // 32)
    rt = -(-n // 128)
    # r = 32 w + 16 rb + lj, c = 8 lh + 2 tq + e
    t = buf.reshape(rt, kt, 4, 2, 4, 4, 16, 2)         # I, K, w, rb, tq, lh, lj, e
    t = t.transpose(0, 2, 3, 6, 1, 5, 4, 7)            # I, w, rb, lj, K, lh, tq, e
    t = t.reshape(rt * 128, kt * 32)
    assert np.all(t[n:, :] == 0) and np.all(t[:, n:] == 0)
    return t[:n, :n]


@pytest.mark.parametrize("n,d,s,kind", MM_CASES)
@pytest.mark.parametrize("stored", [None, "row", "tiled"])
def test_matmat_fp64(ctx, n, d, s, kind, stored):
    g = np.random.default_rng(n + s)
    X = g.random((n, d))
    V = g.standard_normal((n, s))
    Mref = gp.dense_matrix(kind, X, 0.3, 1.3, 1e-2)
    op = make_op(X, kind, 0.3, 1.3, 1e-2)
    if stored:
        op.layout = L.LD_TILED if stored == "tiled" else L.LD_ROW_MAJOR
        op.M = L.kernel_materialize(ctx, op)
        ctx.synchronize()
        M = host(op.M)
        M = untile64(M, n) if stored == "tiled" else M
        np.testing.assert_allclose(M, Mref, rtol=1e-14, atol=1e-15)
    Y = L.kernel_matmat(ctx, op, dev(V))
    ctx.synchronize()
    ref = Mref @ V
    scale = np.abs(Mref) @ np.abs(V)
    assert np.max(np.abs(host(Y) - ref) / scale) < 1e-13


def untile(buf, n):
    """Dense n x n view of an FP32 LD_TILED buffer (128 x 32 tiles; inside a
    tile entry (r, c) at (r/32)*1024 + ((c%16)/4)*256 + (c/16)*128 + (r%32)*4
    + c%4, as documented in logdet.h)."""
    kt = -(-n // 32)
    rt = -(-n // 128)
    # inner index = ((((w*4 + q)*2 + h)*32 + l)*4 + e) with r = 32 w + l, c = 16 h + 4 q + e
    t = buf.reshape(rt, kt, 4, 4, 2, 32, 4)            # I, K, w, q, h, l, e
    t = t.transpose(0, 2, 5, 1, 4, 3, 6)               # I, w, l, K, h, q, e
    t = t.reshape(rt * 128, kt * 32)
    assert np.all(t[n:, :] == 0) and np.all(t[:, n:] == 0)
    return t[:n, :n]


@pytest.mark.parametrize("n,d,s,kind", MM_CASES)
@pytest.mark.parametrize("stored", [None, "row", "tiled"])
def test_matmat_fp32(ctx, n, d, s, kind, stored):
    g = np.random.default_rng(7 * n + s)
    X = g.random((n, d))
    V = g.standard_normal((n, s)).astype(np.float32)
    Mref = gp.dense_matrix(kind, X, 0.3, 1.3, 1e-2)
    op = make_op(X, kind, 0.3, 1.3, 1e-2, precision=L.LD_F32)
    if stored:
        op.layout = L.LD_TILED if stored == "tiled" else L.LD_ROW_MAJOR
        op.M = L.kernel_materialize(ctx, op)
        ctx.synchronize()
        M = host(op.M)
        M = untile(M, n) if stored == "tiled" else M
        np.testing.assert_allclose(M, Mref.astype(np.float32), rtol=1.2e-7, atol=1e-30)
    Y = L.kernel_matmat(ctx, op, dev(V, torch.float32))
    ctx.synchronize()
    ref = Mref @ V.astype(np.float64)
    scale = np.abs(Mref) @ np.abs(V.astype(np.float64))
    assert np.max(np.abs(host(Y) - ref) / scale) < 1e-5


# ------------------------------------------------------- preconditioner --
def _precond_pair(ctx, cfg, precision=L.LD_F64, stored=False):
    X = cfg.X()
    M = gp.dense_matrix(cfg.kind, X, cfg.lengthscale, cfg.variance, cfg.noise)
    op = make_op(X, cfg.kind, cfg.lengthscale, cfg.variance, cfg.noise, precision)
    if stored:
        op.layout = L.LD_TILED if stored == "tiled" else L.LD_ROW_MAJOR
        op.M = L.kernel_materialize(ctx, op)
    P = L.Precond(ctx, op, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed)
    ref = oprec.rsvd(M, cfg.rank, cfg.oversample, cfg.power_iters, cfg.precond_seed,
                     oprec.d_floor(cfg.noise, cfg.variance))
    return X, M, op, P, ref


def test_precond_fp64_matches_oracle(ctx):
    cfg = workloads.C1.with_n(1000, rank=60)
    X, M, op, P, ref = _precond_pair(ctx, cfg)
    U, lam, D = (host(t) for t in P.export())
    np.testing.assert_allclose(lam, ref.lam, rtol=1e-9)
    np.testing.assert_allclose((U * lam) @ U.T, (ref.U * ref.lam) @ ref.U.T, atol=1e-9)
    np.testing.assert_allclose(D, ref.D, rtol=1e-9)
    assert P.logdet == pytest.approx(ref.logdet, rel=1e-11)
    np.testing.assert_allclose(U.T @ U, np.eye(cfg.rank), atol=1e-12)
    # Woodbury apply
    R = np.random.default_rng(3).standard_normal((cfg.n, 5))
    out = host(P.apply_inverse(dev(R), L.LD_F64))
    np.testing.assert_allclose(out, ref.solve(R), rtol=1e-10, atol=1e-10 * np.abs(ref.solve(R)).max())
    out32 = host(P.apply_inverse(dev(R, torch.float32), L.LD_F32))
    np.testing.assert_allclose(out32, ref.solve(R), rtol=0, atol=1e-3 * np.abs(ref.solve(R)).max())


def test_precond_fp32_stored_close_to_oracle(ctx):
    cfg = workloads.C2.with_n(2000, rank=100)
    X, M, op, P, ref = _precond_pair(ctx, cfg, precision=L.LD_F32, stored="tiled")
    U, lam, D = (host(t) for t in P.export())
    np.testing.assert_allclose(lam[:50], ref.lam[:50], rtol=1e-4)
    assert P.logdet == pytest.approx(ref.logdet, rel=1e-4)


# ------------------------------------------------------------- estimate --
def _oracle_estimate(M, ref, k, seed, s):
    Z = oest.probes(seed, M.shape[0], s)
    return oest.estimate_dense(M, ref.dense(), ref.logdet, k, Z)


@pytest.mark.parametrize("k", [1, 3, 5])
def test_estimate_fp64_c1_parity(ctx, k):
    cfg = workloads.C1
    X, M, op, P, ref = _precond_pair(ctx, cfg)
    res, per = L.logdet_estimate(ctx, op, P, k, cfg.probes, cfg.probe_seed, 1e-12, 5000)
    want = _oracle_estimate(M, ref, k, cfg.probe_seed, cfg.probes)
    assert res["status"] == "LD_OK"
    np.testing.assert_allclose(per, want.per_probe, rtol=1e-10)
    assert res["logdet"] == pytest.approx(want.logdet, rel=1e-10)
    assert res["logdet_P"] == pytest.approx(ref.logdet, rel=1e-11)
    assert res["converged_cols"] == cfg.probes


@pytest.mark.parametrize("stored", [False, "row", "tiled"])
@pytest.mark.parametrize("k", [1, 3, 5])
def test_estimate_fp32_parity(ctx, k, stored):
    cfg = workloads.C2.with_n(3000, rank=150)
    X, M, op, P, ref = _precond_pair(ctx, cfg, precision=L.LD_F32, stored=stored)
    res, per = L.logdet_estimate(ctx, op, P, k, cfg.probes, cfg.probe_seed + k, 1e-6, 5000)
    want = _oracle_estimate(M, ref, k, cfg.probe_seed + k, cfg.probes)
    assert res["status"] == "LD_OK"
    assert res["logdet"] == pytest.approx(want.logdet, rel=1e-4)
    np.testing.assert_allclose(per, want.per_probe, rtol=1e-3)


def test_estimate_small_and_single_probe(ctx):
    # n below one tile, s = 1, ragged everything
    cfg = workloads.C1.with_n(50, rank=5)
    X, M, op, P, ref = _precond_pair(ctx, cfg)
    res, per = L.logdet_estimate(ctx, op, P, 3, 1, 99, 1e-12, 1000)
    want = _oracle_estimate(M, ref, 3, 99, 1)
    assert per[0] == pytest.approx(want.per_probe[0], rel=1e-10)
    assert np.isnan(res["std_err"])


def test_estimate_default_precond_and_determinism(ctx):
    cfg = workloads.C1.with_n(700)
    X = cfg.X()
    op = make_op(X, cfg.kind, cfg.lengthscale, cfg.variance, cfg.noise)
    a, pa = L.logdet_estimate(ctx, op, None, 3, 8, 17, 1e-12, 2000)
    b, pb = L.logdet_estimate(ctx, op, None, 3, 8, 17, 1e-12, 2000)
    np.testing.assert_array_equal(pa, pb)
    M = gp.dense_matrix(cfg.kind, X, cfg.lengthscale, cfg.variance, cfg.noise)
    ref = oprec.rsvd(M, 70, 10, 2, 18, oprec.d_floor(cfg.noise, cfg.variance))
    want = _oracle_estimate(M, ref, 3, 17, 8)
    assert a["logdet"] == pytest.approx(want.logdet, rel=1e-10)


def test_estimate_error_within_bias_and_noise_of_exact(ctx):
    cfg = workloads.C1
    X, M, op, P, ref = _precond_pair(ctx, cfg)
    res, _ = L.logdet_estimate(ctx, op, P, 3, cfg.probes, cfg.probe_seed, 1e-12, 5000)
    exact = oest.logdet_exact(M)
    _, bias = oest.expected_estimate(M, ref.dense(), ref.logdet, 3)
    assert abs(res["logdet"] - exact) <= abs(bias) + 4 * res["std_err"]


# --------------------------------------------------------------- errors --
def test_error_paths(ctx):
    cfg = workloads.C1.with_n(300, rank=20)
    X = cfg.X()
    op = make_op(X, cfg.kind, cfg.lengthscale, cfg.variance, cfg.noise)
    with pytest.raises(L.LogdetError) as e:
        L.logdet_estimate(ctx, op, None, 2, 4, 0, 1e-8, 10)
    assert e.value.status == L._binding.LD_EINVAL
    with pytest.raises(L.LogdetError) as e:
        L.Precond(ctx, op, 295, 10, 2, 0)
    assert e.value.status == L._binding.LD_EINVAL
    bad = make_op(X, cfg.kind, -1.0, cfg.variance, cfg.noise)
    with pytest.raises(L.LogdetError) as e:
        L.kernel_matmat(ctx, bad, dev(np.ones((300, 1))))
    assert e.value.status == L._binding.LD_EINVAL
    P = L.Precond(ctx, op, 20, 10, 2, 1)
    res, per = L.logdet_estimate(ctx, op, P, 3, 4, 0, 1e-12, 1, allow_noconv=True)
    assert res["status"] == "LD_ENOCONV" and res["iterations"] == 1
    assert res["converged_cols"] == 0 and np.all(np.isfinite(per))


# --------------------------------------------------- precision form (BF16) --
@pytest.mark.parametrize("n,d,s,kind", MM_CASES)
def test_matmat_bf16_split(ctx, n, d, s, kind):
    g = np.random.default_rng(11 * n + s)
    X = g.random((n, d))
    V = g.standard_normal((n, s)).astype(np.float32)
    Mref = gp.dense_matrix(kind, X, 0.3, 1.3, 1e-2)
    op = make_op(X, kind, 0.3, 1.3, 1e-2, precision=L.LD_BF16)
    Y = L.kernel_matmat(ctx, op, dev(V, torch.float32))
    ctx.synchronize()
    ref = Mref @ V.astype(np.float64)
    scale = np.abs(Mref) @ np.abs(V.astype(np.float64))
    # three-term split-bf16 products: about 2^-16 relative per term
    assert np.max(np.abs(host(Y) - ref) / scale) < 1e-4


@pytest.mark.parametrize("precision", [L.LD_F32, L.LD_BF16])
def test_matmat_column_panels_bitwise(ctx, precision):
    """A fused product wider than 128 columns runs as 128-column panels over
    the strided V; each panel takes the plan of a standalone 128-column call
    on the contiguous slice, so the two agree bit for bit."""
    n, s = 777, 300
    g = np.random.default_rng(17)
    X = g.random((n, 3))
    V = g.standard_normal((n, s)).astype(np.float32)
    op = make_op(X, gp.MATERN52, 0.3, 1.3, 1e-2, precision=precision)
    Y = host(L.kernel_matmat(ctx, op, dev(V, torch.float32)))
    for c in range(0, s, 128):
        w = min(128, s - c)
        Yp = host(L.kernel_matmat(ctx, op, dev(np.ascontiguousarray(V[:, c:c + w]), torch.float32)))
        ctx.synchronize()
        assert np.array_equal(Y[:, c:c + w], Yp), c


@pytest.mark.parametrize("n,d,s,kind", MM_CASES)
def test_matmat_bf16_stored_tiles(ctx, n, d, s, kind):
    """The precision form from stored FP32 tiles: the buffer is the FP32
    LD_TILED matrix, split exactly into three BF16 parts inside the product."""
    g = np.random.default_rng(13 * n + s)
    X = g.random((n, d))
    V = g.standard_normal((n, s)).astype(np.float32)
    Mref = gp.dense_matrix(kind, X, 0.3, 1.3, 1e-2)
    op = make_op(X, kind, 0.3, 1.3, 1e-2, precision=L.LD_BF16)
    op.layout = L.LD_TILED
    op.M = L.kernel_materialize(ctx, op)
    ctx.synchronize()
    assert op.M.dtype == torch.float32
    np.testing.assert_array_equal(untile(host(op.M), n), Mref.astype(np.float32))
    Y = L.kernel_matmat(ctx, op, dev(V, torch.float32))
    ctx.synchronize()
    ref = Mref @ V.astype(np.float64)
    scale = np.abs(Mref) @ np.abs(V.astype(np.float64))
    # V's hi + lo carry 2^-17 relative; the stored entries enter exactly
    assert np.max(np.abs(host(Y) - ref) / scale) < 3e-5


@pytest.mark.parametrize("k", [1, 3, 5])
def test_estimate_bf16_stored_parity(ctx, k):
    cfg = workloads.C2.with_n(3000, rank=150)
    X, M, op, P, ref = _precond_pair(ctx, cfg, precision=L.LD_BF16, stored="tiled")
    res, per = L.logdet_estimate(ctx, op, P, k, cfg.probes, cfg.probe_seed + k, 1e-6, 5000)
    want = _oracle_estimate(M, ref, k, cfg.probe_seed + k, cfg.probes)
    assert res["status"] == "LD_OK"
    assert res["logdet"] == pytest.approx(want.logdet, rel=1e-4)
    np.testing.assert_allclose(per, want.per_probe, rtol=2e-3)


@pytest.mark.parametrize("k", [3, 5])
def test_estimate_bf16_parity(ctx, k):
    cfg = workloads.C3.with_n(3000, rank=200)
    X, M, op, P, ref = _precond_pair(ctx, cfg, precision=L.LD_BF16)
    res, per = L.logdet_estimate(ctx, op, P, k, cfg.probes, cfg.probe_seed, 1e-6, 5000)
    want = _oracle_estimate(M, ref, k, cfg.probe_seed, cfg.probes)
    assert res["status"] == "LD_OK"
    assert res["logdet"] == pytest.approx(want.logdet, rel=1e-4)
    np.testing.assert_allclose(per, want.per_probe, rtol=2e-3)


# ----------------------------------------- tiled storage: ragged and tiny n --
@pytest.mark.parametrize("n", [1, 2, 31, 129, 333])
@pytest.mark.parametrize("precision", [L.LD_F64, L.LD_F32, L.LD_BF16])
def test_matmat_tiled_ragged_and_tiny(ctx, n, precision):
    """Stored LD_TILED products where n leaves most of a 128 x 32 tile as
    padding (n = 1, 2) or cuts through tiles in both directions."""
    g = np.random.default_rng(19 * n + precision)
    X = g.random((n, 3))
    s = 5
    V = g.standard_normal((n, s))
    Mref = gp.dense_matrix(gp.MATERN52, X, 0.3, 1.3, 1e-2)
    op = make_op(X, gp.MATERN52, 0.3, 1.3, 1e-2, precision=precision)
    op.layout = L.LD_TILED
    op.M = L.kernel_materialize(ctx, op)
    dt = torch.float64 if precision == L.LD_F64 else torch.float32
    Y = L.kernel_matmat(ctx, op, dev(V, dt))
    ctx.synchronize()
    Vd = host(dev(V, dt))
    ref = Mref @ Vd
    scale = np.abs(Mref) @ np.abs(Vd)
    tol = {L.LD_F64: 1e-13, L.LD_F32: 1e-5, L.LD_BF16: 3e-5}[precision]
    assert np.max(np.abs(host(Y) - ref) / scale) < tol


@pytest.mark.parametrize("k", [1, 3, 5])
def test_estimate_fp64_tiled_ragged_parity(ctx, k):
    """FP64 estimate from the FP64 LD_TILED matrix at a size that is ragged in
    both tile dimensions: oracle parity at 1e-10 (solves to 1e-11)."""
    cfg = workloads.C2.with_n(1333, rank=60)
    X, M, op, P, ref = _precond_pair(ctx, cfg, precision=L.LD_F64, stored="tiled")
    res, per = L.logdet_estimate(ctx, op, P, k, cfg.probes, cfg.probe_seed + k, 1e-11, 5000)
    want = _oracle_estimate(M, ref, k, cfg.probe_seed + k, cfg.probes)
    assert res["status"] == "LD_OK" and res["converged_cols"] == cfg.probes
    assert res["logdet"] == pytest.approx(want.logdet, rel=1e-10)
    assert res["logdet_P"] == pytest.approx(ref.logdet, rel=1e-11)
    assert np.max(np.abs(per - want.per_probe)) <= 1e-9 * np.max(np.abs(want.per_probe))
