"""GPU parity of the batched form (logdet_estimate_batched): many GP problems
of uneven size through one pass of the Section 2 method, each instance
checked against the FP64 CPU oracle on the same seeded inputs.

Tolerance (FP32 products and vectors): the estimate within 1e-4 relative,
gated as relative only where |log det| >= 0.01 n and as |error|/n <= 1e-5
otherwise (a relative error is meaningless near log det = 0); per-probe
values within 1e-3 relative plus 1e-5 n absolute.

Where the l-th and (l+1)-th Ritz values of the sketch (nearly) tie, the kept
subspace of the preconditioner is not determined by the method (any rotation
within the tied eigenspace is equally correct), so FP32 and FP64 runs pick
different, equally valid P and their estimates differ by more than the
tolerance.  Such an instance is recognised on the oracle side alone: its own
estimate moves by more than 1e-5 relative when M is perturbed elementwise
by 1e-7 relative (FP32 rounding level).  For it the test checks validity
instead: log det P finite and the estimate within six standard errors of
the exact Cholesky log det."""
import numpy as np
import pytest

import workloads
from oracle import estimate as oest
from oracle import gp, precond as oprec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # collected on CPU hosts but never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2405_03474_amd as L  # noqa: E402

OVERSAMPLE = 10
POWER = 2


@pytest.fixture(scope="module")
def ctx():
    c = L.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def items_of(insts):
    return [L.BatchItem(X=dev(g.X()), kind=g.kind, lengthscale=g.lengthscale, variance=g.variance,
                        noise=g.noise, rank=g.rank, precond_seed=g.precond_seed,
                        probe_seed=g.probe_seed) for g in insts]



def check_close(got, want, n, what):
    err = abs(got - want)
    if abs(want) >= 0.01 * n:
        assert err <= 1e-4 * abs(want), f"{what}: {got} vs {want} (rel {err / abs(want):.2e})"
    else:
        assert err <= 1e-5 * n, f"{what}: {got} vs {want} (abs/n {err / n:.2e})"


def small_batch():
    """Uneven sizes across tile boundaries, both kernels, d in {1,2,3,8}."""
    base = workloads.batch_instances(count=6, seed=workloads.BASE_SEED + 7, n_lo=100, n_hi=2500,
                                     probes=16)
    extra = [
        workloads.GPInstance("tiny_d1", n=37, d=1, kind=workloads.MATERN52, lengthscale=0.3,
                             variance=1.3, noise=1e-2, points="uniform", seed=11, rank=3,
                             probe_seed=12, precond_seed=13),
        workloads.GPInstance("tile_edge", n=128, d=2, kind=workloads.RBF, lengthscale=0.25,
                             variance=0.8, noise=3e-3, points="uniform", seed=21, rank=12,
                             probe_seed=22, precond_seed=23),
        workloads.GPInstance("ragged_129", n=129, d=8, kind=workloads.RBF, lengthscale=0.9,
                             variance=1.0, noise=1e-3, points="uniform", seed=31, rank=20,
                             probe_seed=32, precond_seed=33),
        # 20 row tiles of 128: the symmetric form cuts the rows of strips 4..9
        # into runs of at most 8 row tiles (three runs from strip 8 on), so
        # row tiles 17..19 add the transposed sums of three runs
        workloads.GPInstance("two_runs", n=2433, d=3, kind=workloads.MATERN52, lengthscale=0.2,
                             variance=1.1, noise=2e-3, points="uniform", seed=41, rank=40,
                             probe_seed=42, precond_seed=43),
    ]
    return base + extra


def ill_posed(g, M, k, Z, want):
    """True when the oracle's own estimate is not stable at FP32 rounding
    level (a tie at the rank cut of the sketch's Ritz values)."""
    r = np.random.default_rng(5).choice([-1.0, 1.0], size=M.shape)
    Mp = M * (1.0 + 1e-7 * (np.triu(r) + np.triu(r, 1).T))
    ref2 = oprec.rsvd(Mp, g.rank, OVERSAMPLE, POWER, g.precond_seed, oprec.d_floor(g.noise, g.variance))
    moved = oest.estimate_dense(M, ref2.dense(), ref2.logdet, k, Z).logdet
    return abs(moved - want.logdet) > 1e-5 * max(abs(want.logdet), 0.01 * g.n)


def check_instance(g, r, pp, k, s):
    """Parity for a well-posed instance; validity for a tied-subspace one.
    Returns True when parity was checked."""
    M = gp.dense_matrix(g.kind, g.X(), g.lengthscale, g.variance, g.noise)
    ref = oprec.rsvd(M, g.rank, OVERSAMPLE, POWER, g.precond_seed, oprec.d_floor(g.noise, g.variance))
    Z = oest.probes(g.probe_seed, g.n, s)
    want = oest.estimate_dense(M, ref.dense(), ref.logdet, k, Z)
    if not ill_posed(g, M, k, Z, want):
        check_close(r["logdet_P"], ref.logdet, g.n, f"{g.name} log det P")
        check_close(r["logdet"], want.logdet, g.n, f"{g.name} estimate")
        np.testing.assert_allclose(pp, want.per_probe, rtol=1e-3, atol=1e-5 * g.n, err_msg=g.name)
        return True
    exact = oest.logdet_exact(M)
    assert np.isfinite(r["logdet_P"])
    assert abs(r["logdet"] - exact) <= 6 * r["std_err"] + 1e-6 * g.n, (g.name, r, exact)
    return False


@pytest.mark.parametrize("symmetric", [False, True])
@pytest.mark.parametrize("k", [1, 3, 5])
def test_batched_matches_oracle(ctx, k, symmetric):
    insts = small_batch()
    s = 16
    print(f"[batched] k {k} symmetric {symmetric}", flush=True)
    res, per, status = L.logdet_estimate_batched(ctx, items_of(insts), k, s, OVERSAMPLE, POWER,
                                                 tol=1e-6, max_iters=3000, symmetric=symmetric)
    assert status == "LD_OK"
    strict = 0
    for g, r, pp in zip(insts, res, per):
        strict += check_instance(g, r, pp, k, s)
        assert r["converged_cols"] == s and r["k"] == k and r["num_probes"] == s
    assert strict >= len(insts) - 1


@pytest.mark.parametrize("symmetric", [False, True])
def test_batched_graph_equals_eager_and_instances_independent(ctx, symmetric):
    insts = small_batch()
    items = items_of(insts)
    kw = dict(tol=1e-6, symmetric=symmetric)
    eager, pe, _ = L.logdet_estimate_batched(ctx, items, 3, 8, OVERSAMPLE, POWER, **kw)
    graph, pg, _ = L.logdet_estimate_batched(ctx, items, 3, 8, OVERSAMPLE, POWER, graph=True, **kw)
    np.testing.assert_array_equal(pe, pg)
    assert [r["logdet"] for r in eager] == [r["logdet"] for r in graph]
    # an instance alone gives bit-for-bit what it gives inside the batch:
    # nothing leaks across the instance segments
    for j in (0, len(insts) - 1):
        alone, pa, _ = L.logdet_estimate_batched(ctx, [items[j]], 3, 8, OVERSAMPLE, POWER, **kw)
        np.testing.assert_array_equal(pa[0], pe[j])
        assert alone[0]["logdet_P"] == eager[j]["logdet_P"]


def test_batched_single_probe_single_instance(ctx):
    g = small_batch()[-3]  # n = 37, rank 3
    res, per, status = L.logdet_estimate_batched(ctx, items_of([g]), 3, 1, 5, 1, tol=1e-6)
    ref = oprec.rsvd(gp.dense_matrix(g.kind, g.X(), g.lengthscale, g.variance, g.noise), g.rank, 5,
                     1, g.precond_seed, oprec.d_floor(g.noise, g.variance))
    M = gp.dense_matrix(g.kind, g.X(), g.lengthscale, g.variance, g.noise)
    want = oest.estimate_dense(M, ref.dense(), ref.logdet, 3, oest.probes(g.probe_seed, g.n, 1))
    assert status == "LD_OK"
    check_close(res[0]["logdet"], want.logdet, g.n, "n=37 s=1")
    assert np.isnan(res[0]["std_err"])


def test_batched_max_iters_reports_noconv(ctx):
    insts = small_batch()[:3]
    for graph in (False, True):
        res, per, status = L.logdet_estimate_batched(ctx, items_of(insts), 5, 4, OVERSAMPLE, POWER,
                                                     tol=1e-12, max_iters=3, graph=graph,
                                                     allow_noconv=True)
        assert status == "LD_ENOCONV"
        assert all(r["iterations"] == 3 for r in res)
        assert all(np.isfinite(r["logdet"]) for r in res)


def test_batched_error_paths(ctx):
    g = small_batch()[0]
    it = items_of([g])[0]

    def call(items, **kw):
        args = dict(k=3, num_probes=4)
        args.update(kw)
        return L.logdet_estimate_batched(ctx, items, args.pop("k"), args.pop("num_probes"), **args)

    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        call([], k=3)
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        call([it], k=2)
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        call([it], num_probes=65)
    bad = L.BatchItem(**{**it.__dict__, "rank": g.n})
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        call([it, bad])
    X9 = torch.zeros((50, 9), dtype=torch.float64, device="cuda:0")
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        call([L.BatchItem(**{**it.__dict__, "X": X9, "rank": 3})])
    with pytest.raises(L.LogdetError, match="LD_EINVAL"):
        call([L.BatchItem(**{**it.__dict__, "lengthscale": 0.0})])


@pytest.mark.parametrize("symmetric", [False, True])
def test_batched_full_c4_sampled(ctx, symmetric):
    """The 256-instance heterogeneous batch at full size, in the graph launch
    the benchmark times (tuned tile shape, and the symmetric form); the
    smallest instances are checked against the oracle one by one and every
    instance must converge."""
    insts = workloads.batch_instances()
    print(f"[batched] c4 symmetric {symmetric}", flush=True)
    res, per, status = L.logdet_estimate_batched(ctx, items_of(insts), 3, 16, OVERSAMPLE, POWER,
                                                 tol=1e-6, max_iters=3000, graph=True,
                                                 symmetric=symmetric)
    assert status == "LD_OK"
    assert all(r["converged_cols"] == 16 and np.isfinite(r["logdet"]) for r in res)
    order = np.argsort([g.n for g in insts])
    strict = 0
    for i in order[:8]:
        strict += check_instance(insts[i], res[i], per[i], 3, 16)
    assert strict >= 5  # enough well-posed instances among the sampled
    # the five instances farthest from their exact log det (R11 error rule:
    # 17-104% here, the bias of r_3 on the spread spectra of short-lengthscale
    # problems at rank min(200, n/10)) are oracle-matching too
    for i in WORST_VS_EXACT:
        check_instance(insts[i], res[i], per[i], 3, 16)


# Indices of the five c4 instances with the largest error against the exact
# log det in a measured batched run (n = 589, 6,407, 4,259, 3,304, 6,073).
WORST_VS_EXACT = (22, 90, 244, 10, 145)


def test_precond_only_and_eigenvalues(ctx):
    """LD_BATCH_PRECOND_ONLY returns the same log det P as a full run and each
    instance's kept eigenvalues, which match the oracle's Ritz values."""
    insts = small_batch()
    items = items_of(insts)
    full, _, _, lam_full = L.logdet_estimate_batched(ctx, items, 3, 4, OVERSAMPLE, POWER, tol=1e-6,
                                                     want_lambda=True)
    pre, _, status, lam = L.logdet_estimate_batched(ctx, items, 3, 4, OVERSAMPLE, POWER,
                                                    precond_only=True, want_lambda=True)
    assert status == "LD_OK"
    np.testing.assert_array_equal(lam, lam_full)
    for g, a, b, row in zip(insts, full, pre, lam):
        assert b["logdet_P"] == a["logdet_P"] and b["logdet"] == b["logdet_P"]
        assert b["iterations"] == 0 and b["trace_term"] == 0.0
        assert np.all(row[g.rank:] == 0) and np.all(np.diff(row[:g.rank]) <= 0)
        M = gp.dense_matrix(g.kind, g.X(), g.lengthscale, g.variance, g.noise)
        ref = oprec.rsvd(M, g.rank, OVERSAMPLE, POWER, g.precond_seed,
                         oprec.d_floor(g.noise, g.variance))
        # the leading Ritz values are well separated; FP32 products keep them to ~1e-5
        top = min(g.rank, 5)
        np.testing.assert_allclose(row[:top], ref.lam[:top], rtol=1e-4)
