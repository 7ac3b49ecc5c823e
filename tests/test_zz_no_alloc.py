"""kernel_matmat_noalloc (static device scratch, no allocation in the
library) against kernel_matmat on the same inputs: the same kernels on the
same plan, so the products agree bit for bit; two calls in a row, the second
smaller, in every arithmetic and storage; sizes beyond the static scratch
are rejected before anything runs."""
import numpy as np
import pytest

import workloads
from oracle import gp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # collected on CPU hosts but never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2405_03474_amd as L  # noqa: E402

CASES = [
    # precision, layout (None: on the fly), (n1, s1) then (n2, s2)
    (L.LD_F64, None, (3000, 64), (1037, 7)),
    (L.LD_F64, L.LD_TILED, (4500, 64), (777, 33)),
    (L.LD_F64, L.LD_ROW_MAJOR, (2100, 40), (300, 1)),
    (L.LD_F32, None, (5000, 300), (1200, 64)),
    (L.LD_F32, L.LD_TILED, (6000, 64), (513, 16)),
    (L.LD_BF16, None, (4000, 64), (999, 5)),
    (L.LD_BF16, L.LD_TILED, (3000, 64), (700, 64)),
]
DT = {L.LD_F64: torch.float64, L.LD_F32: torch.float32, L.LD_BF16: torch.float32}


@pytest.fixture(scope="module")
def ctx():
    c = L.Context(0)
    yield c
    c.close()


def _op(ctx, precision, layout, n, seed):
    X = np.random.default_rng(seed).random((n, 3))
    op = L.GPOperator(X=torch.as_tensor(X, device="cuda:0"), kind=gp.MATERN52, lengthscale=0.2,
                      variance=1.1, noise=1e-2, precision=precision,
                      layout=layout if layout is not None else L.LD_ROW_MAJOR)
    if layout is not None:
        op.M = L.kernel_materialize(ctx, op)
    return op


@pytest.mark.parametrize("precision,layout,first,second", CASES)
def test_noalloc_equals_kernel_matmat(ctx, precision, layout, first, second):
    for call, (n, s) in enumerate((first, second)):
        print(f"[no_alloc] precision {precision} layout {layout} call {call} n {n} s {s}",
              flush=True)
        op = _op(ctx, precision, layout, n, 100 * n + s)
        V = torch.as_tensor(np.random.default_rng(n + s).standard_normal((n, s)),
                            dtype=DT[precision], device="cuda:0")
        want = L.kernel_matmat(ctx, op, V)
        # a poisoned output buffer: every element must be written
        Y = torch.full_like(V, float("nan"))
        got = L.kernel_matmat_noalloc(ctx, op, V, Y)
        ctx.synchronize()
        assert torch.equal(got, want), (call, n, s)


def test_noalloc_rejects_products_beyond_the_static_scratch(ctx):
    # 64 columns of an FP64 product at n = 60,000 need more than 256 MiB of
    # partial sums: rejected on the host, nothing enqueued (the buffers are
    # never touched)
    n, s = 60000, 64
    X = torch.zeros((n, 3), dtype=torch.float64, device="cuda:0")
    op = L.GPOperator(X=X, kind=gp.RBF, lengthscale=0.3, variance=1.0, noise=1e-2,
                      precision=L.LD_F64)
    V = torch.zeros((n, s), dtype=torch.float64, device="cuda:0")
    with pytest.raises(L.LogdetError) as e:
        L.kernel_matmat_noalloc(ctx, op, V)
    assert e.value.status == L._binding.LD_EINVAL
    assert "static scratch" in str(e.value)
