"""MI355X (gfx950) implementation of the rational-function log-determinant
estimator of Colthurst et al. (arXiv 2405.03474).

The computation lives in liblogdet.so (HIP kernels behind the C ABI of
include/logdet.h); this package is its Python binding.
"""
from ._binding import (  # noqa: F401
    EXPORTED, LD_BATCH_GRAPH, LD_BATCH_PRECOND_ONLY, LD_BATCH_RETUNE, LD_BATCH_NO_SYMMETRIC, LD_BF16, LD_F32, LD_F64,
    LD_LANCZOS_MAX, LD_MATERN52, LD_PRECOND_DIAGONAL, LD_PRECOND_IDENTITY, LD_PRECOND_PCHOL,
    LD_PRECOND_RANK_ONE, LD_PRECOND_RSVD, LD_PRECOND_SCALED, LD_PROBE_GAUSSIAN,
    LD_PROBE_ORTHOGONAL, LD_PROBE_RADEMACHER, LD_RBF, LD_ROW_MAJOR, LD_SUR_BINS, LD_SUR_FEATURES, LD_SUR_WIDTH, LD_SYM_BF16, LD_SYM_F32, LD_TILED,
    BatchItem, Context, GPOperator, LogdetError, Precond, Surrogate, fill_gaussian, fill_probes,
    kernel_materialize, kernel_matmat, kernel_matmat_noalloc, load, logdet_estimate, logdet_estimate_batched,
    logdet_estimate_lanczos, logdet_estimate_lanczos_orders, logdet_estimate_orders,
    logdet_gradient,
    rational_coeffs, stored_elements, surrogate_features, surrogate_param_count, workspace_bytes,
)
