/*
 * logdet.h -- C ABI of liblogdet, an MI355X (gfx950) implementation of the
 * rational-function log-determinant estimator of Colthurst, Vasudevan,
 * Lottes and Patton, "Fast Approximate Determinants Using Rational
 * Functions" (arXiv 2405.03474).
 *
 *   log det M = log det P + tr log(M P^-1)
 *             ~ log det P + (1/s) sum_i z_i^T ( b I + sum_j c_j (M P^-1 + a_j I)^-1 ) z_i
 *
 * (Section 2, Algorithm 1 output and the derivation below Table 1), for M a
 * dense RBF or Matern-5/2 Gaussian-process covariance matrix plus noise
 * (Section 3), r_k = b + sum_j c_j/(x + a_j) the partial-fraction form of the
 * order-k approximant of eq. 1 (Table 1), P a randomized truncated-SVD
 * preconditioner (Section 2; Appendix), z_i Rademacher probes.
 *
 * Conventions for every entry point:
 *  - All matrices are row-major and contiguous.  Pointers named "device" must
 *    point to memory on the context's device; the caller owns them and must
 *    keep them alive until the work enqueued on the context stream finishes.
 *  - Work is enqueued on the stream given to ld_ctx_create.  Entry points that
 *    return host scalars (logdet_precond_build, logdet_estimate) synchronize
 *    that stream before returning; the others are asynchronous.
 *  - Errors are returned as ld_status; no exception crosses the ABI.  On an
 *    error, ld_last_error() gives a message (thread-local, valid until the
 *    next call on the same thread).  Argument checks happen before any work is
 *    enqueued.
 *  - Scratch device memory: by default the library allocates it on first use
 *    (hipMalloc), keeps it in the context, grows it when a call needs more
 *    and frees it in ld_ctx_destroy.  After ld_set_workspace the context uses
 *    the caller's buffer instead and allocates no scratch; preconditioners
 *    (ld_precond) and the surrogate's parameters stay library-owned.
 */
#ifndef LOGDET_H
#define LOGDET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LD_OK = 0,
  LD_EINVAL = -1,   /* invalid argument (sizes, k, kernel kind, null pointer, ...) */
  LD_ENOTSPD = -2,  /* a matrix that must be positive definite is not (Cholesky
                       breakdown in the preconditioner, or a non-positive CG
                       curvature / residual norm in the solver) */
  LD_ENOCONV = -3,  /* the solver hit max_iters; the result is still filled */
  LD_EHIP = -4,     /* a HIP runtime call failed */
  LD_ENOMEM = -5    /* device or pinned-host allocation failed */
} ld_status;

typedef enum { LD_RBF = 0, LD_MATERN52 = 1 } ld_kernel;

/* Arithmetic of the kernel-matrix products and of the solver vectors.
 * Scalar recurrences, reductions, the preconditioner's small dense algebra
 * and log det P are FP64 in every mode.
 *  LD_F64  FP64 products (FP64 matrix cores) and vectors.
 *  LD_F32  FP32 products (FP32 matrix cores) and vectors.
 *  LD_BF16 precision form: products on BF16 matrix cores with FP32
 *          accumulation, vectors FP32 (vector buffers use FP32).  On the
 *          fly: kernel values and distances in FP32, each operand split
 *          into bf16 hi + lo parts, products hi*hi + hi*lo + lo*hi.  From a
 *          stored matrix (FP32, LD_TILED only: the same buffer as LD_F32):
 *          each stored entry split exactly into three bf16 parts, each V
 *          entry into hi + lo, four product terms (see kernel_materialize),
 *          so the stored operator enters exactly as its FP32 values. */
typedef enum { LD_F64 = 0, LD_F32 = 1, LD_BF16 = 2 } ld_precision;

/* The matrix M = K(X, X) + noise * I (Section 3 kernels; formulas are the
 * textbook ones: RBF k(r) = variance * exp(-r^2 / (2 l^2)); Matern-5/2
 * k(r) = variance * (1 + sqrt5 r/l + 5 r^2/(3 l^2)) exp(-sqrt5 r/l)). */
typedef struct {
  const double* X;        /* device, n x d points (FP64) */
  int64_t n;              /* number of points, >= 1 */
  int32_t d;              /* dimension, 1..64; generating entries on the fly
                             (M_stored NULL in any call but kernel_materialize,
                             and every logdet_gradient) needs d <= 16 */
  int32_t kind;           /* ld_kernel */
  double lengthscale;     /* > 0 */
  double variance;        /* signal variance, > 0 */
  double noise;           /* noise variance added to the diagonal, >= 0 */
  int32_t precision;      /* ld_precision */
  const void* M_stored;   /* device matrix M (FP64 for LD_F64, FP32 for LD_F32
                             and LD_BF16; noise included) in layout `layout`,
                             or NULL to generate kernel entries on the fly
                             from X */
  int32_t layout;         /* ld_layout of M_stored (ignored when it is NULL) */
} ld_operator;

/* Storage layouts of a stored M.
 *  LD_ROW_MAJOR: n x n, row-major.
 *  LD_TILED (FP32 and FP64): 128 x 32 tiles, each contiguous; tile (I, K)
 *    covers rows 128 I .. 128 I + 127 and columns 32 K .. 32 K + 31 and
 *    starts at element (I * ceil(n/32) + K) * 4096, so a band of 128 rows is
 *    one contiguous stream.  Entries outside n x n are zero.  Inside a tile,
 *    entry (r, c) (0 <= r < 128, 0 <= c < 32) sits at
 *      FP32: (r/32)*1024 + ((c%16)/4)*256 + (c/16)*128 + (r%32)*4 + c%4,
 *      FP64: (r/32)*1024 + (4*((r/16)%2) + (c%8)/2)*128 + (16*(c/8) + r%16)*2 + c%2,
 *    the order in which the matrix-core A operand of 32-row slices is loaded
 *    as 1 KB blocks (v_mfma_f32_32x32x2f32 and v_mfma_f64_16x16x4f64
 *    respectively).  (Stored split BF16 uses its own tile format, see
 *    kernel_materialize.) */
typedef enum { LD_ROW_MAJOR = 0, LD_TILED = 1 } ld_layout;

/* Number of elements a stored M of order n occupies in `layout` (n^2 for
 * LD_ROW_MAJOR; ceil(n/128)*128 * ceil(n/32)*32 for LD_TILED), or -1 for an
 * invalid argument.  Host only. */
int64_t ld_stored_elements(int64_t n, int32_t layout);

typedef struct ld_ctx ld_ctx;         /* device, stream, cached scratch memory */
typedef struct ld_precond ld_precond; /* library-owned preconditioner factors */

typedef struct {
  double logdet;          /* the estimate of log det M */
  double logdet_P;        /* log det P */
  double trace_term;      /* (1/s) sum_i t_i, the estimate of tr r_k(M P^-1) */
  double std_err;         /* sample std of t_i / sqrt(s) (NaN for s = 1) */
  double rel_resid;       /* max over probes of ||r||_{P^-1} / ||z||_{P^-1} of
                             the smallest-shift system at exit */
  double seconds_precond; /* wall time of the preconditioner build done by
                             this call (P NULL; batched: all instances), else 0 */
  double seconds_solve;   /* wall time of the solve and reduction */
  int32_t iterations;     /* solver iterations run */
  int32_t converged_cols; /* probes that met the tolerance */
  int32_t k;              /* order of r_k */
  int32_t num_probes;     /* s */
} ld_result;

/* Create a context on HIP device `device` that enqueues on `stream` (a
 * hipStream_t, or NULL for the null stream).  *out receives the context. */
ld_status ld_ctx_create(int device, void* stream, ld_ctx** out);
void ld_ctx_destroy(ld_ctx* ctx);
const char* ld_last_error(void);

/* Device scratch bytes that cover, for this operator, kernel_matmat with s
 * columns, logdet_precond_build(rank, oversample) and the other
 * preconditioners of that rank, ld_precond_apply_inverse with s columns, and
 * logdet_estimate / logdet_estimate_orders / logdet_estimate_lanczos (up to
 * LD_LANCZOS_MAX steps) / logdet_gradient with s probes of any kind and a
 * preconditioner of that rank (or P = NULL).  k (1, 3 or 5) is checked;
 * the bound covers every order.  Sized for the current HIP device.  Returns 0
 * on invalid arguments (ld_last_error says which).  The batched form and the
 * surrogate are not covered: with a workspace too small for them they return
 * LD_ENOMEM and ld_last_error gives the bytes needed. */
size_t ld_workspace_bytes(const ld_operator* op, int64_t s, int32_t rank, int32_t oversample,
                          int32_t k);

/* Use the caller's device buffer (256-byte aligned, `bytes` long, on the
 * context's device) as the context's scratch from now on; the library's own
 * scratch block is freed.  The caller keeps the buffer alive until the
 * context is destroyed or another ld_set_workspace call returns, and does
 * not use it meanwhile.  A later call that needs more scratch than `bytes`
 * fails with LD_ENOMEM (nothing enqueued) instead of allocating.
 * ld_set_workspace(ctx, NULL, 0) returns to library-allocated scratch.
 * Synchronizes the context stream (work in flight may use the old block). */
ld_status ld_set_workspace(ld_ctx* ctx, void* dev_ptr, size_t bytes);

/* Instrumentation.  With timing on, the solvers of logdet_estimate and
 * logdet_estimate_batched record HIP events around every launch of their
 * kernel-matrix product kernel (on the stream the kernel runs on; the
 * batched form records them only without LD_BATCH_GRAPH); ld_ctx_read_timing
 * returns the summed elapsed time (ms), the number of launches, and their
 * algorithmic flops (2 n^2 s each; batched: the sum over instances that still
 * have an active probe) and bytes (the stored matrix once, when stored, plus
 * V read and Y written; batched: also the addend and the points).
 * ld_ctx_set_timing resets the totals.  Any output pointer may be NULL. */
ld_status ld_ctx_set_timing(ld_ctx* ctx, int32_t on);

/* Launch overhead.  With graphs on, the multi-shift CG of logdet_estimate,
 * logdet_estimate_orders and logdet_gradient captures its first full chunk of
 * iterations between convergence checks (8 below n = 16,384, else 1) as a HIP
 * graph and replays it for the later chunks, on a side stream of the context
 * that waits for the context stream and is waited for by it (so ordering is
 * as without graphs).  Results are identical; small problems, whose
 * iterations are a dozen short kernels, run faster.  Off by default; ignored
 * while timing is on (events are not recorded inside graphs). */
ld_status ld_ctx_set_graphs(ld_ctx* ctx, int32_t on);

/* Symmetric reuse of generated kernel entries (M is symmetric, Section 2).
 * For the forms whose bit is set, on-the-fly products of 33..64 columns at
 * n >= 16,384 (the solver's products for 64 probes) cut M into 128 x 128
 * blocks and generate only the blocks on and above the diagonal: block
 * (I, J), J > I, is applied as K_IJ V_J to rows I and as K_IJ^T V_I to rows
 * J, so about half of the entries are generated; the transposed products
 * read the generated entries back from LDS with one lane per column.
 *   LD_SYM_F32   FP32 matrix cores (strips of two blocks; partial sums about
 *                n^2 / 2 bytes of device scratch, 20 GB at n = 200,000)
 *   LD_SYM_BF16  split-BF16 matrix cores (strips of four blocks, n^2 / 4
 *                bytes)
 * The default is LD_SYM_F32: at n = 200,000 with 64 columns the FP32 product
 * takes 56.9 ms against 59.1 ms without the split, while the split-BF16 one
 * takes 32.7 ms against 30.7 ms (its transposed products are bound by LDS
 * traffic rather than by generating entries).  Products whose partial sums
 * would exceed 32 GB, or that run on a caller's workspace (ld_set_workspace)
 * too small for them, use the plain split, and so does
 * kernel_matmat_noalloc.  Results are deterministic either way and agree
 * with each other to FP32 rounding of the summation order.  0: every product
 * generates every entry. */
typedef enum { LD_SYM_F32 = 1, LD_SYM_BF16 = 2 } ld_sym_form;
ld_status ld_ctx_set_symmetric(ld_ctx* ctx, int32_t forms);
ld_status ld_ctx_read_timing(ld_ctx* ctx, double* ms, int64_t* calls, double* flops, double* bytes);

/* Probe distributions of Algorithm 1 step 1 (mean 0, variance 1):
 *   LD_PROBE_RADEMACHER  +-1 entries (the default)
 *   LD_PROBE_GAUSSIAN    standard normal entries (counter stream 2, Box-Muller)
 *   LD_PROBE_ORTHOGONAL  'normal orthogonal' probes (Appendix): W = Q S with Q
 *                        the orthonormal QR factor (positive R diagonal) of a
 *                        standard normal n x s block G and S = diag of G's
 *                        column norms (chi with n degrees of freedom,
 *                        independent of Q); needs s <= n
 * The estimators always keep b z^T z inside the per-probe value, as the
 * Method section asks for non-Rademacher probes. */
typedef enum {
  LD_PROBE_RADEMACHER = 0,
  LD_PROBE_GAUSSIAN = 1,
  LD_PROBE_ORTHOGONAL = 2
} ld_probe_kind;

/* Probe distribution used by later logdet_estimate / logdet_estimate_lanczos
 * calls on this context (not by the batched form, which is Rademacher). */
ld_status ld_ctx_set_probes(ld_ctx* ctx, int32_t kind);

/* Partial-fraction form of r_k (Section 2, Table 1), k in {1, 3, 5}:
 * r_k(x) = b + sum_{j<k} c[j] / (x + a[j]), a ascending, c < 0.  Host only;
 * a and c must hold k doubles.  The constants are derived in the library
 * from the closed-form roots of the denominators of eq. 1. */
ld_status ld_rational_coeffs(int32_t k, double* b, double* a, double* c);

/* Probe block of Algorithm 1 step 1: Z (device, n x s, FP64 if precision is
 * LD_F64 else FP32) with Rademacher entries from the counter stream
 * (SplitMix64 finalizer used as a hash; stream 2; index row * s + col). */
ld_status ld_fill_probes(ld_ctx* ctx, uint64_t seed, int64_t n, int64_t s,
                         int32_t precision, void* Z);

/* Standard normal block (device FP64, rows x cols) from the same counter
 * stream family (Box-Muller on two uniforms): the Gaussian test matrix of the
 * randomized range finder uses stream 1. */
ld_status ld_fill_gaussian(ld_ctx* ctx, uint64_t seed, int32_t stream, int64_t rows,
                           int64_t cols, double* out);

/* Y = M V (Section 2: the kernel-matrix times probe-block product that
 * dominates each solver step).  V, Y: device n x s in the operator's
 * precision; Y must not alias V.  Asynchronous. */
ld_status kernel_matmat(ld_ctx* ctx, const ld_operator* op, const void* V, int64_t s, void* Y);

/* kernel_matmat for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same product with the same kernels and bit-identical results (those of
 * kernel_matmat with ld_ctx_set_symmetric off: the symmetric split's partial
 * sums grow as n^2 and are never taken here), with its
 * scratch (the stream-K partial sums and, on the FP32 / split-BF16
 * on-the-fly paths, the scaled FP32 copy of the points) taken from a static
 * device array of 256 MiB, which every device the library runs on holds from
 * the code object's load until the process ends, instead of the context's
 * arena.  The call allocates nothing.  A product whose scratch would exceed
 * 256 MiB fails with LD_EINVAL before anything is enqueued (with 64 columns:
 * FP64 up to about n = 49,000, FP32 and split BF16 up to about n = 114,000;
 * with 16 columns about n = 245,000).  Every call on a device shares that
 * device's array and overwrites it: calls that overlap in time on one device
 * (other streams, contexts or threads) race, and the caller must serialise
 * them.  Nothing in the array needs to start at zero (each partial slot the
 * epilogue reads is written earlier by the same call).  Arguments as for
 * kernel_matmat.  Asynchronous. */
ld_status kernel_matmat_noalloc(ld_ctx* ctx, const ld_operator* op, const void* V, int64_t s,
                                void* Y);

/* Write M = K + noise I (device, ld_stored_elements(n, op->layout) elements,
 * FP64 for LD_F64, FP32 for LD_F32 and LD_BF16) in op->layout so that it can
 * be passed back as op->M_stored.  op->M_stored is ignored.  LD_BF16 needs
 * LD_TILED and writes the same FP32 tiles as LD_F32: its products split each
 * FP32 entry m in registers into h = bf16(m), c = bf16(m - h),
 * l = bf16(m - h - c) (h + c + l = m exactly) and each V entry v into
 * bf16 hi + lo, and take h*hi + h*lo + c*hi + l*hi.  Asynchronous. */
ld_status kernel_materialize(ld_ctx* ctx, const ld_operator* op, void* M_out);

/* Build the randomized truncated-SVD preconditioner P = D + U diag(lam) U^T
 * (Section 2, after Halko et al. Alg. 4.1 / 5.3; Appendix): Gaussian test
 * matrix with rank + oversample columns (counter stream 1, `seed`),
 * power_iters subspace iterations, Rayleigh-Ritz on the sketch, top `rank`
 * eigenpairs, D = diag(M) - rowsum(U^2 lam) floored at the noise variance
 * (or 1e-12 * variance when noise is 0).  Requires 1 <= rank and
 * rank + oversample <= n, oversample >= 0, 0 <= power_iters <= 16.
 * Synchronizes.  *out must be released with ld_precond_free. */
ld_status logdet_precond_build(ld_ctx* ctx, const ld_operator* op, int32_t rank,
                               int32_t oversample, int32_t power_iters, uint64_t seed,
                               ld_precond** out);

/* The Appendix's list of preconditioners, all of the form
 * P = D + U diag(lam) U^T and applied by the same Woodbury kernels:
 *   LD_PRECOND_RSVD       the randomized truncated SVD of logdet_precond_build
 *   LD_PRECOND_IDENTITY   P = I (rank 0)
 *   LD_PRECOND_DIAGONAL   P = diag(M) (rank 0)
 *   LD_PRECOND_RANK_ONE   P = D + lam v v^T with (lam, v) the top Ritz pair of
 *                         the randomized SVD of rank 1
 *   LD_PRECOND_PCHOL      P = D + C C^T, C the greedy pivoted partial Cholesky
 *                         factor of rank `rank` (pivot = largest remaining
 *                         diagonal entry, first index on ties; lam = 1)
 * For the low-rank kinds D = diag(M - low-rank part) floored at the noise
 * variance, or with LD_PRECOND_SCALED ("plus scaling") D = noise * I. */
typedef enum {
  LD_PRECOND_RSVD = 0,
  LD_PRECOND_IDENTITY = 1,
  LD_PRECOND_DIAGONAL = 2,
  LD_PRECOND_RANK_ONE = 3,
  LD_PRECOND_PCHOL = 4
} ld_precond_kind;
#define LD_PRECOND_SCALED 1

/* Build any preconditioner of the list (Appendix).  rank is used by RSVD and
 * PCHOL (PCHOL: 1 <= rank <= min(n, 4096)); oversample, power_iters and seed
 * by RSVD and RANK_ONE (as for logdet_precond_build).  flags: 0 or
 * LD_PRECOND_SCALED (low-rank kinds only; needs noise > 0).  The partial
 * Cholesky factor is computed in FP64 from the stored matrix (FP64 or FP32)
 * or from the points.  Synchronizes; *out is released with ld_precond_free. */
ld_status logdet_precond_build_kind(ld_ctx* ctx, const ld_operator* op, int32_t kind,
                                    int32_t rank, int32_t oversample, int32_t power_iters,
                                    uint64_t seed, int32_t flags, ld_precond** out);

/* Size and log det P of a preconditioner (host outputs; any may be NULL). */
ld_status ld_precond_info(const ld_precond* P, int64_t* n, int32_t* rank, double* logdet_P);

/* Copy the factors to caller device buffers (FP64): U n x rank, lambda rank
 * (descending), D n.  Any pointer may be NULL.  Asynchronous on ctx. */
ld_status ld_precond_export(ld_ctx* ctx, const ld_precond* P, double* U, double* lambda, double* D);

/* OUT = P^-1 R by the Woodbury identity (Section 2: a cheap P^-1 v):
 * P^-1 = D^-1 - F F^T with F = D^-1 U L^-T, L L^T = diag(1/lam) + U^T D^-1 U.
 * R, OUT: device n x s, FP64 if precision is LD_F64 else FP32; OUT must not
 * alias R.  Asynchronous. */
ld_status ld_precond_apply_inverse(ld_ctx* ctx, const ld_precond* P, const void* R, int64_t s,
                                   int32_t precision, void* OUT);

void ld_precond_free(ld_precond* P);

/* The estimator (Algorithm 1 output with its shifted solves run to a
 * tolerance): s Rademacher probes from `probe_seed`, one multi-shift
 * preconditioned CG per probe in the P^-1 inner product seeded with the
 * smallest shift a_1, shifted systems by the scalar recurrences of
 * Jegerlehner's multi-shift CG (Section 2, multi-shift solver paragraph),
 * stopping when ||r||_{P^-1} <= tol * ||z||_{P^-1} for the seed system of every
 * probe, then the Hutchinson mean (Section 1) in FP64.
 *   P          preconditioner for this operator (same n), or NULL to build
 *              one with rank min(100, n/10), oversample 10, 2 power
 *              iterations, seed probe_seed + 1
 *   k          1, 3 or 5
 *   num_probes s >= 1
 *   tol        > 0 (1e-12 typical for LD_F64, 1e-6 for LD_F32)
 *   max_iters  >= 1
 *   out        host, filled on LD_OK and on LD_ENOCONV
 *   per_probe  host array of s doubles receiving t_i, or NULL
 * Synchronizes. */
ld_status logdet_estimate(ld_ctx* ctx, const ld_operator* op, const ld_precond* P, int32_t k,
                          int32_t num_probes, uint64_t probe_seed, double tol, int32_t max_iters,
                          ld_result* out, double* per_probe);

/* Several orders from one Krylov space: the estimates of logdet_estimate for
 * every k in ks[], with one probe block shared by all of them.  The poles of
 * the requested r_k form one shift set (r_1, r_3 and r_5 together have 7
 * distinct poles: 1 is a pole of each), the multi-shift CG runs on its
 * smallest shift, and each order combines the shifted solutions of its own
 * poles with its own partial-fraction coefficients (Table 1).  Each estimate
 * equals logdet_estimate's with the same probe_seed up to the solver
 * tolerance; the estimates share probes, so their errors are correlated.
 *   ks         host array of num_orders distinct values in {1, 3, 5}
 *   num_orders 1..3
 *   P, num_probes, probe_seed, tol, max_iters  as for logdet_estimate
 *   out        host array of num_orders results (filled on LD_OK and on
 *              LD_ENOCONV; iterations and residuals are the shared solver's)
 *   per_probe  host array of num_orders x s doubles (order-major), or NULL
 * Synchronizes. */
ld_status logdet_estimate_orders(ld_ctx* ctx, const ld_operator* op, const ld_precond* P,
                                 int32_t num_orders, const int32_t* ks, int32_t num_probes,
                                 uint64_t probe_seed, double tol, int32_t max_iters,
                                 ld_result* out, double* per_probe);

/* Gradient of log det M with respect to (lengthscale, variance, noise) by
 * Hutchinson's estimator over probe solves (the CG-based gradient the paper
 * tunes its parameters with, Section 3):
 *   d log det M / d theta = tr(M^-1 dM/dtheta) ~ (1/s) sum_i (M^-1 z_i)^T (dM/dtheta) z_i,
 * dM/d noise = I, dM/d variance = K / variance, dM/d l the kernel's
 * derivative (RBF: k r^2 / l^3; Matern-5/2: variance t^2 (1 + t) e^-t / (3 l),
 * t = sqrt5 r / l).  The solves M y = z run as the preconditioned CG of
 * logdet_estimate with shift 0 in the operator's precision (y accumulated
 * from the search directions); the derivative products are generated in
 * FP64 from the points.  Probes follow ld_ctx_set_probes.
 *   P, num_probes, probe_seed, tol, max_iters  as for logdet_estimate
 *   grad       host, 3 doubles: d/d lengthscale, d/d variance, d/d noise
 *   std_err    host, 3 doubles or NULL: Hutchinson standard errors
 *   per_probe  host, 3 x s doubles or NULL: per-probe values, component-major
 *   out        host or NULL: iterations, converged_cols, rel_resid, logdet_P
 * Returns LD_ENOCONV (outputs filled) when a probe's solve did not reach tol.
 * Synchronizes. */
ld_status logdet_gradient(ld_ctx* ctx, const ld_operator* op, const ld_precond* P,
                          int32_t num_probes, uint64_t probe_seed, double tol, int32_t max_iters,
                          double* grad, double* std_err, double* per_probe, ld_result* out);

/* Largest number of Lanczos steps logdet_estimate_lanczos accepts. */
#define LD_LANCZOS_MAX 128

/* Algorithm 1 as printed (Section 2): s Rademacher probes from `probe_seed`;
 * for each probe v, `steps` Lanczos steps on M P^-1 started at v, giving the
 * tridiagonal T; for every pole a_j of r_k (Table 1) the system
 * (T + a_j I) w_j = |v| e_1 solved by the Thomas algorithm; per-probe value
 * t = b v^T v + sum_j c_j v^T Q^T w_j; the Hutchinson mean of t in FP64.
 * The recurrence runs in the inner product x^T P^-1 y, in which M P^-1 is
 * self-adjoint (|v|^2 = v^T P^-1 v; v^T Q^T w = sum_l (v^T q_l) w_l with
 * Euclidean products), so `steps` Lanczos steps reproduce `steps` iterations
 * of logdet_estimate's solver.  A probe whose recurrence reaches an
 * invariant subspace (beta_l <= 1e-12 times its largest |alpha|) stops early
 * with exact solves.  All probes run in lock step: one kernel-matrix product
 * and one Woodbury apply per step.
 *   P, k, num_probes, out, per_probe  as for logdet_estimate
 *   steps      1 .. LD_LANCZOS_MAX (the paper uses 20)
 * On return out->iterations = most steps any probe took, converged_cols =
 * probes that stopped in an invariant subspace, rel_resid = the largest
 * P^-1-norm residual of the smallest-shift system over |v|
 * (beta_m |w_m| / |v|).  LD_ENOTSPD when a norm in the recurrence is
 * negative or not finite (M or P not SPD).  Synchronizes. */
ld_status logdet_estimate_lanczos(ld_ctx* ctx, const ld_operator* op, const ld_precond* P,
                                  int32_t k, int32_t num_probes, uint64_t probe_seed,
                                  int32_t steps, ld_result* out, double* per_probe);

/* Algorithm 1 for several orders from one Lanczos recurrence: the steps do
 * not depend on the poles, so the t-step T of every probe serves every
 * requested r_k; only the tridiagonal solves and the Hutchinson mean are per
 * order.  Each estimate equals logdet_estimate_lanczos's for that k with the
 * same probe_seed (to rounding).
 *   ks, num_orders, out, per_probe  as for logdet_estimate_orders
 *   P, num_probes, probe_seed, steps  as for logdet_estimate_lanczos
 * Synchronizes. */
ld_status logdet_estimate_lanczos_orders(ld_ctx* ctx, const ld_operator* op, const ld_precond* P,
                                         int32_t num_orders, const int32_t* ks,
                                         int32_t num_probes, uint64_t probe_seed, int32_t steps,
                                         ld_result* out, double* per_probe);

/* One problem of a batch: M = K(X, X) + noise * I as in ld_operator (always
 * on the fly, FP32 products), with its own preconditioner rank and seeds. */
typedef struct {
  const double* X;        /* device, n x d points (FP64) */
  int64_t n;              /* >= 1 */
  int32_t d;              /* 1..8 */
  int32_t kind;           /* ld_kernel */
  double lengthscale;     /* > 0 */
  double variance;        /* > 0 */
  double noise;           /* >= 0 */
  int32_t rank;           /* preconditioner rank l >= 1, l + oversample <= n */
  int32_t reserved;       /* must be 0 */
  uint64_t precond_seed;  /* Gaussian test matrix, counter stream 1 */
  uint64_t probe_seed;    /* Rademacher probes, counter stream 2 */
} ld_instance;

/* Flags of logdet_estimate_batched. */
#define LD_BATCH_GRAPH 1   /* capture the solver iterations in a HIP graph and
                              replay it (on a library-owned side stream
                              joined to the context stream) */
#define LD_BATCH_RETUNE 2  /* re-time the product tile shapes even if this
                              context already chose one */
#define LD_BATCH_PRECOND_ONLY 4  /* build the preconditioners only: results carry
                                    logdet_P (logdet = logdet_P, trace_term = 0,
                                    iterations = 0) and lambda_out is filled */
#define LD_BATCH_NO_SYMMETRIC 8  /* up to 16 probes: use the autotuned tile
                                    shapes instead of the symmetric product
                                    form (below) */

/* The estimator of logdet_estimate applied to `count` independent problems
 * of uneven size in one pass (the same method per instance, Section 2 and
 * Algorithm 1): for every instance a randomized truncated-SVD preconditioner
 * (rank_i, oversample, power_iters, precond_seed_i), num_probes Rademacher
 * probes (probe_seed_i), and a multi-shift CG for r_k in the P^-1 inner
 * product stopping per probe at ||r||_{P^-1} <= tol ||z||_{P^-1}.  All
 * instances advance together: every kernel-matrix product, Woodbury apply and
 * reduction covers the whole batch in one launch; an instance's probes that
 * have converged stop updating.  Products and vectors are FP32; the
 * preconditioner's dense algebra, the CG scalars and log det P are FP64.
 * Instance i's probes are the same as those of logdet_estimate with
 * probe_seed_i, and its Gaussian test matrix the same as that of
 * logdet_precond_build with precond_seed_i.
 *   count       1..4096
 *   instances   host array of count descriptors
 *   k           1, 3 or 5
 *   num_probes  1..64
 *   oversample  >= 0;  power_iters 0..16
 *   tol > 0, max_iters >= 1, flags: LD_BATCH_* bits
 *   results     host array of count ld_result (filled on LD_OK / LD_ENOCONV;
 *               seconds_solve and iterations are those of the whole batch)
 *   per_probe   host array of count * num_probes doubles (instance-major), or NULL
 *   lambda_out  host array of count * lambda_stride doubles receiving each
 *               instance's kept eigenvalues (rank_i values, descending, rest
 *               of the row zero), or NULL; lambda_stride >= max rank_i
 * The product kernel's tile shape (matrix-core shape, column blocks, 4 or 2
 * waves per workgroup: up to four candidates for the probe count) is timed
 * on the first call for a probe count and kept in the context.  For up to
 * 16 probes (unless LD_BATCH_NO_SYMMETRIC) the symmetric form is used
 * instead: each instance's kernel matrix in 128 x 128 blocks, only those on
 * and above the diagonal generated, each off-diagonal block applied to its
 * rows and, transposed, to its columns (one workgroup per instance, 256-column
 * strip and run of at most 8 row tiles; partial sums added per row tile by
 * a second kernel in a fixed order; 8 KB of partial sums per (strip, row
 * tile) pair in the scratch arena).  Synchronizes. */
ld_status logdet_estimate_batched(ld_ctx* ctx, int32_t count, const ld_instance* instances,
                                  int32_t k, int32_t num_probes, int32_t oversample,
                                  int32_t power_iters, double tol, int32_t max_iters,
                                  int32_t flags, ld_result* results, double* per_probe,
                                  double* lambda_out, int32_t lambda_stride);

/* ---- learned surrogate of the trace term ----
 * An ensemble of MLPs (38 -> 256 -> 256 -> 256 -> 1, GELU after the first
 * three layers) predicting tr log(M P^-1) / n from 38 features, so that a
 * hyperparameter sweep can skip the shifted solves where the members agree;
 * the estimator itself (logdet_estimate / logdet_estimate_batched) produces
 * the training targets and remains the fallback and the judge of the error.
 * Features (ld_surrogate_features): kernel kind, log lengthscale, log variance,
 * log noise, log n, d, and the normalised histogram of log(lambda_j / n) over
 * the preconditioner's kept eigenvalues lambda_j in LD_SUR_BINS equal bins
 * between fixed edges (values outside fall in the end bins).
 * Training: FP32 forward/backward, MSE on the standardised target, Adam
 * (beta 0.9 / 0.999, eps 1e-8); every member steps on the same minibatch.
 * Inference: BF16 weights and activations on BF16 matrix cores, FP32
 * accumulation; returns the ensemble mean and standard deviation of the
 * de-standardised target.  Initial weights U(-1/sqrt(fan_in), 1/sqrt(fan_in))
 * from counter stream 3 of seed + member; biases 0. */
#define LD_SUR_FEATURES 38
#define LD_SUR_WIDTH 256
#define LD_SUR_BINS 32
typedef struct ld_surrogate ld_surrogate;

/* Parameters per member: W1 (38 x 256), b1, W2 (256 x 256), b2, W3, b3,
 * w4 (256), b4, packed in this order with every tensor starting at a multiple
 * of 64 floats; the count includes that padding.  Host only. */
int64_t ld_surrogate_param_count(void);

/* Host-side feature vector (out: 38 floats) of one problem. lambda: rank kept
 * eigenvalues (> 0); edges: LD_SUR_BINS + 1 increasing values. */
ld_status ld_surrogate_features(const double* lambda, int32_t rank, int32_t kind, double lengthscale,
                                double variance, double noise, int64_t n, int32_t d,
                                const double* edges, float* out);

/* members 1..64.  The surrogate lives on the context's device; free it with
 * ld_surrogate_free.  Synchronizes. */
ld_status ld_surrogate_create(ld_ctx* ctx, int32_t members, uint64_t seed, ld_surrogate** out);
void ld_surrogate_free(ld_surrogate* S);

/* Standardisation: features (x - x_mean) / x_std (host arrays of 38), target
 * (y - y_mean) / y_std.  Defaults: 0, 1, 0, 1.  Synchronizes. */
ld_status ld_surrogate_set_scaling(ld_ctx* ctx, ld_surrogate* S, const float* x_mean,
                                   const float* x_std, double y_mean, double y_std);

/* One Adam step of every member on the minibatch X (device, B x 38 raw
 * features) and y (device, B raw targets); loss (host, members doubles, the
 * MSE on the standardised target before the step) may be NULL (then the call
 * is asynchronous). */
ld_status ld_surrogate_train_step(ld_ctx* ctx, ld_surrogate* S, const float* X, const float* y,
                                  int32_t B, float lr, double* loss);

/* Gradient of member's loss on (X, y) without an update: grad (device,
 * ld_surrogate_param_count() floats, packed like the parameters) and the loss
 * (host, may be NULL).  Synchronizes. */
ld_status ld_surrogate_gradient(ld_ctx* ctx, ld_surrogate* S, int32_t member, const float* X,
                                const float* y, int32_t B, float* grad, double* loss);

/* Copy member's FP32 parameters to out and/or replace them from in (device
 * arrays of ld_surrogate_param_count() floats; either may be NULL). Asynchronous. */
ld_status ld_surrogate_params(ld_ctx* ctx, ld_surrogate* S, int32_t member, float* out,
                              const float* in);

/* BF16 ensemble inference on X (device, N x 38 raw features): mean and stddev
 * (device, N floats each) of the de-standardised target over the members.
 * Asynchronous. */
ld_status ld_surrogate_predict(ld_ctx* ctx, ld_surrogate* S, const float* X, int64_t N, float* mean,
                               float* stddev);

#ifdef __cplusplus
}
#endif

#endif /* LOGDET_H */
