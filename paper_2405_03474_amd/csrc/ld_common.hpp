// Internal declarations shared by the liblogdet translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "logdet.h"

namespace ld {

// ---------------------------------------------------------------- errors --
void set_error(const std::string& msg);
ld_status fail(ld_status st, const std::string& msg);

#define LD_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return ::ld::fail(LD_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LD_TRY(expr)                     \
  do {                                   \
    ld_status s_ = (expr);               \
    if (s_ != LD_OK) return s_;          \
  } while (0)

// ------------------------------------------------------------- constants --
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr int kStreamOmega = 1;
constexpr int kStreamProbes = 2;

// host-side SplitMix64 finalizer (key derivation)
inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline uint64_t stream_key(uint64_t seed, int stream) {
  return mix64(seed + kGolden * (uint64_t)(stream + 1));
}

// ------------------------------------------------------ scratch arena --
// Device scratch arena of a context.  Allocation is a bump pointer over one
// block; reset() frees everything at once.  The block is either the
// library's own (hipMalloc'ed, grown on demand) or the caller's workspace
// (ld_set_workspace: never grown or freed here; a call that needs more fails
// with LD_ENOMEM).
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t top = 0;
  bool external = false;
  ld_status reserve(size_t bytes);  // ensure capacity (only when top == 0)
  void* take(size_t bytes);         // 256-byte aligned; nullptr if out of room
  void reset() { top = 0; }
  void release();
};

}  // namespace ld

struct ld_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 256;
  ld::Arena arena;
  double* pinned = nullptr;  // host pinned staging for small readbacks
  size_t pinned_count = 0;
  // optional event timing of the solver's kernel-matrix product launches
  bool timing = false;
  // replay the solver's iterations from captured HIP graphs (ld_ctx_set_graphs)
  bool graphs = false;
  // on-the-fly products of 33..64 columns that generate each off-diagonal
  // kernel entry once (ld_ctx_set_symmetric): LD_SYM_F32 | LD_SYM_BF16 bits
  int symmetric = LD_SYM_F32;
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  size_t ev_used = 0;          // events recorded and not yet collected
  double mm_ms = 0.0;
  int64_t mm_calls = 0;
  double mm_flops = 0.0;
  double mm_bytes = 0.0;
  std::vector<double> pending_flops, pending_bytes;
  // batched form: side stream for graph replay, its join event, and the
  // product tile shape chosen by timing (-1 until the first batched call)
  hipStream_t side = nullptr;
  hipEvent_t ev_join = nullptr;
  int bvariant = -1;
  int bvariant_cols = -1;  // the column count bvariant was chosen for
  // probe distribution of the single-problem estimators (ld_probe_kind)
  int probe_kind = 0;
  // this device's static scratch (kernel_matmat_noalloc), set at creation
  void* static_scratch = nullptr;
};

struct ld_precond {
  int64_t n = 0;
  int32_t rank = 0;
  int device = 0;
  double logdet = 0.0;
  double* U = nullptr;       // n x rank
  double* lam = nullptr;     // rank, descending
  double* D = nullptr;       // n
  double* F64 = nullptr;     // n x rank : D^-1 U L^-T
  double* Dinv64 = nullptr;  // n
  float* F32 = nullptr;      // n x rp32 : F rounded to FP32, zero columns beyond rank
  float* Dinv32 = nullptr;
  int32_t rp32 = 0;          // rank rounded up to a multiple of 32
  void* block = nullptr;     // single allocation holding all of the above
};

namespace ld {

// Kernel-evaluation parameters derived from ld_operator.
struct KParams {
  int kind;
  double variance;
  double noise;
  double c_rbf;      // 1 / (2 l^2)
  double c_mat;      // sqrt(5) / l
};
KParams make_kparams(const ld_operator& op);

// generate: the call may generate kernel entries on the fly (needs d <= 16)
ld_status check_operator(const ld_operator* op, bool generate = true);
ld_status ensure_pinned(ld_ctx* ctx, size_t count);
// event timing: reserve a (start, stop) pair, and fold finished pairs into
// the totals (call only after the stream has been synchronized)
ld_status timing_pair(ld_ctx* ctx, hipEvent_t* start, hipEvent_t* stop, double flops, double bytes);
void timing_collect(ld_ctx* ctx);

// ------------------------------------------------------------ launchers --
// rng.hip
void launch_fill_rademacher(hipStream_t st, uint64_t key, int64_t n, int64_t s, bool f64, void* Z);
void launch_fill_gaussian(hipStream_t st, uint64_t key, int64_t rows, int64_t cols, double* out);

// matmat.hip
// Y (n x s, ld = s) = M V (+ alpha2 * X2) where M is stored (A != nullptr,
// leading dimension n) or generated from points.  Points: X64 (FP64) for the
// FP64 path, X32 (FP32 copy) for the FP32 path.  Optional column dots:
// dots[blk][c] = sum over rows of block blk of V[i][c] * Y[i][c] (FP64),
// returning the number of row blocks in *dot_blocks.
struct MatmatArgs {
  int64_t n = 0;
  int64_t s = 0;
  int d = 0;
  KParams kp{};
  const void* A = nullptr;   // stored matrix or nullptr
  int layout = LD_ROW_MAJOR; // layout of A
  const void* X = nullptr;   // points in the path's precision (n x d)
  const void* V = nullptr;
  void* Y = nullptr;
  const void* X2 = nullptr;  // optional addend
  double alpha2 = 0.0;
  double* dots = nullptr;    // optional
  int* dot_blocks = nullptr;
  int64_t ld = 0;            // row stride of V, Y and X2 (0: s); wider only for the
                             // column panels of the fused FP32 / split-BF16 products
  bool timed = false;        // record events around the product kernel (ctx->timing)
  bool bf16 = false;         // FP32 path: split-BF16 matrix-core product (on the fly, or
                             // from stored split-BF16 LD_TILED tiles)
};
ld_status matmat(ld_ctx* ctx, bool f64, const MatmatArgs& a);
// kernel_matmat_noalloc's static device scratch: its size, and its address
// on `device` (which must be current), looked up once per device and kept
constexpr size_t kStaticScratchBytes = (size_t)256 << 20;
ld_status static_scratch_address(int device, void** out);
size_t matmat_scratch_bytes(ld_ctx* ctx, bool f64, int64_t n, int64_t s);
constexpr int kEpiRows = 128;  // rows per output tile of the product
constexpr int kEpiSplitMax = 16;  // most epilogue workgroups (dot partial rows) per output tile
// epilogue workgroups per output tile: 4 (8 for 128-column tiles, so that a
// thread keeps at most 8 of the tile's elements), raised for small grids so
// that about 1024 workgroups share the partial sums
inline int epi_split(int64_t tiles, int NT) {
  int sp = NT > 64 ? 8 : 4;
  while (sp < kEpiSplitMax && tiles * sp < 1024) sp *= 2;
  return sp;
}
void launch_materialize(hipStream_t st, const KParams& kp, const double* X, int64_t n, int d,
                        int precision, int layout, void* M);

// Element (i, k) of a stored FP32 matrix in LD_TILED layout: 128 x 32 tiles,
// tile (I, K) at (I * ceil(n/32) + K) * 4096; inside a tile, element (r, c)
// sits where lane r % 32 + 32 (c / 16) of wave r / 32 finds it when the wave
// loads the tile as four consecutive 1 KB blocks q = (c % 16) / 4 of one
// 16-byte chunk per lane (the A-operand order of v_mfma_f32_32x32x2f32 with
// lane half h supplying columns 16 h .. 16 h + 15).
constexpr int kTileRows = 128;
constexpr int kTileCols = 32;
__host__ __device__ inline int tile_offset(int r, int c) {
  return (r >> 5) * 1024 + ((c & 15) >> 2) * 256 + (c >> 4) * 128 + (r & 31) * 4 + (c & 3);
}
__host__ __device__ inline void tile_coords(int w, int* r, int* c) {  // inverse of tile_offset
  *r = (w >> 10) * 32 + ((w >> 2) & 31);
  *c = ((w >> 7) & 1) * 16 + ((w >> 8) & 3) * 4 + (w & 3);
}
__host__ __device__ inline int64_t tiled_index(int64_t i, int64_t k, int64_t n) {
  const int64_t kt = (n + kTileCols - 1) / kTileCols;
  return ((i / kTileRows) * kt + k / kTileCols) * (kTileRows * kTileCols) +
         tile_offset((int)(i % kTileRows), (int)(k % kTileCols));
}
// FP64 LD_TILED: the same 128 x 32 tiles and tile order; inside a tile,
// element (r, c) sits where lane r % 16 + 16 (c / 8) of wave r / 32 finds it
// when the wave loads its 32-row slice as eight consecutive 1 KB blocks
// q = 4 ((r / 16) % 2) + (c % 8) / 2 of one 16-byte pair per lane (the
// A-operand order of v_mfma_f64_16x16x4f64 with lane quarter h supplying
// columns 8 h .. 8 h + 7, two 16-row halves per slice).
__host__ __device__ inline int tile_offset64(int r, int c) {
  return (r >> 5) * 1024 + (((r >> 4) & 1) * 4 + ((c & 7) >> 1)) * 128 +
         ((c >> 3) * 16 + (r & 15)) * 2 + (c & 1);
}
__host__ __device__ inline void tile_coords64(int w, int* r, int* c) {  // inverse of tile_offset64
  const int q = (w >> 7) & 7, lane = (w >> 1) & 63;
  *r = (w >> 10) * 32 + (q >> 2) * 16 + (lane & 15);
  *c = (lane >> 4) * 8 + (q & 3) * 2 + (w & 1);
}
__host__ __device__ inline int64_t tiled_index64(int64_t i, int64_t k, int64_t n) {
  const int64_t kt = (n + kTileCols - 1) / kTileCols;
  return ((i / kTileRows) * kt + k / kTileCols) * (kTileRows * kTileCols) +
         tile_offset64((int)(i % kTileRows), (int)(k % kTileCols));
}
// Element (i, k) of a stored FP64 or FP32 matrix in either layout.
__host__ __device__ inline int64_t stored_index(int64_t i, int64_t k, int64_t n, int layout,
                                                bool f64) {
  if (layout != LD_TILED) return i * n + k;
  return f64 ? tiled_index64(i, k, n) : tiled_index(i, k, n);
}
inline int64_t stored_elements(int64_t n, int layout) {
  if (layout == LD_TILED)
    return ((n + kTileRows - 1) / kTileRows) * kTileRows * ((n + kTileCols - 1) / kTileCols) *
           kTileCols;
  return n * n;
}
void launch_convert_f64_to_f32(hipStream_t st, const double* in, float* out, int64_t count);
// out = (float)(in * scale); the FP32 points of the fused kernels use
// scale = point_scale(kp)
void launch_convert_f64_to_f32_scaled(hipStream_t st, const double* in, float* out, int64_t count,
                                      double scale);
double point_scale(const KParams& kp);
void launch_convert_f32_to_f64(hipStream_t st, const float* in, double* out, int64_t count);

// dense64.hip -- FP64 small/tall dense algebra for the preconditioner
// G (m x m) = A^T diag(w) B, A and B n x m row-major (w may be null).
ld_status gram64(ld_ctx* ctx, const double* A, const double* B, const double* w, int64_t n, int m,
                 double* G);
// in-place upper Cholesky G = R^T R (m x m); writes R (upper, zero below);
// sets the device int *fail_flag to 1 on breakdown (a pivot <= 0 or not
// finite) and leaves it untouched otherwise.
void launch_cholesky_upper(hipStream_t st, double* G, int m, int* fail_flag);
// Rinv = R^-1 for upper-triangular R (m x m)
void launch_tri_inv_upper(hipStream_t st, const double* R, int m, double* Rinv);
// C (n x N) = diag(rs) A (n x K) B (K x N, row stride ldb); rs may be null.
void launch_gemm64(hipStream_t st, const double* A, const double* B, int ldb, const double* rs,
                   int64_t n, int K, int N, double* C);
// symmetric eigendecomposition by parallel cyclic Jacobi; A (m x m) is
// overwritten; on return evals (m, descending) and evecs (m x m, column j is
// the eigenvector of evals[j]).
ld_status jacobi_eigh(ld_ctx* ctx, double* A, int m, double* evals, double* evecs);

// pcg.hip
// Per-column solver scalars of the multi-shift CG (FP64, device arrays;
// column c of ncols, shift j of J stored at j * ncols + c).
struct Scal {
  double* rho;
  double* rho0;
  double* alpha;
  double* beta;
  double* alpha_prev;
  double* beta_prev;
  double* ztz;
  double* zeta;       // J x ncols
  double* zeta_prev;  // J x ncols
  double* ztp;        // J x ncols  z^T p_j
  double* ztx;        // J x ncols  z^T x_j
  int* frozen;        // J x ncols
  int* active;        // ncols
  int* status;        // [0] = active columns, [1] = breakdown flag
};
// Single-workgroup scalar steps; the column dots arrive as nblk partial rows
// of ncols values (nblk = 1 for sums already reduced).
void launch_scal_init(hipStream_t st, const Scal& S, const double* d1, const double* d2, int nblk,
                      int64_t ncols, int J);
void launch_scal_alpha(hipStream_t st, const Scal& S, const double* dots, int nblk, int64_t ncols);
void launch_scal_beta(hipStream_t st, const Scal& S, const double* d1, const double* d2, int nblk,
                      int64_t ncols, int J, const double* delta, double tol);
ld_status woodbury_apply(ld_ctx* ctx, const ld_precond* P, bool f64, const void* R, int64_t s,
                         void* OUT);
size_t woodbury_scratch_bytes(int64_t n, int rank, int64_t s);
// F32 (n x rp, rp >= rank) = F64 (n x rank) rounded, zero columns rank .. rp - 1
void launch_pitch_f32(hipStream_t st, const double* F64, int64_t n, int rank, int rp, float* F32);
// Multi-shift PCG over the probe block Z (n x s) for shifts a_j (ascending,
// shifts[0] seeds the Krylov space).  Returns z^T x_j (J x s, row j = shift j)
// and z^T z per column in host vectors.
// r_k(x) = b + sum_j c_j / (x + a_j) (Table 1), J = k poles, a ascending.
// Shifts a[0..J) (a[0] the smallest: the CG's seed system) and the
// Hutchinson coefficients of one estimate over them: per probe
// b z^T z + sum_j c[j] z^T x_j.  Up to 8 shifts: the union of the poles of
// r_1, r_3 and r_5 has 7 (one estimate's absent poles carry c = 0).
constexpr int kMaxShifts = 8;
struct Coef {
  double b;
  double a[kMaxShifts];
  double c[kMaxShifts];
  int J;
};
ld_status multishift_pcg(ld_ctx* ctx, bool f64, const MatmatArgs& base, const ld_precond* P,
                         const Coef& cf, const void* Z, int64_t s, double tol, int max_iters,
                         std::vector<double>& per_probe, double* mean, double* stderr_,
                         int* iterations, int* converged, double* rel_resid, bool* breakdown,
                         void* ysol = nullptr);
// Several estimates from one Krylov space: the CG runs on the shifts of
// cfs[0] (every cfs[o] must list the same shifts a[0..J)), and estimate o
// combines them with cfs[o]'s coefficients.  per_probe gets ncf x s values,
// mean and stderr_ ncf each.
ld_status multishift_pcg_multi(ld_ctx* ctx, bool f64, const MatmatArgs& base, const ld_precond* P,
                               const Coef* cfs, int ncf, const void* Z, int64_t s, double tol,
                               int max_iters, std::vector<double>& per_probe, double* mean,
                               double* stderr_, int* iterations, int* converged, double* rel_resid,
                               bool* breakdown);
// Hutchinson combination of z^T x_j (J x s) and z^T z (s), device buffers:
// per-probe values (s) and [mean, standard error].
ld_status hutchinson(ld_ctx* ctx, const double* ztx_dev, const double* ztz_dev, int64_t s,
                     const Coef& cf, double* per_probe_dev, double* stats_dev);
// Algorithm 1 as printed: t Lanczos steps per probe and tridiagonal solves.
constexpr int kLzMax = LD_LANCZOS_MAX;
struct LzOut {
  std::vector<double> per_probe;
  double mean = 0.0, stderr_ = 0.0, resid = 0.0;
  int max_steps = 0;  // most steps any probe took
  int exact = 0;      // probes whose recurrence ended in an invariant subspace
  bool breakdown = false;
};
ld_status lanczos_estimate(ld_ctx* ctx, bool f64, const MatmatArgs& base, const ld_precond* P,
                           const Coef& cf, const void* Z, int64_t s, int t, LzOut& out);
// one recurrence, the tridiagonal solves and mean of every cfs[e] (outs[e])
ld_status lanczos_estimate_multi(ld_ctx* ctx, bool f64, const MatmatArgs& base,
                                 const ld_precond* P, const Coef* cfs, int ncf, const void* Z,
                                 int64_t s, int t, LzOut* outs);
size_t lanczos_scratch_bytes(ld_ctx* ctx, bool f64, int64_t n, int rank, int64_t s, int t);
size_t pcg_scratch_bytes(ld_ctx* ctx, bool f64, int64_t n, int rank, int64_t s, int J);

// batch.hip -- the whole estimator over `count` validated instances; shifts
// a_j (ascending), constant b and weights c_j of r_k.
ld_status batched_estimate(ld_ctx* ctx, int count, const ld_instance* in, int J,
                           const double* shifts, double bcoef, const double* ccoef, int s,
                           int oversample, int power_iters, double tol, int max_iters, int flags,
                           ld_result* out, double* per_probe, double* lambda_out, int lambda_stride);

}  // namespace ld
