// C ABI of liblogdet: argument checks, scratch management and the host-side
// orchestration of the estimator (Section 2: Algorithm 1 and the randomized
// truncated-SVD preconditioner).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kfun_dev.hpp"
#include "ld_common.hpp"

namespace ld {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }
ld_status fail(ld_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

// ------------------------------------------------------------------ arena --
ld_status Arena::reserve(size_t bytes) {
  if (bytes <= cap) return LD_OK;
  if (external)
    return fail(LD_ENOMEM, "the workspace set by ld_set_workspace holds " + std::to_string(cap) +
                               " bytes; this call needs " + std::to_string(bytes));
  // the old block may still be read by enqueued work
  if (base) (void)hipDeviceSynchronize();
  release();
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LD_ENOMEM, "device scratch allocation of " + std::to_string(bytes) + " bytes failed");
  }
  base = (char*)p;
  cap = bytes;
  top = 0;
  return LD_OK;
}

void* Arena::take(size_t bytes) {
  const size_t off = (top + 255) & ~(size_t)255;
  if (off + bytes > cap) return nullptr;
  top = off + bytes;
  return base + off;
}

void Arena::release() {
  if (base && !external) (void)hipFree(base);
  base = nullptr;
  cap = 0;
  top = 0;
  external = false;
}

ld_status ensure_pinned(ld_ctx* ctx, size_t count) {
  if (count <= ctx->pinned_count) return LD_OK;
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  ctx->pinned = nullptr;
  ctx->pinned_count = 0;
  void* p = nullptr;
  if (hipHostMalloc(&p, count * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LD_ENOMEM, "pinned host allocation failed");
  }
  ctx->pinned = (double*)p;
  ctx->pinned_count = count;
  return LD_OK;
}

ld_status timing_pair(ld_ctx* ctx, hipEvent_t* start, hipEvent_t* stop, double flops, double bytes) {
  if (ctx->ev_used + 2 > ctx->ev.size()) {
    for (int q = 0; q < 2; ++q) {
      hipEvent_t e;
      LD_HIP(hipEventCreate(&e));
      ctx->ev.push_back(e);
    }
  }
  *start = ctx->ev[ctx->ev_used];
  *stop = ctx->ev[ctx->ev_used + 1];
  ctx->ev_used += 2;
  ctx->pending_flops.push_back(flops);
  ctx->pending_bytes.push_back(bytes);
  return LD_OK;
}

void timing_collect(ld_ctx* ctx) {
  for (size_t i = 0; i + 1 < ctx->ev_used; i += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]) == hipSuccess) {
      ctx->mm_ms += ms;
      ctx->mm_calls += 1;
      ctx->mm_flops += ctx->pending_flops[i / 2];
      ctx->mm_bytes += ctx->pending_bytes[i / 2];
    } else {
      (void)hipGetLastError();
    }
  }
  ctx->ev_used = 0;
  ctx->pending_flops.clear();
  ctx->pending_bytes.clear();
}

// generate: the call may generate kernel entries on the fly from the points
// (all calls but kernel_materialize when M is not stored); the fused
// generation kernels keep a point's coordinates in registers, up to 16
ld_status check_operator(const ld_operator* op, bool generate) {
  if (!op) return fail(LD_EINVAL, "operator is NULL");
  if (!op->X) return fail(LD_EINVAL, "operator X is NULL");
  if (op->n < 1) return fail(LD_EINVAL, "n must be >= 1");
  if (op->d < 1 || op->d > 64) return fail(LD_EINVAL, "d must be in 1..64");
  if (generate && !op->M_stored && op->d > 16)
    return fail(LD_EINVAL, "kernel entries on the fly need d <= 16; store M (kernel_materialize) for larger d");
  if (op->kind != LD_RBF && op->kind != LD_MATERN52) return fail(LD_EINVAL, "unknown kernel kind");
  if (!(op->lengthscale > 0.0) || !std::isfinite(op->lengthscale))
    return fail(LD_EINVAL, "lengthscale must be finite and > 0");
  if (!(op->variance > 0.0) || !std::isfinite(op->variance))
    return fail(LD_EINVAL, "variance must be finite and > 0");
  if (!(op->noise >= 0.0) || !std::isfinite(op->noise))
    return fail(LD_EINVAL, "noise must be finite and >= 0");
  if (op->precision != LD_F64 && op->precision != LD_F32 && op->precision != LD_BF16)
    return fail(LD_EINVAL, "precision must be LD_F64, LD_F32 or LD_BF16");
  if (op->layout != LD_ROW_MAJOR && op->layout != LD_TILED)
    return fail(LD_EINVAL, "layout must be LD_ROW_MAJOR or LD_TILED");
  if (op->precision == LD_BF16 && op->M_stored && op->layout != LD_TILED)
    return fail(LD_EINVAL, "a stored LD_BF16 matrix must use the LD_TILED layout");
  return LD_OK;
}

namespace {

bool is_f64(const ld_operator* op) { return op->precision == LD_F64; }

// Points in the arithmetic of the path: FP64 as given, or an FP32 copy.
ld_status path_points(ld_ctx* ctx, const ld_operator* op, const void** X) {
  if (is_f64(op) || op->M_stored) {
    *X = op->X;
    return LD_OK;
  }
  float* x32 = (float*)ctx->arena.take((size_t)op->n * op->d * sizeof(float));
  if (!x32) return fail(LD_ENOMEM, "scratch arena too small for FP32 points");
  // scaled in FP64 before rounding, so that the fused kernels read squared
  // distances in the kernel's own units (kval32s)
  launch_convert_f64_to_f32_scaled(ctx->stream, op->X, x32, op->n * op->d,
                                   point_scale(make_kparams(*op)));
  *X = x32;
  return LD_OK;
}

MatmatArgs base_args(const ld_operator* op, const void* X) {
  MatmatArgs a;
  a.n = op->n;
  a.d = op->d;
  a.kp = make_kparams(*op);
  a.A = op->M_stored;
  a.layout = op->layout;
  a.bf16 = op->precision == LD_BF16;
  a.X = X;
  return a;
}

// ---------------------------------------------------- rational constants --
// r_k = pref * N_k / D_k (eq. 1).  D_k(z) = sum_i C(2k, 2i) z^i, whose roots
// are -tan^2(pi (2m+1) / (4k)); the residue at a simple root alpha is
// pref * N_k(alpha) / D_k'(alpha); b is the ratio of leading coefficients.
struct Rational {
  double b;
  double a[5];
  double c[5];
};

bool rational_for(int k, Rational* out) {
  static const long double n1[] = {1, -1};
  static const long double n3[] = {7, 27, -27, -7};
  static const long double n5[] = {43, 825, 1150, -1150, -825, -43};
  const long double* num;
  long double pref;
  switch (k) {
    case 1: num = n1; pref = 2.0L; break;
    case 3: num = n3; pref = 2.0L / 3.0L; break;
    case 5: num = n5; pref = 2.0L / 15.0L; break;
    default: return false;
  }
  // denominator coefficients, highest power first: C(2k, 2(k - i))
  long double den[6];
  for (int i = 0; i <= k; ++i) {
    const int e = 2 * (k - i);
    long double cb = 1.0L;
    for (int t = 1; t <= e; ++t) cb = cb * (long double)(2 * k - e + t) / (long double)t;
    den[i] = cb;
  }
  const long double pi = 3.141592653589793238462643383279502884L;
  out->b = (double)(pref * num[0] / den[0]);
  for (int m = 0; m < k; ++m) {
    const long double tq = tanl(pi * (long double)(2 * m + 1) / (long double)(4 * k));
    const long double alpha = -tq * tq;
    long double nv = 0.0L, dv = 0.0L;
    for (int i = 0; i <= k; ++i) nv = nv * alpha + num[i];
    for (int i = 0; i < k; ++i) dv = dv * alpha + den[i] * (long double)(k - i);
    out->a[m] = (double)(-alpha);
    out->c[m] = (double)(pref * nv / dv);
  }
  return true;
}

ld_status check_ctx(ld_ctx* ctx) {
  if (!ctx) return fail(LD_EINVAL, "context is NULL");
  LD_HIP(hipSetDevice(ctx->device));
  return LD_OK;
}

// D = diag(M) - rowsum(U^2 lam) floored at floor_v, or the constant const_d
// when it is positive (identity and "plus scaling" preconditioners).
__global__ void k_d_and_inv(const double* __restrict__ U, const double* __restrict__ lam, int64_t n,
                            int rank, const void* __restrict__ Mst, int mprec, int layout,
                            double diag_const, double floor_v, double const_d,
                            double* __restrict__ D, double* __restrict__ Dinv) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    if (const_d > 0.0) {
      D[i] = const_d;
      Dinv[i] = 1.0 / const_d;
      continue;
    }
    double dm = diag_const;
    const int64_t ii = stored_index(i, i, n, layout, mprec == LD_F64);
    if (Mst) {  // FP64, or FP32 (LD_F32 and the LD_BF16 precision form)
      dm = mprec == LD_F64 ? ((const double*)Mst)[ii] : (double)((const float*)Mst)[ii];
    }
    double low = 0.0;
    for (int j = 0; j < rank; ++j) {
      const double u = U[i * rank + j];
      low = fma(lam[j] * u, u, low);
    }
    double dv = dm - low;
    if (!(dv >= floor_v)) dv = floor_v;
    D[i] = dv;
    Dinv[i] = 1.0 / dv;
  }
}

__global__ void k_sqrt_diag(const double* __restrict__ G, int m, double* __restrict__ out) {
  for (int j = blockIdx.x * 256 + threadIdx.x; j < m; j += gridDim.x * 256)
    out[j] = sqrt(G[(int64_t)j * m + j]);
}

__global__ void k_scale_cols64(double* __restrict__ A, const double* __restrict__ f, int64_t n,
                               int64_t s) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n * s; i += (int64_t)gridDim.x * 256)
    A[i] *= f[i % s];
}

__global__ void k_add_diag_inv(double* __restrict__ C, const double* __restrict__ lam, int rank) {
  for (int j = blockIdx.x * 256 + threadIdx.x; j < rank; j += gridDim.x * 256)
    C[(int64_t)j * rank + j] += 1.0 / lam[j];
}

// shift the Gram diagonal by c * trace(G) (shifted CholeskyQR first pass)
__global__ void k_shift_diag(double* __restrict__ G, int m, double c) {
  __shared__ double red[256];
  double t = 0.0;
  for (int j = threadIdx.x; j < m; j += 256) t += G[(int64_t)j * m + j];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double sh = c * red[0];
  for (int j = threadIdx.x; j < m; j += 256) G[(int64_t)j * m + j] += sh;
}

// out[0] = sum log D, out[1] = sum log lam, out[2] = 2 sum log diag(R)
__global__ void k_logdet_parts(const double* __restrict__ D, int64_t n, const double* __restrict__ lam,
                               const double* __restrict__ R, int rank, double* __restrict__ out) {
  __shared__ double red[3][256];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) a += log(D[i]);
  for (int j = threadIdx.x; j < rank; j += 256) {
    b += log(lam[j]);
    c += 2.0 * log(R[(int64_t)j * rank + j]);
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) out[q] = red[q][0];
}

int grid1(int64_t count) {
  int64_t b = (count + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

// Orthonormal basis of range(Y) by shifted CholeskyQR3 (one shifted pass,
// then two plain passes).  Y (n x m) is consumed; the basis ends in *Q, which
// is one of the two buffers Y / W.
ld_status orthonormalize(ld_ctx* ctx, double* Y, double* W, int64_t n, int m, double* G, double* Rinv,
                         int* ok_dev, int passes, double** Q) {
  hipStream_t st = ctx->stream;
  double* src = Y;
  double* dst = W;
  const double shift_c = 11.0 * ((double)n * m + (double)m * (m + 1)) * 0x1.0p-53;
  LD_HIP(hipMemsetAsync(ok_dev, 0, sizeof(int), st));
  for (int pass = 0; pass < passes; ++pass) {
    const size_t mark = ctx->arena.top;
    LD_TRY(gram64(ctx, src, src, nullptr, n, m, G));
    ctx->arena.top = mark;  // partials are consumed by the reduction already enqueued
    if (pass == 0) hipLaunchKernelGGL(k_shift_diag, dim3(1), dim3(256), 0, st, G, m, shift_c);
    launch_cholesky_upper(st, G, m, ok_dev);
    launch_tri_inv_upper(st, G, m, Rinv);
    launch_gemm64(st, src, Rinv, m, nullptr, n, m, m, dst);
    std::swap(src, dst);
  }
  LD_HIP(hipGetLastError());
  LD_TRY(ensure_pinned(ctx, 1));
  LD_HIP(hipMemcpyAsync(ctx->pinned, ok_dev, sizeof(int), hipMemcpyDeviceToHost, st));
  LD_HIP(hipStreamSynchronize(st));
  if (*(int*)ctx->pinned != 0)
    return fail(LD_ENOTSPD, "CholeskyQR breakdown: sketch Gram matrix not positive definite");
  *Q = src;
  return LD_OK;
}

// Y = M V for an n x m FP64 block, through the operator's arithmetic.
ld_status apply_M64(ld_ctx* ctx, const ld_operator* op, const void* Xp, const double* V, double* Y,
                    int m, float* t1, float* t2) {
  MatmatArgs a = base_args(op, Xp);
  a.s = m;
  const size_t mark = ctx->arena.top;
  if (is_f64(op)) {
    a.V = V;
    a.Y = Y;
    LD_TRY(matmat(ctx, true, a));
  } else {
    launch_convert_f64_to_f32(ctx->stream, V, t1, op->n * (int64_t)m);
    a.V = t1;
    a.Y = t2;
    LD_TRY(matmat(ctx, false, a));
    launch_convert_f32_to_f64(ctx->stream, t2, Y, op->n * (int64_t)m);
  }
  ctx->arena.top = mark;
  return LD_OK;
}

// Library-owned block for the factors of a rank-`rank` preconditioner
// (rank 0: D only).
ld_status alloc_precond(ld_ctx* ctx, int64_t n, int rank, ld_precond** out) {
  ld_precond* P = new ld_precond();
  P->n = n;
  P->rank = rank;
  P->device = ctx->device;
  const size_t nl = (size_t)n * rank;
  P->rp32 = (rank + 31) / 32 * 32;
  const size_t nlp = (size_t)n * P->rp32;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t bytes = al(nl * 8) * 2 + al((size_t)rank * 8) + al((size_t)n * 8) * 2 +
                       al(nlp * 4) + al((size_t)n * 4);
  void* blk = nullptr;
  if (hipMalloc(&blk, bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete P;
    return fail(LD_ENOMEM, "preconditioner allocation failed");
  }
  P->block = blk;
  char* c = (char*)blk;
  P->U = (double*)c; c += al(nl * 8);
  P->F64 = (double*)c; c += al(nl * 8);
  P->lam = (double*)c; c += al((size_t)rank * 8);
  P->D = (double*)c; c += al((size_t)n * 8);
  P->Dinv64 = (double*)c; c += al((size_t)n * 8);
  P->F32 = (float*)c; c += al(nlp * 4);
  P->Dinv32 = (float*)c;
  *out = P;
  return LD_OK;
}

// Given U and lam in P: D (the floored diagonal remainder, or const_d when
// positive), the capacitance C = diag(1/lam) + U^T D^-1 U = R^T R, log det P
// by the determinant lemma, F = D^-1 U R^-1 and the FP32 copies.  G, Rinv
// (rank x rank), ok (int) and parts (3 doubles) are device scratch.  Frees P
// on failure.
ld_status finish_precond(ld_ctx* ctx, const ld_operator* op, ld_precond* P, double const_d,
                         double* G, double* Rinv, int* okd, double* parts) {
  hipStream_t st = ctx->stream;
  const int64_t n = P->n;
  const int rank = P->rank;
  auto bail = [&](ld_status s_) {
    (void)hipStreamSynchronize(st);
    ld_precond_free(P);
    return s_;
  };
  const double floor_v = op->noise > 0.0 ? op->noise : 1e-12 * op->variance;
  hipLaunchKernelGGL(k_d_and_inv, dim3(grid1(n)), dim3(256), 0, st, P->U, P->lam, n, rank,
                     op->M_stored, op->precision, op->layout, op->variance + op->noise, floor_v,
                     const_d, P->D, P->Dinv64);
  if (hipMemsetAsync(okd, 0, sizeof(int), st) != hipSuccess) return bail(fail(LD_EHIP, "memset failed"));
  if (rank > 0) {
    {
      const size_t mark = ctx->arena.top;
      ld_status s_ = gram64(ctx, P->U, P->U, P->Dinv64, n, rank, G);
      ctx->arena.top = mark;
      if (s_ != LD_OK) return bail(s_);
    }
    hipLaunchKernelGGL(k_add_diag_inv, dim3(grid1(rank)), dim3(256), 0, st, G, P->lam, rank);
    launch_cholesky_upper(st, G, rank, okd);
  }
  hipLaunchKernelGGL(k_logdet_parts, dim3(1), dim3(256), 0, st, P->D, n, P->lam, G, rank, parts);
  if (rank > 0) {
    // F = D^-1 U R^-1  (= D^-1 U L^-T with L = R^T)
    launch_tri_inv_upper(st, G, rank, Rinv);
    launch_gemm64(st, P->U, Rinv, rank, P->Dinv64, n, rank, rank, P->F64);
    launch_pitch_f32(st, P->F64, n, rank, P->rp32, P->F32);
  }
  launch_convert_f64_to_f32(st, P->Dinv64, P->Dinv32, n);
  if (hipGetLastError() != hipSuccess) return bail(fail(LD_EHIP, "kernel launch failed"));
  if (ensure_pinned(ctx, 8) != LD_OK) return bail(LD_ENOMEM);
  if (hipMemcpyAsync(ctx->pinned, parts, 3 * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(ctx->pinned + 4, okd, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return bail(fail(LD_EHIP, "readback of log det P failed"));
  if (*(int*)(ctx->pinned + 4) != 0)
    return bail(fail(LD_ENOTSPD, "capacitance matrix Cholesky breakdown"));
  P->logdet = ctx->pinned[0] + ctx->pinned[1] + ctx->pinned[2];
  if (!std::isfinite(P->logdet)) return bail(fail(LD_ENOTSPD, "log det P is not finite"));
  return LD_OK;
}

// ---------------------------------------------------------- scratch sizes --
// Device scratch each call takes from the context's arena; ld_workspace_bytes
// reports the largest of them.

// randomized truncated SVD with rank + oversample sketch columns
size_t rsvd_scratch_bytes(ld_ctx* ctx, const ld_operator* op, int rank, int oversample) {
  const int64_t n = op->n;
  const int m = rank + oversample;
  const bool f64 = is_f64(op);
  const size_t nm = (size_t)n * m;
  const int me = m + (m & 1);
  size_t need = 0;
  need += (size_t)n * op->d * 4 + 512;                     // FP32 points
  need += 2 * nm * 8 + 1024;                               // Q, Y (FP64)
  if (!f64) need += 2 * nm * 4 + 1024;                     // FP32 copies for matmat
  need += 4 * (size_t)m * m * 8 + 2048;                    // G, Rinv, evecs, B
  need += (size_t)m * 8 + 512;                             // evals
  need += 4 * (size_t)me * me * 8 + 16 + 2048;             // Jacobi
  size_t gram_b = std::max((size_t)16 << 20, (size_t)2 * m * m * 8) + 512;
  need += std::max(gram_b, matmat_scratch_bytes(ctx, f64, n, m)) + 1024;
  need += 4096;
  return need;
}

// identity, diagonal (rank 0) and partial Cholesky of the given rank
size_t simple_precond_scratch_bytes(const ld_operator* op, int rank) {
  const int64_t n = op->n;
  return (size_t)n * op->d * 4 + 512 + (size_t)n * 8 + 512 + 2 * (size_t)rank * rank * 8 + 1024 +
         (size_t)rank * 12 + 512 + 4096 + ((size_t)16 << 20);
}

// one kernel_matmat call with s columns
size_t matmat_call_bytes(ld_ctx* ctx, const ld_operator* op, int64_t s) {
  return (size_t)op->n * op->d * 4 + 512 + matmat_scratch_bytes(ctx, is_f64(op), op->n, s);
}

// the estimators' set-up (points, probes, probe drawing) plus the solver's
// own scratch and `extra`
size_t est_scratch_bytes(const ld_operator* op, int64_t s, int probe_kind, size_t solver,
                         size_t extra) {
  const int64_t n = op->n;
  const size_t es = is_f64(op) ? 8 : 4;
  // Gaussian / orthogonal probes are drawn in FP64 first (two n x s blocks
  // and the small Gram factors of the orthonormalisation)
  const size_t probe_tmp = probe_kind == LD_PROBE_RADEMACHER
                               ? 0
                               : 2 * (size_t)n * s * 8 + 3 * (size_t)s * s * 8 + (size_t)s * 8 +
                                     ((size_t)16 << 20) + 4096;
  return (size_t)n * op->d * 4 + 512 + (size_t)n * s * es + 512 + solver + extra + probe_tmp;
}

// logdet_gradient's scratch beyond the solver: y (operator precision), FP64
// copies of z and y, the derivative product, partials and values
size_t gradient_extra_bytes(ld_ctx* ctx, const ld_operator* op, int64_t s) {
  const int64_t n = op->n;
  const size_t es = is_f64(op) ? 8 : 4;
  const int64_t nblk = (n + 255) / 256;
  return (size_t)n * s * es + 3 * (size_t)n * s * 8 + (size_t)nblk * s * 8 + 8 * (size_t)s * 8 +
         8 * 4096 + matmat_scratch_bytes(ctx, true, n, s);
}

// Randomized truncated SVD (rank >= 1) with D the floored diagonal remainder,
// or, with const_d > 0, D = const_d I ("plus scaling").
ld_status build_precond(ld_ctx* ctx, const ld_operator* op, int rank, int oversample, int power_iters,
                        uint64_t seed, ld_precond** out, double const_d) {
  const int64_t n = op->n;
  const int m = rank + oversample;
  const bool f64 = is_f64(op);
  const size_t nm = (size_t)n * m;
  ctx->arena.reset();
  LD_TRY(ctx->arena.reserve(rsvd_scratch_bytes(ctx, op, rank, oversample)));

  const void* Xp = nullptr;
  LD_TRY(path_points(ctx, op, &Xp));
  double* Qb = (double*)ctx->arena.take(nm * 8);
  double* Yb = (double*)ctx->arena.take(nm * 8);
  float* t1 = f64 ? nullptr : (float*)ctx->arena.take(nm * 4);
  float* t2 = f64 ? nullptr : (float*)ctx->arena.take(nm * 4);
  double* G = (double*)ctx->arena.take((size_t)m * m * 8);
  double* Rinv = (double*)ctx->arena.take((size_t)m * m * 8);
  double* evecs = (double*)ctx->arena.take((size_t)m * m * 8);
  double* evals = (double*)ctx->arena.take((size_t)m * 8);
  int* okd = (int*)ctx->arena.take(64);
  if (!Qb || !Yb || (!f64 && (!t1 || !t2)) || !G || !Rinv || !evecs || !evals || !okd)
    return fail(LD_ENOMEM, "precond: scratch arena too small");
  hipStream_t st = ctx->stream;

  // 1-2. Gaussian test matrix and range finder
  launch_fill_gaussian(st, stream_key(seed, kStreamOmega), n, m, Qb);
  LD_TRY(apply_M64(ctx, op, Xp, Qb, Yb, m, t1, t2));
  double* Q = nullptr;
  // intermediate bases are made orthonormal too (a shifted pass and a plain
  // one): after a shifted pass alone the small singular values of the basis
  // are only partly restored, the next product scales them by the ratio of
  // M's extreme eigenvalues again, and over several power iterations the
  // sketch's condition number grows past what CholeskyQR can handle.  The
  // basis used for the Rayleigh-Ritz step gets three passes.
  LD_TRY(orthonormalize(ctx, Yb, Qb, n, m, G, Rinv, okd, power_iters == 0 ? 3 : 2, &Q));
  // 3. subspace iterations
  for (int it = 0; it < power_iters; ++it) {
    double* other = (Q == Qb) ? Yb : Qb;
    LD_TRY(apply_M64(ctx, op, Xp, Q, other, m, t1, t2));
    LD_TRY(orthonormalize(ctx, other, Q, n, m, G, Rinv, okd, it + 1 == power_iters ? 3 : 2, &Q));
  }
  // 4. B = Q^T M Q and its eigenpairs
  double* MQ = (Q == Qb) ? Yb : Qb;
  LD_TRY(apply_M64(ctx, op, Xp, Q, MQ, m, t1, t2));
  {
    const size_t mark = ctx->arena.top;
    LD_TRY(gram64(ctx, Q, MQ, nullptr, n, m, G));
    ctx->arena.top = mark;
  }
  {
    const size_t mark = ctx->arena.top;
    LD_TRY(jacobi_eigh(ctx, G, m, evals, evecs));
    ctx->arena.top = mark;
  }
  LD_TRY(ensure_pinned(ctx, (size_t)m + 8));
  LD_HIP(hipMemcpyAsync(ctx->pinned, evals, (size_t)m * 8, hipMemcpyDeviceToHost, st));
  LD_HIP(hipStreamSynchronize(st));
  for (int j = 0; j < rank; ++j)
    if (!(ctx->pinned[j] > 0.0) || !std::isfinite(ctx->pinned[j]))
      return fail(LD_ENOTSPD, "projected matrix has a non-positive eigenvalue among the kept ones");

  // 5. factors
  ld_precond* P = nullptr;
  LD_TRY(alloc_precond(ctx, n, rank, &P));
  // U = Q V_l, lam = top eigenvalues
  launch_gemm64(st, Q, evecs, m, nullptr, n, m, rank, P->U);
  if (hipMemcpyAsync(P->lam, evals, (size_t)rank * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) {
    ld_precond_free(P);
    return fail(LD_EHIP, "copy of eigenvalues failed");
  }
  const ld_status s_ = finish_precond(ctx, op, P, const_d, G, Rinv, okd, evals);
  if (s_ != LD_OK) return s_;
  *out = P;
  return LD_OK;
}


// ------------------------------------------------- preconditioner family --
// Greedy pivoted partial Cholesky (the Appendix's partial Cholesky
// preconditioner): rank steps of
//   p = argmax res (first index on ties),  C[:, k] = (M[:, p] - C C[p, :]^T) / sqrt(res[p]),
//   res -= C[:, k]^2, res[p] = 0,
// in FP64, with M's column p read from the stored matrix (FP64 or FP32) or
// generated in FP64 from the points.  C is n x rank row-major (the U of
// P = D + C C^T with lam = 1).
__global__ void k_pc_res_init(double* __restrict__ res, int64_t n, const void* __restrict__ Mst,
                              int mprec, int layout, double diag_const) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double dm = diag_const;
    if (Mst) {
      const int64_t ii = stored_index(i, i, n, layout, mprec == LD_F64);
      dm = mprec == LD_F64 ? ((const double*)Mst)[ii] : (double)((const float*)Mst)[ii];
    }
    res[i] = dm;
  }
}

// one workgroup: piv[k] = first index of the largest res, pivval[k] = res[piv]
__global__ __launch_bounds__(1024) void k_pc_argmax(const double* __restrict__ res, int64_t n,
                                                    int k, int* __restrict__ piv,
                                                    double* __restrict__ pivval) {
  __shared__ double bv[1024];
  __shared__ int64_t bi[1024];
  double v = -1.0;
  int64_t idx = n;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double r = res[i];
    if (r > v) {  // strictly larger: keeps the first index among equal values
      v = r;
      idx = i;
    }
  }
  bv[threadIdx.x] = v;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double o = bv[threadIdx.x + w];
      const int64_t oi = bi[threadIdx.x + w];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    piv[k] = (int)bi[0];
    pivval[k] = bv[0];
  }
}

template <int KIND>
__global__ void k_pc_column(const double* __restrict__ X, int d, double var, double c,
                            double noise, const void* __restrict__ Mst, int mprec, int layout,
                            int64_t n, int rank, int k, const int* __restrict__ piv,
                            const double* __restrict__ pivval, double* __restrict__ C,
                            double* __restrict__ res) {
  const int64_t p = piv[k];
  const double inv = 1.0 / sqrt(pivval[k]);
  const double* cp = C + p * rank;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double m;
    if (Mst) {
      const int64_t ii = stored_index(i, p, n, layout, mprec == LD_F64);
      m = mprec == LD_F64 ? ((const double*)Mst)[ii] : (double)((const float*)Mst)[ii];
    } else {
      double r2 = 0.0;
      for (int dd = 0; dd < d; ++dd) {
        const double df = X[i * d + dd] - X[p * d + dd];
        r2 = fma(df, df, r2);
      }
      m = dev::kval64<KIND>(r2, var, c) + (i == p ? noise : 0.0);
    }
    const double* ci = C + i * rank;
    double sdot = 0.0;
    for (int l = 0; l < k; ++l) sdot = fma(ci[l], cp[l], sdot);
    const double v = (m - sdot) * inv;
    C[i * rank + k] = v;
    res[i] = i == p ? 0.0 : res[i] - v * v;
  }
}

__global__ void k_fill(double* __restrict__ a, int64_t count, double v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
    a[i] = v;
}

// Preconditioners of the Appendix's list other than the randomized SVD:
// identity and diagonal (rank 0), and partial Cholesky; const_d > 0 gives
// the "plus scaling" D = const_d I.
ld_status build_precond_simple(ld_ctx* ctx, const ld_operator* op, int kind, int rank,
                               double const_d, ld_precond** out) {
  const int64_t n = op->n;
  if (kind != LD_PRECOND_PCHOL) rank = 0;
  ctx->arena.reset();
  LD_TRY(ctx->arena.reserve(simple_precond_scratch_bytes(op, rank)));
  double* res = (double*)ctx->arena.take((size_t)n * 8);
  double* G = (double*)ctx->arena.take((size_t)std::max(rank, 1) * std::max(rank, 1) * 8);
  double* Rinv = (double*)ctx->arena.take((size_t)std::max(rank, 1) * std::max(rank, 1) * 8);
  int* piv = (int*)ctx->arena.take((size_t)std::max(rank, 1) * 4);
  double* pivval = (double*)ctx->arena.take((size_t)std::max(rank, 1) * 8);
  double* parts = (double*)ctx->arena.take(64);
  int* okd = (int*)ctx->arena.take(64);
  if (!res || !G || !Rinv || !piv || !pivval || !parts || !okd)
    return fail(LD_ENOMEM, "precond: scratch arena too small");
  hipStream_t st = ctx->stream;
  ld_precond* P = nullptr;
  LD_TRY(alloc_precond(ctx, n, rank, &P));
  if (kind == LD_PRECOND_IDENTITY) const_d = 1.0;
  if (kind == LD_PRECOND_PCHOL) {
    const KParams kp = make_kparams(*op);
    const double c = kp.kind == LD_RBF ? kp.c_rbf : kp.c_mat;
    hipLaunchKernelGGL(k_pc_res_init, dim3(grid1(n)), dim3(256), 0, st, res, n, op->M_stored,
                       op->precision, op->layout, op->variance + op->noise);
    for (int k = 0; k < rank; ++k) {
      hipLaunchKernelGGL(k_pc_argmax, dim3(1), dim3(1024), 0, st, res, n, k, piv, pivval);
      if (kp.kind == LD_RBF)
        hipLaunchKernelGGL(k_pc_column<LD_RBF>, dim3(grid1(n)), dim3(256), 0, st,
                           (const double*)op->X, op->d,
                           op->variance, c, op->noise, op->M_stored, op->precision, op->layout, n,
                           rank, k, piv, pivval, P->U, res);
      else
        hipLaunchKernelGGL(k_pc_column<LD_MATERN52>, dim3(grid1(n)), dim3(256), 0, st,
                           (const double*)op->X, op->d, op->variance, c, op->noise, op->M_stored, op->precision,
                           op->layout, n, rank, k, piv, pivval, P->U, res);
    }
    hipLaunchKernelGGL(k_fill, dim3(grid1(rank)), dim3(256), 0, st, P->lam, (int64_t)rank, 1.0);
    if (hipGetLastError() != hipSuccess) {
      ld_precond_free(P);
      return fail(LD_EHIP, "kernel launch failed");
    }
  }
  LD_TRY(finish_precond(ctx, op, P, const_d, G, Rinv, okd, parts));
  *out = P;
  return LD_OK;
}

}  // namespace
}  // namespace ld

using namespace ld;

extern "C" {

const char* ld_last_error(void) { return ld::g_err.c_str(); }

ld_status ld_ctx_create(int device, void* stream, ld_ctx** out) {
  if (!out) return fail(LD_EINVAL, "out is NULL");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return fail(LD_EHIP, "no HIP device available");
  }
  if (device < 0 || device >= count) return fail(LD_EINVAL, "device index out of range");
  LD_HIP(hipSetDevice(device));
  ld_ctx* c = new ld_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0)
    c->num_cu = cu;
  const ld_status st = static_scratch_address(device, &c->static_scratch);
  if (st != LD_OK) {
    delete c;
    return st;
  }
  *out = c;
  return LD_OK;
}

void ld_ctx_destroy(ld_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
  }
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  ctx->arena.release();
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
}

ld_status ld_set_workspace(ld_ctx* ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return fail(LD_EINVAL, "context is NULL");
  if ((dev_ptr == nullptr) != (bytes == 0))
    return fail(LD_EINVAL, "pass a buffer and its size, or NULL and 0");
  if (dev_ptr && ((uintptr_t)dev_ptr & 255) != 0)
    return fail(LD_EINVAL, "the workspace must be 256-byte aligned");
  LD_HIP(hipSetDevice(ctx->device));
  // enqueued work may still use the current block
  LD_HIP(hipStreamSynchronize(ctx->stream));
  if (ctx->side) LD_HIP(hipStreamSynchronize(ctx->side));
  ctx->arena.release();
  if (dev_ptr) {
    ctx->arena.base = (char*)dev_ptr;
    ctx->arena.cap = bytes;
    ctx->arena.external = true;
  }
  return LD_OK;
}

size_t ld_workspace_bytes(const ld_operator* op, int64_t s, int32_t rank, int32_t oversample,
                          int32_t k) {
  if (check_operator(op, false) != LD_OK) return 0;
  Rational rf;
  if (s < 1 || rank < 1 || oversample < 0 || (int64_t)rank + oversample > op->n ||
      !rational_for(k, &rf)) {
    fail(LD_EINVAL, "need s >= 1, 1 <= rank, oversample >= 0, rank + oversample <= n, k in {1, 3, 5}");
    return 0;
  }
  // a context only for sizing: the product's plan depends on the CU count
  ld_ctx sz;
  int dev = 0, cu = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
    sz.num_cu = cu;
  else
    (void)hipGetLastError();
  const bool f64 = is_f64(op);
  const int64_t n = op->n;
  // the default preconditioner logdet_estimate builds when P is NULL
  const int drank = (int)std::min<int64_t>(100, std::max<int64_t>(1, n / 10));
  const int dover = (int)std::min<int64_t>(10, n - drank);
  size_t need = matmat_call_bytes(&sz, op, s);
  need = std::max(need, rsvd_scratch_bytes(&sz, op, rank, oversample));
  need = std::max(need, rsvd_scratch_bytes(&sz, op, drank, dover));
  need = std::max(need, simple_precond_scratch_bytes(op, rank));
  need = std::max(need, woodbury_scratch_bytes(n, rank, s));
  // estimators: any probe kind, up to every pole of r_1, r_3, r_5 at once,
  // Algorithm 1 up to LD_LANCZOS_MAX steps, and the gradient
  const size_t solver = std::max(pcg_scratch_bytes(&sz, f64, n, rank, s, kMaxShifts),
                                 lanczos_scratch_bytes(&sz, f64, n, rank, s, LD_LANCZOS_MAX));
  need = std::max(need, est_scratch_bytes(op, s, LD_PROBE_ORTHOGONAL, solver, 0));
  need = std::max(need, est_scratch_bytes(op, s, LD_PROBE_ORTHOGONAL,
                                          pcg_scratch_bytes(&sz, f64, n, rank, s, 1),
                                          gradient_extra_bytes(&sz, op, s)));
  return need;
}

ld_status ld_ctx_set_timing(ld_ctx* ctx, int32_t on) {
  if (!ctx) return fail(LD_EINVAL, "context is NULL");
  ctx->timing = on != 0;
  ctx->mm_ms = 0.0;
  ctx->mm_calls = 0;
  ctx->mm_flops = 0.0;
  ctx->mm_bytes = 0.0;
  return LD_OK;
}

ld_status ld_ctx_set_graphs(ld_ctx* ctx, int32_t on) {
  if (!ctx) return fail(LD_EINVAL, "context is NULL");
  ctx->graphs = on != 0;
  return LD_OK;
}

ld_status ld_ctx_set_symmetric(ld_ctx* ctx, int32_t forms) {
  if (!ctx) return fail(LD_EINVAL, "context is NULL");
  if (forms & ~(LD_SYM_F32 | LD_SYM_BF16)) return fail(LD_EINVAL, "unknown symmetric-split form bits");
  ctx->symmetric = forms;
  return LD_OK;
}

ld_status ld_ctx_set_probes(ld_ctx* ctx, int32_t kind) {
  if (!ctx) return fail(LD_EINVAL, "context is NULL");
  if (kind != LD_PROBE_RADEMACHER && kind != LD_PROBE_GAUSSIAN && kind != LD_PROBE_ORTHOGONAL)
    return fail(LD_EINVAL, "unknown probe kind");
  ctx->probe_kind = kind;
  return LD_OK;
}

ld_status ld_ctx_read_timing(ld_ctx* ctx, double* ms, int64_t* calls, double* flops, double* bytes) {
  if (!ctx) return fail(LD_EINVAL, "context is NULL");
  if (ctx->ev_used) {
    LD_HIP(hipStreamSynchronize(ctx->stream));
    timing_collect(ctx);
  }
  if (ms) *ms = ctx->mm_ms;
  if (calls) *calls = ctx->mm_calls;
  if (flops) *flops = ctx->mm_flops;
  if (bytes) *bytes = ctx->mm_bytes;
  return LD_OK;
}

int64_t ld_stored_elements(int64_t n, int32_t layout) {
  if (n < 1 || (layout != LD_ROW_MAJOR && layout != LD_TILED)) return -1;
  return stored_elements(n, layout);
}

ld_status ld_rational_coeffs(int32_t k, double* b, double* a, double* c) {
  if (!b || !a || !c) return fail(LD_EINVAL, "null output pointer");
  Rational r;
  if (!rational_for(k, &r)) return fail(LD_EINVAL, "k must be 1, 3 or 5");
  *b = r.b;
  for (int j = 0; j < k; ++j) {
    a[j] = r.a[j];
    c[j] = r.c[j];
  }
  return LD_OK;
}

ld_status ld_fill_probes(ld_ctx* ctx, uint64_t seed, int64_t n, int64_t s, int32_t precision, void* Z) {
  LD_TRY(check_ctx(ctx));
  if (n < 1 || s < 1 || !Z) return fail(LD_EINVAL, "bad probe block arguments");
  if (precision != LD_F64 && precision != LD_F32 && precision != LD_BF16)
    return fail(LD_EINVAL, "bad precision");
  launch_fill_rademacher(ctx->stream, stream_key(seed, kStreamProbes), n, s, precision == LD_F64, Z);
  LD_HIP(hipGetLastError());
  return LD_OK;
}

ld_status ld_fill_gaussian(ld_ctx* ctx, uint64_t seed, int32_t stream, int64_t rows, int64_t cols,
                           double* out) {
  LD_TRY(check_ctx(ctx));
  if (rows < 1 || cols < 1 || !out || stream < 0) return fail(LD_EINVAL, "bad gaussian block arguments");
  launch_fill_gaussian(ctx->stream, stream_key(seed, stream), rows, cols, out);
  LD_HIP(hipGetLastError());
  return LD_OK;
}

ld_status kernel_matmat(ld_ctx* ctx, const ld_operator* op, const void* V, int64_t s, void* Y) {
  LD_TRY(check_ctx(ctx));
  LD_TRY(check_operator(op));
  if (!V || !Y || s < 1) return fail(LD_EINVAL, "bad V / Y / s");
  if (V == Y) return fail(LD_EINVAL, "Y must not alias V");
  const bool f64 = is_f64(op);
  ctx->arena.reset();
  LD_TRY(ctx->arena.reserve(matmat_call_bytes(ctx, op, s)));
  const void* Xp = nullptr;
  LD_TRY(path_points(ctx, op, &Xp));
  MatmatArgs a = base_args(op, Xp);
  a.s = s;
  a.V = V;
  a.Y = Y;
  return matmat(ctx, f64, a);
}

ld_status kernel_matmat_noalloc(ld_ctx* ctx, const ld_operator* op, const void* V, int64_t s,
                                void* Y) {
  LD_TRY(check_ctx(ctx));
  LD_TRY(check_operator(op));
  if (!V || !Y || s < 1) return fail(LD_EINVAL, "bad V / Y / s");
  if (V == Y) return fail(LD_EINVAL, "Y must not alias V");
  // the same path as kernel_matmat without symmetric reuse (whose partial
  // sums grow as n^2), with the context's arena pointed at the static
  // scratch for this call (external: never grown, never freed)
  struct Swap {
    ld_ctx* c;
    Arena saved;
    int symmetric;
    ~Swap() {
      c->arena = saved;
      c->symmetric = symmetric;
    }
  } swap{ctx, ctx->arena, ctx->symmetric};
  ctx->symmetric = 0;
  const size_t need = matmat_call_bytes(ctx, op, s);
  if (need > kStaticScratchBytes)
    return fail(LD_EINVAL, "kernel_matmat_noalloc: this product needs " + std::to_string(need) +
                               " bytes of scratch; the static scratch holds " +
                               std::to_string(kStaticScratchBytes));
  if (!ctx->static_scratch) return fail(LD_EHIP, "kernel_matmat_noalloc: no static scratch");
  ctx->arena = Arena();
  ctx->arena.base = (char*)ctx->static_scratch;
  ctx->arena.cap = kStaticScratchBytes;
  ctx->arena.external = true;
  const void* Xp = nullptr;
  LD_TRY(path_points(ctx, op, &Xp));
  MatmatArgs a = base_args(op, Xp);
  a.s = s;
  a.V = V;
  a.Y = Y;
  return matmat(ctx, is_f64(op), a);
}

ld_status kernel_materialize(ld_ctx* ctx, const ld_operator* op, void* M_out) {
  LD_TRY(check_ctx(ctx));
  LD_TRY(check_operator(op, false));
  if (!M_out) return fail(LD_EINVAL, "M_out is NULL");
  if (op->precision == LD_BF16 && op->layout != LD_TILED)
    return fail(LD_EINVAL, "a stored LD_BF16 matrix must use the LD_TILED layout");
  launch_materialize(ctx->stream, make_kparams(*op), op->X, op->n, op->d, op->precision, op->layout,
                     M_out);
  LD_HIP(hipGetLastError());
  return LD_OK;
}

ld_status logdet_precond_build(ld_ctx* ctx, const ld_operator* op, int32_t rank, int32_t oversample,
                               int32_t power_iters, uint64_t seed, ld_precond** out) {
  LD_TRY(check_ctx(ctx));
  LD_TRY(check_operator(op));
  if (!out) return fail(LD_EINVAL, "out is NULL");
  if (rank < 1 || oversample < 0 || (int64_t)rank + oversample > op->n)
    return fail(LD_EINVAL, "need 1 <= rank and rank + oversample <= n");
  if (rank + oversample > 4096) return fail(LD_EINVAL, "rank + oversample must be <= 4096");
  if (power_iters < 0 || power_iters > 16) return fail(LD_EINVAL, "power_iters must be in 0..16");
  return build_precond(ctx, op, rank, oversample, power_iters, seed, out, 0.0);
}

ld_status logdet_precond_build_kind(ld_ctx* ctx, const ld_operator* op, int32_t kind,
                                    int32_t rank, int32_t oversample, int32_t power_iters,
                                    uint64_t seed, int32_t flags, ld_precond** out) {
  LD_TRY(check_ctx(ctx));
  LD_TRY(check_operator(op));
  if (!out) return fail(LD_EINVAL, "out is NULL");
  if (flags & ~LD_PRECOND_SCALED) return fail(LD_EINVAL, "unknown flags");
  const bool scaled = (flags & LD_PRECOND_SCALED) != 0;
  if (scaled && !(op->noise > 0.0))
    return fail(LD_EINVAL, "LD_PRECOND_SCALED needs noise > 0 (D = noise I)");
  const double const_d = scaled ? op->noise : 0.0;
  switch (kind) {
    case LD_PRECOND_RSVD:
    case LD_PRECOND_RANK_ONE: {
      if (kind == LD_PRECOND_RANK_ONE) rank = 1;
      if (rank < 1 || oversample < 0 || (int64_t)rank + oversample > op->n)
        return fail(LD_EINVAL, "need 1 <= rank and rank + oversample <= n");
      if (rank + oversample > 4096) return fail(LD_EINVAL, "rank + oversample must be <= 4096");
      if (power_iters < 0 || power_iters > 16) return fail(LD_EINVAL, "power_iters must be in 0..16");
      return build_precond(ctx, op, rank, oversample, power_iters, seed, out, const_d);
    }
    case LD_PRECOND_IDENTITY:
    case LD_PRECOND_DIAGONAL:
      if (scaled) return fail(LD_EINVAL, "LD_PRECOND_SCALED applies to low-rank preconditioners");
      return build_precond_simple(ctx, op, kind, 0, 0.0, out);
    case LD_PRECOND_PCHOL:
      if (rank < 1 || rank > op->n || rank > 4096)
        return fail(LD_EINVAL, "partial Cholesky needs 1 <= rank <= min(n, 4096)");
      return build_precond_simple(ctx, op, kind, rank, const_d, out);
    default:
      return fail(LD_EINVAL, "unknown preconditioner kind");
  }
}

ld_status ld_precond_info(const ld_precond* P, int64_t* n, int32_t* rank, double* logdet_P) {
  if (!P) return fail(LD_EINVAL, "preconditioner is NULL");
  if (n) *n = P->n;
  if (rank) *rank = P->rank;
  if (logdet_P) *logdet_P = P->logdet;
  return LD_OK;
}

ld_status ld_precond_export(ld_ctx* ctx, const ld_precond* P, double* U, double* lambda, double* D) {
  LD_TRY(check_ctx(ctx));
  if (!P) return fail(LD_EINVAL, "preconditioner is NULL");
  hipStream_t st = ctx->stream;
  if (U) LD_HIP(hipMemcpyAsync(U, P->U, (size_t)P->n * P->rank * 8, hipMemcpyDeviceToDevice, st));
  if (lambda) LD_HIP(hipMemcpyAsync(lambda, P->lam, (size_t)P->rank * 8, hipMemcpyDeviceToDevice, st));
  if (D) LD_HIP(hipMemcpyAsync(D, P->D, (size_t)P->n * 8, hipMemcpyDeviceToDevice, st));
  return LD_OK;
}

ld_status ld_precond_apply_inverse(ld_ctx* ctx, const ld_precond* P, const void* R, int64_t s,
                                   int32_t precision, void* OUT) {
  LD_TRY(check_ctx(ctx));
  if (!P || !R || !OUT || s < 1) return fail(LD_EINVAL, "bad arguments");
  if (R == OUT) return fail(LD_EINVAL, "OUT must not alias R");
  if (precision != LD_F64 && precision != LD_F32 && precision != LD_BF16)
    return fail(LD_EINVAL, "bad precision");
  ctx->arena.reset();
  LD_TRY(ctx->arena.reserve(woodbury_scratch_bytes(P->n, P->rank, s)));
  return woodbury_apply(ctx, P, precision == LD_F64, R, s, OUT);
}

void ld_precond_free(ld_precond* P) {
  if (!P) return;
  (void)hipSetDevice(P->device);
  (void)hipDeviceSynchronize();
  if (P->block) (void)hipFree(P->block);
  delete P;
}

namespace {

// per-column dot products A^T B (n x s each, FP64) as 256-row block partials
// parts[blk][c], summed in a fixed order
__global__ __launch_bounds__(256) void k_coldot_parts(const double* __restrict__ A,
                                                      const double* __restrict__ B, int64_t n,
                                                      int64_t s, double* __restrict__ parts) {
  __shared__ double red[4][64];
  const int tid = threadIdx.x, cl = tid & 63, grp = tid >> 6;
  const int64_t c = (int64_t)blockIdx.y * 64 + cl;
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  const int64_t r1 = r0 + 256 < n ? r0 + 256 : n;
  double acc = 0.0;
  if (c < s)
    for (int64_t i = r0 + grp; i < r1; i += 4) acc += A[i * s + c] * B[i * s + c];
  red[grp][cl] = acc;
  __syncthreads();
  if (grp == 0 && c < s)
    parts[blockIdx.x * s + c] = ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}

__global__ void k_parts_sum(const double* __restrict__ parts, int64_t nblk, int64_t s,
                            double* __restrict__ out) {
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < s; c += (int64_t)gridDim.x * 256) {
    double acc = 0.0;
    for (int64_t b = 0; b < nblk; ++b) acc += parts[b * s + c];
    out[c] = acc;
  }
}

}  // namespace

namespace {

Coef coef_of(const Rational& rf, int k) {
  Coef cf{};
  cf.b = rf.b;
  cf.J = k;
  for (int j = 0; j < k; ++j) {
    cf.a[j] = rf.a[j];
    cf.c[j] = rf.c[j];
  }
  return cf;
}

bool same_pole(double x, double y) { return std::fabs(x - y) <= 1e-12 * std::max(x, y); }

// Coefficients of several orders over the union of their poles, ascending
// (the smallest is the CG's seed; a pole shared by several orders, such as 1,
// is one shift).  Each order weighs its own poles with its Table 1 residues
// and the others with 0.
ld_status orders_coefs(int32_t num_orders, const int32_t* ks, Coef* cfs) {
  if (!ks) return fail(LD_EINVAL, "ks is NULL");
  if (num_orders < 1 || num_orders > 3) return fail(LD_EINVAL, "num_orders must be in 1..3");
  Rational rf[3];
  for (int o = 0; o < num_orders; ++o) {
    if (!rational_for(ks[o], &rf[o])) return fail(LD_EINVAL, "every k must be 1, 3 or 5");
    for (int q = 0; q < o; ++q)
      if (ks[q] == ks[o]) return fail(LD_EINVAL, "orders must be distinct");
  }
  std::vector<double> sh;
  for (int o = 0; o < num_orders; ++o)
    for (int m = 0; m < ks[o]; ++m) {
      bool seen = false;
      for (double x : sh) seen = seen || same_pole(x, rf[o].a[m]);
      if (!seen) sh.push_back(rf[o].a[m]);
    }
  std::sort(sh.begin(), sh.end());
  for (int o = 0; o < num_orders; ++o) {
    Coef& cf = cfs[o];
    cf = Coef{};
    cf.b = rf[o].b;
    cf.J = (int)sh.size();
    for (int j = 0; j < cf.J; ++j) {
      cf.a[j] = sh[j];
      for (int m = 0; m < ks[o]; ++m)
        if (same_pole(sh[j], rf[o].a[m])) cf.c[j] = rf[o].c[m];
    }
  }
  return LD_OK;
}

// Shared set-up of the single-problem estimators: validation, the default
// preconditioner when P is NULL, the scratch arena, the points in the
// path's precision and the Rademacher probe block (Algorithm 1 step 1).
struct EstSetup {
  Rational rf;
  const ld_precond* P = nullptr;
  ld_precond* own = nullptr;
  bool f64 = false;
  const void* Xp = nullptr;
  void* Z = nullptr;
  double precond_s = 0.0;  // the default preconditioner's build, when P was NULL
  ~EstSetup() {
    if (own) ld_precond_free(own);
  }
};

ld_status est_setup(ld_ctx* ctx, const ld_operator* op, const ld_precond* P, int32_t k,
                    int32_t num_probes, uint64_t probe_seed, size_t solver_bytes_extra,
                    size_t (*solver_bytes)(ld_ctx*, bool, int64_t, int, int64_t, int), int arg,
                    EstSetup& e) {
  LD_TRY(check_ctx(ctx));
  LD_TRY(check_operator(op));
  if (!rational_for(k, &e.rf)) return fail(LD_EINVAL, "k must be 1, 3 or 5");
  if (num_probes < 1) return fail(LD_EINVAL, "num_probes must be >= 1");
  if (P && P->n != op->n) return fail(LD_EINVAL, "preconditioner size does not match the operator");
  if (!P) {
    int rank = (int)std::min<int64_t>(100, std::max<int64_t>(1, op->n / 10));
    int over = (int)std::min<int64_t>(10, op->n - rank);
    const auto tp = std::chrono::steady_clock::now();
    LD_TRY(build_precond(ctx, op, rank, over, 2, probe_seed + 1, &e.own, 0.0));
    e.precond_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - tp).count();
    P = e.own;
  }
  e.P = P;
  e.f64 = is_f64(op);
  const int64_t n = op->n, s = num_probes;
  const int pk = ctx->probe_kind;
  if (pk == LD_PROBE_ORTHOGONAL && s > n)
    return fail(LD_EINVAL, "orthogonal probes need num_probes <= n");
  const size_t es = e.f64 ? 8 : 4;
  ctx->arena.reset();
  LD_TRY(ctx->arena.reserve(est_scratch_bytes(op, s, pk, solver_bytes(ctx, e.f64, n, P->rank, s, arg),
                                              solver_bytes_extra)));
  LD_TRY(path_points(ctx, op, &e.Xp));
  e.Z = ctx->arena.take((size_t)n * s * es);
  if (!e.Z) return fail(LD_ENOMEM, "scratch arena too small for probes");
  const uint64_t key = stream_key(probe_seed, kStreamProbes);
  hipStream_t st = ctx->stream;
  if (pk == LD_PROBE_RADEMACHER) {
    launch_fill_rademacher(st, key, n, s, e.f64, e.Z);
    LD_HIP(hipGetLastError());
    return LD_OK;
  }
  const size_t mark = ctx->arena.top;
  double* Gb = (double*)ctx->arena.take((size_t)n * s * 8);
  double* Wb = (double*)ctx->arena.take((size_t)n * s * 8);
  double* gram = (double*)ctx->arena.take((size_t)s * s * 8);
  double* g2 = (double*)ctx->arena.take((size_t)s * s * 8);
  double* rinv = (double*)ctx->arena.take((size_t)s * s * 8);
  double* norms = (double*)ctx->arena.take((size_t)s * 8);
  int* okd = (int*)ctx->arena.take(64);
  if (!Gb || !Wb || !gram || !g2 || !rinv || !norms || !okd)
    return fail(LD_ENOMEM, "scratch arena too small for probes");
  launch_fill_gaussian(st, key, n, s, Gb);
  const double* W = Gb;
  if (pk == LD_PROBE_ORTHOGONAL) {
    {
      const size_t m2 = ctx->arena.top;
      LD_TRY(gram64(ctx, Gb, Gb, nullptr, n, (int)s, gram));
      ctx->arena.top = m2;
    }
    hipLaunchKernelGGL(k_sqrt_diag, dim3(grid1(s)), dim3(256), 0, st, gram, (int)s, norms);
    double* Q = nullptr;
    LD_TRY(orthonormalize(ctx, Gb, Wb, n, (int)s, g2, rinv, okd, 3, &Q));
    hipLaunchKernelGGL(k_scale_cols64, dim3(grid1(n * s)), dim3(256), 0, st, Q, norms, n, s);
    W = Q;
  }
  if (e.f64)
    LD_HIP(hipMemcpyAsync(e.Z, W, (size_t)n * s * 8, hipMemcpyDeviceToDevice, st));
  else
    launch_convert_f64_to_f32(st, W, (float*)e.Z, n * s);
  LD_HIP(hipGetLastError());
  // the FP64 blocks are free again once the copy above has run (stream order)
  ctx->arena.top = mark;
  return LD_OK;
}

}  // namespace

ld_status logdet_estimate(ld_ctx* ctx, const ld_operator* op, const ld_precond* P, int32_t k,
                          int32_t num_probes, uint64_t probe_seed, double tol, int32_t max_iters,
                          ld_result* out, double* per_probe) {
  if (!out) return fail(LD_EINVAL, "out is NULL");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(LD_EINVAL, "tol must be finite and > 0");
  if (max_iters < 1) return fail(LD_EINVAL, "max_iters must be >= 1");
  EstSetup e;
  LD_TRY(est_setup(ctx, op, P, k, num_probes, probe_seed, 0, pcg_scratch_bytes, k, e));
  const int64_t s = num_probes;
  auto t0 = std::chrono::steady_clock::now();
  std::vector<double> t;
  double mean = 0.0, se = 0.0;
  int iters = 0, conv = 0;
  double rr = 0.0;
  bool breakdown = false;
  LD_TRY(multishift_pcg(ctx, e.f64, base_args(op, e.Xp), e.P, coef_of(e.rf, k), e.Z, s, tol,
                        max_iters, t, &mean, &se, &iters, &conv, &rr, &breakdown));
  auto t1 = std::chrono::steady_clock::now();
  out->trace_term = mean;
  out->logdet_P = e.P->logdet;
  out->logdet = e.P->logdet + mean;
  out->std_err = se;
  out->rel_resid = rr;
  out->seconds_solve = std::chrono::duration<double>(t1 - t0).count();
  out->seconds_precond = e.precond_s;
  out->iterations = iters;
  out->converged_cols = conv;
  out->k = k;
  out->num_probes = num_probes;
  if (per_probe) std::memcpy(per_probe, t.data(), (size_t)s * sizeof(double));
  if (breakdown)
    return fail(LD_ENOTSPD, "non-positive curvature or residual norm in the solver (M or P not SPD?)");
  if (conv < s) return fail(LD_ENOCONV, "max_iters reached before every probe converged");
  return LD_OK;
}

ld_status logdet_estimate_orders(ld_ctx* ctx, const ld_operator* op, const ld_precond* P,
                                 int32_t num_orders, const int32_t* ks, int32_t num_probes,
                                 uint64_t probe_seed, double tol, int32_t max_iters,
                                 ld_result* out, double* per_probe) {
  if (!out) return fail(LD_EINVAL, "out is NULL");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(LD_EINVAL, "tol must be finite and > 0");
  if (max_iters < 1) return fail(LD_EINVAL, "max_iters must be >= 1");
  Coef cfs[3];
  LD_TRY(orders_coefs(num_orders, ks, cfs));
  const int J = cfs[0].J;
  EstSetup e;
  LD_TRY(est_setup(ctx, op, P, ks[0], num_probes, probe_seed, 0, pcg_scratch_bytes, J, e));
  const int64_t s = num_probes;
  auto t0 = std::chrono::steady_clock::now();
  std::vector<double> t;
  double mean[3] = {0.0, 0.0, 0.0}, se[3] = {0.0, 0.0, 0.0};
  int iters = 0, conv = 0;
  double rr = 0.0;
  bool breakdown = false;
  LD_TRY(multishift_pcg_multi(ctx, e.f64, base_args(op, e.Xp), e.P, cfs, num_orders, e.Z, s, tol,
                              max_iters, t, mean, se, &iters, &conv, &rr, &breakdown));
  auto t1 = std::chrono::steady_clock::now();
  for (int o = 0; o < num_orders; ++o) {
    ld_result& r = out[o];
    r = ld_result{};
    r.trace_term = mean[o];
    r.logdet_P = e.P->logdet;
    r.logdet = e.P->logdet + mean[o];
    r.std_err = se[o];
    r.rel_resid = rr;
    r.seconds_solve = std::chrono::duration<double>(t1 - t0).count();
    r.seconds_precond = e.precond_s;
    r.iterations = iters;
    r.converged_cols = conv;
    r.k = ks[o];
    r.num_probes = num_probes;
  }
  if (per_probe) std::memcpy(per_probe, t.data(), (size_t)num_orders * s * sizeof(double));
  if (breakdown)
    return fail(LD_ENOTSPD, "non-positive curvature or residual norm in the solver (M or P not SPD?)");
  if (conv < s) return fail(LD_ENOCONV, "max_iters reached before every probe converged");
  return LD_OK;
}

ld_status logdet_estimate_lanczos(ld_ctx* ctx, const ld_operator* op, const ld_precond* P,
                                  int32_t k, int32_t num_probes, uint64_t probe_seed,
                                  int32_t steps, ld_result* out, double* per_probe) {
  if (!out) return fail(LD_EINVAL, "out is NULL");
  if (steps < 1 || steps > LD_LANCZOS_MAX)
    return fail(LD_EINVAL, "steps must be in 1..LD_LANCZOS_MAX");
  EstSetup e;
  LD_TRY(est_setup(ctx, op, P, k, num_probes, probe_seed, 0, lanczos_scratch_bytes, steps, e));
  const int64_t s = num_probes;
  auto t0 = std::chrono::steady_clock::now();
  LzOut o;
  LD_TRY(lanczos_estimate(ctx, e.f64, base_args(op, e.Xp), e.P, coef_of(e.rf, k), e.Z, s, steps,
                          o));
  auto t1 = std::chrono::steady_clock::now();
  out->trace_term = o.mean;
  out->logdet_P = e.P->logdet;
  out->logdet = e.P->logdet + o.mean;
  out->std_err = o.stderr_;
  out->rel_resid = o.resid;
  out->seconds_solve = std::chrono::duration<double>(t1 - t0).count();
  out->seconds_precond = e.precond_s;
  out->iterations = o.max_steps;
  out->converged_cols = o.exact;
  out->k = k;
  out->num_probes = num_probes;
  if (per_probe) std::memcpy(per_probe, o.per_probe.data(), (size_t)s * sizeof(double));
  if (o.breakdown)
    return fail(LD_ENOTSPD, "non-positive or non-finite norm in the Lanczos recurrence (M or P not SPD?)");
  return LD_OK;
}

ld_status logdet_estimate_lanczos_orders(ld_ctx* ctx, const ld_operator* op, const ld_precond* P,
                                         int32_t num_orders, const int32_t* ks,
                                         int32_t num_probes, uint64_t probe_seed, int32_t steps,
                                         ld_result* out, double* per_probe) {
  if (!out) return fail(LD_EINVAL, "out is NULL");
  if (steps < 1 || steps > LD_LANCZOS_MAX)
    return fail(LD_EINVAL, "steps must be in 1..LD_LANCZOS_MAX");
  Coef cfs[3];
  LD_TRY(orders_coefs(num_orders, ks, cfs));
  EstSetup e;
  LD_TRY(est_setup(ctx, op, P, ks[0], num_probes, probe_seed, 0, lanczos_scratch_bytes, steps, e));
  const int64_t s = num_probes;
  auto t0 = std::chrono::steady_clock::now();
  LzOut o[3];
  LD_TRY(lanczos_estimate_multi(ctx, e.f64, base_args(op, e.Xp), e.P, cfs, num_orders, e.Z, s,
                                steps, o));
  auto t1 = std::chrono::steady_clock::now();
  for (int q = 0; q < num_orders; ++q) {
    ld_result& r = out[q];
    r = ld_result{};
    r.trace_term = o[q].mean;
    r.logdet_P = e.P->logdet;
    r.logdet = e.P->logdet + o[q].mean;
    r.std_err = o[q].stderr_;
    r.rel_resid = o[q].resid;
    r.seconds_solve = std::chrono::duration<double>(t1 - t0).count();
    r.seconds_precond = e.precond_s;
    r.iterations = o[q].max_steps;
    r.converged_cols = o[q].exact;
    r.k = ks[q];
    r.num_probes = num_probes;
    if (per_probe) std::memcpy(per_probe + q * s, o[q].per_probe.data(), (size_t)s * sizeof(double));
  }
  if (o[0].breakdown)
    return fail(LD_ENOTSPD, "non-positive or non-finite norm in the Lanczos recurrence (M or P not SPD?)");
  return LD_OK;
}

ld_status logdet_gradient(ld_ctx* ctx, const ld_operator* op, const ld_precond* P,
                          int32_t num_probes, uint64_t probe_seed, double tol, int32_t max_iters,
                          double* grad, double* std_err, double* per_probe, ld_result* out) {
  LD_TRY(check_ctx(ctx));
  LD_TRY(check_operator(op));
  if (op->d > 16) return fail(LD_EINVAL, "the derivative products are generated on the fly: d <= 16");
  if (!grad) return fail(LD_EINVAL, "grad is NULL");
  if (num_probes < 1) return fail(LD_EINVAL, "num_probes must be >= 1");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(LD_EINVAL, "tol must be finite and > 0");
  if (max_iters < 1) return fail(LD_EINVAL, "max_iters must be >= 1");
  const int64_t n = op->n, s = num_probes;
  const bool f64op = is_f64(op);
  const size_t es = f64op ? 8 : 4;
  const int64_t nblk = (n + 255) / 256;
  const size_t extra = gradient_extra_bytes(ctx, op, s);
  EstSetup e;
  LD_TRY(est_setup(ctx, op, P, 1, num_probes, probe_seed, extra, pcg_scratch_bytes, 1, e));
  hipStream_t st = ctx->stream;
  void* ysol = ctx->arena.take((size_t)n * s * es);
  double* z64 = (double*)ctx->arena.take((size_t)n * s * 8);
  double* y64 = (double*)ctx->arena.take((size_t)n * s * 8);
  double* az = (double*)ctx->arena.take((size_t)n * s * 8);
  double* parts = (double*)ctx->arena.take((size_t)nblk * s * 8);
  double* vals = (double*)ctx->arena.take((size_t)3 * s * 8);
  double* hut = (double*)ctx->arena.take((size_t)3 * (s + 2) * 8);
  if (!ysol || !z64 || !y64 || !az || !parts || !vals || !hut)
    return fail(LD_ENOMEM, "gradient: scratch arena too small");
  // y = M^-1 z by the preconditioned CG (shift 0)
  Coef cf{};
  cf.b = 0.0;
  cf.J = 1;
  cf.a[0] = 0.0;
  cf.c[0] = 1.0;
  std::vector<double> tmp;
  double mean = 0.0, se = 0.0, rr = 0.0;
  int iters = 0, conv = 0;
  bool breakdown = false;
  auto t0 = std::chrono::steady_clock::now();
  LD_TRY(multishift_pcg(ctx, e.f64, base_args(op, e.Xp), e.P, cf, e.Z, s, tol, max_iters, tmp,
                        &mean, &se, &iters, &conv, &rr, &breakdown, ysol));
  if (e.f64) {
    LD_HIP(hipMemcpyAsync(z64, e.Z, (size_t)n * s * 8, hipMemcpyDeviceToDevice, st));
    LD_HIP(hipMemcpyAsync(y64, ysol, (size_t)n * s * 8, hipMemcpyDeviceToDevice, st));
  } else {
    launch_convert_f32_to_f64(st, (const float*)e.Z, z64, n * s);
    launch_convert_f32_to_f64(st, (const float*)ysol, y64, n * s);
  }
  // (M^-1 z)^T (dM/dtheta) z: the derivative products in FP64 from the points
  const KParams kp = make_kparams(*op);
  const dim3 cd_grid((unsigned)nblk, (unsigned)((s + 63) / 64));
  for (int p = 0; p < 3; ++p) {
    const double* B = z64;
    if (p < 2) {
      MatmatArgs a{};
      a.n = n;
      a.s = s;
      a.d = op->d;
      a.kp = kp;
      a.kp.noise = 0.0;
      if (p == 0) {  // d/d lengthscale
        const double l = op->lengthscale;
        a.kp.kind = op->kind == LD_RBF ? dev::kKindRbfDl : dev::kKindMaternDl;
        a.kp.variance = op->kind == LD_RBF ? op->variance / (l * l * l) : op->variance / (3.0 * l);
      } else {  // d/d variance = K / variance
        a.kp.variance = 1.0;
      }
      a.X = op->X;
      a.V = z64;
      a.Y = az;
      const size_t mark = ctx->arena.top;
      LD_TRY(matmat(ctx, true, a));
      ctx->arena.top = mark;
      B = az;
    }
    hipLaunchKernelGGL(k_coldot_parts, cd_grid, dim3(256), 0, st, y64, B, n, s, parts);
    hipLaunchKernelGGL(k_parts_sum, dim3(1), dim3(256), 0, st, parts, nblk, s, vals + p * s);
    Coef one{};
    one.b = 0.0;
    one.J = 1;
    one.c[0] = 1.0;
    LD_TRY(hutchinson(ctx, vals + p * s, vals + p * s, s, one, hut + p * (s + 2),
                      hut + p * (s + 2) + s));
  }
  LD_HIP(hipGetLastError());
  LD_TRY(ensure_pinned(ctx, (size_t)3 * (s + 2) + 8));
  LD_HIP(hipMemcpyAsync(ctx->pinned, hut, (size_t)3 * (s + 2) * 8, hipMemcpyDeviceToHost, st));
  LD_HIP(hipStreamSynchronize(st));
  auto t1 = std::chrono::steady_clock::now();
  const double* hp = ctx->pinned;
  for (int p = 0; p < 3; ++p) {
    grad[p] = hp[p * (s + 2) + s];
    if (std_err) std_err[p] = hp[p * (s + 2) + s + 1];
    if (per_probe) std::memcpy(per_probe + p * s, hp + p * (s + 2), (size_t)s * 8);
  }
  if (out) {
    out->logdet_P = e.P->logdet;
    out->rel_resid = rr;
    out->seconds_solve = std::chrono::duration<double>(t1 - t0).count();
    out->seconds_precond = e.precond_s;
    out->iterations = iters;
    out->converged_cols = conv;
    out->num_probes = num_probes;
  }
  if (breakdown)
    return fail(LD_ENOTSPD, "non-positive curvature or residual norm in the solver (M or P not SPD?)");
  if (conv < s) return fail(LD_ENOCONV, "max_iters reached before every probe converged");
  return LD_OK;
}

ld_status logdet_estimate_batched(ld_ctx* ctx, int32_t count, const ld_instance* instances,
                                  int32_t k, int32_t num_probes, int32_t oversample,
                                  int32_t power_iters, double tol, int32_t max_iters,
                                  int32_t flags, ld_result* results, double* per_probe,
                                  double* lambda_out, int32_t lambda_stride) {
  LD_TRY(check_ctx(ctx));
  if (count < 1 || count > 4096) return fail(LD_EINVAL, "count must be in 1..4096");
  if (!instances || !results) return fail(LD_EINVAL, "instances or results is NULL");
  Rational rf;
  if (!rational_for(k, &rf)) return fail(LD_EINVAL, "k must be 1, 3 or 5");
  if (num_probes < 1 || num_probes > 64) return fail(LD_EINVAL, "num_probes must be in 1..64");
  if (oversample < 0) return fail(LD_EINVAL, "oversample must be >= 0");
  if (power_iters < 0 || power_iters > 16) return fail(LD_EINVAL, "power_iters must be in 0..16");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(LD_EINVAL, "tol must be finite and > 0");
  if (max_iters < 1) return fail(LD_EINVAL, "max_iters must be >= 1");
  if (flags & ~(LD_BATCH_GRAPH | LD_BATCH_RETUNE | LD_BATCH_PRECOND_ONLY | LD_BATCH_NO_SYMMETRIC))
    return fail(LD_EINVAL, "unknown flag bits");
  for (int32_t i = 0; i < count; ++i) {
    const ld_instance& x = instances[i];
    const std::string at = " (instance " + std::to_string(i) + ")";
    if (!x.X) return fail(LD_EINVAL, "X is NULL" + at);
    if (x.n < 1 || x.n > (int64_t)1 << 24) return fail(LD_EINVAL, "n must be in 1..2^24" + at);
    if (x.d < 1 || x.d > 8) return fail(LD_EINVAL, "d must be in 1..8" + at);
    if (x.kind != LD_RBF && x.kind != LD_MATERN52) return fail(LD_EINVAL, "unknown kernel kind" + at);
    if (!(x.lengthscale > 0.0) || !std::isfinite(x.lengthscale))
      return fail(LD_EINVAL, "lengthscale must be finite and > 0" + at);
    if (!(x.variance > 0.0) || !std::isfinite(x.variance))
      return fail(LD_EINVAL, "variance must be finite and > 0" + at);
    if (!(x.noise >= 0.0) || !std::isfinite(x.noise))
      return fail(LD_EINVAL, "noise must be finite and >= 0" + at);
    if (x.rank < 1 || (int64_t)x.rank + oversample > x.n || (int64_t)x.rank + oversample > 1024)
      return fail(LD_EINVAL, "need 1 <= rank and rank + oversample <= min(n, 1024)" + at);
    if (x.reserved != 0) return fail(LD_EINVAL, "reserved must be 0" + at);
    if (lambda_out && x.rank > lambda_stride) return fail(LD_EINVAL, "lambda_stride < rank" + at);
  }
  return batched_estimate(ctx, count, instances, k, rf.a, rf.b, rf.c, num_probes, oversample,
                          power_iters, tol, max_iters, flags, results, per_probe, lambda_out,
                          lambda_stride);
}

}  // extern "C"
