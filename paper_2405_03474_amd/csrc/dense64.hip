// FP64 dense algebra for the randomized truncated-SVD preconditioner
// (Section 2; Halko et al. Alg. 4.1 / 5.3): Gram products A^T diag(w) B,
// Cholesky, triangular inverse, tall GEMM on FP64 matrix cores, and a
// parallel cyclic Jacobi eigen-solver for the small projected matrix.  The
// workgroup-level bodies live in dense_dev.hpp and are shared with the
// batched kernels.
#include <cmath>
#include <vector>

#include "dense_dev.hpp"
#include "ld_common.hpp"

namespace ld {
namespace {

using dev::CT;
using dev::GM_BM;
using dev::GM_BN;

// ------------------------------------------------------------------ Gram --
// Partial G_c = A_c^T diag(w_c) B_c over row chunk c, one 64 x 64 output tile
// per workgroup on FP64 matrix cores (v_mfma_f64_16x16x4f64): wave w owns
// tile rows 32 (w / 2) .. + 32 and columns 32 (w % 2) .. + 32 as 2 x 2 blocks
// of 16 x 16.  Rows of A and B are staged through LDS GR at a time; in each
// 4-row step lane (l % 16, l / 16) supplies A(row l / 16, column l % 16) and
// the same element of B, and output register r of a block holds its row
// l / 16 + 4 r, column l % 16.
constexpr int GT = 64;
constexpr int GR = 32;

__global__ __launch_bounds__(256) void k_gram_partial(const double* __restrict__ A,
                                                      const double* __restrict__ B,
                                                      const double* __restrict__ w, int64_t n,
                                                      int m, int64_t chunk,
                                                      double* __restrict__ part) {
  __shared__ double As[GR][GT + 1];
  __shared__ double Bs[GR][GT + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lj = lane & 15, lh = lane >> 4;
  const int wi = 32 * (wave >> 1), wj = 32 * (wave & 1);
  const int i0 = blockIdx.y * GT, j0 = blockIdx.z * GT;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  int64_t r1 = r0 + chunk;
  if (r1 > n) r1 = n;
  dev::f64x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[x][y][r] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += GR) {
    __syncthreads();
    for (int e = tid; e < GR * GT; e += 256) {
      const int rr = e / GT, cc = e % GT;
      const int64_t row = rb + rr;
      double av = 0.0, bv = 0.0;
      if (row < r1) {
        const double wr = w ? w[row] : 1.0;
        if (i0 + cc < m) av = A[row * m + i0 + cc] * wr;
        if (j0 + cc < m) bv = B[row * m + j0 + cc];
      }
      As[rr][cc] = av;
      Bs[rr][cc] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GR; kk += 4) {
      const double a0 = As[kk + lh][wi + lj], a1 = As[kk + lh][wi + 16 + lj];
      const double b0 = Bs[kk + lh][wj + lj], b1 = Bs[kk + lh][wj + 16 + lj];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  double* dst = part + (int64_t)blockIdx.x * m * m;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wi + 16 * x + lh + 4 * r, j = j0 + wj + 16 * y + lj;
        if (i < m && j < m) dst[(int64_t)i * m + j] = acc[x][y][r];
      }
}

__global__ void k_sum_chunks(const double* __restrict__ part, int chunks, int64_t mm,
                             double* __restrict__ G) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < mm; e += (int64_t)gridDim.x * 256) {
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * mm + e];
    G[e] = s;
  }
}

// ------------------------------------------------------ factorizations --
__global__ __launch_bounds__(CT) void k_cholesky_upper(double* __restrict__ G, int m,
                                                       int* __restrict__ fail_flag) {
  dev::chol_upper_block(G, m, m, fail_flag);
}

__global__ __launch_bounds__(CT) void k_tri_inv_upper(const double* __restrict__ R, int m,
                                                      double* __restrict__ X) {
  dev::tri_inv_upper_block(R, m, m, X, m);
}

__global__ __launch_bounds__(256) void k_gemm64(const double* __restrict__ A,
                                                const double* __restrict__ B, int ldb,
                                                const double* __restrict__ rs, int64_t n, int K,
                                                int N, double* __restrict__ C) {
  dev::gemm64_tile(A, K, B, ldb, rs, n, K, N, C, N, (int64_t)blockIdx.x * GM_BM,
                   blockIdx.y * GM_BN);
}

// ---------------------------------------------------------------- Jacobi --
__global__ __launch_bounds__(256) void k_jacobi_round(const double* __restrict__ A,
                                                      double* __restrict__ A2,
                                                      const double* __restrict__ V,
                                                      double* __restrict__ V2, int me, int r) {
  dev::jacobi_item(A, A2, V, V2, me, r, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// out[0] = sum of squares off the diagonal, out[1] = on the diagonal
__global__ __launch_bounds__(256) void k_offnorm(const double* __restrict__ A, int me,
                                                 double* __restrict__ out) {
  __shared__ double so[256], sd[256];
  double o = 0.0, dg = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)me * me; e += 256) {
    const double v = A[e];
    if (e / me == e % me)
      dg += v * v;
    else
      o += v * v;
  }
  so[threadIdx.x] = o;
  sd[threadIdx.x] = dg;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      so[threadIdx.x] += so[threadIdx.x + w];
      sd[threadIdx.x] += sd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = so[0];
    out[1] = sd[0];
  }
}

__global__ void k_jacobi_init(const double* __restrict__ Ain, int m, int me, double* __restrict__ A,
                              double* __restrict__ V) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)me * me;
       e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / me), j = (int)(e % me);
    A[e] = (i < m && j < m) ? 0.5 * (Ain[(int64_t)i * m + j] + Ain[(int64_t)j * m + i]) : 0.0;
    V[e] = i == j ? 1.0 : 0.0;
  }
}

// sort eigenpairs (diag of A, columns of V) by descending eigenvalue; ties by index
__global__ void k_jacobi_sort(const double* __restrict__ A, const double* __restrict__ V, int m,
                              int me, double* __restrict__ evals, double* __restrict__ evecs) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const double li = A[(int64_t)i * me + i];
  int pos = 0;
  for (int j = 0; j < m; ++j) {
    const double lj = A[(int64_t)j * me + j];
    if (lj > li || (lj == li && j < i)) ++pos;
  }
  evals[pos] = li;
  for (int r = 0; r < m; ++r) evecs[(int64_t)r * m + pos] = V[(int64_t)r * me + i];
}

int grid1(int64_t count) {
  int64_t b = (count + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

}  // namespace

ld_status gram64(ld_ctx* ctx, const double* A, const double* B, const double* w, int64_t n, int m,
                 double* G) {
  const int tiles = (m + GT - 1) / GT;
  int64_t chunks = (int64_t)ctx->num_cu * 2 / ((int64_t)tiles * tiles);
  const int64_t maxc = (n + 255) / 256;
  if (chunks > maxc) chunks = maxc;
  if (chunks < 1) chunks = 1;
  const int64_t chunk = (n + chunks - 1) / chunks;
  chunks = (n + chunk - 1) / chunk;
  double* part = (double*)ctx->arena.take((size_t)chunks * m * m * sizeof(double));
  if (!part) return fail(LD_ENOMEM, "gram64: scratch arena too small");
  hipLaunchKernelGGL(k_gram_partial, dim3((unsigned)chunks, tiles, tiles), dim3(256), 0,
                     ctx->stream, A, B, w, n, m, chunk, part);
  const int64_t mm = (int64_t)m * m;
  hipLaunchKernelGGL(k_sum_chunks, dim3(grid1(mm)), dim3(256), 0, ctx->stream, part, (int)chunks,
                     mm, G);
  LD_HIP(hipGetLastError());
  return LD_OK;
}

void launch_cholesky_upper(hipStream_t st, double* G, int m, int* fail_flag) {
  hipLaunchKernelGGL(k_cholesky_upper, dim3(1), dim3(CT), 0, st, G, m, fail_flag);
}

void launch_tri_inv_upper(hipStream_t st, const double* R, int m, double* Rinv) {
  hipLaunchKernelGGL(k_tri_inv_upper, dim3(1), dim3(CT), 0, st, R, m, Rinv);
}

void launch_gemm64(hipStream_t st, const double* A, const double* B, int ldb, const double* rs,
                   int64_t n, int K, int N, double* C) {
  dim3 grid((unsigned)((n + GM_BM - 1) / GM_BM), (unsigned)((N + GM_BN - 1) / GM_BN));
  hipLaunchKernelGGL(k_gemm64, grid, dim3(256), 0, st, A, B, ldb, rs, n, K, N, C);
}

ld_status jacobi_eigh(ld_ctx* ctx, double* Ain, int m, double* evals, double* evecs) {
  const int me = m + (m & 1);
  const size_t sz = (size_t)me * me;
  double* A0 = (double*)ctx->arena.take(sz * sizeof(double));
  double* A1 = (double*)ctx->arena.take(sz * sizeof(double));
  double* V0 = (double*)ctx->arena.take(sz * sizeof(double));
  double* V1 = (double*)ctx->arena.take(sz * sizeof(double));
  double* nrm = (double*)ctx->arena.take(2 * sizeof(double));
  if (!A0 || !A1 || !V0 || !V1 || !nrm) return fail(LD_ENOMEM, "jacobi: scratch arena too small");
  LD_TRY(ensure_pinned(ctx, 2));
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_jacobi_init, dim3(grid1(sz)), dim3(256), 0, st, Ain, m, me, A0, V0);
  const int h = me / 2;
  const int64_t items = (int64_t)h * h + (int64_t)me * h;
  const int blocks = (int)((items + 255) / 256);
  double* cur = A0;
  double* nxt = A1;
  double* vcur = V0;
  double* vnxt = V1;
  bool done = me < 2;
  double off_prev = -1.0;
  for (int sweep = 0; sweep < 40 && !done; ++sweep) {
    for (int r = 0; r < me - 1; ++r) {
      hipLaunchKernelGGL(k_jacobi_round, dim3(blocks), dim3(256), 0, st, cur, nxt, vcur, vnxt, me, r);
      std::swap(cur, nxt);
      std::swap(vcur, vnxt);
    }
    hipLaunchKernelGGL(k_offnorm, dim3(1), dim3(256), 0, st, cur, me, nrm);
    LD_HIP(hipMemcpyAsync(ctx->pinned, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    LD_HIP(hipStreamSynchronize(st));
    const double off = ctx->pinned[0], dg = ctx->pinned[1];
    if (!std::isfinite(off) || !std::isfinite(dg))
      return fail(LD_ENOTSPD, "jacobi: non-finite entries in the projected matrix");
    done = dev::jacobi_done(off, dg, off_prev);
    off_prev = off;
  }
  if (!done) return fail(LD_ENOCONV, "jacobi: no convergence in 40 sweeps");
  hipLaunchKernelGGL(k_jacobi_sort, dim3((m + 255) / 256), dim3(256), 0, st, cur, vcur, m, me, evals,
                     evecs);
  LD_HIP(hipGetLastError());
  return LD_OK;
}

}  // namespace ld
