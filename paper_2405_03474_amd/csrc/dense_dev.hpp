// Workgroup-level FP64 dense building blocks shared by the single-instance
// kernels (dense64.hip) and the batched ones (batch.hip): blocked Cholesky,
// upper-triangular inverse, an FP64 matrix-core GEMM tile, and the pieces of
// the parallel cyclic Jacobi eigen-solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ld {
namespace dev {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int CB = 64;   // block size of the LDS-blocked factorizations
constexpr int CT = 512;  // threads of a factorization workgroup

// Blocked right-looking Cholesky G = R^T R (R upper) of an m x m matrix with
// leading dimension ld, by one workgroup of CT threads: factor the 64 x 64
// diagonal block in LDS, solve the block row R_kk^T X = G_k,: (one column per
// thread, X in registers), subtract R_k,I^T R_k,J from every trailing upper
// tile.  The strict lower triangle is zeroed.  *fail_flag is set to 1 on a
// pivot that is not positive and finite, and left alone otherwise.
__device__ inline void chol_upper_block(double* __restrict__ G, int m, int ld,
                                        int* __restrict__ fail_flag) {
  __shared__ double Dk[CB][CB + 1];
  __shared__ double PI[CB][CB + 1];
  __shared__ double PJ[CB][CB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  const int nb = (m + CB - 1) / CB;
  for (int kb = 0; kb < nb; ++kb) {
    const int k0 = kb * CB;
    const int w = m - k0 < CB ? m - k0 : CB;
    __syncthreads();
    for (int e = tid; e < CB * CB; e += CT) {
      const int a = e / CB, b = e % CB;
      Dk[a][b] = (a < w && b < w && b >= a) ? G[(int64_t)(k0 + a) * ld + k0 + b] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < w; ++j) {
      if (tid == 0) {
        const double d = Dk[j][j];
        if (!(d > 0.0) || !isfinite(d)) {
          bad = 1;
          Dk[j][j] = 1.0;
        } else {
          Dk[j][j] = sqrt(d);
        }
      }
      __syncthreads();
      const double inv = 1.0 / Dk[j][j];
      for (int t = j + 1 + tid; t < w; t += CT) Dk[j][t] *= inv;
      __syncthreads();
      const int rem = w - j - 1;
      for (int e = tid; e < rem * rem; e += CT) {
        const int a = j + 1 + e / rem, b = j + 1 + e % rem;
        if (b >= a) Dk[a][b] -= Dk[j][a] * Dk[j][b];
      }
      __syncthreads();
    }
    for (int e = tid; e < CB * CB; e += CT) {
      const int a = e / CB, b = e % CB;
      if (a < w && b < w) G[(int64_t)(k0 + a) * ld + k0 + b] = b >= a ? Dk[a][b] : 0.0;
    }
    const int k1 = k0 + w;
    if (k1 >= m) break;
    for (int c = k1 + tid; c < m; c += CT) {
      double x[CB];
#pragma unroll
      for (int i = 0; i < CB; ++i) {
        if (i < w) {
          double v = G[(int64_t)(k0 + i) * ld + c];
#pragma unroll
          for (int t = 0; t < i; ++t) v -= Dk[t][i] * x[t];
          x[i] = v / Dk[i][i];
        }
      }
#pragma unroll
      for (int i = 0; i < CB; ++i)
        if (i < w) G[(int64_t)(k0 + i) * ld + c] = x[i];
    }
    __syncthreads();
    const int nt = (m - k1 + CB - 1) / CB;
    for (int ti = 0; ti < nt; ++ti) {
      for (int tj = ti; tj < nt; ++tj) {
        const int I0 = k1 + ti * CB, J0 = k1 + tj * CB;
        __syncthreads();
        for (int e = tid; e < CB * CB; e += CT) {
          const int t = e / CB, a = e % CB;
          PI[t][a] = (t < w && I0 + a < m) ? G[(int64_t)(k0 + t) * ld + I0 + a] : 0.0;
          PJ[t][a] = (t < w && J0 + a < m) ? G[(int64_t)(k0 + t) * ld + J0 + a] : 0.0;
        }
        __syncthreads();
        const int a0 = tid / 16, b0 = tid % 16;
        double acc[2][4] = {};
        for (int t = 0; t < w; ++t) {
          const double p0 = PI[t][a0], p1 = PI[t][a0 + 32];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double pj = PJ[t][b0 + 16 * q];
            acc[0][q] = fma(p0, pj, acc[0][q]);
            acc[1][q] = fma(p1, pj, acc[1][q]);
          }
        }
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = I0 + a0 + 32 * r, j = J0 + b0 + 16 * q;
            if (i < m && j < m && j >= i) G[(int64_t)i * ld + j] -= acc[r][q];
          }
      }
    }
  }
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)m * m; e += CT) {
    const int i = (int)(e / m), j = (int)(e % m);
    if (j < i) G[(int64_t)i * ld + j] = 0.0;
  }
  if (tid == 0 && bad) *fail_flag = 1;
}

// X = R^-1 for an upper-triangular m x m R (leading dimensions ldr, ldx), one
// workgroup of CT threads: the 64 x 64 diagonal block inverses first (back
// substitution, one column per thread, in LDS), then for each block column j
// and block row i < j (bottom up)  X_ij = -X_ii (sum_{k=i+1..j} R_ik X_kj).
__device__ inline void tri_inv_upper_block(const double* __restrict__ R, int m, int ldr,
                                           double* __restrict__ X, int ldx) {
  __shared__ double Ta[CB][CB + 1];
  __shared__ double Tb[CB][CB + 1];
  __shared__ double Acc[CB][CB + 1];
  const int tid = threadIdx.x;
  const int nb = (m + CB - 1) / CB;
  for (int64_t e = tid; e < (int64_t)m * m; e += CT) X[(e / m) * ldx + e % m] = 0.0;
  __syncthreads();
  for (int ib = 0; ib < nb; ++ib) {
    const int i0 = ib * CB;
    const int w = m - i0 < CB ? m - i0 : CB;
    __syncthreads();
    for (int e = tid; e < CB * CB; e += CT) {
      const int a = e / CB, b = e % CB;
      Ta[a][b] = (a < w && b < w) ? R[(int64_t)(i0 + a) * ldr + i0 + b] : 0.0;
    }
    __syncthreads();
    if (tid < w) {
      const int c = tid;
      for (int i = c; i >= 0; --i) {
        double v = (i == c) ? 1.0 : 0.0;
        for (int t = i + 1; t <= c; ++t) v -= Ta[i][t] * Tb[t][c];
        Tb[i][c] = v / Ta[i][i];
      }
    }
    __syncthreads();
    for (int e = tid; e < CB * CB; e += CT) {
      const int a = e / CB, b = e % CB;
      if (a < w && b < w && b >= a) X[(int64_t)(i0 + a) * ldx + i0 + b] = Tb[a][b];
    }
  }
  __syncthreads();
  const int a0 = tid / 16, b0 = tid % 16;
  for (int jb = 1; jb < nb; ++jb) {
    const int j0 = jb * CB;
    const int wj = m - j0 < CB ? m - j0 : CB;
    for (int ib = jb - 1; ib >= 0; --ib) {
      const int i0 = ib * CB;
      double acc[2][4] = {};
      for (int kb = ib + 1; kb <= jb; ++kb) {
        const int kk0 = kb * CB;
        const int wk = m - kk0 < CB ? m - kk0 : CB;
        __syncthreads();
        for (int e = tid; e < CB * CB; e += CT) {
          const int a = e / CB, b = e % CB;
          Ta[a][b] = (b < wk) ? R[(int64_t)(i0 + a) * ldr + kk0 + b] : 0.0;
          Tb[a][b] = (a < wk && b < wj) ? X[(int64_t)(kk0 + a) * ldx + j0 + b] : 0.0;
        }
        __syncthreads();
        for (int t = 0; t < CB; ++t) {
          const double r0 = Ta[a0][t], r1 = Ta[a0 + 32][t];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double xv = Tb[t][b0 + 16 * q];
            acc[0][q] = fma(r0, xv, acc[0][q]);
            acc[1][q] = fma(r1, xv, acc[1][q]);
          }
        }
      }
      __syncthreads();
      for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 4; ++q) Acc[a0 + 32 * r][b0 + 16 * q] = acc[r][q];
      for (int e = tid; e < CB * CB; e += CT) {
        const int a = e / CB, b = e % CB;
        Ta[a][b] = X[(int64_t)(i0 + a) * ldx + i0 + b];
      }
      __syncthreads();
      double out[2][4] = {};
      for (int t = 0; t < CB; ++t) {
        const double x0 = Ta[a0][t], x1 = Ta[a0 + 32][t];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double av = Acc[t][b0 + 16 * q];
          out[0][q] = fma(x0, av, out[0][q]);
          out[1][q] = fma(x1, av, out[1][q]);
        }
      }
      for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 4; ++q) {
          const int j = j0 + b0 + 16 * q;
          if (j - j0 < wj) X[(int64_t)(i0 + a0 + 32 * r) * ldx + j] = -out[r][q];
        }
    }
  }
}

// One 128 x 64 output tile (rows i0.., columns j0..) of
// C = diag(rs) A (n x K, lda) B (K x N, ldb) into C (ldc) on
// v_mfma_f64_16x16x4f64, by a workgroup of 256 threads (4 waves of 32 rows).
// K is staged 16 at a time; in k-step t lane group h supplies k = 4h + t.
// The 16x16 output of the instruction has row = lane/16 + 4 * register.
constexpr int GM_BM = 128, GM_BN = 64, GM_BK = 16;

__device__ inline void gemm64_tile(const double* __restrict__ A, int64_t lda,
                                   const double* __restrict__ B, int64_t ldb,
                                   const double* __restrict__ rs, int64_t n, int K, int N,
                                   double* __restrict__ C, int64_t ldc, int64_t i0, int j0) {
  constexpr int AS = GM_BK + 2;
  constexpr int BS = GM_BN + 2;
  __shared__ __attribute__((aligned(16))) double As[GM_BM * AS];
  __shared__ double Bs[GM_BK * BS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lj = lane & 15, lh = lane >> 4;
  f64x4 acc[2][4];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[rb][nb][r] = 0.0;
  // the next stage is fetched into registers while this one is multiplied
  constexpr int APT = GM_BM * GM_BK / 256, BPT = GM_BK * GM_BN / 256;
  double pa[APT], pb[BPT];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int j = 0; j < APT; ++j) {
      const int e = tid + 256 * j;
      const int rr = e / GM_BK, kk = e % GM_BK;
      const int64_t row = i0 + rr;
      pa[j] = (row < n && k0 + kk < K) ? A[row * lda + k0 + kk] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int e = tid + 256 * j;
      const int kk = e / GM_BN, cc = e % GM_BN;
      pb[j] = (k0 + kk < K && j0 + cc < N) ? B[(int64_t)(k0 + kk) * ldb + j0 + cc] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += GM_BK) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < APT; ++j) {
      const int e = tid + 256 * j;
      As[(e / GM_BK) * AS + e % GM_BK] = pa[j];
    }
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int e = tid + 256 * j;
      Bs[(e / GM_BN) * BS + e % GM_BN] = pb[j];
    }
    __syncthreads();
    if (k0 + GM_BK < K) fetch(k0 + GM_BK);
    double a[2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const double2* ap = (const double2*)&As[(32 * wave + 16 * rb + lj) * AS + 4 * lh];
      const double2 v0 = ap[0], v1 = ap[1];
      a[rb][0] = v0.x;
      a[rb][1] = v0.y;
      a[rb][2] = v1.x;
      a[rb][3] = v1.y;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double* brow = &Bs[(4 * lh + t) * BS + lj];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const double b = brow[16 * nb];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
          acc[rb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb][t], b, acc[rb][nb], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = i0 + 32 * wave + 16 * rb + lh + 4 * r;
      if (row >= n) continue;
      const double sc = rs ? rs[row] : 1.0;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const int col = j0 + 16 * nb + lj;
        if (col < N) C[row * ldc + col] = sc * acc[rb][nb][r];
      }
    }
}

// ---------------------------------------------------------------- Jacobi --
// Round r of the round-robin tournament on me (even) indices: position 0
// holds index 0, position p > 0 holds ((p - 1 + r) mod (me - 1)) + 1; pair k
// joins positions k and me - 1 - k.
__device__ __forceinline__ int player_at(int pos, int r, int me) {
  return pos == 0 ? 0 : ((pos - 1 + r) % (me - 1)) + 1;
}

__device__ __forceinline__ void pair_of(int k, int r, int me, int& p, int& q) {
  const int a = player_at(k, r, me), b = player_at(me - 1 - k, r, me);
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// rotation that annihilates A[p][q]; A' rows: p <- c*p - s*q, q <- s*p + c*q
__device__ __forceinline__ void rotation(const double* __restrict__ A, int me, int p, int q,
                                         double& c, double& s) {
  const double apq = A[(int64_t)p * me + q];
  const double app = A[(int64_t)p * me + p], aqq = A[(int64_t)q * me + q];
  if (apq == 0.0 || fabs(apq) <= 1e-300) {
    c = 1.0;
    s = 0.0;
    return;
  }
  const double tau = (aqq - app) / (2.0 * apq);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

// Work item e of one Jacobi round (h = me/2): items below h*h update the 2x2
// block of A between pairs (e / h, e % h); the next me*h items rotate the
// columns of V for row e / h and pair e % h.  Reads A, V; writes A2, V2.
__device__ __forceinline__ void jacobi_item(const double* __restrict__ A, double* __restrict__ A2,
                                            const double* __restrict__ V, double* __restrict__ V2,
                                            int me, int r, int64_t e) {
  const int h = me / 2;
  const int64_t nblk = (int64_t)h * h;
  if (e < nblk) {
    const int P = (int)(e / h), Q = (int)(e % h);
    int p1, q1, p2, q2;
    pair_of(P, r, me, p1, q1);
    pair_of(Q, r, me, p2, q2);
    double c1, s1, c2, s2;
    rotation(A, me, p1, q1, c1, s1);
    rotation(A, me, p2, q2, c2, s2);
    const double a11 = A[(int64_t)p1 * me + p2], a12 = A[(int64_t)p1 * me + q2];
    const double a21 = A[(int64_t)q1 * me + p2], a22 = A[(int64_t)q1 * me + q2];
    const double b11 = c1 * a11 - s1 * a21, b12 = c1 * a12 - s1 * a22;
    const double b21 = s1 * a11 + c1 * a21, b22 = s1 * a12 + c1 * a22;
    double o11 = c2 * b11 - s2 * b12, o12 = s2 * b11 + c2 * b12;
    double o21 = c2 * b21 - s2 * b22, o22 = s2 * b21 + c2 * b22;
    if (P == Q) {  // the annihilated pair
      o12 = 0.0;
      o21 = 0.0;
    }
    A2[(int64_t)p1 * me + p2] = o11;
    A2[(int64_t)p1 * me + q2] = o12;
    A2[(int64_t)q1 * me + p2] = o21;
    A2[(int64_t)q1 * me + q2] = o22;
    return;
  }
  const int64_t f = e - nblk;
  if (f >= (int64_t)me * h) return;
  const int row = (int)(f / h), Q = (int)(f % h);
  int p2, q2;
  pair_of(Q, r, me, p2, q2);
  double c2, s2;
  rotation(A, me, p2, q2, c2, s2);
  const double vp = V[(int64_t)row * me + p2], vq = V[(int64_t)row * me + q2];
  V2[(int64_t)row * me + p2] = c2 * vp - s2 * vq;
  V2[(int64_t)row * me + q2] = s2 * vp + c2 * vq;
}

// Stopping rule of the sweeps: off-diagonal mass converged, or stalled at the
// rounding level after quadratic convergence.
__host__ __device__ inline bool jacobi_done(double off, double dg, double off_prev) {
  return off <= 1e-30 * dg || (off <= 1e-22 * dg && off_prev >= 0.0 && off >= 0.25 * off_prev);
}

}  // namespace dev
}  // namespace ld
