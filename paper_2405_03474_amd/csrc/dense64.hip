// FP64 dense algebra for the randomized truncated-SVD preconditioner
// (Section 2; Halko et al. Alg. 4.1 / 5.3): Gram products A^T diag(w) B,
// Cholesky, triangular inverse, tall GEMM on FP64 matrix cores, and a
// parallel cyclic Jacobi eigen-solver for the small projected matrix.
#include <cmath>
#include <vector>

#include "ld_common.hpp"

namespace ld {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ Gram --
// Partial G_c = A_c^T diag(w_c) B_c over row chunk c, 64 x 64 output tile per
// workgroup, 4 x 4 outputs per thread, rows staged through LDS 16 at a time.
constexpr int GT = 64;
constexpr int GR = 16;

__global__ __launch_bounds__(256) void k_gram_partial(const double* __restrict__ A,
                                                      const double* __restrict__ B,
                                                      const double* __restrict__ w, int64_t n,
                                                      int m, int64_t chunk,
                                                      double* __restrict__ part) {
  __shared__ double As[GR][GT + 1];
  __shared__ double Bs[GR][GT + 1];
  const int tid = threadIdx.x;
  const int ti = tid / 16, tj = tid % 16;
  const int i0 = blockIdx.y * GT, j0 = blockIdx.z * GT;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  int64_t r1 = r0 + chunk;
  if (r1 > n) r1 = n;
  double acc[4][4] = {};
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
#pragma unroll 4
    for (int rr = 0; rr < GR; ++rr) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[rr][ti + 16 * q];
        b[q] = Bs[rr][tj + 16 * q];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
    }
  }
  double* dst = part + (int64_t)blockIdx.x * m * m;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = i0 + ti + 16 * x, j = j0 + tj + 16 * y;
      if (i < m && j < m) dst[(int64_t)i * m + j] = acc[x][y];
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

// -------------------------------------------------------------- Cholesky --
// Blocked right-looking Cholesky G = R^T R (R upper) in one workgroup of 512
// threads, 64 x 64 blocks staged in LDS: factor the diagonal block, solve the
// block row R_kk^T X = G_k,: (one column per thread, X in registers), then
// subtract R_k,I^T R_k,J from every trailing upper tile (I <= J).
constexpr int CB = 64;
constexpr int CT = 512;

__global__ __launch_bounds__(CT) void k_cholesky_upper(double* __restrict__ G, int m,
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
      Dk[a][b] = (a < w && b < w && b >= a) ? G[(int64_t)(k0 + a) * m + k0 + b] : 0.0;
    }
    __syncthreads();
    // unblocked factorization of the diagonal block
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
      if (a < w && b < w) G[(int64_t)(k0 + a) * m + k0 + b] = b >= a ? Dk[a][b] : 0.0;
    }
    const int k1 = k0 + w;
    if (k1 >= m) break;
    // block row: R_kk^T x = g for every column right of the block
    for (int c = k1 + tid; c < m; c += CT) {
      double x[CB];
#pragma unroll
      for (int i = 0; i < CB; ++i) {
        if (i < w) {
          double v = G[(int64_t)(k0 + i) * m + c];
#pragma unroll
          for (int t = 0; t < i; ++t) v -= Dk[t][i] * x[t];
          x[i] = v / Dk[i][i];
        }
      }
#pragma unroll
      for (int i = 0; i < CB; ++i)
        if (i < w) G[(int64_t)(k0 + i) * m + c] = x[i];
    }
    __syncthreads();
    // trailing update of the upper triangle
    const int nt = (m - k1 + CB - 1) / CB;
    for (int ti = 0; ti < nt; ++ti) {
      for (int tj = ti; tj < nt; ++tj) {
        const int I0 = k1 + ti * CB, J0 = k1 + tj * CB;
        __syncthreads();
        for (int e = tid; e < CB * CB; e += CT) {
          const int t = e / CB, a = e % CB;
          PI[t][a] = (t < w && I0 + a < m) ? G[(int64_t)(k0 + t) * m + I0 + a] : 0.0;
          PJ[t][a] = (t < w && J0 + a < m) ? G[(int64_t)(k0 + t) * m + J0 + a] : 0.0;
        }
        __syncthreads();
        // 8 outputs per thread: rows a0, a0 + 32; columns b0 + 16 q
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
            if (i < m && j < m && j >= i) G[(int64_t)i * m + j] -= acc[r][q];
          }
      }
    }
  }
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)m * m; e += CT) {
    const int i = (int)(e / m), j = (int)(e % m);
    if (j < i) G[e] = 0.0;
  }
  if (tid == 0 && bad) *fail_flag = 1;
}

// ------------------------------------------------- upper triangular inverse --
// X = R^-1 for upper-triangular R, one workgroup: the 64 x 64 diagonal block
// inverses first (back substitution, one column per thread, in LDS), then for
// each block column j and block row i < j (bottom up)
//   X_ij = -X_ii (sum_{k=i+1..j} R_ik X_kj).
__global__ __launch_bounds__(CT) void k_tri_inv_upper(const double* __restrict__ R, int m,
                                                      double* __restrict__ X) {
  __shared__ double Ta[CB][CB + 1];
  __shared__ double Tb[CB][CB + 1];
  __shared__ double Acc[CB][CB + 1];
  const int tid = threadIdx.x;
  const int nb = (m + CB - 1) / CB;
  for (int64_t e = tid; e < (int64_t)m * m; e += CT) X[e] = 0.0;
  __syncthreads();
  // diagonal blocks
  for (int ib = 0; ib < nb; ++ib) {
    const int i0 = ib * CB;
    const int w = m - i0 < CB ? m - i0 : CB;
    __syncthreads();
    for (int e = tid; e < CB * CB; e += CT) {
      const int a = e / CB, b = e % CB;
      Ta[a][b] = (a < w && b < w) ? R[(int64_t)(i0 + a) * m + i0 + b] : 0.0;
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
      if (a < w && b < w && b >= a) X[(int64_t)(i0 + a) * m + i0 + b] = Tb[a][b];
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
      // T = sum_k R_ik X_kj
      for (int kb = ib + 1; kb <= jb; ++kb) {
        const int kk0 = kb * CB;
        const int wk = m - kk0 < CB ? m - kk0 : CB;
        __syncthreads();
        for (int e = tid; e < CB * CB; e += CT) {
          const int a = e / CB, b = e % CB;
          Ta[a][b] = (b < wk) ? R[(int64_t)(i0 + a) * m + kk0 + b] : 0.0;
          Tb[a][b] = (a < wk && b < wj) ? X[(int64_t)(kk0 + a) * m + j0 + b] : 0.0;
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
        Ta[a][b] = X[(int64_t)(i0 + a) * m + i0 + b];  // X_ii (upper, zero below)
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
          if (j - j0 < wj) X[(int64_t)(i0 + a0 + 32 * r) * m + j] = -out[r][q];
        }
    }
  }
}

// ---------------------------------------------------------------- GEMM64 --
// C (n x N) = diag(rs) A (n x K) B (K x N) with v_mfma_f64_16x16x4f64.
// Workgroup tile 128 x 64, 4 waves of 32 x 64, K staged 16 at a time; in
// k-step t lane group h supplies physical k = 4h + t.
constexpr int GM_BM = 128, GM_BN = 64, GM_BK = 16;

__global__ __launch_bounds__(256) void k_gemm64(const double* __restrict__ A,
                                                const double* __restrict__ B, int ldb,
                                                const double* __restrict__ rs, int64_t n, int K,
                                                int N, double* __restrict__ C) {
  constexpr int AS = GM_BK + 2;
  constexpr int BS = GM_BN + 2;
  __shared__ __attribute__((aligned(16))) double As[GM_BM * AS];
  __shared__ double Bs[GM_BK * BS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lj = lane & 15, lh = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * GM_BM;
  const int j0 = blockIdx.y * GM_BN;
  f64x4 acc[2][4];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[rb][nb][r] = 0.0;
  for (int k0 = 0; k0 < K; k0 += GM_BK) {
    __syncthreads();
    for (int e = tid; e < GM_BM * GM_BK; e += 256) {
      const int rr = e / GM_BK, kk = e % GM_BK;
      const int64_t row = i0 + rr;
      As[rr * AS + kk] = (row < n && k0 + kk < K) ? A[row * K + k0 + kk] : 0.0;
    }
    for (int e = tid; e < GM_BK * GM_BN; e += 256) {
      const int kk = e / GM_BN, cc = e % GM_BN;
      Bs[kk * BS + cc] = (k0 + kk < K && j0 + cc < N) ? B[(int64_t)(k0 + kk) * ldb + j0 + cc] : 0.0;
    }
    __syncthreads();
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
      const int64_t row = i0 + 32 * wave + 16 * rb + lh + 4 * r;  // row = lane/16 + 4 reg
      if (row >= n) continue;
      const double sc = rs ? rs[row] : 1.0;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const int col = j0 + 16 * nb + lj;
        if (col < N) C[row * N + col] = sc * acc[rb][nb][r];
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

__global__ __launch_bounds__(256) void k_jacobi_round(const double* __restrict__ A,
                                                      double* __restrict__ A2,
                                                      const double* __restrict__ V,
                                                      double* __restrict__ V2, int me, int r) {
  const int h = me / 2;
  const int64_t nblk = (int64_t)h * h;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
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
    // rows
    const double b11 = c1 * a11 - s1 * a21, b12 = c1 * a12 - s1 * a22;
    const double b21 = s1 * a11 + c1 * a21, b22 = s1 * a12 + c1 * a22;
    // columns
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

void launch_cholesky_upper(hipStream_t st, double* G, int m, int* ok) {
  hipLaunchKernelGGL(k_cholesky_upper, dim3(1), dim3(CT), 0, st, G, m, ok);
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
  // both buffers must hold every entry: a round rewrites all of A and V
  LD_HIP(hipMemcpyAsync(A1, A0, sz * sizeof(double), hipMemcpyDeviceToDevice, st));
  LD_HIP(hipMemcpyAsync(V1, V0, sz * sizeof(double), hipMemcpyDeviceToDevice, st));
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
      double* t = cur;
      cur = nxt;
      nxt = t;
      t = vcur;
      vcur = vnxt;
      vnxt = t;
    }
    hipLaunchKernelGGL(k_offnorm, dim3(1), dim3(256), 0, st, cur, me, nrm);
    LD_HIP(hipMemcpyAsync(ctx->pinned, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    LD_HIP(hipStreamSynchronize(st));
    const double off = ctx->pinned[0], dg = ctx->pinned[1];
    if (!std::isfinite(off) || !std::isfinite(dg))
      return fail(LD_ENOTSPD, "jacobi: non-finite entries in the projected matrix");
    // converged, or stalled at the rounding level after quadratic convergence
    if (off <= 1e-30 * dg || (off <= 1e-22 * dg && off_prev >= 0.0 && off >= 0.25 * off_prev))
      done = true;
    off_prev = off;
  }
  if (!done) return fail(LD_ENOCONV, "jacobi: no convergence in 40 sweeps");
  hipLaunchKernelGGL(k_jacobi_sort, dim3((m + 255) / 256), dim3(256), 0, st, cur, vcur, m, me, evals,
                     evecs);
  LD_HIP(hipGetLastError());
  return LD_OK;
}

}  // namespace ld
