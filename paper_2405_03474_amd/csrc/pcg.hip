// Woodbury apply of P^-1 and the block multi-shift preconditioned CG with the
// Hutchinson reduction (Section 2: Algorithm 1 steps 2-3 as a multi-shift
// solver, the estimator output, and a cheap P^-1 v; Section 1: Hutchinson).
//
// P = D + U diag(lam) U^T is stored as F = D^-1 U L^-T and D^-1, with
// L L^T = diag(1/lam) + U^T D^-1 U, so P^-1 R = D^-1 R - F (F^T R).
//
// The solver runs CG on A = M P^-1 + a_1 I in the inner product <x, y> =
// x^T P^-1 y, in which M P^-1 is self-adjoint (the paper runs Lanczos on
// M P^-1; this is the inner product that makes that well defined).  One CG
// per probe column, all columns of the block in lock step; each column has
// its own alpha, beta.  Per iteration:
//   q = M w + a_1 p        (w = P^-1 p)          kernel matmat + epilogue
//   alpha = rho / w^T q
//   r -= alpha q ; u = P^-1 r ; rho' = r^T u ; beta = rho' / rho
//   p = r + beta p ; w = u + beta w
// The shifted systems (M P^-1 + a_j I) x_j = z share the Krylov space; their
// residuals are zeta_j r, with Jegerlehner's recurrences for zeta_j,
// alpha_j, beta_j.  Only the scalars z^T x_j are needed by the estimator, and
// z^T x_j, z^T p_j follow from the scalar z^T r per column:
//   z^T x_j += alpha_j z^T p_j ;  z^T p_j = zeta_j z^T r + beta_j z^T p_j,
// so no n-vector is kept per shift.  All scalars are FP64.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ld_common.hpp"

namespace ld {
namespace {

constexpr int WT = 64;  // Woodbury tile (rows of F / columns of R)
constexpr int FR = 32;  // rows of F and R staged per step
typedef double f64x4w __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// t_partial[c] = F_c^T R_c over row chunk c (output rank x s, FP64) on FP64
// matrix cores (v_mfma_f64_16x16x4f64, inputs widened exactly).  Workgroup:
// one row chunk x 64 columns of F x 64 columns of R, cut into 16 x 16 (l, c)
// tiles, at most four per wave.  Stages of 32 rows of F and R go through LDS
// (coalesced row-segment loads, the next stage prefetched in registers).  In
// step t a wave consumes stage rows 4t .. 4t+3, lane group g = lane/16
// supplying row 4t + g; output lane l, register r: tile row l/16 + 4 r,
// column l % 16.
template <typename T>
__global__ __launch_bounds__(256) void k_ft_partial(const T* __restrict__ F,
                                                    const T* __restrict__ R, int64_t n, int rank,
                                                    int64_t s, int64_t chunk,
                                                    double* __restrict__ part) {
  __shared__ double Fs[FR][WT + 1];
  __shared__ double Rs[FR][WT + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int l0 = blockIdx.y * WT;
  const int64_t c0 = (int64_t)blockIdx.z * WT;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;
  const int ltl = (rank - l0 < WT ? rank - l0 + 15 : WT + 15) / 16;
  const int ctl = (int)((s - c0 < WT ? s - c0 + 15 : WT + 15) / 16);
  const int tiles = ltl * ctl;
  f64x4w acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = f64x4w{0.0, 0.0, 0.0, 0.0};
  T pf[8], pr[8];
  auto fetch = [&](int64_t rb) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      const int rr = e / WT, cc = e % WT;
      const int64_t row = rb + rr;
      const bool ok = row < r1;
      pf[j] = (ok && l0 + cc < rank) ? F[row * rank + l0 + cc] : (T)0;
      pr[j] = (ok && c0 + cc < s) ? R[row * s + c0 + cc] : (T)0;
    }
  };
  fetch(r0);
  for (int64_t rb = r0; rb < r1; rb += FR) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      Fs[e / WT][e % WT] = (double)pf[j];
      Rs[e / WT][e % WT] = (double)pr[j];
    }
    __syncthreads();
    if (rb + FR < r1) fetch(rb + FR);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int p = wave + 4 * q;
      if (p < tiles) {
        const int lt = p / ctl, cs = p % ctl;
#pragma unroll
        for (int t = 0; t < FR / 4; ++t) {
          const int k = 4 * t + lg;
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(Fs[k][lt * 16 + li], Rs[k][cs * 16 + li],
                                                        acc[q], 0, 0, 0);
        }
      }
    }
  }
  double* dst = part + (int64_t)blockIdx.x * rank * s;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int p = wave + 4 * q;
    if (p < tiles) {
      const int lt = p / ctl, cs = p % ctl;
      const int64_t c = c0 + cs * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int l = l0 + lt * 16 + lg + 4 * r;
        if (l < rank && c < s) dst[(int64_t)l * s + c] = acc[q][r];
      }
    }
  }
}

// out[e] = sum over the chunks of part[c][e], in chunk order; 64-thread
// workgroups (more of them in flight) with eight chunks' loads issued
// together
__global__ __launch_bounds__(64) void k_sum_parts(const double* __restrict__ part, int chunks,
                                                  int64_t count, double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * 64 + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * 64) {
    double s = 0.0;
    int c = 0;
    for (; c + 8 <= chunks; c += 8) {
      double v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = part[(int64_t)(c + j) * count + e];
#pragma unroll
      for (int j = 0; j < 8; ++j) s += v[j];
    }
    for (; c < chunks; ++c) s += part[(int64_t)c * count + e];
    out[e] = s;
  }
}

// OUT = Dinv .* R - F t (t: rank x s FP64) on a 64-row x 64-column tile, the
// product F t on FP64 matrix cores; wave w owns rows 16 w .. 16 w + 15.  F
// goes from HBM straight into the matrix-core registers: in a stage of 32
// rank indices k0 .. k0 + 31, lane (i, g) = (lane % 16, lane / 16) holds
// F[row i][k0 + 8 q + 2 g + e], q < 4, e < 2 (four 16-byte loads; in each,
// the four lanes of a row read 64 consecutive bytes), fetched two stages
// ahead, and matrix-core step 2 q + e pairs it with t[k0 + 8 q + 2 g + e][c].
// The stage of t (32 x 64, shared by the four waves) is loaded one stage
// ahead into registers and kept k-contiguous per column in a double-buffered
// LDS tile, one barrier per stage.  Optional per-row-tile column dots: dot1 =
// sum R .* OUT, dot2 = sum Z .* R.
constexpr int WK = 32;       // rank indices per stage
constexpr int TKS = WK + 2;  // LDS stride (doubles) of a column of the t stage
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_wood_out(const double* __restrict__ F,
                                                  const double* __restrict__ Dinv,
                                                  const double* __restrict__ t,
                                                  const double* __restrict__ R, int64_t n,
                                                  int rank, int64_t s, double* __restrict__ OUT,
                                                  const double* __restrict__ Z,
                                                  double* __restrict__ dot1,
                                                  double* __restrict__ dot2) {
  typedef double f64x2 __attribute__((ext_vector_type(2)));
  // the column-dot reduction reuses the t stages' LDS after the rank loop
  __shared__ __attribute__((aligned(16))) union {
    double Tt[2][WT * TKS];
    struct {
      double r1[4][64][4];
      double r2[4][64][4];
    } rd;
  } lds;
  auto& red1 = lds.rd.r1;
  auto& red2 = lds.rd.r2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * WT;
  const int64_t c0 = (int64_t)blockIdx.y * WT;
  const int ctl = (int)((s - c0 < WT ? s - c0 + 15 : WT + 15) / 16);
  const int nst = (rank + WK - 1) / WK;
  const int64_t arow = i0 + 16 * wave + li;
  const double* frow = F + arow * rank;
  f64x4w acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = f64x4w{0.0, 0.0, 0.0, 0.0};

  auto kbase = [&](int st) { return st * WK; };
  // this lane's 8 F values of stage st (zero past the rank or the rows)
  auto load_a = [&](int st, double (&a)[8]) {
    const int k0 = kbase(st);
    if (arow < n && k0 + WK <= rank && (rank & 1) == 0) {
      const f64x2* src = (const f64x2*)(frow + k0 + 2 * lg);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f64x2 v = __builtin_nontemporal_load(src + 4 * q);
        a[2 * q] = v.x;
        a[2 * q + 1] = v.y;
      }
      return;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + 8 * (j >> 1) + 2 * lg + (j & 1);
      a[j] = (arow < n && k < rank) ? frow[k] : 0.0;
    }
  };
  // t stage: thread column tid % 64, rank indices 8 (tid / 64) + j
  double tq[8];
  auto load_t = [&](int st) {
    const int k = kbase(st) + 8 * (tid / 64);
    const int64_t col = c0 + tid % 64;
#pragma unroll
    for (int j = 0; j < 8; ++j) tq[j] = (k + j < rank && col < s) ? t[(int64_t)(k + j) * s + col] : 0.0;
  };
  auto store_t = [&](double* tt) {
    f64x2* dst = (f64x2*)&tt[(tid % 64) * TKS + 8 * (tid / 64)];
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = f64x2{tq[2 * q], tq[2 * q + 1]};
  };

  double a[2][8];
  load_a(0, a[0]);
  if (nst > 1) load_a(1, a[1]);
  load_t(0);
  store_t(lds.Tt[0]);
  if (nst > 1) load_t(1);
  __syncthreads();
  for (int st = 0; st < nst; st += 2) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int cur = st + d;
      if (cur < nst) {
        // stage cur + 1 into the other buffer (last read in stage cur - 1,
        // fenced by the barrier that ended it)
        if (cur + 1 < nst) store_t(lds.Tt[(cur + 1) & 1]);
        if (cur + 2 < nst) load_t(cur + 2);
        const double* tt = lds.Tt[cur & 1];
        // two halves of four steps; in each, the four column tiles' chains
        // interleave (independent accumulators back to back; tiles past s
        // multiply the zero columns of the t stage)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          double b[4][4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const f64x2* bp = (const f64x2*)&tt[(c * 16 + li) * TKS + 16 * h + 2 * lg];
            const f64x2 v0 = bp[0], v1 = bp[4];
            b[c][0] = v0.x;
            b[c][1] = v0.y;
            b[c][2] = v1.x;
            b[c][3] = v1.y;
          }
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
#pragma unroll
            for (int c = 0; c < 4; ++c)
              acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[d][4 * h + jj], b[c][jj], acc[c], 0,
                                                            0, 0);
        }
        if (cur + 2 < nst) load_a(cur + 2, a[d]);
        __syncthreads();
      }
    }
  }
  double d1[4] = {0.0, 0.0, 0.0, 0.0}, d2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c >= ctl) continue;
    const int64_t cc = c0 + c * 16 + li;
    if (cc >= s) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = i0 + 16 * wave + lg + 4 * r;
      if (row >= n) continue;
      const int64_t off = row * s + cc;
      const double rv = R[off];
      const double o = Dinv[row] * rv - acc[c][r];
      OUT[off] = o;
      d1[c] += rv * o;
      if (dot2) d2[c] += Z[off] * rv;
    }
  }
  if (dot1) {
    __syncthreads();  // every wave is done reading the staging tiles
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      red1[wave][lane][c] = d1[c];
      red2[wave][lane][c] = d2[c];
    }
    __syncthreads();
    if (tid < WT) {
      const int c = tid / 16, l16 = tid % 16;
      double a = 0.0, b = 0.0;
      for (int w = 0; w < 4; ++w)
        for (int g = 0; g < 4; ++g) {
          a += red1[w][l16 + 16 * g][c];
          b += red2[w][l16 + 16 * g][c];
        }
      const int64_t col = c0 + tid;
      if (col < s) {
        dot1[(int64_t)blockIdx.x * s + col] = a;
        if (dot2) dot2[(int64_t)blockIdx.x * s + col] = b;
      }
    }
  }
}

// ------------------------------------------------- FP32 Woodbury apply --
// The FP32 path keeps F as an n x rp matrix (rp = rank rounded up to a
// multiple of 32, zero columns beyond rank) so that rank stages need no
// bounds checks, and runs both products on FP32 matrix cores
// (v_mfma_f32_32x32x2f32: lane l supplies A[l % 32][l / 32] and
// B[l / 32][l % 32]; output register r of lane l is row 8 (r / 4) +
// 4 (l / 32) + r % 4, column l % 32).  F^T R is summed over row chunks in
// FP32 inside a chunk and in FP64 across chunks; t is rounded to FP32 for
// the output step.
constexpr int W32R = 128;  // rank rows of F^T R per workgroup / rows of OUT per workgroup
constexpr int W32C = 64;   // columns of R per workgroup
constexpr int W32K = 32;   // contraction indices per LDS stage

// part[chunk] (rp x s, FP64) = F_chunk^T R_chunk.  Workgroup: one row chunk
// (a multiple of 32 rows), 128 rank rows, 64 columns; wave w owns rank rows
// 32 w .. 32 w + 31 and both 32-column blocks.  Stages of 32 rows of F
// (16-byte row segments) and R go through LDS, the next stage prefetched in
// registers.  MFMA step j contracts stage rows 2 j + l / 32.
__global__ __launch_bounds__(256) void k_ft32(const float* __restrict__ F,
                                              const float* __restrict__ R, int64_t n, int rp,
                                              int64_t s, int64_t chunk,
                                              double* __restrict__ part) {
  __shared__ float Fs[W32K][W32R + 4];
  __shared__ float Rs[W32K][W32C + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, h = lane >> 5;
  const int l0 = blockIdx.y * W32R;
  const int64_t c0 = (int64_t)blockIdx.z * W32C;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;
  f32x16 acc[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[nb][r] = 0.0f;
  float4 pf[4];
  float pr[8];
  auto fetch = [&](int64_t rb) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = tid + 256 * j;
      const int rr = e >> 5, c4 = e & 31;  // 32 rows x 32 float4
      const int64_t row = rb + rr;
      const int col = l0 + 4 * c4;
      pf[j] = (row < r1 && col < rp) ? *(const float4*)(F + row * rp + col)
                                     : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      const int rr = e >> 6, cc = e & 63;  // 32 rows x 64 columns
      const int64_t row = rb + rr;
      pr[j] = (row < r1 && c0 + cc < s) ? R[row * s + c0 + cc] : 0.0f;
    }
  };
  fetch(r0);
  for (int64_t rb = r0; rb < r1; rb += W32K) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = tid + 256 * j;
      *(float4*)&Fs[e >> 5][4 * (e & 31)] = pf[j];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      Rs[e >> 6][e & 63] = pr[j];
    }
    __syncthreads();
    if (rb + W32K < r1) fetch(rb + W32K);
#pragma unroll
    for (int j = 0; j < W32K / 2; ++j) {
      const int k = 2 * j + h;
      const float a = Fs[k][32 * wave + li];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, Rs[k][32 * nb + li], acc[nb], 0, 0, 0);
    }
  }
  double* dst = part + (int64_t)blockIdx.x * rp * s;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int64_t c = c0 + 32 * nb + li;
    if (c >= s) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int l = l0 + 32 * wave + 8 * (r >> 2) + 4 * h + (r & 3);
      if (l < rp) dst[(int64_t)l * s + c] = (double)acc[nb][r];
    }
  }
}

// t32[e] = (float) sum over chunks of part[chunk][e], e < count, chunks in
// order: four threads per element add contiguous quarters of the chunk list
// (loads issued four at a time), then the quarters are added in order.
__global__ __launch_bounds__(256) void k_sum32(const double* __restrict__ part, int chunks,
                                               int64_t count, float* __restrict__ t32) {
  __shared__ double red[4][64];
  const int tid = threadIdx.x, q = tid >> 6, el = tid & 63;
  const int64_t e = (int64_t)blockIdx.x * 64 + el;
  const int cb = (int)(((int64_t)chunks * q) / 4), ce = (int)(((int64_t)chunks * (q + 1)) / 4);
  double sum = 0.0;
  if (e < count) {
    int c = cb;
    for (; c + 4 <= ce; c += 4) {
      const double v0 = part[(int64_t)c * count + e];
      const double v1 = part[(int64_t)(c + 1) * count + e];
      const double v2 = part[(int64_t)(c + 2) * count + e];
      const double v3 = part[(int64_t)(c + 3) * count + e];
      sum += v0;
      sum += v1;
      sum += v2;
      sum += v3;
    }
    for (; c < ce; ++c) sum += part[(int64_t)c * count + e];
  }
  red[q][el] = sum;
  __syncthreads();
  if (q == 0 && e < count) t32[e] = (float)(((red[0][el] + red[1][el]) + red[2][el]) + red[3][el]);
}

// OUT = Dinv .* R - F t32 on a 128-row x 64-column tile: wave w owns rows
// 32 w .. 32 w + 31; each lane streams 16 consecutive rank indices of its
// row of F per stage (four 16-byte loads, the next stage prefetched), the
// stage's 32 x 64 block of t32 goes through LDS; MFMA step j contracts rank
// index 16 (l / 32) + j.  Optional per-128-row-tile column dots:
// dot1 = sum R .* OUT, dot2 = sum Z .* R.
__global__ __launch_bounds__(256) void k_wood32(const float* __restrict__ F,
                                                const float* __restrict__ Dinv,
                                                const float* __restrict__ t32,
                                                const float* __restrict__ R, int64_t n, int rp,
                                                int64_t s, float* __restrict__ OUT,
                                                const float* __restrict__ Z,
                                                double* __restrict__ dot1,
                                                double* __restrict__ dot2) {
  __shared__ float Ts[W32K][W32C + 4];
  __shared__ double red1[4][64][2];
  __shared__ double red2[4][64][2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, h = lane >> 5;
  const int64_t i0 = (int64_t)blockIdx.x * W32R;
  const int64_t c0 = (int64_t)blockIdx.y * W32C;
  const int64_t myrow = i0 + 32 * wave + li;
  const bool rowok = myrow < n;
  const float* Frow = F + (rowok ? myrow : 0) * rp + 16 * h;
  f32x16 acc[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[nb][r] = 0.0f;
  float4 fa[4], fn[4];
  float pt[8];
  auto fetch = [&](int k0, float4* dstv) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      dstv[j] = rowok ? *(const float4*)(Frow + k0 + 4 * j) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      const int kk = e >> 6, cc = e & 63;  // 32 rank indices x 64 columns
      pt[j] = (c0 + cc < s) ? t32[(int64_t)(k0 + kk) * s + c0 + cc] : 0.0f;
    }
  };
  fetch(0, fa);
  for (int k0 = 0; k0 < rp; k0 += W32K) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      Ts[e >> 6][e & 63] = pt[j];
    }
    __syncthreads();
    const bool more = k0 + W32K < rp;
    if (more) fetch(k0 + W32K, fn);
    float av[16];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      av[4 * j] = fa[j].x;
      av[4 * j + 1] = fa[j].y;
      av[4 * j + 2] = fa[j].z;
      av[4 * j + 3] = fa[j].w;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k = 16 * h + j;
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[j], Ts[k][32 * nb + li], acc[nb], 0, 0, 0);
    }
    if (more) {
#pragma unroll
      for (int j = 0; j < 4; ++j) fa[j] = fn[j];
    }
  }
  double d1[2] = {0.0, 0.0}, d2[2] = {0.0, 0.0};
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int64_t cc = c0 + 32 * nb + li;
    if (cc >= s) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t row = i0 + 32 * wave + 8 * (r >> 2) + 4 * h + (r & 3);
      if (row >= n) continue;
      const int64_t off = row * s + cc;
      const float rv = R[off];
      const float o = Dinv[row] * rv - acc[nb][r];
      OUT[off] = o;
      d1[nb] += (double)rv * (double)o;
      if (dot2) d2[nb] += (double)Z[off] * (double)rv;
    }
  }
  if (dot1) {
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      red1[wave][lane][nb] = d1[nb];
      red2[wave][lane][nb] = d2[nb];
    }
    __syncthreads();
    if (tid < W32C) {
      const int nb = tid >> 5, l32 = tid & 31;
      double a = 0.0, b = 0.0;
      for (int w = 0; w < 4; ++w)
        for (int g = 0; g < 2; ++g) {
          a += red1[w][l32 + 32 * g][nb];
          b += red2[w][l32 + 32 * g][nb];
        }
      const int64_t col = c0 + tid;
      if (col < s) {
        dot1[(int64_t)blockIdx.x * s + col] = a;
        if (dot2) dot2[(int64_t)blockIdx.x * s + col] = b;
      }
    }
  }
}

// Rank-0 preconditioner (identity, diagonal): OUT = Dinv .* R with the same
// per-row-block column dots as the Woodbury kernels (rows per block `rb`).
template <typename T>
__global__ __launch_bounds__(256) void k_wood_diag(const T* __restrict__ Dinv,
                                                   const T* __restrict__ R, int64_t n, int64_t s,
                                                   int rb, T* __restrict__ OUT,
                                                   const T* __restrict__ Z,
                                                   double* __restrict__ dot1,
                                                   double* __restrict__ dot2) {
  __shared__ double red1[4][64];
  __shared__ double red2[4][64];
  const int tid = threadIdx.x, cl = tid & 63, grp = tid >> 6;
  const int64_t c = (int64_t)blockIdx.y * 64 + cl;
  const int64_t r0 = (int64_t)blockIdx.x * rb;
  const int64_t r1 = r0 + rb < n ? r0 + rb : n;
  double a = 0.0, b = 0.0;
  if (c < s)
    for (int64_t i = r0 + grp; i < r1; i += 4) {
      const int64_t off = i * s + c;
      const T rv = R[off];
      const T o = (T)((double)Dinv[i] * (double)rv);
      OUT[off] = o;
      a += (double)rv * (double)o;
      if (dot2) b += (double)Z[off] * (double)rv;
    }
  red1[grp][cl] = a;
  red2[grp][cl] = b;
  __syncthreads();
  if (grp == 0 && c < s && dot1) {
    dot1[blockIdx.x * s + c] = ((red1[0][cl] + red1[1][cl]) + red1[2][cl]) + red1[3][cl];
    if (dot2) dot2[blockIdx.x * s + c] = ((red2[0][cl] + red2[1][cl]) + red2[2][cl]) + red2[3][cl];
  }
}

__global__ void k_pitch_f32(const double* __restrict__ in, int64_t n, int rank, int rp,
                            float* __restrict__ out) {
  const int64_t total = n * rp;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    const int64_t row = i / rp;
    const int k = (int)(i % rp);
    out[i] = k < rank ? (float)in[row * rank + k] : 0.0f;
  }
}

// ------------------------------------------------------------------ PCG --

template <typename T>
__global__ void k_copy2(const T* __restrict__ src, T* __restrict__ a, T* __restrict__ b,
                        int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    const T v = src[i];
    a[i] = v;
    if (b) b[i] = v;
  }
}

// First level of the column reductions: out[seg][c] = sum of parts[b][c]
// over the seg-th contiguous range of row blocks b (fixed order), so that the
// single-workgroup scalar kernels add only kSeg values per column.
constexpr int kSeg = 32;

// one workgroup's share: columns 64 x .. 64 x + 63, segment seg
__device__ void colsum_seg_block(const double* __restrict__ parts, int nblk, int64_t s,
                                 double* __restrict__ out, int64_t x, int seg) {
  __shared__ double red[4][64];
  const int cl = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t c = x * 64 + cl;
  const int chunk = (nblk + kSeg - 1) / kSeg;
  const int b0 = seg * chunk;
  const int b1 = b0 + chunk < nblk ? b0 + chunk : nblk;
  double acc = 0.0;
  if (c < s) {
    int b = b0 + q;
    for (; b + 12 < b1; b += 16) {
      const double v0 = parts[(int64_t)b * s + c], v1 = parts[(int64_t)(b + 4) * s + c];
      const double v2 = parts[(int64_t)(b + 8) * s + c], v3 = parts[(int64_t)(b + 12) * s + c];
      acc += v0;
      acc += v1;
      acc += v2;
      acc += v3;
    }
    for (; b < b1; b += 4) acc += parts[(int64_t)b * s + c];
  }
  red[q][cl] = acc;
  __syncthreads();
  if (q == 0 && c < s) out[(int64_t)seg * s + c] = ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}

__global__ __launch_bounds__(256) void k_colsum_seg(const double* __restrict__ parts, int nblk,
                                                    int64_t s, double* __restrict__ out) {
  colsum_seg_block(parts, nblk, s, out, blockIdx.x, blockIdx.y);
}

// True in every thread of the workgroup that finishes last among the grid's
// workgroups (device-scope counter, which that workgroup resets to 0 for the
// next launch); every workgroup's global writes before the call are then
// visible to it.  No workgroup waits for another.
__device__ bool last_workgroup(int* counter) {
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const int total = (int)(gridDim.x * gridDim.y * gridDim.z);
    last = atomicAdd(counter, 1) == total - 1;
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  if (threadIdx.x == 0) atomicExch(counter, 0);
  return true;
}

// sum over b of parts[b][c] in order b = 0, 1, ...; the loads are issued
// eight at a time (the single-workgroup scalar kernels are latency bound)
__device__ double block_colsum(const double* __restrict__ parts, int nblk, int64_t s, int64_t c) {
  double acc = 0.0;
  int b = 0;
  for (; b + 8 <= nblk; b += 8) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = parts[(int64_t)(b + j) * s + c];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += v[j];
  }
  for (; b < nblk; ++b) acc += parts[(int64_t)b * s + c];
  return acc;
}

// initial state after u0 = P^-1 z: rho0 = z^T u0 (dots1), ztz = z^T z (dots2)
__global__ void k_scal_init(Scal S, const double* __restrict__ dots1, const double* __restrict__ dots2,
                            int nblk, int64_t s, int J) {
  for (int64_t c = threadIdx.x; c < s; c += blockDim.x) {
    const double rho = block_colsum(dots1, nblk, s, c);
    const double ztz = block_colsum(dots2, nblk, s, c);
    S.rho[c] = rho;
    S.rho0[c] = rho;
    S.ztz[c] = ztz;
    S.alpha[c] = 0.0;
    S.beta[c] = 0.0;
    S.alpha_prev[c] = 1.0;
    S.beta_prev[c] = 0.0;
    const bool ok = rho > 0.0 && isfinite(rho);
    S.active[c] = ok ? 1 : 0;
    if (!ok) atomicOr(&S.status[1], 1);
    for (int j = 0; j < J; ++j) {
      S.zeta[j * s + c] = 1.0;
      S.zeta_prev[j * s + c] = 1.0;
      S.ztp[j * s + c] = ztz;
      S.ztx[j * s + c] = 0.0;
      S.frozen[j * s + c] = 0;
    }
  }
}

__device__ void scal_alpha_body(const Scal& S, const double* __restrict__ dots, int nblk,
                                int64_t s) {
  for (int64_t c = threadIdx.x; c < s; c += blockDim.x) {
    double a = 0.0;
    if (S.active[c]) {
      const double wq = block_colsum(dots, nblk, s, c);
      if (!(wq > 0.0) || !isfinite(wq)) {
        atomicOr(&S.status[1], 1);
        S.active[c] = 0;
      } else {
        a = S.rho[c] / wq;
      }
    }
    S.alpha[c] = a;
  }
}

__global__ void k_scal_alpha(Scal S, const double* __restrict__ dots, int nblk, int64_t s) {
  scal_alpha_body(S, dots, nblk, s);
}

// k_colsum_seg over the product's dot blocks, then (last workgroup) the
// alpha step on the kSeg partial sums: one launch, the same sums
__global__ __launch_bounds__(256) void k_colsum_alpha(Scal S, const double* __restrict__ parts,
                                                      int nblk, int64_t s,
                                                      double* __restrict__ sg, int* counter) {
  colsum_seg_block(parts, nblk, s, sg, blockIdx.x, blockIdx.y);
  if (last_workgroup(counter)) scal_alpha_body(S, sg, kSeg, s);
}

// r -= alpha q and y += alpha w (w = P^-1 p): y converges to M^-1 z when the
// seed shift is 0 (x = P y solves M P^-1 x = z)
template <typename T>
__global__ void k_update_ry(T* __restrict__ r, const T* __restrict__ q, T* __restrict__ y,
                            const T* __restrict__ w, const double* __restrict__ alpha, int64_t n,
                            int64_t s) {
  const int64_t total = n * s;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    const int64_t c = i % s;
    const double a = alpha[c];
    r[i] = (T)((double)r[i] - a * (double)q[i]);
    y[i] = (T)((double)y[i] + a * (double)w[i]);
  }
}

template <typename T>
__global__ void k_update_r(T* __restrict__ r, const T* __restrict__ q, const double* __restrict__ alpha,
                           int64_t n, int64_t s) {
  const int64_t total = n * s;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    const int64_t c = i % s;
    r[i] = (T)((double)r[i] - alpha[c] * (double)q[i]);
  }
}

// rho' = r^T u (dots1), z^T r (dots2); beta; shifted recurrences; convergence.
__device__ void scal_beta_body(const Scal& S, const double* __restrict__ dots1,
                               const double* __restrict__ dots2, int nblk, int64_t s, int J,
                               const double* __restrict__ delta, double tol) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int64_t c = threadIdx.x; c < s; c += blockDim.x) {
    if (!S.active[c]) {
      S.beta[c] = 0.0;
      continue;
    }
    const double rho_new = block_colsum(dots1, nblk, s, c);
    const double ztr = block_colsum(dots2, nblk, s, c);
    if (!(rho_new >= 0.0) || !isfinite(rho_new)) {
      atomicOr(&S.status[1], 1);
      S.active[c] = 0;
      S.beta[c] = 0.0;
      continue;
    }
    const double alpha = S.alpha[c];
    const double beta = rho_new / S.rho[c];
    const double ap = S.alpha_prev[c], bp = S.beta_prev[c];
    const double rel = sqrt(rho_new / S.rho0[c]);
    for (int j = 0; j < J; ++j) {
      const int64_t o = (int64_t)j * s + c;
      if (S.frozen[o]) continue;
      const double z = S.zeta[o], zp = S.zeta_prev[o];
      const double zn = z * zp * ap / (ap * zp * (1.0 + alpha * delta[j]) + alpha * bp * (zp - z));
      const double ratio = zn / z;
      const double aj = alpha * ratio;
      const double bj = beta * ratio * ratio;
      S.ztx[o] += aj * S.ztp[o];
      S.ztp[o] = zn * ztr + bj * S.ztp[o];
      S.zeta_prev[o] = z;
      S.zeta[o] = zn;
      if (!isfinite(zn) || fabs(zn) * rel < 1e-2 * tol || fabs(zn) < 1e-200) S.frozen[o] = 1;
    }
    S.alpha_prev[c] = alpha;
    S.beta_prev[c] = beta;
    S.rho[c] = rho_new;
    if (rel <= tol) {
      S.active[c] = 0;
      S.beta[c] = 0.0;
    } else {
      S.beta[c] = beta;
      ++mine;
    }
  }
  atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) S.status[0] = cnt;
}

__global__ void k_scal_beta(Scal S, const double* __restrict__ dots1, const double* __restrict__ dots2,
                            int nblk, int64_t s, int J, const double* __restrict__ delta, double tol) {
  scal_beta_body(S, dots1, dots2, nblk, s, J, delta, tol);
}

// k_colsum_seg over both Woodbury dot arrays (blockIdx.z), then (last
// workgroup) the beta step: one launch, the same sums
__global__ __launch_bounds__(256) void k_colsum_beta(Scal S, const double* __restrict__ d1,
                                                     const double* __restrict__ d2, int nblk,
                                                     int64_t s, double* __restrict__ sg1,
                                                     double* __restrict__ sg2, int J,
                                                     const double* __restrict__ delta, double tol,
                                                     int* counter) {
  if (blockIdx.z == 0)
    colsum_seg_block(d1, nblk, s, sg1, blockIdx.x, blockIdx.y);
  else
    colsum_seg_block(d2, nblk, s, sg2, blockIdx.x, blockIdx.y);
  if (last_workgroup(counter)) scal_beta_body(S, sg1, sg2, kSeg, s, J, delta, tol);
}

template <typename T>
__global__ void k_update_pw(T* __restrict__ p, T* __restrict__ w, const T* __restrict__ r,
                            const T* __restrict__ u, const double* __restrict__ beta,
                            const int* __restrict__ active, int64_t n, int64_t s) {
  const int64_t total = n * s;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    const int64_t c = i % s;
    if (!active[c]) continue;
    const double b = beta[c];
    p[i] = (T)((double)r[i] + b * (double)p[i]);
    w[i] = (T)((double)u[i] + b * (double)w[i]);
  }
}

int grid1(int64_t count) {
  int64_t b = (count + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

struct WoodPlan {
  int64_t chunks, chunk;
  int ltiles, ctiles;
  int64_t rtiles;
};

WoodPlan wood_plan(ld_ctx* ctx, int64_t n, int rank, int64_t s) {
  WoodPlan w{};
  w.ltiles = (rank + WT - 1) / WT;
  w.ctiles = (int)((s + WT - 1) / WT);
  // three workgroups of k_ft_partial fit a CU (registers): one wave of them
  int64_t chunks = (int64_t)ctx->num_cu * 3 / ((int64_t)w.ltiles * w.ctiles);
  const int64_t maxc = (n + 255) / 256;
  if (chunks > maxc) chunks = maxc;
  if (chunks < 1) chunks = 1;
  w.chunk = (n + chunks - 1) / chunks;
  w.chunks = (n + w.chunk - 1) / w.chunk;
  w.rtiles = (n + WT - 1) / WT;
  return w;
}

// P^-1 R into OUT; optional column dots per row tile (64 rows in FP64, 128
// rows in FP32: wood_dot_blocks).  Takes its scratch from the arena.
template <typename T>
ld_status wood_apply_t(ld_ctx* ctx, const ld_precond* P, const T* R, int64_t s, T* OUT,
                       const T* Z, double* dot1, double* dot2);

template <typename T>
ld_status wood_apply_diag(ld_ctx* ctx, const T* Dinv, int64_t n, const T* R, int64_t s, int rb,
                          T* OUT, const T* Z, double* dot1, double* dot2) {
  hipLaunchKernelGGL(k_wood_diag<T>, dim3((unsigned)((n + rb - 1) / rb), (unsigned)((s + 63) / 64)),
                     dim3(256), 0, ctx->stream, Dinv, R, n, s, rb, OUT, Z, dot1, dot2);
  LD_HIP(hipGetLastError());
  return LD_OK;
}

template <>
ld_status wood_apply_t<double>(ld_ctx* ctx, const ld_precond* P, const double* R, int64_t s,
                               double* OUT, const double* Z, double* dot1, double* dot2) {
  const int64_t n = P->n;
  const int rank = P->rank;
  if (rank == 0) return wood_apply_diag<double>(ctx, P->Dinv64, n, R, s, WT, OUT, Z, dot1, dot2);
  WoodPlan w = wood_plan(ctx, n, rank, s);
  double* part = (double*)ctx->arena.take((size_t)w.chunks * rank * s * sizeof(double));
  double* t = (double*)ctx->arena.take((size_t)rank * s * sizeof(double));
  if (!part || !t) return fail(LD_ENOMEM, "woodbury: scratch arena too small");
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_ft_partial<double>, dim3((unsigned)w.chunks, w.ltiles, w.ctiles), dim3(256),
                     0, st, P->F64, R, n, rank, s, w.chunk, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(grid1((int64_t)rank * s * 4)), dim3(64), 0, st, part,
                     (int)w.chunks, (int64_t)rank * s, t);
  hipLaunchKernelGGL(k_wood_out, dim3((unsigned)w.rtiles, w.ctiles), dim3(256), 0, st,
                     P->F64, P->Dinv64, t, R, n, rank, s, OUT, Z, dot1, dot2);
  LD_HIP(hipGetLastError());
  return LD_OK;
}

template <>
ld_status wood_apply_t<float>(ld_ctx* ctx, const ld_precond* P, const float* R, int64_t s,
                              float* OUT, const float* Z, double* dot1, double* dot2) {
  const int64_t n = P->n;
  const int rp = P->rp32;
  if (P->rank == 0) return wood_apply_diag<float>(ctx, P->Dinv32, n, R, s, W32R, OUT, Z, dot1, dot2);
  const int ltiles = (rp + W32R - 1) / W32R;
  const int ctiles = (int)((s + W32C - 1) / W32C);
  int64_t target = (int64_t)ctx->num_cu * 2 / ((int64_t)ltiles * ctiles);
  if (target < 1) target = 1;
  int64_t chunk = (n + target - 1) / target;
  chunk = (chunk + W32K - 1) / W32K * W32K;
  const int64_t chunks = (n + chunk - 1) / chunk;
  double* part = (double*)ctx->arena.take((size_t)chunks * rp * s * sizeof(double));
  float* t32 = (float*)ctx->arena.take((size_t)rp * s * sizeof(float));
  if (!part || !t32) return fail(LD_ENOMEM, "woodbury: scratch arena too small");
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_ft32, dim3((unsigned)chunks, ltiles, ctiles), dim3(256), 0, st, P->F32, R,
                     n, rp, s, chunk, part);
  const int64_t count = (int64_t)rp * s;
  hipLaunchKernelGGL(k_sum32, dim3((unsigned)((count + 63) / 64)), dim3(256), 0, st, part,
                     (int)chunks, count, t32);
  hipLaunchKernelGGL(k_wood32, dim3((unsigned)((n + W32R - 1) / W32R), ctiles), dim3(256), 0, st,
                     P->F32, P->Dinv32, t32, R, n, rp, s, OUT, Z, dot1, dot2);
  LD_HIP(hipGetLastError());
  return LD_OK;
}

int64_t wood_dot_blocks(bool f64, int64_t n) { return f64 ? (n + WT - 1) / WT : (n + W32R - 1) / W32R; }

}  // namespace

size_t woodbury_scratch_bytes(int64_t n, int rank, int64_t s) {
  // upper bound on chunks: num_cu * 4 <= 1024 (at most 256 CUs); FP32 rank
  // rows padded to a multiple of 32
  const int64_t chunks = 1024;
  const int64_t rp = (rank + 31) / 32 * 32;
  (void)n;
  return (size_t)(chunks + 1) * rp * s * sizeof(double) + 4096;
}

void launch_pitch_f32(hipStream_t st, const double* F64, int64_t n, int rank, int rp, float* F32) {
  hipLaunchKernelGGL(k_pitch_f32, dim3(grid1(n * rp)), dim3(256), 0, st, F64, n, rank, rp, F32);
}

ld_status woodbury_apply(ld_ctx* ctx, const ld_precond* P, bool f64, const void* R, int64_t s,
                         void* OUT) {
  if (f64)
    return wood_apply_t<double>(ctx, P, (const double*)R, s, (double*)OUT, nullptr, nullptr,
                                nullptr);
  return wood_apply_t<float>(ctx, P, (const float*)R, s, (float*)OUT, nullptr, nullptr, nullptr);
}

// ------------------------------------------------ Hutchinson combination --
// Section 1 / the output of Algorithm 1: t_i = b z_i^T z_i + sum_j c_j
// z_i^T x_ij per probe, then their mean and standard error, in FP64 and in a
// fixed order (one workgroup).
namespace {

__global__ void k_hutchinson(const double* __restrict__ ztx, const double* __restrict__ ztz,
                             int64_t s, Coef cf, double* __restrict__ per_probe,
                             double* __restrict__ stats) {
  for (int64_t c = threadIdx.x; c < s; c += blockDim.x) {
    double v = cf.b * ztz[c];
    for (int j = 0; j < cf.J; ++j) v += cf.c[j] * ztx[(int64_t)j * s + c];
    per_probe[c] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mean = 0.0;
    for (int64_t c = 0; c < s; ++c) mean += per_probe[c];
    mean /= (double)s;
    double var = 0.0;
    for (int64_t c = 0; c < s; ++c) var += (per_probe[c] - mean) * (per_probe[c] - mean);
    stats[0] = mean;
    stats[1] = s > 1 ? sqrt(var / (double)(s - 1) / (double)s) : (double)NAN;
  }
}

// ------------------------------------------------------------- Lanczos --
// Algorithm 1 as printed (Section 2): t Lanczos steps on A = M P^-1 per probe
// (all probes of the block in lock step), then for every pole a tridiagonal
// solve (T + a_j I) w = |v| e_1 by the Thomas algorithm and the output
// v^T Q^T w = sum_l (v^T q_l) w_l.  The recurrence runs in the inner product
// <x, y> = x^T P^-1 y, in which M P^-1 is self-adjoint: the vectors q_l are
// P^-1-orthonormal, q_1 = v / |v| with |v|^2 = v^T P^-1 v, so the right side
// of the shifted systems is |v| e_1, and v^T q_l are Euclidean products
// tracked as the recurrence runs (no Q is stored).  Per step:
//   y = M u_l                 (u_l = P^-1 q_l)           kernel matmat
//   alpha_l = u_l^T y                                    its epilogue dots
//   r = y - alpha_l q_l - beta_{l-1} q_{l-1}
//   r~ = P^-1 r ; beta_l^2 = r^T r~ ; v^T r               Woodbury + dots
//   q_{l+1} = r / beta_l ; u_{l+1} = r~ / beta_l
// A probe whose beta_l falls to 1e-12 times its largest |alpha| has reached
// an invariant subspace and stops (its T then gives the exact solves).
constexpr double kLzBreak = 1e-12;

struct Lz {
  double* alpha;  // steps x s
  double* beta;   // steps x s
  double* g;      // (steps + 1) x s : v^T q_l
  double* nv;     // |v|
  double* ztz;    // v^T v
  double* amax;   // largest |alpha| so far
  double* inv;    // 1 / (scale of the next Lanczos vector)
  double* bprev;  // beta of the previous step
  int* steps;     // steps taken
  int* active;
  int* status;    // [0] active probes, [1] breakdown (non-positive or non-finite norm)
};

__global__ void k_lz_init(Lz L, const double* __restrict__ d1, const double* __restrict__ d2,
                          int nblk, int64_t s) {
  for (int64_t c = threadIdx.x; c < s; c += blockDim.x) {
    const double nv2 = block_colsum(d1, nblk, s, c);
    const double zz = block_colsum(d2, nblk, s, c);
    const bool ok = nv2 > 0.0 && isfinite(nv2);
    const double nv = ok ? sqrt(nv2) : 0.0;
    L.nv[c] = nv;
    L.ztz[c] = zz;
    L.g[c] = ok ? zz / nv : 0.0;
    L.inv[c] = ok ? 1.0 / nv : 0.0;
    L.amax[c] = 0.0;
    L.bprev[c] = 0.0;
    L.steps[c] = 0;
    L.active[c] = ok ? 1 : 0;
    if (!ok) atomicOr(&L.status[1], 1);
  }
}

template <typename T>
__global__ void k_lz_scale(T* __restrict__ a, T* __restrict__ b, const double* __restrict__ inv,
                           const int* __restrict__ active, int64_t n, int64_t s) {
  const int64_t total = n * s;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    const int64_t c = i % s;
    if (!active[c]) continue;
    const double f = inv[c];
    a[i] = (T)((double)a[i] * f);
    b[i] = (T)((double)b[i] * f);
  }
}

__device__ void lz_alpha_body(const Lz& L, const double* __restrict__ dots, int nblk, int64_t s,
                              int l) {
  for (int64_t c = threadIdx.x; c < s; c += blockDim.x) {
    if (!L.active[c]) continue;
    const double a = block_colsum(dots, nblk, s, c);
    if (!isfinite(a)) {
      atomicOr(&L.status[1], 1);
      L.active[c] = 0;
      continue;
    }
    L.alpha[(int64_t)l * s + c] = a;
    L.amax[c] = fmax(L.amax[c], fabs(a));
  }
}

// column sums of the product's dot blocks, then (last workgroup) alpha_l
__global__ __launch_bounds__(256) void k_colsum_lz_alpha(Lz L, const double* __restrict__ parts,
                                                         int nblk, int64_t s,
                                                         double* __restrict__ sg, int l,
                                                         int* counter) {
  colsum_seg_block(parts, nblk, s, sg, blockIdx.x, blockIdx.y);
  if (last_workgroup(counter)) lz_alpha_body(L, sg, kSeg, s, l);
}

template <typename T>
__global__ void k_lz_resid(T* __restrict__ r, const T* __restrict__ q, const T* __restrict__ qp,
                           const double* __restrict__ alpha, const double* __restrict__ bprev,
                           const int* __restrict__ active, int64_t n, int64_t s) {
  const int64_t total = n * s;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    const int64_t c = i % s;
    if (!active[c]) continue;
    r[i] = (T)((double)r[i] - alpha[c] * (double)q[i] - bprev[c] * (double)qp[i]);
  }
}

__device__ void lz_beta_body(const Lz& L, const double* __restrict__ d1,
                             const double* __restrict__ d2, int nblk, int64_t s, int l) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int64_t c = threadIdx.x; c < s; c += blockDim.x) {
    if (!L.active[c]) continue;
    const double b2 = block_colsum(d1, nblk, s, c);
    const double vr = block_colsum(d2, nblk, s, c);
    L.steps[c] = l + 1;
    if (!(b2 >= 0.0) || !isfinite(b2)) {
      atomicOr(&L.status[1], 1);
      L.beta[(int64_t)l * s + c] = 0.0;
      L.active[c] = 0;
      continue;
    }
    const double b = sqrt(b2);
    L.beta[(int64_t)l * s + c] = b;
    if (b <= kLzBreak * L.amax[c]) {  // invariant subspace: T is exact
      L.active[c] = 0;
      continue;
    }
    L.inv[c] = 1.0 / b;
    L.bprev[c] = b;
    L.g[(int64_t)(l + 1) * s + c] = vr / b;
    ++mine;
  }
  atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) L.status[0] = cnt;
}

// column sums of both Woodbury dot arrays (blockIdx.z), then (last
// workgroup) beta_l
__global__ __launch_bounds__(256) void k_colsum_lz_beta(Lz L, const double* __restrict__ d1,
                                                        const double* __restrict__ d2, int nblk,
                                                        int64_t s, double* __restrict__ sg1,
                                                        double* __restrict__ sg2, int l,
                                                        int* counter) {
  if (blockIdx.z == 0)
    colsum_seg_block(d1, nblk, s, sg1, blockIdx.x, blockIdx.y);
  else
    colsum_seg_block(d2, nblk, s, sg2, blockIdx.x, blockIdx.y);
  if (last_workgroup(counter)) lz_beta_body(L, sg1, sg2, kSeg, s, l);
}

// Per probe: the Thomas algorithm for (T + a_j I) w = |v| e_1 (T + a_j I is
// SPD, no pivoting), the output b v^T v + sum_j c_j g^T w_j, and the P^-1
// residual of the smallest-shift system relative to |v|,
// beta_m |w_m| / |v|; then the Hutchinson mean and standard error.
__global__ void k_lz_finish(Lz L, int64_t s, Coef cf, double* __restrict__ per_probe,
                            double* __restrict__ resid, double* __restrict__ stats) {
  for (int64_t c = threadIdx.x; c < s; c += blockDim.x) {
    const int m = L.steps[c];
    const double nv = L.nv[c];
    if (m == 0) {
      per_probe[c] = (double)NAN;
      resid[c] = (double)NAN;
      continue;
    }
    double cp[kLzMax], yp[kLzMax];
    double val = cf.b * L.ztz[c];
    for (int j = 0; j < cf.J; ++j) {
      const double aj = cf.a[j];
      double den = L.alpha[c] + aj;
      cp[0] = m > 1 ? L.beta[c] / den : 0.0;
      yp[0] = nv / den;
      for (int l = 1; l < m; ++l) {
        const double e = L.beta[(int64_t)(l - 1) * s + c];
        den = L.alpha[(int64_t)l * s + c] + aj - e * cp[l - 1];
        cp[l] = l + 1 < m ? L.beta[(int64_t)l * s + c] / den : 0.0;
        yp[l] = -e * yp[l - 1] / den;
      }
      // back substitution, accumulating g^T w from the last row up
      double w = yp[m - 1];
      double gw = L.g[(int64_t)(m - 1) * s + c] * w;
      if (j == 0) resid[c] = L.beta[(int64_t)(m - 1) * s + c] * fabs(w) / nv;
      for (int l = m - 2; l >= 0; --l) {
        w = yp[l] - cp[l] * w;
        gw += L.g[(int64_t)l * s + c] * w;
      }
      val += cf.c[j] * gw;
    }
    per_probe[c] = val;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mean = 0.0, worst = 0.0;
    for (int64_t c = 0; c < s; ++c) {
      mean += per_probe[c];
      worst = fmax(worst, resid[c]);
    }
    mean /= (double)s;
    double var = 0.0;
    for (int64_t c = 0; c < s; ++c) var += (per_probe[c] - mean) * (per_probe[c] - mean);
    stats[0] = mean;
    stats[1] = s > 1 ? sqrt(var / (double)(s - 1) / (double)s) : (double)NAN;
    stats[2] = worst;
  }
}

template <typename T>
ld_status lanczos_run(ld_ctx* ctx, bool f64, const MatmatArgs& base, const ld_precond* P,
                      const Coef* cfs, int ncf, const T* Z, int64_t s, int t, LzOut* outs) {
  const int64_t n = base.n;
  const size_t vec = (size_t)n * s;
  hipStream_t st = ctx->stream;
  T* q = (T*)ctx->arena.take(vec * sizeof(T));
  T* qp = (T*)ctx->arena.take(vec * sizeof(T));
  T* r = (T*)ctx->arena.take(vec * sizeof(T));
  T* u = (T*)ctx->arena.take(vec * sizeof(T));
  T* ut = (T*)ctx->arena.take(vec * sizeof(T));
  const int64_t mrt = (n + kEpiRows - 1) / kEpiRows * kEpiSplitMax;
  const int64_t wrt = wood_dot_blocks(f64, n);
  double* dwq = (double*)ctx->arena.take((size_t)mrt * s * sizeof(double));
  double* d1 = (double*)ctx->arena.take((size_t)wrt * s * sizeof(double));
  double* d2 = (double*)ctx->arena.take((size_t)wrt * s * sizeof(double));
  double* sg1 = (double*)ctx->arena.take((size_t)kSeg * s * sizeof(double));
  double* sg2 = (double*)ctx->arena.take((size_t)kSeg * s * sizeof(double));
  double* sc = (double*)ctx->arena.take(((size_t)(3 * t + 1) * s + 8 * s + 3) * sizeof(double));
  int* isc = (int*)ctx->arena.take((size_t)(2 * s + 4) * sizeof(int));
  if (!q || !qp || !r || !u || !ut || !dwq || !d1 || !d2 || !sg1 || !sg2 || !sc || !isc)
    return fail(LD_ENOMEM, "lanczos: scratch arena too small");
  Lz L;
  L.alpha = sc;
  L.beta = L.alpha + (size_t)t * s;
  L.g = L.beta + (size_t)t * s;
  L.nv = L.g + (size_t)(t + 1) * s;
  L.ztz = L.nv + s;
  L.amax = L.ztz + s;
  L.inv = L.amax + s;
  L.bprev = L.inv + s;
  double* per_probe = L.bprev + s;
  double* resid = per_probe + s;
  double* stats = resid + s;
  L.steps = isc;
  L.active = isc + s;
  L.status = isc + 2 * s;
  int* counters = L.status + 2;  // last-workgroup counters of the fused scalar steps
  LD_TRY(ensure_pinned(ctx, (size_t)(2 * s + 8)));
  LD_HIP(hipMemsetAsync(L.status, 0, 4 * sizeof(int), st));
  LD_HIP(hipMemsetAsync(qp, 0, vec * sizeof(T), st));
  const size_t mark = ctx->arena.top;
  const dim3 cs_grid((unsigned)((s + 63) / 64), kSeg);

  // q_1 = v / |v|, u_1 = P^-1 q_1
  hipLaunchKernelGGL(k_copy2<T>, dim3(grid1(vec)), dim3(256), 0, st, Z, q, (T*)nullptr,
                     (int64_t)vec);
  LD_TRY(wood_apply_t<T>(ctx, P, q, s, u, Z, d1, d2));
  ctx->arena.top = mark;
  hipLaunchKernelGGL(k_colsum_seg, cs_grid, dim3(256), 0, st, d1, (int)wrt, s, sg1);
  hipLaunchKernelGGL(k_colsum_seg, cs_grid, dim3(256), 0, st, d2, (int)wrt, s, sg2);
  hipLaunchKernelGGL(k_lz_init, dim3(1), dim3(256), 0, st, L, sg1, sg2, kSeg, s);
  hipLaunchKernelGGL(k_lz_scale<T>, dim3(grid1(vec)), dim3(256), 0, st, q, u, L.inv, L.active, n, s);
  LD_HIP(hipGetLastError());

  const int check_every = n >= 16384 ? 1 : 8;
  for (int l = 0; l < t; ++l) {
    ctx->arena.top = mark;
    MatmatArgs a = base;
    a.s = s;
    a.V = u;
    a.Y = r;
    a.X2 = nullptr;
    a.alpha2 = 0.0;
    a.dots = dwq;
    a.timed = true;
    int nb = 0;
    a.dot_blocks = &nb;
    LD_TRY(matmat(ctx, f64, a));
    hipLaunchKernelGGL(k_colsum_lz_alpha, cs_grid, dim3(256), 0, st, L, dwq, nb, s, sg1, l,
                       counters);
    hipLaunchKernelGGL(k_lz_resid<T>, dim3(grid1(vec)), dim3(256), 0, st, r, q, qp,
                       L.alpha + (size_t)l * s, L.bprev, L.active, n, s);
    ctx->arena.top = mark;
    LD_TRY(wood_apply_t<T>(ctx, P, r, s, ut, Z, d1, d2));
    hipLaunchKernelGGL(k_colsum_lz_beta, dim3(cs_grid.x, cs_grid.y, 2), dim3(256), 0, st, L, d1,
                       d2, (int)wrt, s, sg1, sg2, l, counters + 1);
    hipLaunchKernelGGL(k_lz_scale<T>, dim3(grid1(vec)), dim3(256), 0, st, r, ut, L.inv, L.active,
                       n, s);
    LD_HIP(hipGetLastError());
    // q_{l-1} <- q_l, q_l <- q_{l+1} (in r), u_l <- u_{l+1} (in ut)
    T* tq = qp;
    qp = q;
    q = r;
    r = tq;
    T* tu = u;
    u = ut;
    ut = tu;
    if ((l + 1) % check_every == 0 && l + 1 < t) {
      LD_HIP(hipMemcpyAsync(ctx->pinned, L.status, sizeof(int), hipMemcpyDeviceToHost, st));
      LD_HIP(hipStreamSynchronize(st));
      timing_collect(ctx);
      if (*(const int*)ctx->pinned == 0) break;
    }
  }
  ctx->arena.top = mark;
  // the recurrence does not depend on the shifts: every estimate's
  // tridiagonal solves and Hutchinson mean come from the same T
  for (int e = 0; e < ncf; ++e) {
    LzOut& o = outs[e];
    hipLaunchKernelGGL(k_lz_finish, dim3(1), dim3(256), 0, st, L, s, cfs[e], per_probe, resid,
                       stats);
    LD_HIP(hipGetLastError());
    double* hp = ctx->pinned;
    LD_HIP(hipMemcpyAsync(hp, per_probe, (size_t)s * sizeof(double), hipMemcpyDeviceToHost, st));
    LD_HIP(hipMemcpyAsync(hp + s, stats, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    LD_HIP(hipMemcpyAsync(hp + s + 3, L.steps, (size_t)s * sizeof(int), hipMemcpyDeviceToHost, st));
    LD_HIP(hipMemcpyAsync((int*)(hp + s + 3) + s, L.status, 2 * sizeof(int),
                          hipMemcpyDeviceToHost, st));
    LD_HIP(hipStreamSynchronize(st));
    if (e == 0) timing_collect(ctx);
    o.per_probe.assign(hp, hp + s);
    o.mean = hp[s];
    o.stderr_ = hp[s + 1];
    o.resid = hp[s + 2];
    const int* steps = (const int*)(hp + s + 3);
    o.max_steps = 0;
    o.exact = 0;
    for (int64_t c = 0; c < s; ++c) {
      o.max_steps = std::max(o.max_steps, steps[c]);
      if (steps[c] < t) ++o.exact;
    }
    o.breakdown = ((const int*)(hp + s + 3))[s + 1] != 0;
  }
  return LD_OK;
}

}  // namespace

ld_status lanczos_estimate(ld_ctx* ctx, bool f64, const MatmatArgs& base, const ld_precond* P,
                           const Coef& cf, const void* Z, int64_t s, int t, LzOut& out) {
  if (f64) return lanczos_run<double>(ctx, true, base, P, &cf, 1, (const double*)Z, s, t, &out);
  return lanczos_run<float>(ctx, false, base, P, &cf, 1, (const float*)Z, s, t, &out);
}

ld_status lanczos_estimate_multi(ld_ctx* ctx, bool f64, const MatmatArgs& base,
                                 const ld_precond* P, const Coef* cfs, int ncf, const void* Z,
                                 int64_t s, int t, LzOut* outs) {
  if (f64) return lanczos_run<double>(ctx, true, base, P, cfs, ncf, (const double*)Z, s, t, outs);
  return lanczos_run<float>(ctx, false, base, P, cfs, ncf, (const float*)Z, s, t, outs);
}

size_t lanczos_scratch_bytes(ld_ctx* ctx, bool f64, int64_t n, int rank, int64_t s, int t) {
  const size_t es = f64 ? 8 : 4;
  size_t b = 5 * (size_t)n * s * es + 1280;
  b += ((n + kEpiRows - 1) / kEpiRows * kEpiSplitMax + 2 * ((n + 63) / 64)) * (size_t)s * 8 + 768;
  b += 2 * (size_t)kSeg * s * 8 + 512;
  b += ((size_t)(3 * t + 1) * s + 8 * s + 3) * 8 + (size_t)(2 * s + 4) * 4 + 512;
  b += std::max(matmat_scratch_bytes(ctx, f64, n, s), woodbury_scratch_bytes(n, rank, s)) + 1024;
  return b;
}

ld_status hutchinson(ld_ctx* ctx, const double* ztx_dev, const double* ztz_dev, int64_t s,
                     const Coef& cf, double* per_probe_dev, double* stats_dev) {
  hipLaunchKernelGGL(k_hutchinson, dim3(1), dim3(256), 0, ctx->stream, ztx_dev, ztz_dev, s, cf,
                     per_probe_dev, stats_dev);
  LD_HIP(hipGetLastError());
  return LD_OK;
}

// --------------------------------------------------------------- driver --
namespace {

struct PcgOut {
  int iterations = 0;
  int converged = 0;
  double rel_resid = 0.0;
  bool breakdown = false;
};

// While a solve replays captured chunks it runs on the context's side stream
// (the caller's stream may be the null stream, which cannot be captured):
// the side stream first waits for the work already on the context stream,
// and on scope exit the context stream waits for the side stream and is
// restored, so stream order is as if everything ran on it.
struct SideStream {
  ld_ctx* ctx = nullptr;
  hipStream_t orig = nullptr;
  ld_status enter(ld_ctx* c) {
    if (!c->side) LD_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    if (!c->ev_join) LD_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    LD_HIP(hipEventRecord(c->ev_join, c->stream));
    LD_HIP(hipStreamWaitEvent(c->side, c->ev_join, 0));
    ctx = c;
    orig = c->stream;
    c->stream = c->side;
    return LD_OK;
  }
  ~SideStream() {
    if (!ctx) return;
    if (hipEventRecord(ctx->ev_join, ctx->side) == hipSuccess)
      (void)hipStreamWaitEvent(orig, ctx->ev_join, 0);
    ctx->stream = orig;
  }
};

// A captured chunk of solver iterations (HIP graph), replayed on the same
// stream.  If capture or instantiation is refused, `failed` is set and the
// caller runs the chunk eagerly; the stream always leaves capture mode.
struct GraphChunk {
  hipGraphExec_t exec = nullptr;
  bool failed = false;
  template <typename F>
  ld_status capture(hipStream_t st, F&& enqueue) {
    if (hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) != hipSuccess) {
      (void)hipGetLastError();
      failed = true;
      return LD_OK;
    }
    const ld_status body = enqueue();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (body != LD_OK) {
      if (g) (void)hipGraphDestroy(g);
      return body;
    }
    if (e != hipSuccess || !g || hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGetLastError();
      exec = nullptr;
      failed = true;
    }
    if (g) (void)hipGraphDestroy(g);
    return LD_OK;
  }
  ~GraphChunk() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

template <typename T>
ld_status pcg_run(ld_ctx* ctx, bool f64, const MatmatArgs& base, const ld_precond* P,
                  const double* shifts, int J, const Coef* cfs, int ncf, const T* Z, int64_t s,
                  double tol, int max_iters, std::vector<double>& per_probe, double* mean,
                  double* stderr_, PcgOut& res, T* ysol) {
  const int64_t n = base.n;
  const size_t vec = (size_t)n * s;
  hipStream_t st = ctx->stream;
  T* r = (T*)ctx->arena.take(vec * sizeof(T));
  T* u = (T*)ctx->arena.take(vec * sizeof(T));
  T* p = (T*)ctx->arena.take(vec * sizeof(T));
  T* w = (T*)ctx->arena.take(vec * sizeof(T));
  T* q = (T*)ctx->arena.take(vec * sizeof(T));
  const int64_t mrt = (n + kEpiRows - 1) / kEpiRows * kEpiSplitMax;  // matmat dot blocks
  const int64_t wrt = wood_dot_blocks(f64, n);  // woodbury dot blocks
  double* dwq = (double*)ctx->arena.take((size_t)mrt * s * sizeof(double));
  double* d1 = (double*)ctx->arena.take((size_t)wrt * s * sizeof(double));
  double* d2 = (double*)ctx->arena.take((size_t)wrt * s * sizeof(double));
  double* scal = (double*)ctx->arena.take((size_t)(7 * s + 4 * J * s + J) * sizeof(double));
  int* iscal = (int*)ctx->arena.take((size_t)(J * s + s + 4) * sizeof(int));
  double* sg1 = (double*)ctx->arena.take((size_t)kSeg * s * sizeof(double));
  double* sg2 = (double*)ctx->arena.take((size_t)kSeg * s * sizeof(double));
  double* hut = (double*)ctx->arena.take((size_t)ncf * (s + 2) * sizeof(double));
  if (!r || !u || !p || !w || !q || !dwq || !d1 || !d2 || !scal || !iscal || !sg1 || !sg2 || !hut)
    return fail(LD_ENOMEM, "pcg: scratch arena too small");
  Scal S;
  S.rho = scal;
  S.rho0 = scal + s;
  S.alpha = scal + 2 * s;
  S.beta = scal + 3 * s;
  S.alpha_prev = scal + 4 * s;
  S.beta_prev = scal + 5 * s;
  S.ztz = scal + 6 * s;
  S.zeta = scal + 7 * s;
  S.zeta_prev = S.zeta + J * s;
  S.ztp = S.zeta_prev + J * s;
  S.ztx = S.ztp + J * s;
  double* delta = S.ztx + J * s;
  S.frozen = iscal;
  S.active = iscal + J * s;
  S.status = iscal + J * s + s;
  int* counters = S.status + 2;  // last-workgroup counters of the fused scalar steps

  std::vector<double> dl(J);
  for (int j = 0; j < J; ++j) dl[j] = shifts[j] - shifts[0];
  LD_TRY(ensure_pinned(ctx, (size_t)(2 * J * s + (ncf + 2) * s + 2 * ncf + 8)));
  std::copy(dl.begin(), dl.end(), ctx->pinned);
  LD_HIP(hipMemcpyAsync(delta, ctx->pinned, J * sizeof(double), hipMemcpyHostToDevice, st));
  LD_HIP(hipMemsetAsync(S.status, 0, 4 * sizeof(int), st));
  // wait for the small upload before the pinned buffer is reused below
  LD_HIP(hipStreamSynchronize(st));

  // The arena top after the persistent buffers: the scratch of each matmat /
  // Woodbury call is taken from here and handed back once its consumer is
  // enqueued (stream order keeps the reuse safe).
  const size_t mark = ctx->arena.top;

  // r = z, p = z; u = P^-1 r, w = u; rho0 = r^T u; z^T z
  if (ysol) LD_HIP(hipMemsetAsync(ysol, 0, vec * sizeof(T), st));
  hipLaunchKernelGGL(k_copy2<T>, dim3(grid1(vec)), dim3(256), 0, st, Z, r, p, (int64_t)vec);
  LD_TRY(wood_apply_t<T>(ctx, P, r, s, u, Z, d1, d2));
  ctx->arena.top = mark;
  hipLaunchKernelGGL(k_copy2<T>, dim3(grid1(vec)), dim3(256), 0, st, u, w, (T*)nullptr,
                     (int64_t)vec);
  const dim3 cs_grid((unsigned)((s + 63) / 64), kSeg);
  hipLaunchKernelGGL(k_colsum_seg, cs_grid, dim3(256), 0, st, d1, (int)wrt, s, sg1);
  hipLaunchKernelGGL(k_colsum_seg, cs_grid, dim3(256), 0, st, d2, (int)wrt, s, sg2);
  hipLaunchKernelGGL(k_scal_init, dim3(1), dim3(256), 0, st, S, sg1, sg2, kSeg, s, J);
  LD_HIP(hipGetLastError());

  const int check_every = n >= 16384 ? 1 : 8;
  // one CG iteration, every shift (all device work; the same buffers and
  // launch shapes each time, so a chunk of them can be captured and replayed)
  auto iteration = [&]() -> ld_status {
    ctx->arena.top = mark;
    MatmatArgs a = base;
    a.s = s;
    a.V = w;
    a.Y = q;
    a.X2 = p;
    a.alpha2 = shifts[0];
    a.dots = dwq;
    a.timed = true;
    int nb = 0;
    a.dot_blocks = &nb;
    LD_TRY(matmat(ctx, f64, a));
    hipLaunchKernelGGL(k_colsum_alpha, cs_grid, dim3(256), 0, st, S, dwq, nb, s, sg1, counters);
    if (ysol)
      hipLaunchKernelGGL(k_update_ry<T>, dim3(grid1(vec)), dim3(256), 0, st, r, q, ysol, w,
                         S.alpha, n, s);
    else
      hipLaunchKernelGGL(k_update_r<T>, dim3(grid1(vec)), dim3(256), 0, st, r, q, S.alpha, n, s);
    ctx->arena.top = mark;
    LD_TRY(wood_apply_t<T>(ctx, P, r, s, u, Z, d1, d2));
    hipLaunchKernelGGL(k_colsum_beta, dim3(cs_grid.x, cs_grid.y, 2), dim3(256), 0, st, S, d1, d2,
                       (int)wrt, s, sg1, sg2, J, delta, tol, counters + 1);
    hipLaunchKernelGGL(k_update_pw<T>, dim3(grid1(vec)), dim3(256), 0, st, p, w, r, u, S.beta,
                       S.active, n, s);
    LD_HIP(hipGetLastError());
    return LD_OK;
  };
  // Optional replay (ld_ctx_set_graphs; not while timing events are on):
  // the first full chunk of check_every iterations is captured once and
  // replayed for every later full chunk; a shorter last chunk runs eagerly.
  GraphChunk chunk;
  const bool replay = ctx->graphs && !ctx->timing;
  int it = 0;
  int active = (int)s;
  while (it < max_iters && active > 0) {
    const int todo = std::min(check_every, max_iters - it);
    if (replay && todo == check_every && !chunk.exec && !chunk.failed)
      LD_TRY(chunk.capture(st, [&]() -> ld_status {
        for (int k = 0; k < todo; ++k) LD_TRY(iteration());
        return LD_OK;
      }));
    if (replay && todo == check_every && chunk.exec) {
      LD_HIP(hipGraphLaunch(chunk.exec, st));
    } else {
      for (int k = 0; k < todo; ++k) LD_TRY(iteration());
    }
    it += todo;
    LD_HIP(hipMemcpyAsync(ctx->pinned, S.status, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    LD_HIP(hipStreamSynchronize(st));
    timing_collect(ctx);
    const int* stt = (const int*)ctx->pinned;
    active = stt[0];
    if (stt[1]) res.breakdown = true;
  }
  ctx->arena.top = mark;
  res.iterations = it;

  // Hutchinson combination of every estimate on the device; read back the
  // per-probe values, means, standard errors, rho and rho0
  const int64_t hs = s + 2;
  for (int o = 0; o < ncf; ++o) LD_TRY(hutchinson(ctx, S.ztx, S.ztz, s, cfs[o], hut + o * hs, hut + o * hs + s));
  double* hp = ctx->pinned;
  LD_HIP(hipMemcpyAsync(hp, hut, (size_t)(ncf * hs) * sizeof(double), hipMemcpyDeviceToHost, st));
  double* hr = hp + ncf * hs;
  LD_HIP(hipMemcpyAsync(hr, S.rho, s * sizeof(double), hipMemcpyDeviceToHost, st));
  LD_HIP(hipMemcpyAsync(hr + s, S.rho0, s * sizeof(double), hipMemcpyDeviceToHost, st));
  LD_HIP(hipStreamSynchronize(st));
  per_probe.resize((size_t)ncf * s);
  for (int o = 0; o < ncf; ++o) {
    std::copy(hp + o * hs, hp + o * hs + s, per_probe.begin() + o * s);
    mean[o] = hp[o * hs + s];
    stderr_[o] = hp[o * hs + s + 1];
  }
  double worst = 0.0;
  int conv = 0;
  for (int64_t c = 0; c < s; ++c) {
    const double rr = std::sqrt(std::max(0.0, hr[c] / hr[s + c]));
    worst = std::max(worst, rr);
    if (rr <= tol) ++conv;
  }
  res.rel_resid = worst;
  res.converged = conv;
  return LD_OK;
}

}  // namespace

ld_status multishift_pcg(ld_ctx* ctx, bool f64, const MatmatArgs& base, const ld_precond* P,
                         const Coef& cf, const void* Z, int64_t s, double tol, int max_iters,
                         std::vector<double>& per_probe, double* mean, double* stderr_,
                         int* iterations, int* converged, double* rel_resid, bool* breakdown,
                         void* ysol) {
  PcgOut o;
  ld_status stt;
  SideStream side;
  if (ctx->graphs && !ctx->timing) LD_TRY(side.enter(ctx));
  if (f64)
    stt = pcg_run<double>(ctx, true, base, P, cf.a, cf.J, &cf, 1, (const double*)Z, s, tol,
                          max_iters, per_probe, mean, stderr_, o, (double*)ysol);
  else
    stt = pcg_run<float>(ctx, false, base, P, cf.a, cf.J, &cf, 1, (const float*)Z, s, tol,
                         max_iters, per_probe, mean, stderr_, o, (float*)ysol);
  *iterations = o.iterations;
  *converged = o.converged;
  *rel_resid = o.rel_resid;
  *breakdown = o.breakdown;
  return stt;
}

ld_status multishift_pcg_multi(ld_ctx* ctx, bool f64, const MatmatArgs& base, const ld_precond* P,
                               const Coef* cfs, int ncf, const void* Z, int64_t s, double tol,
                               int max_iters, std::vector<double>& per_probe, double* mean,
                               double* stderr_, int* iterations, int* converged, double* rel_resid,
                               bool* breakdown) {
  PcgOut o;
  ld_status stt;
  SideStream side;
  if (ctx->graphs && !ctx->timing) LD_TRY(side.enter(ctx));
  if (f64)
    stt = pcg_run<double>(ctx, true, base, P, cfs[0].a, cfs[0].J, cfs, ncf, (const double*)Z, s,
                          tol, max_iters, per_probe, mean, stderr_, o, (double*)nullptr);
  else
    stt = pcg_run<float>(ctx, false, base, P, cfs[0].a, cfs[0].J, cfs, ncf, (const float*)Z, s,
                         tol, max_iters, per_probe, mean, stderr_, o, (float*)nullptr);
  *iterations = o.iterations;
  *converged = o.converged;
  *rel_resid = o.rel_resid;
  *breakdown = o.breakdown;
  return stt;
}

void launch_scal_init(hipStream_t st, const Scal& S, const double* d1, const double* d2, int nblk,
                      int64_t ncols, int J) {
  hipLaunchKernelGGL(k_scal_init, dim3(1), dim3(256), 0, st, S, d1, d2, nblk, ncols, J);
}

void launch_scal_alpha(hipStream_t st, const Scal& S, const double* dots, int nblk, int64_t ncols) {
  hipLaunchKernelGGL(k_scal_alpha, dim3(1), dim3(256), 0, st, S, dots, nblk, ncols);
}

void launch_scal_beta(hipStream_t st, const Scal& S, const double* d1, const double* d2, int nblk,
                      int64_t ncols, int J, const double* delta, double tol) {
  hipLaunchKernelGGL(k_scal_beta, dim3(1), dim3(256), 0, st, S, d1, d2, nblk, ncols, J, delta, tol);
}

size_t pcg_scratch_bytes(ld_ctx* ctx, bool f64, int64_t n, int rank, int64_t s, int J) {
  const size_t es = f64 ? 8 : 4;
  size_t b = 5 * (size_t)n * s * es + 1280;
  b += ((n + kEpiRows - 1) / kEpiRows * kEpiSplitMax + 2 * ((n + 63) / 64)) * (size_t)s * 8 + 768;
  b += (size_t)(7 * s + 4 * J * s + J) * 8 + (size_t)(J * s + s + 4) * 4 + 512;
  b += 2 * (size_t)kSeg * s * 8 + 3 * (size_t)(s + 2) * 8 + 768;   // up to 3 estimates
  b += std::max(matmat_scratch_bytes(ctx, f64, n, s), woodbury_scratch_bytes(n, rank, s)) + 1024;
  return b;
}

}  // namespace ld
