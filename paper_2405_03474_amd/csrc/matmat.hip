// Kernel-matrix times block products Y = M V (Section 2: the product that
// dominates every Krylov step, cost O(n^2) per column) on CDNA4 matrix cores.
//
// Two sources for the left operand:
//   stored : M (n x n, row-major) streamed from HBM through LDS
//   on the fly : every lane evaluates its own MFMA A-fragment entries
//            k(x_i, x_k) from the points, so the n x n matrix never exists
// and two arithmetic paths:
//   FP32 : v_mfma_f32_32x32x2f32, wave tile 32 rows x 32*NB columns
//   FP64 : v_mfma_f64_16x16x4f64, wave tile 32 rows x 16*NB columns
// A workgroup is 4 waves stacked along rows (128 rows).  Work is split
// stream-K style: the (tile, k-stage) index space is cut into G equal
// contiguous ranges, one per workgroup, so every CU gets the same number of
// MFMA stages whatever n is.  Each workgroup writes the partial sums of every
// tile it touched to a scratch slot; an epilogue kernel adds the slots of a
// tile in a fixed order (deterministic), adds noise * V for the on-the-fly
// path, an optional alpha2 * X2 term, and optional per-column dots V^T Y.
//
// The k index inside a stage is permuted so that every lane reads contiguous
// LDS words: in MFMA k-step t, lane half h supplies physical column
// h * (BK / halves) + t for both operands.
#include <algorithm>

#include <cmath>
#include <mutex>
#include <type_traits>

#include "kfun_dev.hpp"
#include "ld_common.hpp"
#include "sym_split.hpp"

namespace ld {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128;  // rows per workgroup tile
constexpr int BK = 32;   // k per stage
constexpr int DMAX = 16; // max point dimension on the fly
constexpr float kLog2e = 1.4426950408889634f;
constexpr int kMaxContrib = 64;  // partial slots summed per output tile (bounded by the plan)

// Work split.  The S k-stages are cut into nx contiguous chunks, one per XCD
// (workgroup g runs on XCD g mod nx), so the slice of V a chunk needs stays
// in that XCD's L2; inside a chunk, the (tile, stage) units are cut into
// G/nx equal contiguous ranges, one per workgroup of that XCD (stream-K).
struct SK {
  int64_t n, s;
  int64_t ld;     // row stride of V, Y and X2 (s, or wider for a column panel)
  int64_t tiles;  // row tiles * column tiles
  int rt;         // row tiles
  int S;          // stages per tile
  int G;          // workgroups, a multiple of nx
  int nx;         // k chunks
  int J;          // partial slots per workgroup
};

struct WGRange {
  int sb;          // first stage of the workgroup's k chunk
  int Sx;          // stages in the chunk
  int64_t u, uend; // unit range inside the chunk
};

__host__ __device__ inline WGRange wg_range(const SK& p, int g) {
  const int x = g % p.nx, lg = g / p.nx, Gx = p.G / p.nx;
  WGRange r;
  r.sb = (int)(((int64_t)p.S * x) / p.nx);
  r.Sx = (int)(((int64_t)p.S * (x + 1)) / p.nx) - r.sb;
  const int64_t Ux = p.tiles * r.Sx;
  r.u = Ux * lg / Gx;
  r.uend = Ux * (lg + 1) / Gx;
  return r;
}

// ---------------------------------------------------------- kernel values --
// FP32 kernel values from pre-scaled points: kval32s (kfun_dev.hpp), shared
// with the batched path.
using dev::kval32s;
using dev::kval64;


// ---------------------------------------------------- FP32 on the fly --
// Every lane evaluates its own A-fragment entries k(x_i, x_k) in FP32 (row
// point in registers, the stage's 32 points in LDS); B is transposed in LDS,
// double buffered, with the next stage (B tile and points) prefetched into
// registers while the current stage's MFMAs run.
template <int NB>
struct FlyTile {
  float v[4 * NB];  // 32 x 32*NB V tile
  float x[2];       // stage points (32 x d <= 32 x 16 floats over 256 threads)
};

template <int NB, int DT>
__device__ __forceinline__ void fly_load(FlyTile<NB>& t, const float* __restrict__ Xp, int d,
                                         const float* __restrict__ V, int64_t n, int64_t s,
                                         int64_t ld, int64_t c0, int64_t k0, int tid) {
  constexpr int NT = 32 * NB;
  constexpr int RT = 4 * NB;  // consecutive k rows per thread (32 rows over 256 / NT threads)
  const int dd_n = DT > 0 ? DT : d;
  // load j of this thread: column c0 + tid % NT, row k0 + RT (tid / NT) + j
  const int64_t col = c0 + tid % NT;
  const int64_t kr0 = k0 + RT * (tid / NT);
  const float* p = V + kr0 * ld + col;
  if (col < s && k0 + BK <= n) {
#pragma unroll
    for (int j = 0; j < RT; ++j) t.v[j] = p[j * ld];
  } else {
#pragma unroll
    for (int j = 0; j < RT; ++j) t.v[j] = (col < s && kr0 + j < n) ? p[j * ld] : 0.f;
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int e = tid + 256 * j;
    const int kk = e / DMAX, dd = e % DMAX;
    const int64_t kr = k0 + kk;
    t.x[j] = (dd < dd_n && kr < n) ? Xp[kr * dd_n + dd] : 0.f;
  }
}

// the stage tile into LDS: V transposed (row stride AS, k contiguous), a
// thread's RT consecutive k of one column as 16-byte writes (consecutive
// lanes take consecutive columns, so a write's lanes fall in distinct banks)
template <int NB>
__device__ __forceinline__ void fly_store(const FlyTile<NB>& t, float* __restrict__ bt,
                                          float* __restrict__ xs, int tid) {
  constexpr int NT = 32 * NB;
  constexpr int RT = 4 * NB;
  constexpr int AS = BK + 4;
  float4* dst = (float4*)&bt[(tid % NT) * AS + RT * (tid / NT)];
#pragma unroll
  for (int q = 0; q < RT / 4; ++q)
    dst[q] = make_float4(t.v[4 * q], t.v[4 * q + 1], t.v[4 * q + 2], t.v[4 * q + 3]);
#pragma unroll
  for (int j = 0; j < 2; ++j) xs[tid + 256 * j] = t.x[j];
}

template <int NB, int KIND, int DT>
// (128-column tiles with d other than 2 or 3 take one wave per SIMD rather
// than spill)
__global__ __launch_bounds__(256, (NB == 4 && DT != 2 && DT != 3) ? 1 : 2) void k_mm32_fly(
    const float* __restrict__ Xp, int d, float var, const float* __restrict__ V,
    float* __restrict__ part, SK p) {
  constexpr int NT = 32 * NB;
  constexpr int AS = BK + 4;
  __shared__ __attribute__((aligned(16))) float Bt[2][NT * AS];
  __shared__ float Xs[2][BK * DMAX];
  const int dd_n = DT > 0 ? DT : d;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, lh = lane >> 5;
  const int64_t n = p.n, s = p.s;

  const WGRange wr = wg_range(p, blockIdx.x);
  int64_t u = wr.u;
  const int64_t uend = wr.uend;
  int seg = 0;
  while (u < uend) {
    const int64_t T = u / wr.Sx;
    const int l0 = (int)(u - T * wr.Sx);
    const int l1 = (int)((int64_t)wr.Sx < l0 + (uend - u) ? (int64_t)wr.Sx : l0 + (uend - u));
    const int st0 = wr.sb + l0, st1 = wr.sb + l1;
    const int rtile = (int)(T % p.rt);
    const int64_t i0 = (int64_t)rtile * BM;
    const int64_t c0 = (T / p.rt) * NT;

    f32x16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;
    float xr[DMAX];
    {
      const int64_t row = i0 + 32 * wave + li;
#pragma unroll
      for (int dd = 0; dd < DMAX; ++dd)
        if (dd < dd_n) xr[dd] = row < n ? Xp[row * dd_n + dd] : 0.f;
    }

    FlyTile<NB> tl;
    fly_load<NB, DT>(tl, Xp, d, V, n, s, p.ld, c0, (int64_t)st0 * BK, tid);
    __syncthreads();  // the previous segment is done with both buffers
    int buf = 0;
    for (int st = st0; st < st1; ++st) {
      float* bt = Bt[buf];
      float* xs = Xs[buf];
      fly_store<NB>(tl, bt, xs, tid);
      __syncthreads();
      if (st + 1 < st1) fly_load<NB, DT>(tl, Xp, d, V, n, s, p.ld, c0, (int64_t)(st + 1) * BK, tid);
      float a[16], b[NB][16];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float4* bp = (const float4*)&bt[(nb * 32 + li) * AS + lh * 16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 v = bp[q];
          b[nb][4 * q + 0] = v.x;
          b[nb][4 * q + 1] = v.y;
          b[nb][4 * q + 2] = v.z;
          b[nb][4 * q + 3] = v.w;
        }
      }
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const float* xk = &xs[(lh * 16 + t) * DMAX];
        float r2 = 0.f;
#pragma unroll
        for (int dd = 0; dd < DMAX; ++dd)
          if (dd < dd_n) {
            const float df = xr[dd] - xk[dd];
            r2 = __builtin_fmaf(df, df, r2);
          }
        a[t] = kval32s<KIND>(r2, var);
      }
#pragma unroll
      for (int t = 0; t < 16; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t], b[nb][t], acc[nb], 0, 0, 0);
      buf ^= 1;
    }

    float* dst = part + ((int64_t)blockIdx.x * p.J + seg) * (int64_t)(BM * NT);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * wave + 8 * (r >> 2) + 4 * lh + (r & 3);
        dst[row * NT + nb * 32 + li] = acc[nb][r];
      }
    ++seg;
    u += st1 - st0;
  }
}

// ------------------------------------------------- FP32 stored, pipelined --
// The stored-matrix FP32 product is an HBM stream of M: each stage's tiles
// are fetched into registers one stage ahead (the loads fly while the
// previous stage's MFMAs run) and LDS is double buffered, so a stage costs
// one barrier.  B is kept transposed in LDS (column-major, k contiguous) so
// that each lane fetches its 16 k-values of a column with four 16-byte
// reads; all fragment reads of a stage are issued before its MFMAs.
template <int NB>
struct StTile {
  float4 a[4];        // 128 x 32 A tile: 1024 float4 / 256 threads
  float b[4 * NB];    // 32 x 32*NB B tile: 1024*NB floats / 256 threads
};

template <int NB>
__device__ __forceinline__ void st_load(StTile<NB>& t, const float* __restrict__ A,
                                        const float* __restrict__ V, int64_t n, int64_t s,
                                        int64_t i0, int64_t c0, int64_t k0, int tid, bool a_vec) {
  constexpr int NT = 32 * NB;
  typedef float f32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int e = tid + 256 * j;
    const int rr = e >> 3, kq = e & 7;
    const int64_t row = i0 + rr, kc = k0 + 4 * kq;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (row < n) {
      const float* src = A + row * n + kc;
      if (a_vec && kc + 3 < n) {
        const f32x4 w = __builtin_nontemporal_load((const f32x4*)src);
        v = make_float4(w.x, w.y, w.z, w.w);
      } else {
        if (kc + 0 < n) v.x = src[0];
        if (kc + 1 < n) v.y = src[1];
        if (kc + 2 < n) v.z = src[2];
        if (kc + 3 < n) v.w = src[3];
      }
    }
    t.a[j] = v;
  }
  // B: one column per lane, consecutive lanes on consecutive columns
#pragma unroll
  for (int j = 0; j < 4 * NB; ++j) {
    const int e = tid + 256 * j;
    const int kk = e / NT, cc = e % NT;
    const int64_t kr = k0 + kk, col = c0 + cc;
    t.b[j] = (kr < n && col < s) ? V[kr * s + col] : 0.f;
  }
}

constexpr int ST_AS = BK + 4;  // row stride (floats) of the A tile and of transposed B

template <int NB>
__device__ __forceinline__ void st_store(const StTile<NB>& t, float* __restrict__ as,
                                         float* __restrict__ bt, int tid) {
  constexpr int NT = 32 * NB;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int e = tid + 256 * j;
    *(float4*)&as[(e >> 3) * ST_AS + 4 * (e & 7)] = t.a[j];
  }
#pragma unroll
  for (int j = 0; j < 4 * NB; ++j) {
    const int e = tid + 256 * j;
    bt[(e % NT) * ST_AS + e / NT] = t.b[j];
  }
}

template <int NB>
__device__ __forceinline__ void st_compute(const float* __restrict__ as,
                                           const float* __restrict__ bt, f32x16* acc, int wave,
                                           int li, int lh) {
  float a[16], b[NB][16];
  const float4* ap = (const float4*)&as[(32 * wave + li) * ST_AS + lh * 16];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 v = ap[q];
    a[4 * q + 0] = v.x;
    a[4 * q + 1] = v.y;
    a[4 * q + 2] = v.z;
    a[4 * q + 3] = v.w;
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const float4* bp = (const float4*)&bt[(nb * 32 + li) * ST_AS + lh * 16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 v = bp[q];
      b[nb][4 * q + 0] = v.x;
      b[nb][4 * q + 1] = v.y;
      b[nb][4 * q + 2] = v.z;
      b[nb][4 * q + 3] = v.w;
    }
  }
#pragma unroll
  for (int t = 0; t < 16; ++t)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t], b[nb][t], acc[nb], 0, 0, 0);
}

template <int NB>
__global__ __launch_bounds__(256, 2) void k_mm32_st(const float* __restrict__ A,
                                                    const float* __restrict__ V,
                                                    float* __restrict__ part, SK p) {
  constexpr int NT = 32 * NB;
  constexpr int AS = BK + 4;  // row stride (floats) of the A tile and of transposed B
  __shared__ __attribute__((aligned(16))) float As[2][BM * AS];
  __shared__ __attribute__((aligned(16))) float Bt[2][NT * AS];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, lh = lane >> 5;
  const int64_t n = p.n, s = p.s;
  const bool a_vec = (n & 3) == 0;

  const WGRange wr = wg_range(p, blockIdx.x);
  int64_t u = wr.u;
  const int64_t uend = wr.uend;
  int seg = 0;
  while (u < uend) {
    const int64_t T = u / wr.Sx;
    const int l0 = (int)(u - T * wr.Sx);
    const int l1 = (int)((int64_t)wr.Sx < l0 + (uend - u) ? (int64_t)wr.Sx : l0 + (uend - u));
    const int st0 = wr.sb + l0, st1 = wr.sb + l1;
    const int rtile = (int)(T % p.rt);
    const int64_t i0 = (int64_t)rtile * BM;
    const int64_t c0 = (T / p.rt) * NT;

    f32x16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;

    // two register stages in flight: tiles st+1 and st+2 load while st computes
    StTile<NB> ta, tb;
    st_load<NB>(ta, A, V, n, s, i0, c0, (int64_t)st0 * BK, tid, a_vec);
    if (st0 + 1 < st1)
      st_load<NB>(tb, A, V, n, s, i0, c0, (int64_t)(st0 + 1) * BK, tid, a_vec);
    __syncthreads();  // the previous segment's last stage is done with both buffers
    for (int st = st0; st < st1; st += 2) {
      st_store<NB>(ta, As[0], Bt[0], tid);
      __syncthreads();
      if (st + 2 < st1)
        st_load<NB>(ta, A, V, n, s, i0, c0, (int64_t)(st + 2) * BK, tid, a_vec);
      st_compute<NB>(As[0], Bt[0], acc, wave, li, lh);
      if (st + 1 >= st1) break;
      st_store<NB>(tb, As[1], Bt[1], tid);
      __syncthreads();
      if (st + 3 < st1)
        st_load<NB>(tb, A, V, n, s, i0, c0, (int64_t)(st + 3) * BK, tid, a_vec);
      st_compute<NB>(As[1], Bt[1], acc, wave, li, lh);
    }

    float* dst = part + ((int64_t)blockIdx.x * p.J + seg) * (int64_t)(BM * NT);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * wave + 8 * (r >> 2) + 4 * lh + (r & 3);
        dst[row * NT + nb * 32 + li] = acc[nb][r];
      }
    ++seg;
    u += st1 - st0;
  }
}

// ------------------------------------- FP32 stored, LD_TILED fragment tiles --
// The fragment order of LD_TILED tiles (tile_offset) lets each wave load its
// 32 rows x 32 k of a stage straight into the registers that feed
// v_mfma_f32_32x32x2f32: four 16-byte loads per lane, each one coalesced
// 1 KB block, no LDS round trip (the rows of A are private to the wave).  A
// is fetched two stages ahead.  B (a 32 x NT block of V, shared by the four
// waves) is loaded one stage ahead into registers and kept transposed in a
// double-buffered LDS tile as in k_mm32_st, one barrier per stage.  Lane half
// h supplies k = 16 h + t in MFMA step t for both operands.
template <int NB>
__global__ __launch_bounds__(256, 2) void k_mm32_tf(const float* __restrict__ A,
                                                    const float* __restrict__ V,
                                                    float* __restrict__ part, SK p) {
  constexpr int NT = 32 * NB;
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  __shared__ __attribute__((aligned(16))) float Bt[2][NT * ST_AS];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, lh = lane >> 5;
  const int64_t n = p.n, s = p.s;

  const WGRange wr = wg_range(p, blockIdx.x);
  int64_t u = wr.u;
  const int64_t uend = wr.uend;
  int seg = 0;
  while (u < uend) {
    const int64_t T = u / wr.Sx;
    const int l0 = (int)(u - T * wr.Sx);
    const int l1 = (int)((int64_t)wr.Sx < l0 + (uend - u) ? (int64_t)wr.Sx : l0 + (uend - u));
    const int st0 = wr.sb + l0, st1 = wr.sb + l1;
    const int rtile = (int)(T % p.rt);
    const int64_t c0 = (T / p.rt) * NT;
    // this wave's quarter of tile (rtile, 0); stage st is st * 4096 floats further
    const f32x4* abase = (const f32x4*)(A + (int64_t)rtile * p.S * (BM * BK) + wave * 1024) + lane;

    f32x16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;

    f32x4 aq[2][4];
    float bq[4 * NB];
    auto load_a = [&](int st, f32x4* dst) {
      const f32x4* src = abase + (int64_t)st * (BM * BK / 4);
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[q] = __builtin_nontemporal_load(src + 64 * q);
    };
    auto load_b = [&](int st) {
      const int64_t k0 = (int64_t)st * BK;
      if (k0 + BK <= n && c0 + NT <= s) {
        // the whole stage is inside V (uniform over the workgroup): no
        // per-element branches, all loads in flight together
        const float* src = V + (k0 + tid / NT) * s + c0 + tid % NT;
#pragma unroll
        for (int j = 0; j < 4 * NB; ++j) bq[j] = src[(int64_t)(256 / NT) * j * s];
        return;
      }
#pragma unroll
      for (int j = 0; j < 4 * NB; ++j) {
        const int e = tid + 256 * j;
        const int64_t kr = k0 + e / NT, col = c0 + e % NT;
        bq[j] = (kr < n && col < s) ? V[kr * s + col] : 0.f;
      }
    };
    auto store_b = [&](float* bt) {
#pragma unroll
      for (int j = 0; j < 4 * NB; ++j) {
        const int e = tid + 256 * j;
        bt[(e % NT) * ST_AS + e / NT] = bq[j];
      }
    };

    load_a(st0, aq[0]);
    if (st0 + 1 < st1) load_a(st0 + 1, aq[1]);
    load_b(st0);
    __syncthreads();  // the previous segment is done with both B buffers
    store_b(Bt[0]);
    if (st0 + 1 < st1) load_b(st0 + 1);
    __syncthreads();
    for (int st = st0; st < st1; st += 2) {
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const int cur = st + d;
        if (cur < st1) {
          const float* bt = Bt[(cur - st0) & 1];
          float b[NB][16];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const float4* bp = (const float4*)&bt[(nb * 32 + li) * ST_AS + lh * 16];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float4 v = bp[q];
              b[nb][4 * q + 0] = v.x;
              b[nb][4 * q + 1] = v.y;
              b[nb][4 * q + 2] = v.z;
              b[nb][4 * q + 3] = v.w;
            }
          }
          float a[16];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            a[4 * q + 0] = aq[d][q].x;
            a[4 * q + 1] = aq[d][q].y;
            a[4 * q + 2] = aq[d][q].z;
            a[4 * q + 3] = aq[d][q].w;
          }
          if (cur + 2 < st1) load_a(cur + 2, aq[d]);
          // stage cur + 1 into the other buffer (last read in stage cur - 1,
          // fenced by the barrier that ended it)
          if (cur + 1 < st1) store_b(Bt[(cur + 1 - st0) & 1]);
          if (cur + 2 < st1) load_b(cur + 2);
#pragma unroll
          for (int t = 0; t < 16; ++t)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
              acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t], b[nb][t], acc[nb], 0, 0, 0);
          __syncthreads();
        }
      }
    }

    float* dst = part + ((int64_t)blockIdx.x * p.J + seg) * (int64_t)(BM * NT);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * wave + 8 * (r >> 2) + 4 * lh + (r & 3);
        dst[row * NT + nb * 32 + li] = acc[nb][r];
      }
    ++seg;
    u += st1 - st0;
  }
}

// ------------------------------------------------- split-BF16 on the fly --
// Precision form of the on-the-fly product: each FP32 kernel value and each
// FP32 entry of V is split into bf16 hi + lo parts and the product takes the
// three significant terms hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16
// with FP32 accumulation (relative error of a term about 2^-16 instead of the
// 2^-8 of one BF16 rounding, which would perturb M by far more than the
// noise variance).  Kernel values and distances are computed in FP32 by the
// lane that feeds them to the matrix core.  Stage = 64 k (4 MFMA k-steps of
// 16); in k-step q lane half h supplies k = 16 q + 8 h + j, j = 0..7, for both
// operands.  B (hi and lo) is kept transposed in LDS, double buffered, with
// the next stage prefetched into registers.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int BK16 = 64;

// x -> bf16 hi + bf16 lo (round to nearest both times) for a pair of values,
// packed two per 32-bit word (element 0 in the low half)
__device__ __forceinline__ void split2(float x0, float x1, uint32_t& hi, uint32_t& lo) {
  const f32x2 v = {x0, x1};
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
  const float h0 = __builtin_bit_cast(float, hi << 16);
  const float h1 = __builtin_bit_cast(float, hi & 0xffff0000u);
  const f32x2 r = {x0 - h0, x1 - h1};
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2));
}
constexpr int BS16 = BK16 + 8;  // bf16 row stride of transposed B (144 bytes)

template <int NB>
struct F16Tile {
  float v[8 * NB];  // 64 x 32*NB V tile: NB runs of 8 consecutive k of one column
  float x[4];       // stage points (64 x d <= 64 x 16 floats over 256 threads)
};

template <int NB, int DT>
__device__ __forceinline__ void f16_load(F16Tile<NB>& t, const float* __restrict__ Xp, int d,
                                         const float* __restrict__ V, int64_t n, int64_t s,
                                         int64_t ld, int64_t c0, int64_t k0, int tid) {
  constexpr int NT = 32 * NB;
  constexpr int G = 256 / NT;  // threads per column
  const int dd_n = DT > 0 ? DT : d;
  // run h of this thread: column c0 + tid % NT, rows k0 + 8 (tid / NT + G h) + r, r < 8
  const int64_t col = c0 + tid % NT;
  const int64_t kr0 = k0 + 8 * (tid / NT);
  const float* p = V + kr0 * ld + col;
  if (col < s && k0 + BK16 <= n) {
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
      for (int r = 0; r < 8; ++r) t.v[8 * h + r] = p[(8 * G * h + r) * ld];
  } else {
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t kr = kr0 + 8 * G * h + r;
        t.v[8 * h + r] = (col < s && kr < n) ? p[(8 * G * h + r) * ld] : 0.f;
      }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int e = tid + 256 * j;
    const int kk = e / DMAX, dd = e % DMAX;
    const int64_t kr = k0 + kk;
    t.x[j] = (dd < dd_n && kr < n) ? Xp[kr * dd_n + dd] : 0.f;
  }
}

// a run of 8 consecutive k split into planes and written as one 16-byte word
// per plane (consecutive lanes take consecutive columns)
__device__ __forceinline__ void split_store8(const float* v, __bf16* __restrict__ bh,
                                             __bf16* __restrict__ bl) {
  u32x4 hw, lw;
#pragma unroll
  for (int jp = 0; jp < 4; ++jp) {
    uint32_t h, l;
    split2(v[2 * jp], v[2 * jp + 1], h, l);
    hw[jp] = h;
    lw[jp] = l;
  }
  *(u32x4*)bh = hw;
  *(u32x4*)bl = lw;
}

template <int NB>
__device__ __forceinline__ void f16_store(const F16Tile<NB>& t, __bf16* __restrict__ bh,
                                          __bf16* __restrict__ bl, float* __restrict__ xs,
                                          int tid) {
  constexpr int NT = 32 * NB;
  constexpr int G = 256 / NT;
  const int cc = tid % NT;
#pragma unroll
  for (int h = 0; h < NB; ++h) {
    const int off = cc * BS16 + 8 * (tid / NT + G * h);
    split_store8(&t.v[8 * h], &bh[off], &bl[off]);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) xs[tid + 256 * j] = t.x[j];
}

template <int NB, int KIND, int DT>
__device__ __forceinline__ void f16_compute(const __bf16* __restrict__ bh,
                                            const __bf16* __restrict__ bl,
                                            const float* __restrict__ xs, const float* xr, int d,
                                            float var, f32x16* acc, int li, int lh) {
  const int dd_n = DT > 0 ? DT : d;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float kv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float* xk = &xs[(16 * q + 8 * lh + j) * DMAX];
      float r2 = 0.f;
#pragma unroll
      for (int dd = 0; dd < DMAX; ++dd)
        if (dd < dd_n) {
          const float df = xr[dd] - xk[dd];
          r2 = __builtin_fmaf(df, df, r2);
        }
      kv[j] = kval32s<KIND>(r2, var);
    }
    u32x4 hw, lw;
#pragma unroll
    for (int jp = 0; jp < 4; ++jp) {
      uint32_t h, l;
      split2(kv[2 * jp], kv[2 * jp + 1], h, l);
      hw[jp] = h;
      lw[jp] = l;
    }
    const bf16x8 ah = __builtin_bit_cast(bf16x8, hw);
    const bf16x8 al = __builtin_bit_cast(bf16x8, lw);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int off = (nb * 32 + li) * BS16 + 16 * q + 8 * lh;
      const bf16x8 bhv = *(const bf16x8*)&bh[off];
      const bf16x8 blv = *(const bf16x8*)&bl[off];
      acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bhv, acc[nb], 0, 0, 0);
      acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, blv, acc[nb], 0, 0, 0);
      acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bhv, acc[nb], 0, 0, 0);
    }
  }
}

// Precision form from a stored FP32 matrix (LD_TILED fragment tiles, the
// same buffer as the FP32 path): each FP32 entry m is split in registers
// into three BF16 parts h = bf16(m), c = bf16(m - h), l = bf16(m - h - c),
// whose sum is m exactly (each rounding leaves at most 8 significant bits
// for the next part); each FP32 entry v of V into bf16 hi + lo (2^-17
// relative).  The product takes h*hi + h*lo + c*hi + l*hi on BF16 matrix
// cores with FP32 accumulation: against the high part of V the stored
// operator enters exactly as its FP32 values; what is dropped (V's bits
// below 2^-16 of each entry, and c*lo, l*lo, about 2^-16 and 2^-24 of each
// term) depends on V and changes from one product to the next, like the
// rounding of V itself, rather than perturbing the operator.  The four BF16
// matrix-core steps per 16 k take a quarter of the FP32 matrix-core time of
// k_mm32_tf; the splitting work on the vector ALUs is what remains.
// A arrives straight into registers as in k_mm32_tf (lane half h holds
// k = 16 h + t, t < 16, of its row); in BF16 k-step q lane half h supplies
// k = 16 h + 8 q + j (j < 8) for both operands.  B is split by the loader
// into hi and lo planes, kept transposed (k contiguous) and double buffered
// in LDS.
constexpr int S16 = BK + 8;  // bf16 row stride of transposed B (80 bytes)

// x -> three bf16 parts (a pair at a time, packed two per word)
__device__ __forceinline__ void split3(float x0, float x1, uint32_t& h, uint32_t& c, uint32_t& l) {
  const f32x2 v = {x0, x1};
  h = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
  const f32x2 r = {x0 - __builtin_bit_cast(float, h << 16),
                   x1 - __builtin_bit_cast(float, h & 0xffff0000u)};
  c = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2));
  const f32x2 q = {r.x - __builtin_bit_cast(float, c << 16),
                   r.y - __builtin_bit_cast(float, c & 0xffff0000u)};
  l = __builtin_bit_cast(uint32_t, __builtin_convertvector(q, bf16x2));
}

template <int NB>
__global__ __launch_bounds__(256, 2) void k_mm16_tf(const float* __restrict__ A,
                                                    const float* __restrict__ V,
                                                    float* __restrict__ part, SK p) {
  constexpr int NT = 32 * NB;
  constexpr int BP = 2 * NB;  // pairs of V values per thread per stage (32 x NT / 512)
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][NT * S16];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][NT * S16];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, lh = lane >> 5;
  const int64_t n = p.n, s = p.s;

  const WGRange wr = wg_range(p, blockIdx.x);
  int64_t u = wr.u;
  const int64_t uend = wr.uend;
  int seg = 0;
  while (u < uend) {
    const int64_t T = u / wr.Sx;
    const int l0 = (int)(u - T * wr.Sx);
    const int l1 = (int)((int64_t)wr.Sx < l0 + (uend - u) ? (int64_t)wr.Sx : l0 + (uend - u));
    const int st0 = wr.sb + l0, st1 = wr.sb + l1;
    const int rtile = (int)(T % p.rt);
    const int64_t c0 = (T / p.rt) * NT;
    // this wave's quarter of tile (rtile, 0); stage st is st * 4096 floats further
    const f32x4* abase = (const f32x4*)(A + (int64_t)rtile * p.S * (BM * BK) + wave * 1024) + lane;

    f32x16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;

    // the same load schedule as k_mm32_tf: identical loads on every path, B
    // issued before A, two stages of A in flight
    const int last = st1 - 1;
    auto clampst = [&](int st) { return st < last ? st : last; };
    f32x4 aq[2][4];
    float bq[2 * BP];  // pairs (k, k + 1) of one column
    auto load_a = [&](int st, f32x4* dst) {
      const f32x4* src = abase + (int64_t)st * (BM * BK / 4);
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[q] = __builtin_nontemporal_load(src + 64 * q);
    };
    // thread column c0 + tid % NT, 2 BP consecutive rows from 2 BP (tid / NT);
    // clamped addresses, masked in store_b (both paths issue the same loads;
    // a stage inside V, uniform over the workgroup, needs no clamping or
    // masking); the planes are stored as one 8- or 16-byte write per thread
    // whose lanes fall in distinct banks
    auto inside = [&](int st) { return (int64_t)st * BK + BK <= n && c0 + NT <= s; };
    auto load_b = [&](int st) {
      const int64_t k0 = (int64_t)st * BK + 2 * BP * (tid / NT);
      const int64_t col = c0 + tid % NT;
      if (inside(st)) {
        const float* src = V + k0 * s + col;
#pragma unroll
        for (int j = 0; j < 2 * BP; ++j) bq[j] = src[(int64_t)j * s];
        return;
      }
      const int64_t cl = col < s ? col : s - 1;
#pragma unroll
      for (int j = 0; j < 2 * BP; ++j) {
        const int64_t r = k0 + j < n ? k0 + j : n - 1;
        bq[j] = V[r * s + cl];
      }
    };
    auto store_b = [&](__bf16* bh, __bf16* bl, int st) {
      const int64_t k0 = (int64_t)st * BK + 2 * BP * (tid / NT);
      const bool full = inside(st);
      const bool cv = c0 + tid % NT < s;
      uint32_t hw[BP], lw[BP];
#pragma unroll
      for (int j = 0; j < BP; ++j) {
        float v0 = bq[2 * j], v1 = bq[2 * j + 1];
        if (!full) {
          v0 *= (cv && k0 + 2 * j < n) ? 1.f : 0.f;
          v1 *= (cv && k0 + 2 * j + 1 < n) ? 1.f : 0.f;
        }
        split2(v0, v1, hw[j], lw[j]);
      }
      const int off = (tid % NT) * S16 + 2 * BP * (tid / NT);
      if constexpr (BP == 4) {
        *(u32x4*)&bh[off] = u32x4{hw[0], hw[1], hw[2], hw[3]};
        *(u32x4*)&bl[off] = u32x4{lw[0], lw[1], lw[2], lw[3]};
      } else {
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        *(u32x2*)&bh[off] = u32x2{hw[0], hw[1]};
        *(u32x2*)&bl[off] = u32x2{lw[0], lw[1]};
      }
    };
    auto stage = [&](int cur, auto dc) {
      constexpr int D = decltype(dc)::value;
      const int buf = (cur - st0) & 1;
      // the three parts of this lane's 16 A values (k = 16 lh + t)
      u32x4 ah[2], ac[2], al[2];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t h0, c0w, l0w, h1, c1w, l1w;
        split3(aq[D][q].x, aq[D][q].y, h0, c0w, l0w);
        split3(aq[D][q].z, aq[D][q].w, h1, c1w, l1w);
        const int w = 2 * (q & 1);
        ah[q >> 1][w] = h0;
        ac[q >> 1][w] = c0w;
        al[q >> 1][w] = l0w;
        ah[q >> 1][w + 1] = h1;
        ac[q >> 1][w + 1] = c1w;
        al[q >> 1][w + 1] = l1w;
      }
      // stage cur + 1 into the other buffer (last read in stage cur - 1,
      // fenced by the barrier that ended it; past the end it is not read)
      store_b(Bh[buf ^ 1], Bl[buf ^ 1], cur + 1);
      load_b(clampst(cur + 2));
      // keep B's loads ahead of A's (the scheduler would interleave them)
      __builtin_amdgcn_sched_barrier(0);
      load_a(clampst(cur + 2), aq[D]);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const bf16x8 a_h = __builtin_bit_cast(bf16x8, ah[q]);
        const bf16x8 a_c = __builtin_bit_cast(bf16x8, ac[q]);
        const bf16x8 a_l = __builtin_bit_cast(bf16x8, al[q]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int boff = (nb * 32 + li) * S16 + 16 * lh + 8 * q;
          const bf16x8 b_h = *(const bf16x8*)&Bh[buf][boff];
          const bf16x8 b_l = *(const bf16x8*)&Bl[buf][boff];
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, b_h, acc[nb], 0, 0, 0);
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_h, b_l, acc[nb], 0, 0, 0);
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_c, b_h, acc[nb], 0, 0, 0);
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_l, b_h, acc[nb], 0, 0, 0);
        }
      }
      __syncthreads();
    };

    load_b(st0);
    load_a(st0, aq[0]);
    __syncthreads();  // the previous segment is done with both B buffers
    store_b(Bh[0], Bl[0], st0);
    load_b(clampst(st0 + 1));
    load_a(clampst(st0 + 1), aq[1]);
    __syncthreads();
    int st = st0;
    for (; st + 1 < st1; st += 2) {
      stage(st, std::integral_constant<int, 0>{});
      stage(st + 1, std::integral_constant<int, 1>{});
    }
    if (st < st1) stage(st, std::integral_constant<int, 0>{});

    float* dst = part + ((int64_t)blockIdx.x * p.J + seg) * (int64_t)(BM * NT);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * wave + 8 * (r >> 2) + 4 * lh + (r & 3);
        dst[row * NT + nb * 32 + li] = acc[nb][r];
      }
    ++seg;
    u += st1 - st0;
  }
}

template <int NB, int KIND, int DT>
// 128-column tiles (NB = 4) need more than the 256 registers of two waves per
// SIMD here, so they run one wave per SIMD rather than spill
__global__ __launch_bounds__(256, NB == 4 ? 1 : 2) void k_mm16(const float* __restrict__ Xp, int d, float var,
                                                 const float* __restrict__ V,
                                                 float* __restrict__ part, SK p) {
  constexpr int NT = 32 * NB;
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][NT * BS16];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][NT * BS16];
  __shared__ float Xs[2][BK16 * DMAX];
  const int dd_n = DT > 0 ? DT : d;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, lh = lane >> 5;
  const int64_t n = p.n, s = p.s;

  const WGRange wr = wg_range(p, blockIdx.x);
  int64_t u = wr.u;
  const int64_t uend = wr.uend;
  int seg = 0;
  while (u < uend) {
    const int64_t T = u / wr.Sx;
    const int l0 = (int)(u - T * wr.Sx);
    const int l1 = (int)((int64_t)wr.Sx < l0 + (uend - u) ? (int64_t)wr.Sx : l0 + (uend - u));
    const int st0 = wr.sb + l0, st1 = wr.sb + l1;
    const int rtile = (int)(T % p.rt);
    const int64_t i0 = (int64_t)rtile * BM;
    const int64_t c0 = (T / p.rt) * NT;

    f32x16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;
    float xr[DMAX];
    {
      const int64_t row = i0 + 32 * wave + li;
#pragma unroll
      for (int dd = 0; dd < DMAX; ++dd)
        if (dd < dd_n) xr[dd] = row < n ? Xp[row * dd_n + dd] : 0.f;
    }

    F16Tile<NB> tl;
    f16_load<NB, DT>(tl, Xp, d, V, n, s, p.ld, c0, (int64_t)st0 * BK16, tid);
    __syncthreads();  // the previous segment is done with both buffers
    int buf = 0;
    for (int st = st0; st < st1; ++st) {
      f16_store<NB>(tl, Bh[buf], Bl[buf], Xs[buf], tid);
      __syncthreads();
      if (st + 1 < st1) f16_load<NB, DT>(tl, Xp, d, V, n, s, p.ld, c0, (int64_t)(st + 1) * BK16, tid);
      f16_compute<NB, KIND, DT>(Bh[buf], Bl[buf], Xs[buf], xr, d, var, acc, li, lh);
      buf ^= 1;
    }

    float* dst = part + ((int64_t)blockIdx.x * p.J + seg) * (int64_t)(BM * NT);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * wave + 8 * (r >> 2) + 4 * lh + (r & 3);
        dst[row * NT + nb * 32 + li] = acc[nb][r];
      }
    ++seg;
    u += st1 - st0;
  }
}

// ------------------------------------------------------------ FP64 path --
template <int NB, bool FLY, int KIND, int DT>
__global__ __launch_bounds__(256, 2) void k_mm64(const double* __restrict__ A,
                                                 const double* __restrict__ Xp, int d, double var,
                                                 double c, const double* __restrict__ V,
                                                 double* __restrict__ part, SK p) {
  constexpr int NT = 16 * NB;
  constexpr int BS = NT + 2;
  constexpr int AS = BK + 2;
  __shared__ __attribute__((aligned(16))) double As[FLY ? 2 : BM * AS];
  __shared__ double Bs[BK * BS];
  __shared__ double Xs[FLY ? BK * DMAX : 1];
  const int dd_n = DT > 0 ? DT : d;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lj = lane & 15, lh = lane >> 4;  // lh in 0..3
  const int64_t n = p.n, s = p.s;

  const WGRange wr = wg_range(p, blockIdx.x);
  int64_t u = wr.u;
  const int64_t uend = wr.uend;
  int seg = 0;
  while (u < uend) {
    const int64_t T = u / wr.Sx;
    const int l0 = (int)(u - T * wr.Sx);
    const int l1 = (int)((int64_t)wr.Sx < l0 + (uend - u) ? (int64_t)wr.Sx : l0 + (uend - u));
    const int st0 = wr.sb + l0, st1 = wr.sb + l1;
    const int rtile = (int)(T % p.rt);
    const int64_t ctile = T / p.rt;
    const int64_t i0 = (int64_t)rtile * BM;
    const int64_t c0 = ctile * NT;

    f64x4 acc[2][NB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[rb][nb][r] = 0.0;

    double xr[2][FLY ? DMAX : 1];
    if (FLY) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const int64_t row = i0 + 32 * wave + 16 * rb + lj;
#pragma unroll
        for (int dd = 0; dd < DMAX; ++dd)
          if (dd < dd_n) xr[rb][dd] = row < n ? Xp[row * dd_n + dd] : 0.0;
      }
    }

    for (int st = st0; st < st1; ++st) {
      const int64_t k0 = (int64_t)st * BK;
      __syncthreads();
      for (int e = tid; e < BK * NT; e += 256) {
        const int kk = e / NT, cc = e - kk * NT;
        const int64_t kr = k0 + kk, col = c0 + cc;
        Bs[kk * BS + cc] = (kr < n && col < s) ? V[kr * s + col] : 0.0;
      }
      if (FLY) {
        for (int e = tid; e < BK * dd_n; e += 256) {
          const int kk = e / dd_n, dd = e - kk * dd_n;
          const int64_t kr = k0 + kk;
          Xs[kk * DMAX + dd] = kr < n ? Xp[kr * dd_n + dd] : 0.0;
        }
      } else {
        const bool vec_ok = (n & 1) == 0;
        for (int e = tid; e < BM * (BK / 2); e += 256) {
          const int rr = e / (BK / 2), kq = e - rr * (BK / 2);
          const int64_t row = i0 + rr, kc = k0 + 2 * kq;
          double2 v = make_double2(0.0, 0.0);
          if (row < n) {
            const double* src = A + row * n + kc;
            if (vec_ok && kc + 1 < n) {
              v = *(const double2*)src;
            } else {
              if (kc + 0 < n) v.x = src[0];
              if (kc + 1 < n) v.y = src[1];
            }
          }
          *(double2*)&As[rr * AS + 2 * kq] = v;
        }
      }
      __syncthreads();

      double a[2][8];
      if (FLY) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const double* xk = &Xs[(lh * 8 + t) * DMAX];
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) {
            double r2 = 0.0;
#pragma unroll
            for (int dd = 0; dd < DMAX; ++dd)
              if (dd < dd_n) {
                const double df = xr[rb][dd] - xk[dd];
                r2 = fma(df, df, r2);
              }
            a[rb][t] = kval64<KIND>(r2, var, c);
          }
        }
      } else {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
          const double2* ap = (const double2*)&As[(32 * wave + 16 * rb + lj) * AS + lh * 8];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double2 v = ap[q];
            a[rb][2 * q + 0] = v.x;
            a[rb][2 * q + 1] = v.y;
          }
        }
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const double* brow = &Bs[(lh * 8 + t) * BS + lj];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const double b = brow[nb * 16];
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
            acc[rb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb][t], b, acc[rb][nb], 0, 0, 0);
        }
      }
    }

    double* dst = part + ((int64_t)blockIdx.x * p.J + seg) * (int64_t)(BM * NT);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 32 * wave + 16 * rb + lh + 4 * r;  // f64 16x16 output: row = lane/16 + 4 reg
          dst[row * NT + nb * 16 + lj] = acc[rb][nb][r];
        }
    ++seg;
    u += st1 - st0;
  }
}

// ------------------------------------- FP64 stored, LD_TILED fragment tiles --
// The FP64 form of k_mm32_tf on v_mfma_f64_16x16x4f64.  tile_offset64 orders
// each tile so that a wave's 32 rows x 32 k of a stage (8 KB) arrive as eight
// 16-byte loads per lane, each one coalesced 1 KB block, straight into the
// registers that feed the matrix core: 16-byte pair q holds rows 16 (q / 4) +
// lane % 16 and k = 8 (lane / 16) + 2 (q % 4) + {0, 1}.  A is fetched two
// stages ahead; after the first (second) half of a stage's MFMA steps the
// pairs that half consumed are reloaded for the stage two ahead.  B (a
// 32 x NT block of V shared by the four waves) is loaded one stage ahead into
// registers and kept transposed in a double-buffered LDS tile, one barrier
// per stage.  In MFMA step t lane quarter h supplies k = 8 h + t for both
// operands.
constexpr int ST64 = BK + 2;  // row stride (doubles) of transposed B

template <int NB>
__global__ __launch_bounds__(256, 2) void k_mm64_tf(const double* __restrict__ A,
                                                    const double* __restrict__ V,
                                                    double* __restrict__ part, SK p) {
  constexpr int NT = 16 * NB;
  constexpr int BL = 2 * NB;  // B values per thread per stage (32 x NT / 256)
  typedef double f64x2 __attribute__((ext_vector_type(2)));
  __shared__ __attribute__((aligned(16))) double Bt[2][NT * ST64];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lj = lane & 15, lh = lane >> 4;
  const int64_t n = p.n, s = p.s;

  const WGRange wr = wg_range(p, blockIdx.x);
  int64_t u = wr.u;
  const int64_t uend = wr.uend;
  int seg = 0;
  while (u < uend) {
    const int64_t T = u / wr.Sx;
    const int l0 = (int)(u - T * wr.Sx);
    const int l1 = (int)((int64_t)wr.Sx < l0 + (uend - u) ? (int64_t)wr.Sx : l0 + (uend - u));
    const int st0 = wr.sb + l0, st1 = wr.sb + l1;
    const int rtile = (int)(T % p.rt);
    const int64_t c0 = (T / p.rt) * NT;
    // this wave's slice of tile (rtile, 0); stage st is st * 4096 doubles further
    const f64x2* abase =
        (const f64x2*)(A + (int64_t)rtile * p.S * (BM * BK) + wave * 1024) + lane;

    f64x4 acc[2][NB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[rb][nb][r] = 0.0;

    f64x2 aq[2][8];
    double bq[BL];
    // pairs q of stage st for MFMA half h: q = 4 rb + 2 h + {0, 1}
    auto load_a_half = [&](int st, f64x2* dst, int h) {
      const f64x2* src = abase + (int64_t)st * (BM * BK / 2);
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int q = 4 * rb + 2 * h + e;
          dst[q] = __builtin_nontemporal_load(src + 64 * q);
        }
    };
    // B: thread column tid % NT, BL consecutive k from BL (tid / NT), so that
    // the transposed store is BL / 2 16-byte writes whose lanes fall in
    // distinct banks
    auto load_b = [&](int st) {
      const int64_t k0 = (int64_t)st * BK + BL * (tid / NT);
      const int64_t col = c0 + tid % NT;
      const double* src = V + k0 * s + col;
      if ((int64_t)st * BK + BK <= n && c0 + NT <= s) {
        // the whole stage is inside V (uniform over the workgroup)
#pragma unroll
        for (int j = 0; j < BL; ++j) bq[j] = src[(int64_t)j * s];
        return;
      }
#pragma unroll
      for (int j = 0; j < BL; ++j) bq[j] = (k0 + j < n && col < s) ? src[(int64_t)j * s] : 0.0;
    };
    auto store_b = [&](double* bt) {
      f64x2* dst = (f64x2*)&bt[(tid % NT) * ST64 + BL * (tid / NT)];
#pragma unroll
      for (int j = 0; j < BL / 2; ++j) dst[j] = f64x2{bq[2 * j], bq[2 * j + 1]};
    };

    load_a_half(st0, aq[0], 0);
    load_a_half(st0, aq[0], 1);
    if (st0 + 1 < st1) {
      load_a_half(st0 + 1, aq[1], 0);
      load_a_half(st0 + 1, aq[1], 1);
    }
    load_b(st0);
    __syncthreads();  // the previous segment is done with both B buffers
    store_b(Bt[0]);
    if (st0 + 1 < st1) load_b(st0 + 1);
    __syncthreads();
    for (int st = st0; st < st1; st += 2) {
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const int cur = st + d;
        if (cur < st1) {
          const double* bt = Bt[(cur - st0) & 1];
          // stage cur + 1 into the other buffer (last read in stage cur - 1,
          // fenced by the barrier that ended it)
          if (cur + 1 < st1) store_b(Bt[(cur + 1 - st0) & 1]);
          if (cur + 2 < st1) load_b(cur + 2);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            double b[NB][4];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
              const f64x2* bp = (const f64x2*)&bt[(nb * 16 + lj) * ST64 + lh * 8 + 4 * h];
              const f64x2 v0 = bp[0], v1 = bp[1];
              b[nb][0] = v0.x;
              b[nb][1] = v0.y;
              b[nb][2] = v1.x;
              b[nb][3] = v1.y;
            }
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
              const int t = 4 * h + tt;
#pragma unroll
              for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int rb = 0; rb < 2; ++rb) {
                  const f64x2 av = aq[d][4 * rb + (t >> 1)];
                  acc[rb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64((t & 1) ? av.y : av.x,
                                                                      b[nb][tt], acc[rb][nb], 0,
                                                                      0, 0);
                }
            }
            if (cur + 2 < st1) load_a_half(cur + 2, aq[d], h);
          }
          __syncthreads();
        }
      }
    }

    double* dst = part + ((int64_t)blockIdx.x * p.J + seg) * (int64_t)(BM * NT);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 32 * wave + 16 * rb + lh + 4 * r;
          dst[row * NT + nb * 16 + lj] = acc[rb][nb][r];
        }
    ++seg;
    u += st1 - st0;
  }
}

// --------------------------------------------------------------- epilogue --
// gridDim.y workgroups per output tile (epi_split: 4 or 8, up to 16 for small
// grids), one per row slice (blockIdx.y): Y = sum of the tile's partial slots
// in slot order (+ noise * V on the fly) (+ alpha2 * X2); optional
// dots[split rtile + slice][c].  Each thread keeps up to eight elements, so
// a slot's loads are issued together.
template <typename T>
__global__ __launch_bounds__(256) void k_epilogue(const T* __restrict__ part, SK p, int NT,
                                                  T* __restrict__ Y, const T* __restrict__ V,
                                                  double noise, const T* __restrict__ X2,
                                                  double alpha2, double* __restrict__ dots) {
  __shared__ double red[256];
  __shared__ int64_t slot[kMaxContrib];
  __shared__ int nslot;
  const int tid = threadIdx.x;
  const int64_t Tt = blockIdx.x;
  const int quarter = blockIdx.y;  // row slice of the tile (gridDim.y slices)
  const int split = gridDim.y;
  const int rtile = (int)(Tt % p.rt);
  const int64_t c0 = (Tt / p.rt) * NT;
  const int64_t i0 = (int64_t)rtile * BM;
  if (tid == 0) {
    // for every k chunk, the workgroups whose unit range intersects the tile
    int cnt = 0;
    const int Gx = p.G / p.nx;
    for (int x = 0; x < p.nx; ++x) {
      const WGRange w0 = wg_range(p, x);
      const int Sx = w0.Sx;
      if (Sx == 0) continue;
      const int64_t Ux = p.tiles * Sx;
      const int64_t ub = Tt * Sx, ue = ub + Sx;
      int lg = (int)((ub * Gx) / Ux);
      if (lg >= Gx) lg = Gx - 1;
      while (lg > 0 && (Ux * lg) / Gx > ub) --lg;
      while (lg + 1 < Gx && (Ux * (lg + 1)) / Gx <= ub) ++lg;
      for (; lg < Gx && cnt < kMaxContrib; ++lg) {
        const int64_t b0 = (Ux * lg) / Gx, b1 = (Ux * (lg + 1)) / Gx;
        if (b0 >= ue) break;
        if (b1 <= b0) continue;
        const int64_t g = (int64_t)lg * p.nx + x;
        slot[cnt++] = (g * p.J + (Tt - b0 / Sx)) * (int64_t)(BM * NT);
      }
    }
    nslot = cnt;
  }
  __syncthreads();
  const int ns = nslot;
  const int col = tid % NT;  // 256 is a multiple of NT
  const int cnt = (BM / split) * NT;  // elements of the slice (<= 8 per thread: epi_split)
  const int e0 = quarter * cnt;
  double sum[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) sum[j] = 0.0;
  // four slots' loads in flight at a time (the partial tiles were written by
  // other XCDs, so each load goes past this XCD's L2); added in slot order
  int q = 0;
  for (; q + 4 <= ns; q += 4) {
    T v[4][8];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T* src = part + slot[q + u] + e0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = tid + 256 * j;
        v[u][j] = e < cnt ? src[e] : (T)0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < 8; ++j) sum[j] += (double)v[u][j];
  }
  for (; q < ns; ++q) {
    const T* src = part + slot[q] + e0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      if (e < cnt) sum[j] += (double)src[e];
    }
  }
  double dacc = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int e = tid + 256 * j;
    if (e >= cnt) continue;
    const int row = (e0 + e) / NT;
    const int64_t i = i0 + row, c = c0 + col;
    if (i < p.n && c < p.s) {
      const int64_t off = i * p.ld + c;
      double v = sum[j];
      if (noise != 0.0) v += noise * (double)V[off];
      if (X2) v += alpha2 * (double)X2[off];
      const T y = (T)v;
      Y[off] = y;
      if (dots) dacc += (double)V[off] * (double)y;
    }
  }
  if (dots) {
    red[tid] = dacc;
    __syncthreads();
    if (tid < NT) {
      double t = 0.0;
      for (int q = tid; q < 256; q += NT) t += red[q];
      const int64_t c = c0 + tid;
      if (c < p.s) dots[((int64_t)rtile * split + quarter) * p.s + c] = t;
    }
  }
}

// ------------------------------------------ on the fly, symmetric blocks --
// M is symmetric, so a fused product can generate each off-diagonal entry
// once (the split and its slot indices: sym_split.hpp).  Block (I, J) with
// J > I is used twice, Y_I += K_IJ V_J (direct: the lane-per-row A fragments
// of k_mm32_fly) and Y_J += K_IJ^T V_I (transposed); diagonal blocks are
// applied directly in full and blocks below the diagonal are skipped, so
// about half of the entries are generated.  For the transposed product the
// generated fragments go to LDS column-major and come back with one lane per
// column: it runs on 16x16x4 FP32 matrix cores, wave w taking probe columns
// 16 w .. 16 w + 15 (so a launch takes 33 to 64 columns), with V_I kept in
// LDS, column-major, for the row tile.  Per stage a wave does as much
// transposed matrix-core work as direct work.  A workgroup keeps the
// transposed sums of its current strip in registers across row tiles and
// writes them once per strip it touches; it writes the direct sum of each
// unit to the unit's own slot.
constexpr int SBK = 128;  // block edge of the symmetric split (= BM)

template <int MS>
__device__ __forceinline__ void sym_flush(f32x4 (&accT)[MS][4][2], float* __restrict__ dst,
                                          int wave, int lq, int lg) {
#pragma unroll
  for (int b = 0; b < MS; ++b)
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 32 * st + 16 * mt + 4 * lg + r;
          dst[(int64_t)b * (BM * 64) + row * 64 + 16 * wave + lq] = accT[b][st][mt][r];
          accT[b][st][mt][r] = 0.f;
        }
}

template <int KIND, int DT, int MS>
__global__ __launch_bounds__(256, 2) void k_mm32_sym(const float* __restrict__ Xp, int d,
                                                     float var, const float* __restrict__ V,
                                                     float* __restrict__ part, SY p) {
  constexpr int NB = 2, NT = 64;
  constexpr int AS = BK + 4;
  constexpr int KS = SBK + 4;  // row stride of the stage's column-major K
  __shared__ __attribute__((aligned(16))) float Bt[2][NT * AS];
  __shared__ float Xs[2][BK * DMAX];
  __shared__ __attribute__((aligned(16))) float Kt[BK * KS];
  __shared__ __attribute__((aligned(16))) float Vt[NT * KS];
  const int dd_n = DT > 0 ? DT : d;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, lh = lane >> 5;
  const int lq = lane & 15, lg = lane >> 4;
  const int64_t n = p.n, s = p.s;
  const int g = blockIdx.x;
  int64_t u = sy_start(p, g);
  const int64_t uend = sy_start(p, g + 1);
  if (u >= uend) return;
  int S = sy_strip(p, u);
  int I = (int)(u - sy_u0(p, S));
  const int Sfirst = S;

  f32x4 accT[MS][4][2];
#pragma unroll
  for (int b = 0; b < MS; ++b)
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) accT[b][st][mt][r] = 0.f;

  FlyTile<NB> tl;
  fly_load<NB, DT>(tl, Xp, d, V, n, s, p.ld, 0, (int64_t)SBK * (I > MS * S ? I : MS * S), tid);
  int buf = 0;
  while (true) {
    const int mS = MS * S;
    const int me = sy_me(p, S);
    const int64_t i0 = (int64_t)SBK * I;
    int Sn = S, In = I + 1;
    if (In >= me) {
      Sn = S + 1;
      In = 0;
    }
    // first column of the next unit (its stage is prefetched by this one's last)
    const int64_t ncol = u + 1 < uend ? (int64_t)SBK * (In > MS * Sn ? In : MS * Sn) : -1;

    float xr[DMAX];
    {
      const int64_t row = i0 + 32 * wave + li;
#pragma unroll
      for (int dd = 0; dd < DMAX; ++dd)
        if (dd < dd_n) xr[dd] = row < n ? Xp[row * dd_n + dd] : 0.f;
    }
    // V_I, the transposed product's B operand, column-major in LDS (after
    // the previous unit's last reads of it)
    __syncthreads();
    {
      // thread: column tid % 64, rows tid / 64 + 4 j
      const int c = tid % NT;
      const int64_t r0 = i0 + tid / NT;
      const float* vp = V + r0 * p.ld + c;
      const int64_t step = 4 * p.ld;
      float* vt = &Vt[c * KS + tid / NT];
      float v[32];
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        v[j] = (c < s && r0 + 4 * j < n) ? *vp : 0.f;
        vp += step;
      }
#pragma unroll
      for (int j = 0; j < 32; ++j) vt[4 * j] = v[j];
    }
    f32x16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;

#pragma unroll
    for (int b = 0; b < MS; ++b) {
      const int J = mS + b;
      if (J < I || J >= me) continue;
      const bool sym = J > I;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int64_t col0 = (int64_t)SBK * J + BK * st;
        float* bt = Bt[buf];
        float* xs = Xs[buf];
        fly_store<NB>(tl, bt, xs, tid);
        __syncthreads();
        const int64_t nc = col0 + BK < (int64_t)SBK * me ? col0 + BK : ncol;
        if (nc >= 0) fly_load<NB, DT>(tl, Xp, d, V, n, s, p.ld, 0, nc, tid);
        float a[16], bv[NB][16];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const float4* bp = (const float4*)&bt[(nb * 32 + li) * AS + lh * 16];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float4 v = bp[q];
            bv[nb][4 * q + 0] = v.x;
            bv[nb][4 * q + 1] = v.y;
            bv[nb][4 * q + 2] = v.z;
            bv[nb][4 * q + 3] = v.w;
          }
        }
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const float* xk = &xs[(lh * 16 + t) * DMAX];
          float r2 = 0.f;
#pragma unroll
          for (int dd = 0; dd < DMAX; ++dd)
            if (dd < dd_n) {
              const float df = xr[dd] - xk[dd];
              r2 = __builtin_fmaf(df, df, r2);
            }
          a[t] = kval32s<KIND>(r2, var);
        }
#pragma unroll
        for (int t = 0; t < 16; ++t)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t], bv[nb][t], acc[nb], 0, 0, 0);
        if (sym) {
          // lane (li, lh) of wave w holds K[32 w + li][16 lh + t]: store it as
          // Kt[column][row], then read a column per lane
#pragma unroll
          for (int t = 0; t < 16; ++t) Kt[(16 * lh + t) * KS + 32 * wave + li] = a[t];
          __syncthreads();
          // A: K[32 lg + k][16 mt + lq];  B: V_I[32 lg + k][16 wave + lq]
          const float4* vp = (const float4*)&Vt[(16 * wave + lq) * KS + 32 * lg];
          const float4* kp0 = (const float4*)&Kt[lq * KS + 32 * lg];
          const float4* kp1 = (const float4*)&Kt[(16 + lq) * KS + 32 * lg];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const float4 vv = vp[q], k0 = kp0[q], k1 = kp1[q];
            f32x4 c0 = accT[b][st][0], c1 = accT[b][st][1];
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(k0.x, vv.x, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(k1.x, vv.x, c1, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(k0.y, vv.y, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(k1.y, vv.y, c1, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(k0.z, vv.z, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(k1.z, vv.z, c1, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(k0.w, vv.w, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(k1.w, vv.w, c1, 0, 0, 0);
            accT[b][st][0] = c0;
            accT[b][st][1] = c1;
          }
        }
        buf ^= 1;
      }
    }

    float* dst = part + sy_dir_slot(p, S, I) * (int64_t)(BM * NT);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * wave + 8 * (r >> 2) + 4 * lh + (r & 3);
        dst[row * NT + nb * 32 + li] = acc[nb][r];
      }
    ++u;
    if (u >= uend) break;
    if (Sn != S)
      sym_flush<MS>(accT, part + sy_tr_slot(p, g, Sfirst, S, MS * S) * (int64_t)(BM * NT), wave,
                    lq, lg);
    S = Sn;
    I = In;
  }
  sym_flush<MS>(accT, part + sy_tr_slot(p, g, Sfirst, S, MS * S) * (int64_t)(BM * NT), wave, lq,
                lg);
}

// Split-BF16 product on the fly over the symmetric split: the arithmetic of
// k_mm16 (kernel values and V split into bf16 hi + lo, hi*hi + hi*lo + lo*hi
// with FP32 accumulation) with each off-diagonal block generated once.  One
// workgroup of 8 waves per CU shares the 160 KB of LDS: per 64-column stage,
// wave (rg, ch) generates rows 32 rg .. + 31 of the row tile against stage
// columns 32 ch .. + 31 and applies them directly (32x32x16 BF16 matrix
// cores); the hi and lo planes of the generated entries go to LDS
// column-major, and wave (ts, ch) applies stage columns 32 ch .. + 31
// transposed against V_I's probe columns 16 ts .. + 15 (16x16x32 BF16 matrix
// cores), so the direct and transposed work per wave and stage are equal.
// Strips are four blocks (512 columns), so each wave keeps 64 transposed
// sums per lane; V_I (split into planes) is double buffered in LDS and the
// next row tile's is loaded while the current one's first stage runs.  The
// two column halves' direct sums of a unit are added through LDS before the
// unit's slot is written.
constexpr int kSym16MS = 4;  // blocks per strip of the split-BF16 form

struct S16Tile {
  float v[8];  // 64 x 64 V tile: 8 consecutive k of one column
  float x[2];  // stage points (64 x d <= 64 x 16 floats over 512 threads)
};

template <int DT>
__device__ __forceinline__ void s16_load(S16Tile& t, const float* __restrict__ Xp, int d,
                                         const float* __restrict__ V, int64_t n, int64_t s,
                                         int64_t ld, int64_t k0, int tid) {
  const int dd_n = DT > 0 ? DT : d;
  // column tid % 64, rows k0 + 8 (tid / 64) + r, r < 8
  const int64_t col = tid % 64;
  const int64_t kr0 = k0 + 8 * (tid / 64);
  const float* q = V + kr0 * ld + col;
  if (col < s && k0 + BK16 <= n) {
#pragma unroll
    for (int r = 0; r < 8; ++r) t.v[r] = q[r * ld];
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r) t.v[r] = (col < s && kr0 + r < n) ? q[r * ld] : 0.f;
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int e = tid + 512 * j;
    const int kk = e / DMAX, dd = e % DMAX;
    const int64_t kr = k0 + kk;
    t.x[j] = (dd < dd_n && kr < n) ? Xp[kr * dd_n + dd] : 0.f;
  }
}

template <int KIND, int DT>
__global__ __launch_bounds__(512, 1) void k_mm16_sym(const float* __restrict__ Xp, int d,
                                                     float var, const float* __restrict__ V,
                                                     float* __restrict__ part, SY p) {
  constexpr int NB = 2, NT = 64, MS = kSym16MS;
  constexpr int KS16 = SBK + 8;  // bf16 row stride of the column-major K and V_I planes
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][NT * BS16];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][NT * BS16];
  __shared__ float Xs[2][BK16 * DMAX];
  __shared__ __attribute__((aligned(16))) __bf16 Kt[2][BK16 * KS16];      // [plane][col][row]
  __shared__ __attribute__((aligned(16))) __bf16 Vt[2][2][NT * KS16];     // [buf][plane][col][row]
  float* cmb = (float*)&Kt[0][0];  // 128 x 64 direct sums of the upper column half
  const int dd_n = DT > 0 ? DT : d;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int rg = wave & 3, ch = wave >> 2;
  const int li = lane & 31, lh = lane >> 5;
  const int lq = lane & 15, lg = lane >> 4;
  const int64_t n = p.n, s = p.s;
  const int g = blockIdx.x;
  int64_t u = sy_start(p, g);
  const int64_t uend = sy_start(p, g + 1);
  if (u >= uend) return;
  int S = sy_strip(p, u);
  int I = (int)(u - sy_u0(p, S));
  const int Sfirst = S;

  // V_I of row tile I into planes: thread column tid % 64, row pairs tid / 64 + 8 j
  auto vi_load = [&](int It, float (&vr)[16]) {
    const int c = tid % 64;
    const int64_t r0 = (int64_t)SBK * It + 2 * (tid / 64);
    const float* q = V + r0 * p.ld + c;
    const int64_t step = 16 * p.ld;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t r = r0 + 16 * j;
      vr[2 * j] = (c < s && r < n) ? q[0] : 0.f;
      vr[2 * j + 1] = (c < s && r + 1 < n) ? q[p.ld] : 0.f;
      q += step;
    }
  };
  auto vi_store = [&](int vb, const float (&vr)[16]) {
    const int c = tid % 64;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int row = 2 * (tid / 64) + 16 * j;
      uint32_t h, l;
      split2(vr[2 * j], vr[2 * j + 1], h, l);
      *(uint32_t*)&Vt[vb][0][c * KS16 + row] = h;
      *(uint32_t*)&Vt[vb][1][c * KS16 + row] = l;
    }
  };

  f32x4 accT[MS][2][2];
#pragma unroll
  for (int b = 0; b < MS; ++b)
#pragma unroll
    for (int sg = 0; sg < 2; ++sg)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) accT[b][sg][mt][r] = 0.f;
  auto flushT = [&](int Sx) {
    float* dst = part + sy_tr_slot(p, g, Sfirst, Sx, MS * Sx) * (int64_t)(BM * NT);
#pragma unroll
    for (int b = 0; b < MS; ++b)
#pragma unroll
      for (int sg = 0; sg < 2; ++sg)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 64 * sg + 32 * ch + 16 * mt + 4 * lg + r;
            dst[(int64_t)b * (BM * NT) + row * NT + 16 * rg + lq] = accT[b][sg][mt][r];
            accT[b][sg][mt][r] = 0.f;
          }
  };

  int vb = 0;
  {
    float vr[16];
    vi_load(I, vr);
    vi_store(0, vr);
  }
  S16Tile tl;
  s16_load<DT>(tl, Xp, d, V, n, s, p.ld, (int64_t)SBK * (I > MS * S ? I : MS * S), tid);
  int buf = 0;
  while (true) {
    const int mS = MS * S;
    const int me = sy_me(p, S);
    const int64_t i0 = (int64_t)SBK * I;
    int Sn = S, In = I + 1;
    if (In >= me) {
      Sn = S + 1;
      In = 0;
    }
    const bool more = u + 1 < uend;
    const int64_t ncol = more ? (int64_t)SBK * (In > MS * Sn ? In : MS * Sn) : -1;
    float xr[DMAX];
    {
      const int64_t row = i0 + 32 * rg + li;
#pragma unroll
      for (int dd = 0; dd < DMAX; ++dd)
        if (dd < dd_n) xr[dd] = row < n ? Xp[row * dd_n + dd] : 0.f;
    }
    // the next row tile's V_I: loads issued now, stored after the first stage
    float vn[16];
    if (more) vi_load(In, vn);
    bool first = true;
    f32x16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;

#pragma unroll
    for (int b = 0; b < MS; ++b) {
      const int J = mS + b;
      if (J < I || J >= me) continue;
      const bool sym = J > I;
#pragma unroll
      for (int sg = 0; sg < 2; ++sg) {
        const int64_t col0 = (int64_t)SBK * J + BK16 * sg;
        {
          // stage tile: V split into planes (transposed, k contiguous), points
          const int off = (tid % 64) * BS16 + 8 * (tid / 64);
          split_store8(tl.v, &Bh[buf][off], &Bl[buf][off]);
#pragma unroll
          for (int j = 0; j < 2; ++j) Xs[buf][tid + 512 * j] = tl.x[j];
        }
        __syncthreads();
        const int64_t nc = col0 + BK16 < (int64_t)SBK * me ? col0 + BK16 : ncol;
        if (nc >= 0) s16_load<DT>(tl, Xp, d, V, n, s, p.ld, nc, tid);
        const float* xs = Xs[buf];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          // columns 32 ch + 16 q + 8 lh + j of the stage, row 32 rg + li
          const int cb = 32 * ch + 16 * q + 8 * lh;
          float kv[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const float* xk = &xs[(cb + j) * DMAX];
            float r2 = 0.f;
#pragma unroll
            for (int dd = 0; dd < DMAX; ++dd)
              if (dd < dd_n) {
                const float df = xr[dd] - xk[dd];
                r2 = __builtin_fmaf(df, df, r2);
              }
            kv[j] = kval32s<KIND>(r2, var);
          }
          u32x4 hw, lw;
#pragma unroll
          for (int jp = 0; jp < 4; ++jp) {
            uint32_t h, l;
            split2(kv[2 * jp], kv[2 * jp + 1], h, l);
            hw[jp] = h;
            lw[jp] = l;
          }
          const bf16x8 ah = __builtin_bit_cast(bf16x8, hw);
          const bf16x8 al = __builtin_bit_cast(bf16x8, lw);
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const int off = (nb * 32 + li) * BS16 + cb;
            const bf16x8 bhv = *(const bf16x8*)&Bh[buf][off];
            const bf16x8 blv = *(const bf16x8*)&Bl[buf][off];
            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bhv, acc[nb], 0, 0, 0);
            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, blv, acc[nb], 0, 0, 0);
            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bhv, acc[nb], 0, 0, 0);
          }
          if (sym) {
            // planes column-major, Kt[plane][column][row], written a word (two
            // rows) at a time: lanes 2i and 2i + 1 (rows r, r + 1) swap half
            // of their columns, the even lane then writes columns cb .. cb + 3
            // and the odd lane cb + 4 .. cb + 7
            const bool odd = li & 1;
            const int cA = cb + (odd ? 4 : 0);
            const int rE = 32 * rg + (li & ~1);
#pragma unroll
            for (int pl = 0; pl < 2; ++pl) {
              const u32x4 w = pl ? lw : hw;
              const uint32_t x0 = odd ? w[0] : w[2], x1 = odd ? w[1] : w[3];
              // swap with the neighbouring lane (DPP quad_perm 1, 0, 3, 2)
              const uint32_t y0 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x0, 0xB1, 0xF, 0xF, false);
              const uint32_t y1 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x1, 0xB1, 0xF, 0xF, false);
              const uint32_t m0 = odd ? y0 : w[0], m1 = odd ? w[2] : y0;  // rows r, r + 1
              const uint32_t m2 = odd ? y1 : w[1], m3 = odd ? w[3] : y1;
              __bf16* kt = &Kt[pl][cA * KS16 + rE];
              *(uint32_t*)&kt[0] = __builtin_amdgcn_perm(m1, m0, 0x05040100u);
              *(uint32_t*)&kt[KS16] = __builtin_amdgcn_perm(m1, m0, 0x07060302u);
              *(uint32_t*)&kt[2 * KS16] = __builtin_amdgcn_perm(m3, m2, 0x05040100u);
              *(uint32_t*)&kt[3 * KS16] = __builtin_amdgcn_perm(m3, m2, 0x07060302u);
            }
          }
        }
        if (sym) {
          __syncthreads();
          // A: K[32 k + 8 lg + j][32 ch + 16 mt + lq];  B: V_I[32 k + 8 lg + j][16 rg + lq]
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int r0 = 32 * k + 8 * lg;
            const int vo = (16 * rg + lq) * KS16 + r0;
            const bf16x8 vh = *(const bf16x8*)&Vt[vb][0][vo];
            const bf16x8 vl = *(const bf16x8*)&Vt[vb][1][vo];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
              const int ko = (32 * ch + 16 * mt + lq) * KS16 + r0;
              const bf16x8 kh = *(const bf16x8*)&Kt[0][ko];
              const bf16x8 kl = *(const bf16x8*)&Kt[1][ko];
              f32x4 c = accT[b][sg][mt];
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh, vh, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh, vl, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kl, vh, c, 0, 0, 0);
              accT[b][sg][mt] = c;
            }
          }
        }
        if (first) {
          // the next row tile's V_I goes to the other buffer (last read by the
          // unit before this one, which every wave has finished)
          if (more) vi_store(vb ^ 1, vn);
          first = false;
        }
        buf ^= 1;
      }
    }

    // direct sums: the upper column half through LDS, then one slot per unit
    __syncthreads();  // every wave is done with Kt
    if (ch == 1) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 32 * rg + 8 * (r >> 2) + 4 * lh + (r & 3);
          cmb[row * NT + nb * 32 + li] = acc[nb][r];
        }
    }
    __syncthreads();
    if (ch == 0) {
      float* dst = part + sy_dir_slot(p, S, I) * (int64_t)(BM * NT);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 32 * rg + 8 * (r >> 2) + 4 * lh + (r & 3);
          dst[row * NT + nb * 32 + li] = acc[nb][r] + cmb[row * NT + nb * 32 + li];
        }
    }
    ++u;
    if (!more) break;
    if (Sn != S) flushT(S);
    S = Sn;
    I = In;
    vb ^= 1;
  }
  flushT(S);
}

// Epilogue of the symmetric split, grid (blocks, epi_split): row tile R =
// blockIdx.x, row slice blockIdx.y; the same outputs as k_epilogue.  A
// thread keeps up to two float4 of the slice (the same four columns in
// each) and has eight slots' loads in flight; slots are added in order.
template <int MS>
__global__ __launch_bounds__(256) void k_sym_epilogue(const float* __restrict__ part, SY p,
                                                      float* __restrict__ Y,
                                                      const float* __restrict__ V, double noise,
                                                      const float* __restrict__ X2, double alpha2,
                                                      double* __restrict__ dots) {
  constexpr int NT = 64;
  constexpr int64_t TILE = BM * NT;
  constexpr int QF = 8;  // slots in flight
  __shared__ double red[4][257];
  __shared__ int64_t slot[kMaxContrib];
  __shared__ int nslot;
  const int tid = threadIdx.x;
  const int R = blockIdx.x;
  const int quarter = blockIdx.y, split = gridDim.y;
  const int SR = R / MS;
  if (tid == 0) nslot = sy_tr_list(p, R, slot, kMaxContrib);
  __syncthreads();
  const int ndir = p.ns - SR;
  const int64_t dbase = sy_dir_base(p, R);  // == sy_dir_slot(p, SR, R)
  const int ntot = ndir + (nslot < kMaxContrib ? nslot : kMaxContrib);
  const int nf = (BM / split) * NT / 4;  // float4 of the slice (<= 512)
  const int f0 = quarter * nf;
  double sum[2][4];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int c = 0; c < 4; ++c) sum[j][c] = 0.0;
  int q = 0;
  for (; q + QF <= ntot; q += QF) {
    float4 v[QF][2];
#pragma unroll
    for (int w = 0; w < QF; ++w) {
      const int qq = q + w;
      const int64_t off = (qq < ndir ? dbase + qq : slot[qq - ndir]) * TILE;
      const float4* src = (const float4*)(part + off) + f0;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int f = tid + 256 * j;
        v[w][j] = f < nf ? src[f] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int w = 0; w < QF; ++w)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        sum[j][0] += (double)v[w][j].x;
        sum[j][1] += (double)v[w][j].y;
        sum[j][2] += (double)v[w][j].z;
        sum[j][3] += (double)v[w][j].w;
      }
  }
  for (; q < ntot; ++q) {
    const int64_t off = (q < ndir ? dbase + q : slot[q - ndir]) * TILE;
    const float4* src = (const float4*)(part + off) + f0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int f = tid + 256 * j;
      if (f < nf) {
        const float4 v = src[f];
        sum[j][0] += (double)v.x;
        sum[j][1] += (double)v.y;
        sum[j][2] += (double)v.z;
        sum[j][3] += (double)v.w;
      }
    }
  }
  const int64_t i0 = (int64_t)R * BM;
  const int cb = (4 * tid) % NT;  // this thread's four columns
  double dacc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int f = tid + 256 * j;
    if (f >= nf) continue;
    const int64_t i = i0 + (4 * (f0 + f)) / NT;
    if (i >= p.n) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int col = cb + c;
      if (col >= p.s) continue;
      const int64_t off = i * p.ld + col;
      double v = sum[j][c];
      if (noise != 0.0) v += noise * (double)V[off];
      if (X2) v += alpha2 * (double)X2[off];
      const float y = (float)v;
      Y[off] = y;
      dacc[c] += (double)V[off] * (double)y;
    }
  }
  if (dots) {
#pragma unroll
    for (int c = 0; c < 4; ++c) red[c][tid] = dacc[c];
    __syncthreads();
    if (tid < NT) {
      // column tid: component tid % 4 of the threads whose column group is tid / 4
      double t = 0.0;
      for (int k = tid / 4; k < 256; k += NT / 4) t += red[tid % 4][k];
      if (tid < p.s) dots[((int64_t)R * split + quarter) * p.s + tid] = t;
    }
  }
}

// ------------------------------------------------------------ materialize --
// DM = DMAX (the fused kernels' limit) or 64 (the largest d the ABI takes)
template <typename T, int KIND, int DM>
__global__ __launch_bounds__(256) void k_materialize(const double* __restrict__ X, int64_t n, int d,
                                                     double var, double c, double noise,
                                                     T* __restrict__ M) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double xj[DM];
#pragma unroll
  for (int dd = 0; dd < DM; ++dd) xj[dd] = (dd < d && j < n) ? X[j * d + dd] : 0.0;
  for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
    if (j >= n) continue;
    double r2 = 0.0;
#pragma unroll
    for (int dd = 0; dd < DM; ++dd)
      if (dd < d) {
        const double df = X[i * d + dd] - xj[dd];
        r2 = fma(df, df, r2);
      }
    double v = kval64<KIND>(r2, var, c);
    if (i == j) v += noise;
    M[i * n + j] = (T)v;
  }
}

// LD_TILED (FP32, fragment order inside the tile: tile_offset): walk the
// storage linearly (coalesced writes), zero the padding.
template <int KIND>
__global__ __launch_bounds__(256) void k_materialize_tiled(const double* __restrict__ X, int64_t n,
                                                           int d, double var, double c,
                                                           double noise, int64_t total,
                                                           float* __restrict__ M) {
  const int64_t kt = (n + kTileCols - 1) / kTileCols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t tile = e / (kTileRows * kTileCols);
    int tr, tc;
    tile_coords((int)(e % (kTileRows * kTileCols)), &tr, &tc);
    const int64_t i = (tile / kt) * kTileRows + tr;
    const int64_t k = (tile % kt) * kTileCols + tc;
    float out = 0.f;
    if (i < n && k < n) {
      double r2 = 0.0;
      for (int dd = 0; dd < d; ++dd) {
        const double df = X[i * d + dd] - X[k * d + dd];
        r2 = fma(df, df, r2);
      }
      double v = kval64<KIND>(r2, var, c);
      if (i == k) v += noise;
      out = (float)v;
    }
    M[e] = out;
  }
}

// LD_TILED (FP64, fragment order inside the tile: tile_offset64)
template <int KIND>
__global__ __launch_bounds__(256) void k_materialize_tiled64(const double* __restrict__ X,
                                                             int64_t n, int d, double var,
                                                             double c, double noise,
                                                             int64_t total,
                                                             double* __restrict__ M) {
  const int64_t kt = (n + kTileCols - 1) / kTileCols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t tile = e / (kTileRows * kTileCols);
    int tr, tc;
    tile_coords64((int)(e % (kTileRows * kTileCols)), &tr, &tc);
    const int64_t i = (tile / kt) * kTileRows + tr;
    const int64_t k = (tile % kt) * kTileCols + tc;
    double out = 0.0;
    if (i < n && k < n) {
      double r2 = 0.0;
      for (int dd = 0; dd < d; ++dd) {
        const double df = X[i * d + dd] - X[k * d + dd];
        r2 = fma(df, df, r2);
      }
      out = kval64<KIND>(r2, var, c);
      if (i == k) out += noise;
    }
    M[e] = out;
  }
}

__global__ void k_f64_to_f32(const double* __restrict__ in, float* __restrict__ out, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
    out[i] = (float)in[i];
}
__global__ void k_f32_to_f64(const float* __restrict__ in, double* __restrict__ out, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
    out[i] = (double)in[i];
}

int grid1(int64_t count) {
  int64_t b = (count + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

// ---------------------------------------------------------------- dispatch --
struct Plan {
  int NT;
  SK p;
  size_t part_bytes;
};

// wide: the fused FP32 and split-BF16 kernels, which also take 128-column
// tiles; every kernel entry they generate then feeds twice the matrix-core
// work, so products wider than 64 columns (the range finder) regenerate M
// half as often
Plan make_plan(ld_ctx* ctx, bool f64, int64_t n, int64_t s, int bk = BK, bool wide = false) {
  Plan pl{};
  if (f64)
    pl.NT = s > 32 ? 64 : (s > 16 ? 32 : 16);
  else
    pl.NT = (wide && s > 64) ? 128 : (s > 32 ? 64 : 32);
  SK& p = pl.p;
  p.n = n;
  p.s = s;
  p.ld = s;
  p.rt = (int)((n + BM - 1) / BM);
  const int64_t ct = (s + pl.NT - 1) / pl.NT;
  p.tiles = (int64_t)p.rt * ct;
  p.S = (int)((n + bk - 1) / bk);
  const int64_t U = p.tiles * p.S;
  // one k chunk per XCD when the device has 8 (otherwise a single chunk), and
  // at least 4 stages per chunk
  int nx = (ctx->num_cu % 8 == 0) ? 8 : 1;
  while (nx > 1 && p.S < 4 * nx) nx /= 2;
  p.nx = nx;
  const int64_t gmax = (int64_t)ctx->num_cu * 2;
  const int64_t min_units = 8;
  int64_t G = (U + min_units - 1) / min_units;
  if (G > gmax) G = gmax;
  // keep every tile split over few workgroups per chunk
  if (G > p.tiles * nx * (kMaxContrib / (2 * nx) - 1)) G = p.tiles * nx * (kMaxContrib / (2 * nx) - 1);
  G = (G / nx) * nx;
  if (G < nx) G = nx;
  p.G = (int)G;
  const int64_t Sxmax = (p.S + nx - 1) / nx;
  const int64_t per = (p.tiles * Sxmax + G / nx - 1) / (G / nx);
  p.J = (int)((per + Sxmax - 1) / Sxmax + 1);
  pl.part_bytes = (size_t)p.G * p.J * BM * pl.NT * (f64 ? sizeof(double) : sizeof(float));
  return pl;
}

template <int KIND, int DT>
void launch_fly32(int NB, dim3 g, hipStream_t st, const float* X, int d, float var,
                  const float* V, float* part, const SK& p) {
  if (NB == 4)
    hipLaunchKernelGGL((k_mm32_fly<4, KIND, DT>), g, dim3(256), 0, st, X, d, var, V, part, p);
  else if (NB == 2)
    hipLaunchKernelGGL((k_mm32_fly<2, KIND, DT>), g, dim3(256), 0, st, X, d, var, V, part, p);
  else
    hipLaunchKernelGGL((k_mm32_fly<1, KIND, DT>), g, dim3(256), 0, st, X, d, var, V, part, p);
}

template <int KIND, int DT>
void launch_fly64(int NB, dim3 g, hipStream_t st, const double* X, int d, double var, double c,
                  const double* V, double* part, const SK& p) {
  if (NB == 4)
    hipLaunchKernelGGL((k_mm64<4, true, KIND, DT>), g, dim3(256), 0, st, nullptr, X, d, var, c, V,
                       part, p);
  else if (NB == 2)
    hipLaunchKernelGGL((k_mm64<2, true, KIND, DT>), g, dim3(256), 0, st, nullptr, X, d, var, c, V,
                       part, p);
  else
    hipLaunchKernelGGL((k_mm64<1, true, KIND, DT>), g, dim3(256), 0, st, nullptr, X, d, var, c, V,
                       part, p);
}

template <int KIND, int DT>
void launch_fly16(int NB, dim3 g, hipStream_t st, const float* X, int d, float var,
                  const float* V, float* part, const SK& p) {
  if (NB == 4)
    hipLaunchKernelGGL((k_mm16<4, KIND, DT>), g, dim3(256), 0, st, X, d, var, V, part, p);
  else if (NB == 2)
    hipLaunchKernelGGL((k_mm16<2, KIND, DT>), g, dim3(256), 0, st, X, d, var, V, part, p);
  else
    hipLaunchKernelGGL((k_mm16<1, KIND, DT>), g, dim3(256), 0, st, X, d, var, V, part, p);
}

template <int KIND>
void fly16_by_d(int NB, dim3 g, hipStream_t st, const float* X, int d, float var,
                const float* V, float* part, const SK& p) {
  switch (d) {
    case 2: launch_fly16<KIND, 2>(NB, g, st, X, d, var, V, part, p); break;
    case 3: launch_fly16<KIND, 3>(NB, g, st, X, d, var, V, part, p); break;
    case 8: launch_fly16<KIND, 8>(NB, g, st, X, d, var, V, part, p); break;
    default: launch_fly16<KIND, 0>(NB, g, st, X, d, var, V, part, p); break;
  }
}

template <int KIND>
void fly32_by_d(int NB, dim3 g, hipStream_t st, const float* X, int d, float var,
                const float* V, float* part, const SK& p) {
  switch (d) {
    case 2: launch_fly32<KIND, 2>(NB, g, st, X, d, var, V, part, p); break;
    case 3: launch_fly32<KIND, 3>(NB, g, st, X, d, var, V, part, p); break;
    case 8: launch_fly32<KIND, 8>(NB, g, st, X, d, var, V, part, p); break;
    default: launch_fly32<KIND, 0>(NB, g, st, X, d, var, V, part, p); break;
  }
}

template <int KIND>
void fly64_by_d(int NB, dim3 g, hipStream_t st, const double* X, int d, double var, double c,
                const double* V, double* part, const SK& p) {
  switch (d) {
    case 2: launch_fly64<KIND, 2>(NB, g, st, X, d, var, c, V, part, p); break;
    case 3: launch_fly64<KIND, 3>(NB, g, st, X, d, var, c, V, part, p); break;
    case 8: launch_fly64<KIND, 8>(NB, g, st, X, d, var, c, V, part, p); break;
    default: launch_fly64<KIND, 0>(NB, g, st, X, d, var, c, V, part, p); break;
  }
}

template <int KIND, int DT>
void launch_sym32(dim3 g, hipStream_t st, const float* X, int d, float var, const float* V,
                  float* part, const SY& p);

template <int KIND>
void sym32_by_d(dim3 g, hipStream_t st, const float* X, int d, float var, const float* V,
                float* part, const SY& p) {
  switch (d) {
    case 2: launch_sym32<KIND, 2>(g, st, X, d, var, V, part, p); break;
    case 3: launch_sym32<KIND, 3>(g, st, X, d, var, V, part, p); break;
    case 8: launch_sym32<KIND, 8>(g, st, X, d, var, V, part, p); break;
    default: launch_sym32<KIND, 0>(g, st, X, d, var, V, part, p); break;
  }
}

// ------------------------------------------------- symmetric split: plan --
constexpr int kSymMS = 2;                          // blocks per strip (256 columns)
constexpr int64_t kSymMinN = 16384;                // smaller products keep the plain split
constexpr size_t kSymMaxBytes = (size_t)32 << 30;  // partial sums of one product

template <int KIND, int DT>
void launch_sym32(dim3 g, hipStream_t st, const float* X, int d, float var, const float* V,
                  float* part, const SY& p) {
  hipLaunchKernelGGL((k_mm32_sym<KIND, DT, kSymMS>), g, dim3(256), 0, st, X, d, var, V, part, p);
}

template <int KIND, int DT>
void launch_sym16(dim3 g, hipStream_t st, const float* X, int d, float var, const float* V,
                  float* part, const SY& p) {
  hipLaunchKernelGGL((k_mm16_sym<KIND, DT>), g, dim3(512), 0, st, X, d, var, V, part, p);
}

template <int KIND>
void sym16_by_d(dim3 g, hipStream_t st, const float* X, int d, float var, const float* V,
                float* part, const SY& p) {
  switch (d) {
    case 2: launch_sym16<KIND, 2>(g, st, X, d, var, V, part, p); break;
    case 3: launch_sym16<KIND, 3>(g, st, X, d, var, V, part, p); break;
    case 8: launch_sym16<KIND, 8>(g, st, X, d, var, V, part, p); break;
    default: launch_sym16<KIND, 0>(g, st, X, d, var, V, part, p); break;
  }
}

struct SymPlan {
  SY p;
  size_t bytes;  // direct slots of every unit, then G * Jt * ms transposed slots
};

// The symmetric split of an n x s on-the-fly product, if it applies: 33..64
// columns, n >= kSymMinN, partial sums within kSymMaxBytes, and every output
// tile fed by at most kMaxContrib transposed slots.  bf16: the split-BF16
// form (strips of kSym16MS blocks, one 8-wave workgroup per CU); otherwise
// the FP32 form (strips of kSymMS blocks, two 4-wave workgroups per CU).
// Either gets fewer workgroups when one would have under four units' worth
// of blocks.
bool make_sym_plan(ld_ctx* ctx, int64_t n, int64_t s, bool bf16, SymPlan* out) {
  if (!(ctx->symmetric & (bf16 ? LD_SYM_BF16 : LD_SYM_F32)) || s <= 32 || s > 64 || n < kSymMinN)
    return false;
  struct Entry {
    SymPlan sp;
    int cu = -1;
    bool ok = false;
  };
  thread_local Entry cache[2];
  Entry& e = cache[bf16 ? 1 : 0];
  if (e.cu == ctx->num_cu && e.sp.p.n == n && e.sp.p.s == s) {
    if (e.ok) *out = e.sp;
    return e.ok;
  }
  const SY p = bf16 ? sy_plan(n, s, kSym16MS, ctx->num_cu) : sy_plan(n, s, kSymMS, ctx->num_cu * 2);
  e.sp = SymPlan{p, (size_t)(p.units + (int64_t)p.G * p.Jt * p.ms) * BM * 64 * sizeof(float)};
  e.cu = ctx->num_cu;
  e.ok = e.sp.bytes <= kSymMaxBytes && sy_max_tr_list(p) <= kMaxContrib;
  if (e.ok) *out = e.sp;
  return e.ok;
}

// ------------------------------------------------------- static scratch --
// Scratch of kernel_matmat_noalloc: a file-scope device array that every
// device the library runs on holds from the code object's load until the
// process ends.  In host code `scratch` names a host-side stand-in, not a
// device address: host code uses only the per-device address that
// static_scratch_address looks up.
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

}  // namespace

ld_status static_scratch_address(int device, void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return fail(LD_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    LD_HIP(hipGetDevice(&cur));
    if (cur != device) return fail(LD_EINVAL, "static scratch lookup: device is not current");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return fail(LD_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    addr[device] = p;
  }
  *out = addr[device];
  return LD_OK;
}

KParams make_kparams(const ld_operator& op) {
  KParams kp{};
  kp.kind = op.kind;
  kp.variance = op.variance;
  kp.noise = op.noise;
  kp.c_rbf = 1.0 / (2.0 * op.lengthscale * op.lengthscale);
  kp.c_mat = 2.23606797749978969640917366873128 / op.lengthscale;
  return kp;
}

// Products of the fused FP32 / split-BF16 kernels wider than this run as
// column panels of this width, one after another: all of a launch's column
// tiles are in flight together, so a single wide launch streams the whole of
// V (n x s) through the caches for every row block, while one panel of V
// (n x 128 x 4 bytes = 100 MB at n = 200,000) stays resident in the
// last-level cache.
constexpr int64_t kFusedPanel = 128;

size_t matmat_scratch_bytes(ld_ctx* ctx, bool f64, int64_t n, int64_t s) {
  size_t b = make_plan(ctx, f64, n, s).part_bytes;
  // column panels (products that return dot blocks run at full width)
  if (!f64 && s > kFusedPanel) b = std::max(b, matmat_scratch_bytes(ctx, f64, n, kFusedPanel) - 1024);
  if (!f64) {
    b = std::max(b, make_plan(ctx, false, n, s, BK16).part_bytes);
    b = std::max(b, make_plan(ctx, false, n, s, BK, true).part_bytes);
    b = std::max(b, make_plan(ctx, false, n, s, BK16, true).part_bytes);
    // the symmetric split, when the arena can grow for it (a caller's
    // workspace that is too small gets the plain split instead)
    SymPlan sp;
    if (!ctx->arena.external && make_sym_plan(ctx, n, s, false, &sp)) b = std::max(b, sp.bytes);
    if (!ctx->arena.external && make_sym_plan(ctx, n, s, true, &sp)) b = std::max(b, sp.bytes);
  }
  return b + 1024;
}

// the on-the-fly product over the symmetric split (FP32 or split-BF16 matrix cores)
ld_status matmat_sym(ld_ctx* ctx, const MatmatArgs& a, const SY& p, bool bf16, float* part) {
  hipStream_t st = ctx->stream;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (a.timed && ctx->timing) {
    const double nn = (double)a.n * (double)a.n;
    LD_TRY(timing_pair(ctx, &ev0, &ev1, 2.0 * nn * (double)a.s, 2.0 * (double)a.n * a.s * 4.0));
    LD_HIP(hipEventRecord(ev0, st));
  }
  const int kind = a.kp.kind;
  const float var = (float)(kind == LD_RBF ? std::log2(a.kp.variance) : a.kp.variance);
  const float* X = (const float*)a.X;
  const float* V = (const float*)a.V;
  if (bf16 && kind == LD_RBF)
    sym16_by_d<LD_RBF>(dim3(p.G), st, X, a.d, var, V, part, p);
  else if (bf16)
    sym16_by_d<LD_MATERN52>(dim3(p.G), st, X, a.d, var, V, part, p);
  else if (kind == LD_RBF)
    sym32_by_d<LD_RBF>(dim3(p.G), st, X, a.d, var, V, part, p);
  else
    sym32_by_d<LD_MATERN52>(dim3(p.G), st, X, a.d, var, V, part, p);
  if (ev1) LD_HIP(hipEventRecord(ev1, st));
  const int split = epi_split(p.nblk, 64);
  if (p.ms == kSym16MS)
    hipLaunchKernelGGL((k_sym_epilogue<kSym16MS>), dim3((unsigned)p.nblk, split), dim3(256), 0,
                       st, part, p, (float*)a.Y, V, a.kp.noise, (const float*)a.X2, a.alpha2,
                       a.dots);
  else
    hipLaunchKernelGGL((k_sym_epilogue<kSymMS>), dim3((unsigned)p.nblk, split), dim3(256), 0, st,
                       part, p, (float*)a.Y, V, a.kp.noise, (const float*)a.X2, a.alpha2,
                       a.dots);
  if (a.dot_blocks) *a.dot_blocks = p.nblk * split;
  LD_HIP(hipGetLastError());
  return LD_OK;
}

ld_status matmat(ld_ctx* ctx, bool f64, const MatmatArgs& a) {
  if (a.n <= 0 || a.s <= 0) return LD_OK;
  const bool split16 = !f64 && a.bf16 && a.A == nullptr;
  const bool fused32 = !f64 && a.A == nullptr;
  if (a.ld != 0 && a.ld != a.s && !fused32)
    return fail(LD_EINVAL, "matmat: a row stride other than s needs a fused FP32 product");
  if (fused32 && a.s > kFusedPanel && a.dots == nullptr) {
    const size_t es = sizeof(float);
    for (int64_t c = 0; c < a.s; c += kFusedPanel) {
      MatmatArgs b = a;
      b.s = std::min(kFusedPanel, a.s - c);
      b.ld = a.ld ? a.ld : a.s;
      b.V = (const char*)a.V + c * es;
      b.Y = (char*)a.Y + c * es;
      if (a.X2) b.X2 = (const char*)a.X2 + c * es;
      // each panel takes the same partial buffer: the launches are ordered
      // on the stream
      const size_t mark = ctx->arena.top;
      LD_TRY(matmat(ctx, f64, b));
      ctx->arena.top = mark;
    }
    return LD_OK;
  }
  if (fused32) {
    SymPlan sp;
    if (make_sym_plan(ctx, a.n, a.s, split16, &sp)) {
      sp.p.ld = a.ld ? a.ld : a.s;
      float* part = (float*)ctx->arena.take(sp.bytes);
      if (part) return matmat_sym(ctx, a, sp.p, split16, part);
    }
  }
  Plan pl = make_plan(ctx, f64, a.n, a.s, split16 ? BK16 : BK, fused32);
  if (a.ld) pl.p.ld = a.ld;
  void* part = ctx->arena.take(pl.part_bytes);
  if (!part) return fail(LD_ENOMEM, "matmat: scratch arena too small");
  hipStream_t st = ctx->stream;
  const bool fly = a.A == nullptr;
  const int kind = a.kp.kind;
  dim3 grid(pl.p.G);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (a.timed && ctx->timing) {
    const double nn = (double)a.n * (double)a.n;
    const double es = f64 ? 8.0 : 4.0;
    // algorithmic traffic: the stored matrix once, V read and Y written once
    const double bytes = (fly ? 0.0 : nn * es) + 2.0 * (double)a.n * a.s * es;
    LD_TRY(timing_pair(ctx, &ev0, &ev1, 2.0 * nn * (double)a.s, bytes));
    LD_HIP(hipEventRecord(ev0, st));
  }
  if (f64) {
    const int NB = pl.NT / 16;
    const double c = (kind == LD_RBF || kind == dev::kKindRbfDl) ? a.kp.c_rbf : a.kp.c_mat;
    const double* V = (const double*)a.V;
    double* P = (double*)part;
    if (fly) {
      if (kind == LD_RBF)
        fly64_by_d<LD_RBF>(NB, grid, st, (const double*)a.X, a.d, a.kp.variance, c, V, P, pl.p);
      else if (kind == dev::kKindRbfDl)
        fly64_by_d<dev::kKindRbfDl>(NB, grid, st, (const double*)a.X, a.d, a.kp.variance, c, V, P,
                                    pl.p);
      else if (kind == dev::kKindMaternDl)
        fly64_by_d<dev::kKindMaternDl>(NB, grid, st, (const double*)a.X, a.d, a.kp.variance, c, V,
                                       P, pl.p);
      else
        fly64_by_d<LD_MATERN52>(NB, grid, st, (const double*)a.X, a.d, a.kp.variance, c, V, P, pl.p);
    } else if (a.layout == LD_TILED) {
      const double* A = (const double*)a.A;
      if (NB == 4)
        hipLaunchKernelGGL((k_mm64_tf<4>), grid, dim3(256), 0, st, A, V, P, pl.p);
      else if (NB == 2)
        hipLaunchKernelGGL((k_mm64_tf<2>), grid, dim3(256), 0, st, A, V, P, pl.p);
      else
        hipLaunchKernelGGL((k_mm64_tf<1>), grid, dim3(256), 0, st, A, V, P, pl.p);
    } else {
      const double* A = (const double*)a.A;
      if (NB == 4)
        hipLaunchKernelGGL((k_mm64<4, false, 0, 1>), grid, dim3(256), 0, st, A, nullptr, 1, 0.0,
                           0.0, V, P, pl.p);
      else if (NB == 2)
        hipLaunchKernelGGL((k_mm64<2, false, 0, 1>), grid, dim3(256), 0, st, A, nullptr, 1, 0.0,
                           0.0, V, P, pl.p);
      else
        hipLaunchKernelGGL((k_mm64<1, false, 0, 1>), grid, dim3(256), 0, st, A, nullptr, 1, 0.0,
                           0.0, V, P, pl.p);
    }
    if (ev1) LD_HIP(hipEventRecord(ev1, st));
    const int64_t tiles = (int64_t)pl.p.rt * ((a.s + pl.NT - 1) / pl.NT);
    hipLaunchKernelGGL(k_epilogue<double>, dim3((unsigned)tiles, epi_split(tiles, pl.NT)), dim3(256), 0, st, P, pl.p, pl.NT,
                       (double*)a.Y, V, fly ? a.kp.noise : 0.0, (const double*)a.X2, a.alpha2,
                       a.dots);
  } else {
    const int NB = pl.NT / 32;
    // kval32s: the FP32 points arrive scaled by point_scale (path_points), so
    // r2 is already in the kernel's units; RBF carries log2(variance)
    const float var = (float)(kind == LD_RBF ? std::log2(a.kp.variance) : a.kp.variance);
    const float* V = (const float*)a.V;
    float* P = (float*)part;
    if (split16) {
      if (kind == LD_RBF)
        fly16_by_d<LD_RBF>(NB, grid, st, (const float*)a.X, a.d, var, V, P, pl.p);
      else
        fly16_by_d<LD_MATERN52>(NB, grid, st, (const float*)a.X, a.d, var, V, P, pl.p);
    } else if (fly) {
      if (kind == LD_RBF)
        fly32_by_d<LD_RBF>(NB, grid, st, (const float*)a.X, a.d, var, V, P, pl.p);
      else
        fly32_by_d<LD_MATERN52>(NB, grid, st, (const float*)a.X, a.d, var, V, P, pl.p);
    } else {
      const float* A = (const float*)a.A;
      const bool tiled = a.layout == LD_TILED;
      if (a.bf16) {  // precision form from the stored FP32 tiles
        if (NB == 2)
          hipLaunchKernelGGL((k_mm16_tf<2>), grid, dim3(256), 0, st, A, V, P, pl.p);
        else
          hipLaunchKernelGGL((k_mm16_tf<1>), grid, dim3(256), 0, st, A, V, P, pl.p);
      } else if (NB == 2 && tiled)
        hipLaunchKernelGGL((k_mm32_tf<2>), grid, dim3(256), 0, st, A, V, P, pl.p);
      else if (NB == 2)
        hipLaunchKernelGGL((k_mm32_st<2>), grid, dim3(256), 0, st, A, V, P, pl.p);
      else if (tiled)
        hipLaunchKernelGGL((k_mm32_tf<1>), grid, dim3(256), 0, st, A, V, P, pl.p);
      else
        hipLaunchKernelGGL((k_mm32_st<1>), grid, dim3(256), 0, st, A, V, P, pl.p);
    }
    if (ev1) LD_HIP(hipEventRecord(ev1, st));
    const int64_t tiles = (int64_t)pl.p.rt * ((a.s + pl.NT - 1) / pl.NT);
    hipLaunchKernelGGL(k_epilogue<float>, dim3((unsigned)tiles, epi_split(tiles, pl.NT)), dim3(256), 0, st, P, pl.p, pl.NT,
                       (float*)a.Y, V,
                       fly ? a.kp.noise : 0.0,
                       (const float*)a.X2, a.alpha2, a.dots);
  }
  if (a.dot_blocks)
    *a.dot_blocks = pl.p.rt * epi_split((int64_t)pl.p.rt * ((a.s + pl.NT - 1) / pl.NT), pl.NT);
  LD_HIP(hipGetLastError());
  return LD_OK;
}

template <typename T>
void materialize_rm(hipStream_t st, int kind, bool small_d, dim3 grid, const double* X, int64_t n,
                    int d, double var, double c, double noise, T* M) {
  if (kind == LD_RBF && small_d)
    hipLaunchKernelGGL((k_materialize<T, LD_RBF, DMAX>), grid, dim3(256), 0, st, X, n, d, var, c, noise, M);
  else if (kind == LD_RBF)
    hipLaunchKernelGGL((k_materialize<T, LD_RBF, 64>), grid, dim3(256), 0, st, X, n, d, var, c, noise, M);
  else if (small_d)
    hipLaunchKernelGGL((k_materialize<T, LD_MATERN52, DMAX>), grid, dim3(256), 0, st, X, n, d, var, c,
                       noise, M);
  else
    hipLaunchKernelGGL((k_materialize<T, LD_MATERN52, 64>), grid, dim3(256), 0, st, X, n, d, var, c,
                       noise, M);
}

void launch_materialize(hipStream_t st, const KParams& kp, const double* X, int64_t n, int d,
                        int precision, int layout, void* M) {
  const double c = kp.kind == LD_RBF ? kp.c_rbf : kp.c_mat;
  const bool f64 = precision == LD_F64;
  if (layout == LD_TILED && f64) {
    const int64_t total = stored_elements(n, LD_TILED);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (kp.kind == LD_RBF)
      hipLaunchKernelGGL((k_materialize_tiled64<LD_RBF>), dim3((unsigned)blocks), dim3(256), 0, st,
                         X, n, d, kp.variance, c, kp.noise, total, (double*)M);
    else
      hipLaunchKernelGGL((k_materialize_tiled64<LD_MATERN52>), dim3((unsigned)blocks), dim3(256),
                         0, st, X, n, d, kp.variance, c, kp.noise, total, (double*)M);
    return;
  }
  if (layout == LD_TILED) {
    const int64_t total = stored_elements(n, LD_TILED);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (kp.kind == LD_RBF)
      hipLaunchKernelGGL((k_materialize_tiled<LD_RBF>), dim3((unsigned)blocks), dim3(256), 0, st, X,
                         n, d, kp.variance, c, kp.noise, total, (float*)M);
    else
      hipLaunchKernelGGL((k_materialize_tiled<LD_MATERN52>), dim3((unsigned)blocks), dim3(256), 0,
                         st, X, n, d, kp.variance, c, kp.noise, total, (float*)M);
    return;
  }
  int64_t gy = n < 256 ? n : 256;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)gy);
  if (f64)
    materialize_rm<double>(st, kp.kind, d <= DMAX, grid, X, n, d, kp.variance, c, kp.noise,
                           (double*)M);
  else
    materialize_rm<float>(st, kp.kind, d <= DMAX, grid, X, n, d, kp.variance, c, kp.noise,
                          (float*)M);
}

__global__ void k_f64_to_f32_scaled(const double* __restrict__ in, float* __restrict__ out,
                                    int64_t count, double scale) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
    out[i] = (float)(in[i] * scale);
}

void launch_convert_f64_to_f32_scaled(hipStream_t st, const double* in, float* out, int64_t count,
                                      double scale) {
  if (count > 0)
    hipLaunchKernelGGL(k_f64_to_f32_scaled, dim3(grid1(count)), dim3(256), 0, st, in, out, count,
                       scale);
}

double point_scale(const KParams& kp) {
  const double l2e = 1.4426950408889634;
  return kp.kind == LD_RBF ? std::sqrt(kp.c_rbf * l2e) : kp.c_mat * l2e;
}

void launch_convert_f64_to_f32(hipStream_t st, const double* in, float* out, int64_t count) {
  if (count > 0) hipLaunchKernelGGL(k_f64_to_f32, dim3(grid1(count)), dim3(256), 0, st, in, out, count);
}
void launch_convert_f32_to_f64(hipStream_t st, const float* in, double* out, int64_t count) {
  if (count > 0) hipLaunchKernelGGL(k_f32_to_f64, dim3(grid1(count)), dim3(256), 0, st, in, out, count);
}

}  // namespace ld
