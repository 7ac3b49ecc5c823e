// Batched form of the estimator: many independent GP problems of uneven size
// carried through the whole hot path together (Section 2 method applied to
// each instance).  The batch is a block-diagonal operator diag(M_1..M_B):
// instance i owns rows [row0_i, row0_i + n_i) of every batch matrix, padded
// to a multiple of 128 rows, and every reduction is segmented by instance.
//
//  - kernel-matrix products: one workgroup per (instance, row block, column
//    block), launched in decreasing n (longest first), each running the full
//    k range on FP32 matrix cores and applying the epilogue itself, so no
//    partial sums leave the workgroup; the candidate tile shapes (matrix-core
//    shape, column blocks, 4 or 2 waves) are timed once per context and the
//    fastest is kept (autotuner);
//  - preconditioner: batched range finder, CholeskyQR, Rayleigh-Ritz with
//    one-workgroup-per-instance Cholesky and triangular inverse
//    (dense_dev.hpp) and a Householder + implicit QL eigen-solver, Woodbury
//    factors per instance;
//  - solver: multi-shift CG with per-(instance, probe) scalars; the
//    iterations can be captured in a HIP graph and replayed in chunks.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <functional>
#include <numeric>
#include <string>
#include <vector>

#include "dense_dev.hpp"
#include "kfun_dev.hpp"
#include "ld_common.hpp"
#include "rng_dev.hpp"

namespace ld {
namespace {

constexpr int BROWS = 128;  // row padding of every instance
constexpr int BDX = 8;      // point stride (max dimension of a batched instance)
constexpr int BBK = 32;     // k per stage
constexpr int BLK = 64;     // row block of the segmented reductions
constexpr int kChunk = 8;   // solver iterations per host check / graph replay
constexpr int FTC = 256;    // rows per partial of the Woodbury projection F^T R
constexpr int GCH = 2048;   // rows per partial of the preconditioner's Gram products
// Stage points in LDS: point k of a BBK-point stage starts at xrow(k), eight
// floats further per block of eight points, so that lanes reading points 8
// (or 16) apart hit different banks; element e = k BDX + dd sits at xs_pos(e)
constexpr int XSTAGE = BBK * BDX + 8 * (BBK / 8);
__device__ __forceinline__ int xrow(int k) { return k * BDX + 8 * (k >> 3); }
__device__ __forceinline__ int xs_pos(int e) { return e + 8 * (e >> 6); }

struct BInst {
  const double* X64;
  int64_t n, row0;
  int d, kind, m, rank;
  int ch0, nch;  // first FTC-row chunk (global index) and chunk count
  int gp0, gnch; // GCH-row chunks of the Gram products; first partial slot when gnch > 1
  float kv, noise;       // kv: log2(variance) for RBF, variance for Matern
  double pscale;         // FP32 points are stored times this (see kval32s)
  double diag, floor_v, shift_c;
  uint64_t key_omega, key_probe;
};

struct BItem {
  int inst, rb, cb, pad;  // instance, row block, column block
};

using dev::f64x4;

// ------------------------------------------------------------ fill kernels --
__global__ void k_bx32(const BInst* __restrict__ inst, const int* __restrict__ blk_inst,
                       int64_t R, float* __restrict__ X32) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < R * BDX;
       e += (int64_t)gridDim.x * 256) {
    const int64_t row = e / BDX;
    const int dd = (int)(e % BDX);
    const BInst& I = inst[blk_inst[row / BLK]];
    const int64_t lr = row - I.row0;
    X32[e] = (lr < I.n && dd < I.d) ? (float)(I.X64[lr * I.d + dd] * I.pscale) : 0.f;
  }
}

// Gaussian test matrix, instance i drawing its own stream (index lr * m_i + c)
__global__ void k_bomega(const BInst* __restrict__ inst, const int* __restrict__ blk_inst,
                         int64_t R, int mmax, double* __restrict__ Om) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < R * mmax;
       e += (int64_t)gridDim.x * 256) {
    const int64_t row = e / mmax;
    const int c = (int)(e % mmax);
    const BInst& I = inst[blk_inst[row / BLK]];
    const int64_t lr = row - I.row0;
    Om[e] = (lr < I.n && c < I.m) ? dev::rng_gaussian(I.key_omega, (uint64_t)(lr * I.m + c)) : 0.0;
  }
}

__global__ void k_bprobes(const BInst* __restrict__ inst, const int* __restrict__ blk_inst,
                          int64_t R, int s, float* __restrict__ Z) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < R * s;
       e += (int64_t)gridDim.x * 256) {
    const int64_t row = e / s;
    const int c = (int)(e % s);
    const BInst& I = inst[blk_inst[row / BLK]];
    const int64_t lr = row - I.row0;
    Z[e] = lr < I.n ? dev::rng_rademacher(I.key_probe, (uint64_t)(lr * s + c)) : 0.f;
  }
}

// ------------------------------------------------------- batched product --
// Y = M V (+ noise V + alpha2 X2) on one instance's rows; padded rows of Y
// are written as zero.  dots[b][c] = sum over the 64-row block b of V .* Y.
//
// One workgroup per work item (instance, row block of 32 * WAVES rows,
// column block of NT columns) runs the whole k range: each stage stages 32
// points and a 32 x NT block of V in LDS (double buffered, the next stage
// prefetched in registers), every lane generates kernel entries for its
// rows, and the matrix cores multiply them into the accumulators.  The
// instance's kernel kind and dimension select a specialised inner loop
// (dimension padded to 2, 3, 4 or 8), so no lane evaluates a branch per
// entry.
//  MF = 32: v_mfma_f32_32x32x2f32, NT = 32 * NB; lane half h supplies
//           k = 16 h + t in step t (t < 16).
//  MF = 16: v_mfma_f32_16x16x4f32 for narrow blocks (NT = 16): each wave
//           covers two 16-row halves; lane group g supplies k = 8 g + t in
//           step t (t < 8).  Output lane l, register r: row 4 (l / 16) + r,
//           column l % 16.
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

template <int MF, int NB>
struct BmmShape {
  static constexpr int NT = MF * NB;  // columns per workgroup
  static constexpr int AS = BBK + 4;  // LDS row stride of the transposed V tile
};

template <int MF, int NB>
struct BmmAcc;
template <int NB>
struct BmmAcc<32, NB> {
  f32x16 v[NB];
};
template <int NB>
struct BmmAcc<16, NB> {
  f32x4v v[2][NB];
};

template <int MF, int NB, int WAVES, int KIND, int D>
__device__ __forceinline__ void bmm_body(const BInst& I, const BItem& it, const float* __restrict__ X32,
                                         const float* __restrict__ V, int ld, float* __restrict__ Y,
                                         const float* __restrict__ X2, float alpha2,
                                         double* __restrict__ dots, float* __restrict__ Bt,
                                         float* __restrict__ Xs, double* __restrict__ red) {
  constexpr int NT = BmmShape<MF, NB>::NT;
  constexpr int AS = BmmShape<MF, NB>::AS;
  constexpr int NTH = 64 * WAVES;
  constexpr int BMW = 32 * WAVES;
  constexpr int VPT = BBK * NT / NTH;   // V values per thread per stage
  constexpr int XPT = BBK * BDX / NTH;  // point values per thread per stage
  static_assert(VPT * NTH == BBK * NT && XPT * NTH == BBK * BDX, "stage split");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = I.n;
  const int64_t r0 = I.row0 + (int64_t)it.rb * BMW;  // first global row of the block
  const int c0 = it.cb * NT;
  const float* Vi = V + I.row0 * ld;
  const float kv = I.kv;

  // this lane's row points (MF = 32: one row; MF = 16: one per half)
  constexpr int NR = MF == 32 ? 1 : 2;
  float xr[NR][D];
#pragma unroll
  for (int h = 0; h < NR; ++h) {
    const int lr_in = MF == 32 ? 32 * wave + (lane & 31) : 32 * wave + 16 * h + (lane & 15);
    const int64_t lr = r0 - I.row0 + lr_in;
#pragma unroll
    for (int dd = 0; dd < D; ++dd) xr[h][dd] = lr < n ? X32[(I.row0 + lr) * BDX + dd] : 0.f;
  }
  BmmAcc<MF, NB> acc;
  if constexpr (MF == 32) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc.v[nb][r] = 0.f;
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc.v[h][nb][r] = 0.f;
  }

  const int S = (int)((n + BBK - 1) / BBK);
  // V stage: where the (column, 4 consecutive k) units divide evenly over the
  // threads, a thread loads such units and stores each as one 16-byte write
  // (lanes on consecutive columns, AS apart: distinct banks); otherwise one
  // value per thread and step
  constexpr bool VEC = (NT * (BBK / 4)) % NTH == 0;
  float tv[VPT], tx[XPT];
  auto load = [&](int st) {
    const int64_t k0 = (int64_t)st * BBK;
    if constexpr (VEC) {
#pragma unroll
      for (int j = 0; j < VPT / 4; ++j) {
        const int u = tid + NTH * j;
        const int kq = u / NT, cc = u % NT;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t kk = k0 + 4 * kq + i;
          tv[4 * j + i] = (kk < n && c0 + cc < ld) ? Vi[kk * ld + c0 + cc] : 0.f;
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < VPT; ++j) {
        const int e = tid + NTH * j;
        const int kk = e / NT, cc = e % NT;
        tv[j] = (k0 + kk < n && c0 + cc < ld) ? Vi[(k0 + kk) * ld + c0 + cc] : 0.f;
      }
    }
#pragma unroll
    for (int j = 0; j < XPT; ++j) {
      const int e = tid + NTH * j;
      const int64_t kr = k0 + e / BDX;
      tx[j] = kr < n ? X32[(I.row0 + kr) * BDX + e % BDX] : 0.f;
    }
  };
  auto entry = [&](const float* xr_, const float* xk) {
    float r2 = 0.f;
#pragma unroll
    for (int dd = 0; dd < D; ++dd) {
      const float df = xr_[dd] - xk[dd];
      r2 = __builtin_fmaf(df, df, r2);
    }
    return dev::kval32s<KIND>(r2, kv);
  };
  load(0);
  int buf = 0;
  for (int st = 0; st < S; ++st) {
    float* bt = Bt + buf * NT * AS;
    float* xs = Xs + buf * XSTAGE;
    if constexpr (VEC) {
#pragma unroll
      for (int j = 0; j < VPT / 4; ++j) {
        const int u = tid + NTH * j;
        *(float4*)&bt[(u % NT) * AS + 4 * (u / NT)] =
            make_float4(tv[4 * j], tv[4 * j + 1], tv[4 * j + 2], tv[4 * j + 3]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < VPT; ++j) {
        const int e = tid + NTH * j;
        bt[(e % NT) * AS + e / NT] = tv[j];
      }
    }
#pragma unroll
    for (int j = 0; j < XPT; ++j) xs[xs_pos(tid + NTH * j)] = tx[j];
    __syncthreads();
    if (st + 1 < S) load(st + 1);
    if constexpr (MF == 32) {
      const int li = lane & 31, lh = lane >> 5;
#pragma unroll
      for (int t4 = 0; t4 < 16; t4 += 4) {
        float a[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) a[t] = entry(xr[0], &xs[xrow(lh * 16 + t4 + t)]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const float4 b = *(const float4*)&bt[(nb * 32 + li) * AS + lh * 16 + t4];
          acc.v[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0], b.x, acc.v[nb], 0, 0, 0);
          acc.v[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1], b.y, acc.v[nb], 0, 0, 0);
          acc.v[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2], b.z, acc.v[nb], 0, 0, 0);
          acc.v[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[3], b.w, acc.v[nb], 0, 0, 0);
        }
      }
    } else {
      const int lj = lane & 15, lg = lane >> 4;
#pragma unroll
      for (int t4 = 0; t4 < 8; t4 += 4) {
        float a[2][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const float* xk = &xs[xrow(lg * 8 + t4 + t)];
          a[0][t] = entry(xr[0], xk);
          a[1][t] = entry(xr[1], xk);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const float4 b = *(const float4*)&bt[(nb * 16 + lj) * AS + lg * 8 + t4];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            acc.v[h][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][0], b.x, acc.v[h][nb], 0, 0, 0);
            acc.v[h][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][1], b.y, acc.v[h][nb], 0, 0, 0);
            acc.v[h][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][2], b.z, acc.v[h][nb], 0, 0, 0);
            acc.v[h][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][3], b.w, acc.v[h][nb], 0, 0, 0);
          }
        }
      }
    }
    buf ^= 1;
  }

  // epilogue: this workgroup owns its rows, so it writes Y directly
  double dsum[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) dsum[nb] = 0.0;
  auto put = [&](int nb, int row, int c, float a) {
    if (c >= ld) return;
    const int64_t grow = r0 + row;
    float y = 0.f;
    if (grow - I.row0 < n) {
      const int64_t off = grow * ld + c;
      double v = (double)a + (double)I.noise * (double)V[off];
      if (X2) v += (double)alpha2 * (double)X2[off];
      y = (float)v;
      dsum[nb] += (double)V[off] * (double)y;
    }
    Y[grow * ld + c] = y;
  };
  if constexpr (MF == 32) {
    const int li = lane & 31, lh = lane >> 5;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        put(nb, 32 * wave + 8 * (r >> 2) + 4 * lh + (r & 3), c0 + nb * 32 + li, acc.v[nb][r]);
  } else {
    const int lj = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          put(nb, 32 * wave + 16 * h + 4 * lg + r, c0 + nb * 16 + lj, acc.v[h][nb][r]);
  }
  if (dots) {
    // red[wave][lane][nb]; the 64-row block q gathers waves 2q and 2q + 1,
    // and within them every lane that holds column c
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) red[(wave * 64 + lane) * NB + nb] = dsum[nb];
    __syncthreads();
    constexpr int LPC = 64 / MF;  // lanes of a wave holding one column
    for (int e = tid; e < (BMW / BLK) * NT; e += NTH) {
      const int q = e / NT, c = e % NT;
      const int nb = c / MF, cl = c % MF;
      double t = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < 2; ++w2)
#pragma unroll
        for (int j = 0; j < LPC; ++j) t += red[((2 * q + w2) * 64 + cl + MF * j) * NB + nb];
      if (c0 + c < ld) dots[((r0 / BLK) + q) * (int64_t)ld + c0 + c] = t;
    }
  }
}

// The 224-column range-finder shape (NB = 7) runs two waves per SIMD: its
// 112 accumulators then share the 256 registers with the rest (about 33
// spilled), which still beats one wave per SIMD (51.6 against 60.1 ms per
// launch on the 256-instance batch)
template <int MF, int NB, int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(NB == 7 ? 2 : 1))) void k_bmm(const BInst* __restrict__ inst,
                                                    const BItem* __restrict__ items,
                                                    const float* __restrict__ X32,
                                                    const float* __restrict__ V, int ld,
                                                    float* __restrict__ Y,
                                                    const float* __restrict__ X2, float alpha2,
                                                    double* __restrict__ dots,
                                                    const int* __restrict__ iact) {
  constexpr int NT = BmmShape<MF, NB>::NT;
  constexpr int AS = BmmShape<MF, NB>::AS;
  __shared__ __attribute__((aligned(16))) float Bt[2 * NT * AS];
  __shared__ __attribute__((aligned(16))) float Xs[2 * XSTAGE];
  __shared__ double red[WAVES * 64 * NB];
  const BItem it = items[blockIdx.x];
  if (iact && !iact[it.inst]) return;  // every probe of this instance has converged
  const BInst I = inst[it.inst];
  const int dcat = I.d <= 2 ? 2 : (I.d == 3 ? 3 : (I.d == 4 ? 4 : 8));
#define LD_BMM_CASE(KIND, DD)                                                                   \
  bmm_body<MF, NB, WAVES, KIND, DD>(I, it, X32, V, ld, Y, X2, alpha2, dots, Bt, Xs, red)
  if (I.kind == LD_RBF) {
    switch (dcat) {
      case 2: LD_BMM_CASE(LD_RBF, 2); break;
      case 3: LD_BMM_CASE(LD_RBF, 3); break;
      case 4: LD_BMM_CASE(LD_RBF, 4); break;
      default: LD_BMM_CASE(LD_RBF, 8); break;
    }
  } else {
    switch (dcat) {
      case 2: LD_BMM_CASE(LD_MATERN52, 2); break;
      case 3: LD_BMM_CASE(LD_MATERN52, 3); break;
      case 4: LD_BMM_CASE(LD_MATERN52, 4); break;
      default: LD_BMM_CASE(LD_MATERN52, 8); break;
    }
  }
#undef LD_BMM_CASE
}

// -------------------------------------------- batched product, symmetric --
// M_i is symmetric, so each instance's off-diagonal kernel entries can be
// generated once: 128 x 128 blocks on and above the diagonal only, block
// (I, J), J > I, applied to rows I directly and to rows J transposed.  One
// workgroup per work item (instance, strip of SMS blocks, range of row
// tiles), for up to 16 probe columns: it runs the row tiles I of its range
// (unit (S, I): the blocks J >= I of the strip), each wave generating its 32
// rows of a 32-column stage.  The direct product is k_bmm's 16x16x4 path.
// For the transposed one a wave writes its generated 32 x 32 entries
// column-major to its own LDS slice and reads them back one column per lane
// (no wave waits for another), with the V rows of the wave in registers.
// Each wave keeps the transposed sums of its rows over the whole item; they
// are added across the four waves in LDS once per item (always in wave
// order) and written to the item's SMS transposed slots.  A strip's row
// tiles are cut into items of at most SCH, so that no item runs more than
// SCH SMS blocks (the last strips of a large instance would otherwise be the
// critical path of the launch once the small instances have converged).
// Each unit's direct sum goes to its own slot; k_bsym_reduce adds, per row
// tile, the direct slots of the strips from its own to the last, then the
// transposed slots of the items of its own strip that hold rows above it,
// in item order.
constexpr int SMS = 2;    // blocks of 128 per strip (256 columns)
constexpr int SCH = 8;    // row tiles per item at most
constexpr int SBB = 128;  // block edge
constexpr int STILE = SBB * 16;  // floats per partial slot (128 rows x 16 columns)

struct BSym {     // an instance's partial slots (in tiles of STILE floats)
  int64_t dir;    // first direct slot; row tile R's slots start dir + base(R)
  int nblk, ns;   // blocks, strips
};
struct BSItem {   // product work item: row tiles [i0, i1) of strip S
  int inst, S, i0, i1;
  int64_t tr;     // its SMS transposed slots (one per block of the strip)
};
struct BRItem {   // reduce work item: row tile R
  int inst, R, ntr;  // ntr transposed slots, SMS apart from tr
  int64_t tr;
};

// first direct slot of row tile R of an instance (the row tiles before it
// have ns - R' / SMS slots each: one per strip at or right of their own)
__host__ __device__ inline int64_t bsym_dir_base(int ns, int64_t R) {
  const int64_t q = R / SMS, r = R % SMS;
  return R * ns - (SMS * (q * (q - 1) / 2) + q * r);
}

template <int KIND, int D>
__device__ __forceinline__ void bsym_body(const BInst& I, const BSym& Q, const BSItem& it,
                                          const float* __restrict__ X32,
                                          const float* __restrict__ V, int ld,
                                          float* __restrict__ part, float* __restrict__ Bt,
                                          float* __restrict__ Xs, float* __restrict__ Kw,
                                          float* __restrict__ red) {
  constexpr int AS = BBK + 4;   // row stride of the transposed V stage
  constexpr int KWS = 32 + 4;   // row stride of a wave's column-major K slice
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lj = lane & 15, lg = lane >> 4;
  const int64_t n = I.n;
  const float kv = I.kv;
  const float* Vi = V + I.row0 * ld;
  const float* Xi = X32 + I.row0 * BDX;
  float* kw = Kw + wave * (32 * KWS);
  const int S = it.S;
  const int mS = SMS * S;
  const int me = mS + SMS < Q.nblk ? mS + SMS : Q.nblk;

  f32x4v accT[SMS][4][2];
#pragma unroll
  for (int b = 0; b < SMS; ++b)
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) accT[b][st][mt] = f32x4v{0.f, 0.f, 0.f, 0.f};

  // stage prefetch: V rows k0 + 2 (tid / 16) (+1) of column tid % 16, one
  // point coordinate
  float tv[2], tx;
  auto load = [&](int64_t k0) {
    const int c = tid % 16;
    const int64_t r = k0 + 2 * (tid / 16);
    tv[0] = (r < n && c < ld) ? Vi[r * ld + c] : 0.f;
    tv[1] = (r + 1 < n && c < ld) ? Vi[(r + 1) * ld + c] : 0.f;
    const int64_t kr = k0 + tid / BDX;
    tx = kr < n ? Xi[kr * BDX + tid % BDX] : 0.f;
  };
  auto entry = [&](const float* xr_, const float* xk) {
    float r2 = 0.f;
#pragma unroll
    for (int dd = 0; dd < D; ++dd) {
      const float df = xr_[dd] - xk[dd];
      r2 = __builtin_fmaf(df, df, r2);
    }
    return dev::kval32s<KIND>(r2, kv);
  };
  load((int64_t)SBB * (it.i0 > mS ? it.i0 : mS));
  int buf = 0;
  for (int I0 = it.i0; I0 < it.i1; ++I0) {
    const int64_t i0 = (int64_t)SBB * I0;
    const int jf = I0 > mS ? I0 : mS;
    const int64_t ncol = I0 + 1 < it.i1 ? (int64_t)SBB * (I0 + 1 > mS ? I0 + 1 : mS) : -1;
    float xr[2][D];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t lr = i0 + 32 * wave + 16 * h + lj;
#pragma unroll
      for (int dd = 0; dd < D; ++dd) xr[h][dd] = lr < n ? Xi[lr * BDX + dd] : 0.f;
    }
    // V rows of this wave as the transposed product's B operand: rows
    // 32 wave + 8 lg + t, column lj
    float vi[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t lr = i0 + 32 * wave + 8 * lg + t;
      vi[t] = (lr < n && lj < ld) ? Vi[lr * ld + lj] : 0.f;
    }
    f32x4v acc[2];
    acc[0] = f32x4v{0.f, 0.f, 0.f, 0.f};
    acc[1] = acc[0];
#pragma unroll
    for (int b = 0; b < SMS; ++b) {
      const int J = mS + b;
      if (J < jf || J >= me) continue;
      const bool sym = J > I0;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int64_t col0 = (int64_t)SBB * J + BBK * st;
        float* bt = Bt + buf * 16 * AS;
        float* xs = Xs + buf * XSTAGE;
        *(float2*)&bt[(tid % 16) * AS + 2 * (tid / 16)] = make_float2(tv[0], tv[1]);
        xs[xs_pos(tid)] = tx;
        __syncthreads();
        const int64_t nc = col0 + BBK < (int64_t)SBB * me ? col0 + BBK : ncol;
        if (nc >= 0) load(nc);
        float a[2][8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const float* xk = &xs[xrow(lg * 8 + t)];
          a[0][t] = entry(xr[0], xk);
          a[1][t] = entry(xr[1], xk);
        }
#pragma unroll
        for (int t4 = 0; t4 < 8; t4 += 4) {
          const float4 bv = *(const float4*)&bt[lj * AS + lg * 8 + t4];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][t4 + 0], bv.x, acc[h], 0, 0, 0);
            acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][t4 + 1], bv.y, acc[h], 0, 0, 0);
            acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][t4 + 2], bv.z, acc[h], 0, 0, 0);
            acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][t4 + 3], bv.w, acc[h], 0, 0, 0);
          }
        }
        if (sym) {
          // lane (lj, lg) holds K[16 h + lj][8 lg + t] of the wave's rows:
          // store column-major, read a column per lane.  Column c keeps its
          // two 16-row halves swapped when bits 3 and 4 of c differ, so
          // that the four lane groups of a store (columns 8 apart) fall in
          // different banks; a read stays four consecutive rows.
          const int sw = 16 * ((lg & 1) ^ (lg >> 1));
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            kw[(8 * lg + t) * KWS + (lj ^ sw)] = a[0][t];
            kw[(8 * lg + t) * KWS + ((16 + lj) ^ sw)] = a[1][t];
          }
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            const int sr = 16 * (((lj >> 3) & 1) ^ mt);
            const float4* kp = (const float4*)&kw[(16 * mt + lj) * KWS + ((8 * lg) ^ sr)];
            const float4 k0v = kp[0], k1v = kp[1];
            f32x4v c = accT[b][st][mt];
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(k0v.x, vi[0], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(k0v.y, vi[1], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(k0v.z, vi[2], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(k0v.w, vi[3], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(k1v.x, vi[4], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(k1v.y, vi[5], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(k1v.z, vi[6], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(k1v.w, vi[7], c, 0, 0, 0);
            accT[b][st][mt] = c;
          }
          __builtin_amdgcn_wave_barrier();
        }
        buf ^= 1;
      }
    }
    // the unit's direct sum (rows 32 wave + 16 h + 4 lg + r, column lj)
    float* dst = part + (Q.dir + bsym_dir_base(Q.ns, I0) + (S - I0 / SMS)) * STILE;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[(32 * wave + 16 * h + 4 * lg + r) * 16 + lj] = acc[h][r];
  }
  // transposed sums: rows (columns of M) 32 st + 16 mt + 4 lg + r of block
  // b, column lj; added over the waves in order
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int b = 0; b < SMS; ++b)
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
          for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int e = b * STILE + (32 * st + 16 * mt + 4 * lg + r) * 16 + lj;
              red[e] = w == 0 ? accT[b][st][mt][r] : red[e] + accT[b][st][mt][r];
            }
    }
    __syncthreads();
  }
  float* dst = part + it.tr * STILE;
  for (int e = tid; e < SMS * STILE; e += 256) dst[e] = red[e];
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_bmm_sym(const BInst* __restrict__ inst,
                                                 const BSym* __restrict__ sym,
                                                 const BSItem* __restrict__ items,
                                                 const float* __restrict__ X32,
                                                 const float* __restrict__ V, int ld,
                                                 float* __restrict__ part,
                                                 const int* __restrict__ iact) {
  __shared__ __attribute__((aligned(16))) float Bt[2 * 16 * (BBK + 4)];
  __shared__ __attribute__((aligned(16))) float Xs[2 * XSTAGE];
  __shared__ __attribute__((aligned(16))) float Kw[4 * 32 * (32 + 4)];
  __shared__ float red[SMS * STILE];
  const BSItem it = items[blockIdx.x];
  if (iact && !iact[it.inst]) return;  // every probe of this instance has converged
  const BInst I = inst[it.inst];
  const BSym Q = sym[it.inst];
  const int dcat = I.d <= 2 ? 2 : (I.d == 3 ? 3 : (I.d == 4 ? 4 : 8));
#define LD_BSYM_CASE(KIND, DD) \
  bsym_body<KIND, DD>(I, Q, it, X32, V, ld, part, Bt, Xs, Kw, red)
  if (I.kind == LD_RBF) {
    switch (dcat) {
      case 2: LD_BSYM_CASE(LD_RBF, 2); break;
      case 3: LD_BSYM_CASE(LD_RBF, 3); break;
      case 4: LD_BSYM_CASE(LD_RBF, 4); break;
      default: LD_BSYM_CASE(LD_RBF, 8); break;
    }
  } else {
    switch (dcat) {
      case 2: LD_BSYM_CASE(LD_MATERN52, 2); break;
      case 3: LD_BSYM_CASE(LD_MATERN52, 3); break;
      case 4: LD_BSYM_CASE(LD_MATERN52, 4); break;
      default: LD_BSYM_CASE(LD_MATERN52, 8); break;
    }
  }
#undef LD_BSYM_CASE
}

// Y of row tile (instance, R) = its direct slots in strip order + its
// transposed slots in item order (+ noise V + alpha2 X2); padded rows
// written as zero;
// dots[b][c] = sum over the 64-row block b of V .* Y (the outputs of k_bmm).
__global__ __launch_bounds__(256) void k_bsym_reduce(const BInst* __restrict__ inst,
                                                     const BSym* __restrict__ sym,
                                                     const BRItem* __restrict__ items,
                                                     const float* __restrict__ part,
                                                     const float* __restrict__ V, int ld,
                                                     float* __restrict__ Y,
                                                     const float* __restrict__ X2, float alpha2,
                                                     double* __restrict__ dots,
                                                     const int* __restrict__ iact) {
  __shared__ double red[256];
  const BRItem it = items[blockIdx.x];
  if (iact && !iact[it.inst]) return;
  const BInst I = inst[it.inst];
  const BSym Q = sym[it.inst];
  const int R = it.R;
  const int tid = threadIdx.x;
  const int SR = R / SMS;
  const int ndir = Q.ns - SR;
  const float* dir = part + (Q.dir + bsym_dir_base(Q.ns, R)) * STILE;
  const int c = tid % 16;  // 256 threads: rows tid / 16 + 16 j, column c
  double sum[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) sum[j] = 0.0;
  int q = 0;
  for (; q + 4 <= ndir; q += 4) {
    float v[4][8];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < 8; ++j) v[u][j] = dir[(int64_t)(q + u) * STILE + tid + 256 * j];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < 8; ++j) sum[j] += (double)v[u][j];
  }
  for (; q < ndir; ++q)
#pragma unroll
    for (int j = 0; j < 8; ++j) sum[j] += (double)dir[(int64_t)q * STILE + tid + 256 * j];
  for (int c = 0; c < it.ntr; ++c) {
    const float* trs = part + (it.tr + (int64_t)SMS * c) * STILE;
#pragma unroll
    for (int j = 0; j < 8; ++j) sum[j] += (double)trs[tid + 256 * j];
  }
  double dq[2] = {0.0, 0.0};
  const int64_t r0 = I.row0 + (int64_t)SBB * R;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int row = tid / 16 + 16 * j;
    if (c >= ld) continue;
    const int64_t grow = r0 + row;
    float y = 0.f;
    if ((int64_t)SBB * R + row < I.n) {
      const int64_t off = grow * ld + c;
      double v = sum[j] + (double)I.noise * (double)V[off];
      if (X2) v += (double)alpha2 * (double)X2[off];
      y = (float)v;
      dq[row / BLK] += (double)V[off] * (double)y;
    }
    Y[grow * ld + c] = y;
  }
  if (dots) {
    // 64-row block q: rows 64 q .. 64 q + 63, threads tid / 16 + 16 j with j in 4 q .. 4 q + 3
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) {
      red[tid] = dq[qb];
      __syncthreads();
      if (tid < 16 && tid < ld) {
        double tsum = 0.0;
        for (int k = tid; k < 256; k += 16) tsum += red[k];
        dots[(r0 / BLK + qb) * (int64_t)ld + tid] = tsum;
      }
      __syncthreads();
    }
  }
}

// -------------------------------------------------------- dense, batched --
// G_i (mdim_i x mdim_i, leading dimension mdim_i, at i * gstride) =
// A_i^T diag(w_i) B_i over the instance's rows; 64 x 64 tile per workgroup
// and GCH-row chunk (work item blockIdx.z = (instance, chunk)): an instance
// of one chunk writes G_i, one of several writes a partial per chunk that
// k_bgram_sum adds in chunk order (a single workgroup streaming all the rows
// of a 20,000-point instance was the launch's critical path).  With sym
// (B = A) only the tiles on and above the diagonal are computed and each
// off-diagonal one is also written transposed.
__global__ __launch_bounds__(256) void k_bgram(const BInst* __restrict__ inst,
                                               const int2* __restrict__ gitems, int use_rank,
                                               const double* __restrict__ A, int lda,
                                               const double* __restrict__ B, int ldb,
                                               const double* __restrict__ w,
                                               double* __restrict__ G, double* __restrict__ gpart,
                                               int64_t gstride, int sym) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int2 gi = gitems[blockIdx.z];
  const BInst I = inst[gi.x];
  const int md = use_rank ? I.rank : I.m;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  if (i0 >= md || j0 >= md || (sym && i0 > j0)) return;
  const int64_t r0 = (int64_t)gi.y * GCH;
  const int64_t r1 = r0 + GCH < I.n ? r0 + GCH : I.n;
  const int tid = threadIdx.x, ti = tid / 16, tj = tid % 16;
  double acc[4][4] = {};
  for (int64_t rb = r0; rb < r1; rb += 16) {
    __syncthreads();
    for (int e = tid; e < 16 * 64; e += 256) {
      const int rr = e / 64, cc = e % 64;
      const int64_t lr = rb + rr, row = I.row0 + lr;
      double av = 0.0, bv = 0.0;
      if (lr < r1) {
        const double wr = w ? w[row] : 1.0;
        if (i0 + cc < md) av = A[row * lda + i0 + cc] * wr;
        if (j0 + cc < md) bv = B[row * ldb + j0 + cc];
      }
      As[rr][cc] = av;
      Bs[rr][cc] = bv;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < 16; ++rr) {
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
  double* Gi = I.gnch > 1 ? gpart + (I.gp0 + gi.y) * gstride : G + gi.x * gstride;
  const bool mirror = sym && i0 < j0;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = i0 + ti + 16 * x, j = j0 + tj + 16 * y;
      if (i < md && j < md) {
        Gi[(int64_t)i * md + j] = acc[x][y];
        if (mirror) Gi[(int64_t)j * md + i] = acc[x][y];
      }
    }
}

// G_i = sum of its chunk partials, in chunk order (instances of several
// GCH-row chunks only); grid (instances, mmax^2 / 256)
__global__ __launch_bounds__(256) void k_bgram_sum(const BInst* __restrict__ inst, int use_rank,
                                                   const double* __restrict__ gpart,
                                                   double* __restrict__ G, int64_t gstride) {
  const BInst I = inst[blockIdx.x];
  if (I.gnch <= 1) return;
  const int md = use_rank ? I.rank : I.m;
  const int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (e >= (int64_t)md * md) return;
  const double* src = gpart + I.gp0 * gstride + e;
  double v = 0.0;
  for (int c = 0; c < I.gnch; ++c) v += src[c * gstride];
  G[blockIdx.x * gstride + e] = v;
}

__global__ __launch_bounds__(256) void k_bshift(const BInst* __restrict__ inst,
                                                double* __restrict__ G, int64_t gstride) {
  __shared__ double red[256];
  const BInst I = inst[blockIdx.x];
  double* Gi = G + blockIdx.x * gstride;
  double t = 0.0;
  for (int j = threadIdx.x; j < I.m; j += 256) t += Gi[(int64_t)j * I.m + j];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double sh = I.shift_c * red[0];
  for (int j = threadIdx.x; j < I.m; j += 256) Gi[(int64_t)j * I.m + j] += sh;
}

__global__ __launch_bounds__(dev::CT) void k_bchol(const BInst* __restrict__ inst, int use_rank,
                                                   double* __restrict__ G, int64_t gstride,
                                                   int* __restrict__ fail) {
  const BInst I = inst[blockIdx.x];
  const int md = use_rank ? I.rank : I.m;
  dev::chol_upper_block(G + blockIdx.x * gstride, md, md, fail + blockIdx.x);
}

__global__ __launch_bounds__(dev::CT) void k_btrinv(const BInst* __restrict__ inst, int use_rank,
                                                    const double* __restrict__ R,
                                                    double* __restrict__ X, int64_t gstride) {
  const BInst I = inst[blockIdx.x];
  const int md = use_rank ? I.rank : I.m;
  dev::tri_inv_upper_block(R + blockIdx.x * gstride, md, md, X + blockIdx.x * gstride, md);
}

// C_i = diag(rs) A_i B_i with A_i the instance's rows of A (lda), B_i the
// instance's K x N matrix at i * bstride (leading dimension ldb_i = N_i when
// bld < 0, else the instance's m), K_i / N_i from (m | rank).
__global__ __launch_bounds__(256) void k_bgemm(const BInst* __restrict__ inst, int k_is_rank,
                                               int n_is_rank, const double* __restrict__ A,
                                               int lda, const double* __restrict__ B,
                                               int64_t bstride, int b_ld_is_m,
                                               const double* __restrict__ rs,
                                               double* __restrict__ C, int ldc) {
  const BInst I = inst[blockIdx.z];
  const int K = k_is_rank ? I.rank : I.m;
  const int N = n_is_rank ? I.rank : I.m;
  const int64_t i0 = (int64_t)blockIdx.x * dev::GM_BM;
  const int j0 = blockIdx.y * dev::GM_BN;
  if (i0 >= I.n || j0 >= N) return;
  const int ldb = b_ld_is_m ? I.m : N;
  dev::gemm64_tile(A + I.row0 * lda, lda, B + blockIdx.z * bstride, ldb,
                   rs ? rs + I.row0 : nullptr, I.n, K, N, C + I.row0 * ldc, ldc, i0, j0);
}

// Symmetric eigen-decomposition of G_i (m_i x m_i, symmetrised) by one
// workgroup of 1024 threads: Householder reduction to tridiagonal form
// T = H^T G H, implicit QL iterations with Wilkinson-type shifts on T whose
// plane rotations are accumulated into Z (Z = I initially), and the
// back-transformation X = H Z; eigenpairs sorted by descending eigenvalue
// into evals (stride emax) and evecs_i (m_i x m_i, column j = eigenvector of
// evals[j]).  One thread runs the scalar QL recurrence; the other threads
// apply each sweep's rotations to the rows of Z.  Work area per instance:
// 2 m^2 doubles (the reduced matrix holding the reflectors, then Z).
// status[i] = 1 when an eigenvalue needs more than 60 QL iterations.
// Requires m_i <= 1024.
__global__ __launch_bounds__(1024) void k_beigh(const BInst* __restrict__ inst,
                                                const double* __restrict__ G, int64_t gstride,
                                                double* __restrict__ work, int64_t wstride,
                                                double* __restrict__ evals, int emax,
                                                double* __restrict__ evecs,
                                                int* __restrict__ status) {
  __shared__ double sd[1024], se[1024];  // diagonal, off-diagonal of T
  __shared__ double su[1024], sp[1024];  // reflector, matrix-vector product
  __shared__ double red[1024];
  __shared__ double rc[1024], rs[1024];  // rotations (i, i+1) of one QL sweep
  __shared__ double sh_v[3];
  __shared__ int sh_flag, sh_lo, sh_hi, sh_fail;
  const BInst I = inst[blockIdx.x];
  const int m = I.m;
  const int tid = threadIdx.x;
  const double* Gi = G + blockIdx.x * gstride;
  double* A = work + blockIdx.x * wstride;
  double* Z = A + (int64_t)m * m;
  for (int64_t e = tid; e < (int64_t)m * m; e += 1024) {
    const int i = (int)(e / m), j = (int)(e % m);
    A[e] = 0.5 * (Gi[(int64_t)i * m + j] + Gi[(int64_t)j * m + i]);
    Z[e] = i == j ? 1.0 : 0.0;
  }
  if (tid == 0) sh_fail = 0;
  __syncthreads();

  auto block_sum = [&](double v) {  // all threads must call; returns the sum to all
    red[tid] = v;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
  };

  // ---- 1. Householder tridiagonalization (H_k = I - u u^T, |u|^2 = 2)
  for (int k = 0; k + 2 < m; ++k) {
    const int n2 = m - k - 1;  // trailing rows / columns k+1 .. m-1
    double t = 0.0;
    for (int i = k + 2 + tid; i < m; i += 1024) {
      const double x = A[(int64_t)i * m + k];
      t += x * x;
    }
    const double sigma = block_sum(t);
    if (tid == 0) {
      const double x0 = A[(int64_t)(k + 1) * m + k];
      sd[k] = A[(int64_t)k * m + k];
      if (sigma == 0.0) {
        se[k] = x0;
        sh_flag = 0;
      } else {
        const double alpha = -copysign(sqrt(x0 * x0 + sigma), x0);
        const double v0 = x0 - alpha;
        se[k] = alpha;
        sh_v[0] = sqrt(2.0 / (v0 * v0 + sigma));  // scale of v to u
        sh_v[1] = v0;
        sh_flag = 1;
      }
    }
    __syncthreads();
    if (!sh_flag) {
      for (int j = tid; j < n2; j += 1024) A[(int64_t)(k + 1 + j) * m + k] = 0.0;  // H_k = I
      __syncthreads();
      continue;
    }
    const double sc = sh_v[0];
    for (int j = tid; j < n2; j += 1024) {
      const double v = j == 0 ? sh_v[1] : A[(int64_t)(k + 1 + j) * m + k];
      su[j] = v * sc;
      A[(int64_t)(k + 1 + j) * m + k] = v * sc;  // kept for the back-transformation
    }
    __syncthreads();
    // p = A22 u (A22 symmetric: thread (grp, j) sums rows grp, grp + ng, ...)
    const int ng = 1024 / n2;
    {
      const int j = tid % n2, grp = tid / n2;
      double acc = 0.0;
      if (grp < ng) {
        const double* col = A + (int64_t)(k + 1) * m + (k + 1 + j);
#pragma unroll 4
        for (int i = grp; i < n2; i += ng) acc = fma(col[(int64_t)i * m], su[i], acc);
      }
      red[tid] = acc;
    }
    __syncthreads();
    double pj = 0.0;
    if (tid < n2) {
      for (int g = 0; g < ng; ++g) pj += red[g * n2 + tid];
    }
    __syncthreads();
    const double K = block_sum(tid < n2 ? pj * su[tid] : 0.0);
    if (tid < n2) sp[tid] = pj - 0.5 * K * su[tid];  // w
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)n2 * n2; e += 1024) {
      const int i = (int)(e / n2), j = (int)(e % n2);
      A[(int64_t)(k + 1 + i) * m + (k + 1 + j)] -= su[i] * sp[j] + sp[i] * su[j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (m >= 2) {
      sd[m - 2] = A[(int64_t)(m - 2) * m + (m - 2)];
      se[m - 2] = A[(int64_t)(m - 1) * m + (m - 2)];
    }
    sd[m - 1] = A[(int64_t)(m - 1) * m + (m - 1)];
    se[m - 1] = 0.0;
  }
  __syncthreads();

  // ---- 2. implicit QL on (sd, se); se[i] couples sd[i] and sd[i+1]
  for (int l = 0; l < m; ++l) {
    int iter = 0;
    while (true) {
      if (tid == 0) {
        int mm = l;
        for (; mm < m - 1; ++mm) {
          const double dd = fabs(sd[mm]) + fabs(sd[mm + 1]);
          if (fabs(se[mm]) <= 0x1.0p-52 * dd) break;
        }
        if (mm == l || iter >= 60) {
          if (mm != l) sh_fail = 1;
          sh_flag = 0;
        } else {
          ++iter;
          double g = (sd[l + 1] - sd[l]) / (2.0 * se[l]);
          double r = hypot(g, 1.0);
          g = sd[mm] - sd[l] + se[l] / (g + copysign(r, g));
          double s = 1.0, c = 1.0, p = 0.0;
          int i = mm - 1;
          bool under = false;
          for (; i >= l; --i) {
            const double f = s * se[i], b = c * se[i];
            r = hypot(f, g);
            se[i + 1] = r;
            if (r == 0.0) {
              sd[i + 1] -= p;
              se[mm] = 0.0;
              under = true;
              break;
            }
            s = f / r;
            c = g / r;
            g = sd[i + 1] - p;
            r = (sd[i] - g) * s + 2.0 * c * b;
            p = s * r;
            sd[i + 1] = g + p;
            g = c * r - b;
            rc[i] = c;
            rs[i] = s;
          }
          sh_hi = mm - 1;
          sh_lo = under ? i + 1 : l;
          if (!under) {
            sd[l] -= p;
            se[l] = g;
            se[mm] = 0.0;
          }
          sh_flag = 1;
        }
      }
      __syncthreads();
      if (!sh_flag) break;
      if (tid < m) {
        double* zr = Z + (int64_t)tid * m;
        for (int i = sh_hi; i >= sh_lo; --i) {
          const double c = rc[i], s = rs[i];
          const double f = zr[i + 1], zi = zr[i];
          zr[i + 1] = s * zi + c * f;
          zr[i] = c * zi - s * f;
        }
      }
      __syncthreads();
    }
    __syncthreads();
  }

  // ---- 3. back-transformation Z <- H_0 H_1 ... H_{m-3} Z (thread per column)
  for (int k = m - 3; k >= 0; --k) {
    const int n2 = m - k - 1;
    for (int j = tid; j < n2; j += 1024) su[j] = A[(int64_t)(k + 1 + j) * m + k];
    __syncthreads();
    if (tid < m) {
      double y = 0.0;
#pragma unroll 4
      for (int i = 0; i < n2; ++i) y = fma(su[i], Z[(int64_t)(k + 1 + i) * m + tid], y);
#pragma unroll 4
      for (int i = 0; i < n2; ++i) Z[(int64_t)(k + 1 + i) * m + tid] -= su[i] * y;
    }
    __syncthreads();
  }

  // ---- sorted output
  if (tid == 0 && sh_fail) status[blockIdx.x] = 1;
  double* ev = evals + (int64_t)blockIdx.x * emax;
  double* vec = evecs + blockIdx.x * gstride;
  for (int i = tid; i < m; i += 1024) {
    const double li = sd[i];
    int pos = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = sd[j];
      if (lj > li || (lj == li && j < i)) ++pos;
    }
    ev[pos] = li;
    for (int r = 0; r < m; ++r) vec[(int64_t)r * m + pos] = Z[(int64_t)r * m + i];
  }
}

// D = diag(M) - rowsum(U^2 lam) floored; padded rows get D = 1, Dinv = 0
__global__ void k_bd(const BInst* __restrict__ inst, const int* __restrict__ blk_inst, int64_t R,
                     const double* __restrict__ U, int ldu, const double* __restrict__ lam,
                     int emax, double* __restrict__ D, double* __restrict__ Dinv) {
  for (int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x; row < R;
       row += (int64_t)gridDim.x * 256) {
    const int ii = blk_inst[row / BLK];
    const BInst& I = inst[ii];
    if (row - I.row0 >= I.n) {
      D[row] = 1.0;
      Dinv[row] = 0.0;
      continue;
    }
    double low = 0.0;
    const double* li = lam + (int64_t)ii * emax;
    for (int j = 0; j < I.rank; ++j) {
      const double u = U[row * ldu + j];
      low = fma(li[j] * u, u, low);
    }
    double dv = I.diag - low;
    if (!(dv >= I.floor_v)) dv = I.floor_v;
    D[row] = dv;
    Dinv[row] = 1.0 / dv;
  }
}

__global__ void k_bcapdiag(const BInst* __restrict__ inst, double* __restrict__ C, int64_t gstride,
                           const double* __restrict__ lam, int emax) {
  const BInst I = inst[blockIdx.x];
  for (int j = threadIdx.x; j < I.rank; j += 256)
    C[blockIdx.x * gstride + (int64_t)j * I.rank + j] += 1.0 / lam[(int64_t)blockIdx.x * emax + j];
}

// log det P_i = sum log D + sum log lam + 2 sum log diag(chol C)
__global__ __launch_bounds__(256) void k_blogdet(const BInst* __restrict__ inst,
                                                 const double* __restrict__ D,
                                                 const double* __restrict__ lam, int emax,
                                                 const double* __restrict__ Rc, int64_t gstride,
                                                 double* __restrict__ out) {
  __shared__ double red[256];
  const BInst I = inst[blockIdx.x];
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < I.n; i += 256) t += log(D[I.row0 + i]);
  for (int j = threadIdx.x; j < I.rank; j += 256)
    t += log(lam[(int64_t)blockIdx.x * emax + j]) +
         2.0 * log(Rc[blockIdx.x * gstride + (int64_t)j * I.rank + j]);
  red[threadIdx.x] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// ----------------------------------------------------------- solver pieces --
// Partial projections of the Woodbury apply: for row chunk g (FTC rows of one
// instance) part_g (rank_i x s, at g * lmax * s) = F_g^T R_g, on FP64 matrix
// cores (v_mfma_f64_16x16x4f64; FP32 inputs widened exactly, FP64
// accumulation).  Stages of 32 rows of F (one pass covers up to FT_PW of
// the rank columns) and of R are loaded with 16-byte reads, prefetched in
// registers while the previous stage is multiplied out of LDS.  The output is
// cut into 16 x 16 (l, c) tiles, at most FT_TW per wave per pass (128-column
// passes: three waves per SIMD, where 256-column passes held two); in step t a
// wave consumes rows 4t .. 4t+3 of the stage, lane group g = lane/16
// supplying row 4t + g.  Output lane l, register r: tile row l/16 + 4 r,
// column l % 16.  Requires ldf % 4 == 0 (16-byte rows of F) and s <= 64.
constexpr int FT_ROWS = 32;
constexpr int FT_PW = 128;  // widest column pass (s <= 16; 64 for s <= 32, 32 above)
constexpr int FT_F4 = FT_ROWS * FT_PW / 4 / 256;  // float4 of the F stage per thread
constexpr int FT_TW = FT_PW / 64;                 // 16 x 16 tiles per wave at most
__global__ __launch_bounds__(256) void k_bft(const BInst* __restrict__ inst,
                                             const int* __restrict__ ch_inst,
                                             const float* __restrict__ F, int ldf,
                                             const float* __restrict__ R, int s, int lmax,
                                             double* __restrict__ part,
                                             const int* __restrict__ iact) {
  constexpr int FS = FT_PW + 4;  // LDS row stride of the F stage
  constexpr int RS = 64 + 4;     // LDS row stride of the R stage
  __shared__ __attribute__((aligned(16))) float Fs[FT_ROWS * FS];
  __shared__ __attribute__((aligned(16))) float Rs[FT_ROWS * RS];
  const int g = blockIdx.x;
  const int ii = ch_inst[g];
  if (iact && !iact[ii]) return;
  const BInst I = inst[ii];
  const int64_t lo = (int64_t)(g - I.ch0) * FTC;
  const int64_t hi = lo + FTC < I.n ? lo + FTC : I.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int ct = (s + 15) / 16;
  const int pw = ct <= 1 ? FT_PW : (ct == 2 ? FT_PW / 2 : FT_PW / 4);  // columns per pass
  double* out = part + (int64_t)g * lmax * s;
  for (int lbase = 0; lbase < I.rank; lbase += pw) {
    const int lw = I.rank - lbase < pw ? I.rank - lbase : pw;  // columns this pass
    const int lw4 = (lw + 3) / 4;
    const int tiles = ((lw + 15) / 16) * ct;  // <= 4 FT_TW
    f64x4 acc[FT_TW];
#pragma unroll
    for (int q = 0; q < FT_TW; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
    // register prefetch of one stage: F as float4 (FT_F4 per thread), R as
    // floats (the stage's 32 rows of R are contiguous: <= 8 per thread)
    float4 pf[FT_F4];
    float pr[8];
    auto fetch = [&](int64_t row0) {
#pragma unroll
      for (int j = 0; j < FT_F4; ++j) {
        const int e = tid + 256 * j;  // float4 index within the stage
        const int rr = e / lw4, c4 = e % lw4;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (rr < FT_ROWS && row0 + rr < hi) {
          const float* src = F + (I.row0 + row0 + rr) * (int64_t)ldf + lbase + 4 * c4;
          v = *(const float4*)src;
        }
        pf[j] = v;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = tid + 256 * j;
        const int rr = e / s;
        pr[j] = (rr < FT_ROWS && row0 + rr < hi) ? R[(I.row0 + row0) * (int64_t)s + e] : 0.f;
      }
    };
    fetch(lo);
    for (int64_t row0 = lo; row0 < hi; row0 += FT_ROWS) {
      __syncthreads();  // the previous stage has been consumed
#pragma unroll
      for (int j = 0; j < FT_F4; ++j) {
        const int e = tid + 256 * j;
        const int rr = e / lw4, c4 = e % lw4;
        if (rr < FT_ROWS) {
          // columns past the rank (padding of the F rows) are stored as zero
          const int l0 = 4 * c4;
          float4 v = pf[j];
          if (l0 + 1 >= lw) v.y = 0.f;
          if (l0 + 2 >= lw) v.z = 0.f;
          if (l0 + 3 >= lw) v.w = 0.f;
          *(float4*)&Fs[rr * FS + l0] = v;
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = tid + 256 * j;
        const int rr = e / s;
        if (rr < FT_ROWS) Rs[rr * RS + e % s] = pr[j];
      }
      __syncthreads();
      if (row0 + FT_ROWS < hi) fetch(row0 + FT_ROWS);
#pragma unroll
      for (int q = 0; q < FT_TW; ++q) {
        const int p = wave + 4 * q;
        if (p < tiles) {
          const int lt = p / ct, cs = p % ct;
#pragma unroll
          for (int t = 0; t < FT_ROWS / 4; ++t) {
            const int k = 4 * t + lg;
            const double a = (double)Fs[k * FS + lt * 16 + li];
            const double b = (double)Rs[k * RS + cs * 16 + li];
            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < FT_TW; ++q) {
      const int p = wave + 4 * q;
      if (p < tiles) {
        const int lt = p / ct, cs = p % ct;
        const int c = cs * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int l = lbase + lt * 16 + lg + 4 * r;
          if (l < I.rank && l - lbase < lw && c < s) out[(int64_t)l * s + c] = acc[q][r];
        }
      }
    }
    __syncthreads();
  }
}

// t_i = sum of the instance's chunk partials (rank_i x s at i * lmax * s);
// grid (instances, lmax * s / 64): workgroup (i, y) sums elements 64 y ..
// 64 y + 63, one per thread
__global__ __launch_bounds__(64) void k_bft_sum(const BInst* __restrict__ inst, int s, int lmax,
                                                const double* __restrict__ part,
                                                double* __restrict__ t,
                                                const int* __restrict__ iact) {
  if (iact && !iact[blockIdx.x]) return;
  const BInst I = inst[blockIdx.x];
  const int64_t cnt = (int64_t)I.rank * s;
  const int64_t cs = (int64_t)lmax * s;  // stride between chunks
  const int64_t e = (int64_t)blockIdx.y * 64 + threadIdx.x;
  if (e < cnt) {
    const double* src = part + (int64_t)I.ch0 * cs + e;
    double v = 0.0;
    int g = 0;
    // in chunk order, eight chunks' loads issued together
    for (; g + 8 <= I.nch; g += 8) {
      double x[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) x[j] = src[(int64_t)(g + j) * cs];
#pragma unroll
      for (int j = 0; j < 8; ++j) v += x[j];
    }
    for (; g < I.nch; ++g) v += src[(int64_t)g * cs];
    t[(int64_t)blockIdx.x * lmax * s + e] = v;
  }
}

// OUT = Dinv R - F t on one 64-row block (wave w: rows 16 w .. 16 w + 15) on
// FP64 matrix cores over stages of 32 rank indices; dots dot1 = R .* OUT and
// dot2 = Z .* R per column (s <= 64).  F goes straight into the matrix-core
// registers: in stage k0, lane (i, g) = (lane % 16, lane / 16) holds
// F[row i][k0 + 16 h + 4 g + e], h < 2, e < 4 (two 16-byte loads; the four
// lanes of a row read 64 consecutive bytes), fetched two stages ahead, and
// step 4 h + e pairs it with t[k0 + 16 h + 4 g + e][c].  The t stage (32 x
// 64, zero past the instance's rank) is kept k-contiguous per column in a
// double-buffered LDS tile, loaded one stage ahead, one barrier per stage.
// F's rows hold ldf (a multiple of 16) values; those at or past the rank
// enter as zero.
constexpr int BTK = 32 + 2;  // LDS stride (doubles) of a column of the t stage
template <int CT>  // 16-column tiles of the output (ceil(s / 16))
__global__ __launch_bounds__(256) void k_bwout(const BInst* __restrict__ inst,
                                               const int* __restrict__ blk_inst,
                                               const float* __restrict__ F, int ldf,
                                               const float* __restrict__ Dinv,
                                               const double* __restrict__ t, int lmax,
                                               const float* __restrict__ R, int s,
                                               float* __restrict__ OUT, const float* __restrict__ Z,
                                               double* __restrict__ dot1, double* __restrict__ dot2,
                                               const int* __restrict__ iact) {
  typedef double f64x2 __attribute__((ext_vector_type(2)));
  __shared__ __attribute__((aligned(16))) union {
    double Tt[2][64 * BTK];
    struct {
      double r1[4][64][4];
      double r2[4][64][4];
    } rd;
  } lds;
  auto& red1 = lds.rd.r1;
  auto& red2 = lds.rd.r2;
  const int ii = blk_inst[blockIdx.x];
  if (iact && !iact[ii]) return;
  const BInst I = inst[ii];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t b0 = (int64_t)blockIdx.x * 64;
  const int64_t nrow = I.row0 + I.n;  // rows at or past nrow are padding
  const double* tin = t + (int64_t)ii * lmax * s;
  const int rank = I.rank;
  const int nst = (rank + 31) / 32;
  const int64_t arow = b0 + 16 * wave + li;  // the row this lane feeds as A operand
  const bool av_ok = arow < nrow;
  const float* frow = F + arow * (int64_t)ldf;
  f64x4 acc[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};

  auto load_a = [&](int st, float (&a)[8]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = 32 * st + 16 * h + 4 * lg;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (av_ok && 32 * st + 16 * h < ldf) v = *(const float4*)(frow + k);
      a[4 * h + 0] = k + 0 < rank ? v.x : 0.f;
      a[4 * h + 1] = k + 1 < rank ? v.y : 0.f;
      a[4 * h + 2] = k + 2 < rank ? v.z : 0.f;
      a[4 * h + 3] = k + 3 < rank ? v.w : 0.f;
    }
  };
  // t stage: thread column tid % 64, rank indices 8 (tid / 64) + j
  double tq[8];
  auto load_t = [&](int st) {
    const int k = 32 * st + 8 * (tid / 64);
    const int col = tid % 64;
#pragma unroll
    for (int j = 0; j < 8; ++j) tq[j] = (k + j < rank && col < s) ? tin[(int64_t)(k + j) * s + col] : 0.0;
  };
  auto store_t = [&](double* tt) {
    f64x2* dst = (f64x2*)&tt[(tid % 64) * BTK + 8 * (tid / 64)];
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = f64x2{tq[2 * q], tq[2 * q + 1]};
  };

  if (nst > 0) {
    float a[2][8];
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
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            double b[CT][4];
#pragma unroll
            for (int c = 0; c < CT; ++c) {
              const f64x2* bp = (const f64x2*)&tt[(c * 16 + li) * BTK + 16 * h + 4 * lg];
              const f64x2 v0 = bp[0], v1 = bp[1];
              b[c][0] = v0.x;
              b[c][1] = v0.y;
              b[c][2] = v1.x;
              b[c][3] = v1.y;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
              for (int c = 0; c < CT; ++c)
                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a[d][4 * h + e], b[c][e],
                                                              acc[c], 0, 0, 0);
          }
          if (cur + 2 < nst) load_a(cur + 2, a[d]);
          __syncthreads();
        }
      }
    }
  }
  double d1[4] = {0.0, 0.0, 0.0, 0.0}, d2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const int cc = c * 16 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = b0 + 16 * wave + lg + 4 * r;
      if (cc >= s) continue;
      const int64_t off = row * s + cc;
      if (row >= nrow) {
        OUT[off] = 0.f;
        continue;
      }
      const double rv = (double)R[off];
      const float o = (float)((double)Dinv[row] * rv - acc[c][r]);
      OUT[off] = o;
      d1[c] += rv * (double)o;
      d2[c] += (double)Z[off] * rv;
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    red1[wave][lane][c] = d1[c];
    red2[wave][lane][c] = d2[c];
  }
  __syncthreads();
  if (threadIdx.x < s) {
    const int c = threadIdx.x / 16, l16 = threadIdx.x % 16;
    double a = 0.0, b = 0.0;
    for (int w = 0; w < 4; ++w)
      for (int g = 0; g < 4; ++g) {
        a += red1[w][l16 + 16 * g][c];
        b += red2[w][l16 + 16 * g][c];
      }
    dot1[blockIdx.x * (int64_t)s + threadIdx.x] = a;
    dot2[blockIdx.x * (int64_t)s + threadIdx.x] = b;
  }
}

// out[i * s + c] = sum of parts[b][c] over the 64-row blocks of instance i
__global__ __launch_bounds__(256) void k_bsegsum(const BInst* __restrict__ inst, int s,
                                                 const double* __restrict__ parts,
                                                 double* __restrict__ out) {
  __shared__ double red[256];
  const BInst I = inst[blockIdx.x];
  const int groups = 256 / s;
  const int c = threadIdx.x % s, q = threadIdx.x / s;
  const int64_t b0 = I.row0 / BLK, nb = (I.n + BLK - 1) / BLK;
  double acc = 0.0;
  if (q < groups)
    for (int64_t b = q; b < nb; b += groups) acc += parts[(b0 + b) * s + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < s) {
    double t = 0.0;
    for (int g = 0; g < groups; ++g) t += red[g * s + threadIdx.x];
    out[(int64_t)blockIdx.x * s + threadIdx.x] = t;
  }
}

// Vector updates over the whole batch; padding rows are left at zero.
__global__ void k_bupdate_r(const BInst* __restrict__ inst, const int* __restrict__ blk_inst,
                            int64_t R, int s, float* __restrict__ r, const float* __restrict__ q,
                            const double* __restrict__ alpha, const int* __restrict__ iact) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < R * s;
       e += (int64_t)gridDim.x * 256) {
    const int64_t row = e / s;
    const int c = (int)(e % s);
    const int ii = blk_inst[row / BLK];
    // a converged instance has alpha = 0 in every column: r is unchanged
    if (!iact[ii] || row - inst[ii].row0 >= inst[ii].n) continue;
    const double a = alpha[(int64_t)ii * s + c];
    r[e] = (float)((double)r[e] - a * (double)q[e]);
  }
}

__global__ void k_bupdate_pw(const BInst* __restrict__ inst, const int* __restrict__ blk_inst,
                             int64_t R, int s, float* __restrict__ p, float* __restrict__ w,
                             const float* __restrict__ r, const float* __restrict__ u,
                             const double* __restrict__ beta, const int* __restrict__ active,
                             const int* __restrict__ iact) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < R * s;
       e += (int64_t)gridDim.x * 256) {
    const int64_t row = e / s;
    const int c = (int)(e % s);
    const int ii = blk_inst[row / BLK];
    // iact (from the start of the iteration) is 0 only when every column of
    // the instance was already inactive
    if (!iact[ii] || row - inst[ii].row0 >= inst[ii].n) continue;
    const int64_t g = (int64_t)ii * s + c;
    if (!active[g]) continue;
    const double b = beta[g];
    p[e] = (float)((double)r[e] + b * (double)p[e]);
    w[e] = (float)((double)u[e] + b * (double)w[e]);
  }
}

// Hutchinson combination of every instance on the device, in FP64: per probe
// t_c = b z^T z + sum_j c_j z^T x_j (the estimator's output, Algorithm 1),
// then the instance's mean, standard error (sample deviation over sqrt(s)),
// largest P^-1 residual ratio of its seed systems and converged count.  One
// workgroup of 64 threads per instance (s <= 64), sums in probe order.
struct BCoef {
  double b;
  double c[kMaxShifts];
  int J;
};
__global__ __launch_bounds__(64) void k_bhutchinson(int s, int64_t ncol, BCoef cf,
                                                    const double* __restrict__ ztx,
                                                    const double* __restrict__ ztz,
                                                    const double* __restrict__ rho,
                                                    const double* __restrict__ rho0, double tol,
                                                    double* __restrict__ per_probe,
                                                    double* __restrict__ stats) {
  __shared__ double tt[64], rr[64];
  const int i = blockIdx.x, c = threadIdx.x;
  if (c < s) {
    const int64_t g = (int64_t)i * s + c;
    double v = cf.b * ztz[g];
    for (int j = 0; j < cf.J; ++j) v += cf.c[j] * ztx[(int64_t)j * ncol + g];
    tt[c] = v;
    rr[c] = sqrt(fmax(0.0, rho[g] / rho0[g]));
    per_probe[g] = v;
  }
  __syncthreads();
  if (c == 0) {
    double mean = 0.0, worst = 0.0, conv = 0.0;
    for (int q = 0; q < s; ++q) {
      mean += tt[q];
      worst = fmax(worst, rr[q]);
      if (rr[q] <= tol) conv += 1.0;
    }
    mean /= s;
    double var = 0.0;
    for (int q = 0; q < s; ++q) var += (tt[q] - mean) * (tt[q] - mean);
    stats[4 * i + 0] = mean;
    stats[4 * i + 1] = s > 1 ? sqrt(var / (s - 1) / s) : (double)NAN;
    stats[4 * i + 2] = worst;
    stats[4 * i + 3] = conv;
  }
}

// iact[i] = 1 while any probe column of instance i is still active
__global__ void k_binst_active(int B, int s, const int* __restrict__ active, int* __restrict__ iact) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < B; i += gridDim.x * 256) {
    int a = 0;
    for (int c = 0; c < s; ++c) a |= active[(int64_t)i * s + c];
    iact[i] = a;
  }
}

// Instrumentation: algorithmic work of the next product launch (instances
// with an active probe): acc[0] += sum 2 n_i^2 s flops, acc[1] += bytes of
// V and X2 read and Y written (FP32) plus the points.  One workgroup.
__global__ __launch_bounds__(256) void k_bwork(const BInst* __restrict__ inst,
                                               const int* __restrict__ iact, int B, int s,
                                               double* __restrict__ acc) {
  __shared__ double rf[256], rb[256];
  double f = 0.0, by = 0.0;
  for (int i = threadIdx.x; i < B; i += 256)
    if (iact[i]) {
      const double n = (double)inst[i].n;
      f += 2.0 * n * n * s;
      by += 4.0 * n * (3.0 * s + BDX);
    }
  rf[threadIdx.x] = f;
  rb[threadIdx.x] = by;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rf[threadIdx.x] += rf[threadIdx.x + w];
      rb[threadIdx.x] += rb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    acc[0] += rf[0];
    acc[1] += rb[0];
  }
}

__global__ void k_bcopy2(const float* __restrict__ src, float* __restrict__ a,
                         float* __restrict__ b, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    const float v = src[i];
    a[i] = v;
    if (b) b[i] = v;
  }
}

int grid1(int64_t count) {
  int64_t b = (count + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

// ------------------------------------------------------------------ host --
struct Batch {
  int B = 0;
  int s = 0;
  int64_t R = 0;       // padded rows
  int64_t nblk = 0;    // 64-row blocks
  int mmax = 0;        // max m (rank + oversample)
  int lmax = 0;        // max rank
  int64_t gstride = 0; // mmax^2
  std::vector<BInst> h;
  BInst* d_inst = nullptr;
  int* d_blk_inst = nullptr;
  float* X32 = nullptr;
  int2* d_gitems = nullptr;  // Gram work items (instance, GCH-row chunk)
  int ngitems = 0;
  double* gpart = nullptr;   // Gram partials of the instances of several chunks
};

// grid rows of k_bgram_sum (mmax^2 elements per instance)
unsigned gsum_rows(const Batch& b) { return (unsigned)((b.gstride + 255) / 256); }

// Work items of the batched product, longest instances first.
std::vector<BItem> make_items(const Batch& b, int bmw, int ncols, int nt) {
  std::vector<int> order(b.B);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b.h[x].n > b.h[y].n; });
  std::vector<BItem> items;
  const int cbs = (ncols + nt - 1) / nt;
  for (int i : order) {
    const int rbs = (int)((b.h[i].n + bmw - 1) / bmw);
    for (int rb = 0; rb < rbs; ++rb)
      for (int cb = 0; cb < cbs; ++cb) items.push_back(BItem{i, rb, cb, 0});
  }
  return items;
}

struct ProductPlan {
  BItem* d_items = nullptr;
  int count = 0;
  int waves = 4;  // 4 waves x 128 rows or 2 waves x 64 rows per workgroup
  int mf = 32;    // matrix-core shape (32: 32x32x2, 16: 16x16x4)
  int nb = 1;     // column sub-blocks: NT = mf * nb columns per workgroup
  // the symmetric form (k_bmm_sym + k_bsym_reduce; up to 16 columns)
  bool sym = false;
  BSym* d_sym = nullptr;
  BSItem* d_sitems = nullptr;  // (instance, strip, row tiles), most blocks first
  BRItem* d_ritems = nullptr;  // (instance, row tile)
  int nsitems = 0, nritems = 0;
  float* part = nullptr;
};

// the symmetric form's slots and work items for the batch's instances:
// direct slots of every instance first, then the transposed slots (SMS per
// item, an instance's items in strip order and, within a strip, in row order)
struct SymLayout {
  std::vector<BSym> sym;
  std::vector<BSItem> items;
  std::vector<BRItem> ritems;
  int64_t slots = 0;
};
SymLayout sym_layout(const Batch& b) {
  SymLayout L;
  int64_t dir = 0;
  for (int i = 0; i < b.B; ++i) {
    BSym q{};
    q.nblk = (int)((b.h[i].n + SBB - 1) / SBB);
    q.ns = (q.nblk + SMS - 1) / SMS;
    q.dir = dir;
    dir += bsym_dir_base(q.ns, q.nblk);  // one slot per (strip, row tile) unit
    L.sym.push_back(q);
  }
  std::vector<std::pair<int64_t, BSItem>> cost;
  int64_t tr = dir;
  for (int i = 0; i < b.B; ++i) {
    const BSym& q = L.sym[i];
    std::vector<int64_t> first(q.ns);  // first transposed slot of each strip
    for (int S = 0; S < q.ns; ++S) {
      const int mS = SMS * S, me = std::min(mS + SMS, q.nblk);
      first[S] = tr;
      for (int i0 = 0; i0 < me; i0 += SCH) {
        const int i1 = std::min(i0 + SCH, me);
        int64_t c = 0;  // blocks the item runs
        for (int I0 = i0; I0 < i1; ++I0) c += me - std::max(I0, mS);
        cost.push_back({c, BSItem{i, S, i0, i1, tr}});
        tr += SMS;
      }
    }
    // row tile R takes the items of its strip that hold rows above it
    for (int R = 0; R < q.nblk; ++R) {
      const int SR = R / SMS;
      L.ritems.push_back(BRItem{i, R, (R + SCH - 1) / SCH, first[SR] + (R - SMS * SR)});
    }
  }
  L.slots = tr;
  std::stable_sort(cost.begin(), cost.end(),
                   [](const auto& x, const auto& y) { return x.first > y.first; });
  for (const auto& c : cost) L.items.push_back(c.second);
  return L;
}

size_t sym_scratch_bytes(const Batch& b) {
  const SymLayout L = sym_layout(b);
  return L.sym.size() * sizeof(BSym) + L.items.size() * sizeof(BSItem) +
         L.ritems.size() * sizeof(BRItem) + (size_t)L.slots * STILE * sizeof(float) + 4 * 256;
}

// The product tile shapes the autotuner times for ncols columns: matrix-core
// shape (16x16x4 or 32x32x2), column sub-blocks and waves per workgroup (4
// waves: 128 rows, 2 waves: 64 rows, which doubles the work items and evens
// out the tail of small instances).  Every candidate covers ncols (at most
// 224 columns per block; wider products repeat the block).
struct Shape {
  int mf, nb, waves;
};
std::vector<Shape> product_shapes(int ncols) {
  if (ncols <= 16) return {{16, 1, 4}, {16, 1, 2}, {32, 1, 4}, {32, 1, 2}};
  if (ncols <= 32) return {{32, 1, 4}, {32, 1, 2}, {32, 2, 4}, {32, 2, 2}};
  if (ncols <= 64) return {{32, 2, 4}, {32, 2, 2}, {32, 4, 4}};
  if (ncols <= 128) return {{32, 4, 4}, {32, 7, 4}};
  return {{32, 7, 4}};
}

// the symmetric form is the plan after the tile shapes; it serves products
// of up to 16 columns unless the tile shapes are asked for (the autotuner
// does not time it: its first launch, every instance active, does not show
// the late launches where only the large instances remain)
bool sym_form(int ncols, int flags) { return !(flags & LD_BATCH_NO_SYMMETRIC) && ncols <= 16; }

ld_status plan_product(ld_ctx* ctx, const Batch& b, int ncols, int variant, ProductPlan* pp) {
  const std::vector<Shape> shapes = product_shapes(ncols);
  if (ncols <= 16 && variant == (int)shapes.size()) {
    const SymLayout L = sym_layout(b);
    pp->sym = true;
    pp->d_sym = (BSym*)ctx->arena.take(L.sym.size() * sizeof(BSym));
    pp->d_sitems = (BSItem*)ctx->arena.take(L.items.size() * sizeof(BSItem));
    pp->d_ritems = (BRItem*)ctx->arena.take(L.ritems.size() * sizeof(BRItem));
    pp->part = (float*)ctx->arena.take((size_t)L.slots * STILE * sizeof(float));
    if (!pp->d_sym || !pp->d_sitems || !pp->d_ritems || !pp->part)
      return fail(LD_ENOMEM, "batch: scratch arena too small for the symmetric product");
    LD_HIP(hipMemcpyAsync(pp->d_sym, L.sym.data(), L.sym.size() * sizeof(BSym),
                          hipMemcpyHostToDevice, ctx->stream));
    LD_HIP(hipMemcpyAsync(pp->d_sitems, L.items.data(), L.items.size() * sizeof(BSItem),
                          hipMemcpyHostToDevice, ctx->stream));
    LD_HIP(hipMemcpyAsync(pp->d_ritems, L.ritems.data(), L.ritems.size() * sizeof(BRItem),
                          hipMemcpyHostToDevice, ctx->stream));
    LD_HIP(hipStreamSynchronize(ctx->stream));  // the host vectors are released on return
    pp->nsitems = (int)L.items.size();
    pp->nritems = (int)L.ritems.size();
    return LD_OK;
  }
  const Shape sh = shapes[variant < (int)shapes.size() ? variant : 0];
  const int mf = sh.mf, nb = sh.nb, waves = sh.waves;
  std::vector<BItem> items = make_items(b, 32 * waves, ncols, mf * nb);
  pp->d_items = (BItem*)ctx->arena.take(items.size() * sizeof(BItem));
  if (!pp->d_items) return fail(LD_ENOMEM, "batch: scratch arena too small for work items");
  LD_HIP(hipMemcpyAsync(pp->d_items, items.data(), items.size() * sizeof(BItem),
                        hipMemcpyHostToDevice, ctx->stream));
  LD_HIP(hipStreamSynchronize(ctx->stream));  // `items` is released on return
  pp->count = (int)items.size();
  pp->waves = waves;
  pp->mf = mf;
  pp->nb = nb;
  return LD_OK;
}

void launch_product(hipStream_t st, const Batch& b, const ProductPlan& pp, const float* V, int ld,
                    float* Y, const float* X2, float alpha2, double* dots, const int* iact) {
  if (pp.sym) {
    hipLaunchKernelGGL(k_bmm_sym, dim3(pp.nsitems), dim3(256), 0, st, b.d_inst, pp.d_sym,
                       pp.d_sitems, b.X32, V, ld, pp.part, iact);
    hipLaunchKernelGGL(k_bsym_reduce, dim3(pp.nritems), dim3(256), 0, st, b.d_inst, pp.d_sym,
                       pp.d_ritems, pp.part, V, ld, Y, X2, alpha2, dots, iact);
    return;
  }
  const dim3 g(pp.count);
#define LD_BMM_LAUNCH(MF, NB, W)                                                               \
  hipLaunchKernelGGL((k_bmm<MF, NB, W>), g, dim3(64 * W), 0, st, b.d_inst, pp.d_items, b.X32, V, \
                     ld, Y, X2, alpha2, dots, iact)
  const bool w4 = pp.waves == 4;
  if (pp.mf == 16) {
    if (w4) LD_BMM_LAUNCH(16, 1, 4); else LD_BMM_LAUNCH(16, 1, 2);
  } else if (pp.nb == 1) {
    if (w4) LD_BMM_LAUNCH(32, 1, 4); else LD_BMM_LAUNCH(32, 1, 2);
  } else if (pp.nb == 2) {
    if (w4) LD_BMM_LAUNCH(32, 2, 4); else LD_BMM_LAUNCH(32, 2, 2);
  } else if (pp.nb == 4) {
    LD_BMM_LAUNCH(32, 4, 4);
  } else {
    LD_BMM_LAUNCH(32, 7, 4);
  }
  // (plan_product only produces the shapes above: product_shapes)
#undef LD_BMM_LAUNCH
}

}  // namespace

// ------------------------------------------------------------------ driver --
namespace {

struct Bufs {
  double *Q, *Y, *G, *Rinv, *evecs, *evals, *jwork, *U, *F64, *D, *Dinv64, *ldP;
  float *V32, *Y32, *F32, *Dinv32;
  int *fail, *jstat;
};

ld_status read_ints(ld_ctx* ctx, hipStream_t st, const int* d, int count, std::vector<int>& h) {
  LD_TRY(ensure_pinned(ctx, (size_t)count / 2 + 8));
  LD_HIP(hipMemcpyAsync(ctx->pinned, d, (size_t)count * sizeof(int), hipMemcpyDeviceToHost, st));
  LD_HIP(hipStreamSynchronize(st));
  h.assign((const int*)ctx->pinned, (const int*)ctx->pinned + count);
  return LD_OK;
}

dim3 gemm_grid(const Batch& b, int ncols) {
  int64_t maxrows = 0;
  for (const BInst& I : b.h) maxrows = std::max(maxrows, I.n);
  return dim3((unsigned)((maxrows + dev::GM_BM - 1) / dev::GM_BM),
              (unsigned)((ncols + dev::GM_BN - 1) / dev::GM_BN), (unsigned)b.B);
}

// Orthonormal basis of range(Y_i) for every instance: shifted CholeskyQR on
// the first pass, plain passes after it.  The basis ends in *Q (Y or W).
void b_orth(hipStream_t st, const Batch& b, Bufs& f, double* Y, double* W, int passes,
            double** Q) {
  const int tiles = (b.mmax + 63) / 64;
  double* src = Y;
  double* dst = W;
  for (int pass = 0; pass < passes; ++pass) {
    hipLaunchKernelGGL(k_bgram, dim3(tiles, tiles, b.ngitems), dim3(256), 0, st, b.d_inst, b.d_gitems,
                       0, src, b.mmax, src, b.mmax, (const double*)nullptr, f.G, b.gpart,
                       b.gstride, 1);
    hipLaunchKernelGGL(k_bgram_sum, dim3(b.B, gsum_rows(b)), dim3(256), 0, st, b.d_inst, 0, b.gpart, f.G,
                       b.gstride);
    if (pass == 0)
      hipLaunchKernelGGL(k_bshift, dim3(b.B), dim3(256), 0, st, b.d_inst, f.G, b.gstride);
    hipLaunchKernelGGL(k_bchol, dim3(b.B), dim3(dev::CT), 0, st, b.d_inst, 0, f.G, b.gstride,
                       f.fail);
    hipLaunchKernelGGL(k_btrinv, dim3(b.B), dim3(dev::CT), 0, st, b.d_inst, 0, f.G, f.Rinv,
                       b.gstride);
    hipLaunchKernelGGL(k_bgemm, gemm_grid(b, b.mmax), dim3(256), 0, st, b.d_inst, 0, 0, src,
                       b.mmax, f.Rinv, b.gstride, 1, (const double*)nullptr, dst, b.mmax);
    std::swap(src, dst);
  }
  *Q = src;
}

// Y64 = M Q64 for every instance through the FP32 batched product
void b_apply(hipStream_t st, const Batch& b, Bufs& f, const ProductPlan& pp, const double* Qin,
             double* Yout) {
  const int64_t cnt = b.R * b.mmax;
  launch_convert_f64_to_f32(st, Qin, f.V32, cnt);
  launch_product(st, b, pp, f.V32, b.mmax, f.Y32, nullptr, 0.f, nullptr, nullptr);
  launch_convert_f32_to_f64(st, f.Y32, Yout, cnt);
}

ld_status with_stream(ld_ctx* ctx, hipStream_t st, const Batch& b, int ncols, int variant,
                      ProductPlan* pp) {
  const hipStream_t keep = ctx->stream;
  ctx->stream = st;
  const ld_status r = plan_product(ctx, b, ncols, variant, pp);
  ctx->stream = keep;
  return r;
}

}  // namespace

ld_status batched_estimate(ld_ctx* ctx, int count, const ld_instance* in, int J,
                           const double* shifts, double bcoef, const double* ccoef, int s,
                           int oversample, int power_iters, double tol, int max_iters, int flags,
                           ld_result* out, double* per_probe, double* lambda_out,
                           int lambda_stride) {
  // ---- layout: instance i owns padded rows [row0_i, row0_i + ceil(n_i/128)*128)
  Batch b;
  b.B = count;
  b.s = s;
  int64_t row0 = 0;
  int nchunks = 0;
  int ngpart = 0;  // Gram partial slots
  for (int i = 0; i < count; ++i) {
    const ld_instance& x = in[i];
    BInst I{};
    I.X64 = x.X;
    I.n = x.n;
    I.row0 = row0;
    I.d = x.d;
    I.kind = x.kind;
    I.rank = x.rank;
    I.m = x.rank + oversample;
    I.ch0 = nchunks;
    I.nch = (int)((x.n + FTC - 1) / FTC);
    nchunks += I.nch;
    I.gnch = (int)((x.n + GCH - 1) / GCH);
    I.gp0 = ngpart;
    if (I.gnch > 1) ngpart += I.gnch;
    // points pre-scaled so that r2 is the base-2 exponent (RBF) or its
    // square root is (Matern): kval32s
    const double l2e = 1.4426950408889634;
    I.pscale = x.kind == LD_RBF ? std::sqrt(l2e / (2.0 * x.lengthscale * x.lengthscale))
                                : 2.23606797749978969640917366873128 * l2e / x.lengthscale;
    I.kv = (float)(x.kind == LD_RBF ? std::log2(x.variance) : x.variance);
    I.noise = (float)x.noise;
    I.diag = x.variance + x.noise;
    I.floor_v = x.noise > 0.0 ? x.noise : 1e-12 * x.variance;
    I.shift_c = 11.0 * ((double)x.n * I.m + (double)I.m * (I.m + 1)) * 0x1.0p-53;
    I.key_omega = stream_key(x.precond_seed, kStreamOmega);
    I.key_probe = stream_key(x.probe_seed, kStreamProbes);
    b.h.push_back(I);
    row0 += (x.n + BROWS - 1) / BROWS * BROWS;
    b.mmax = std::max(b.mmax, I.m);
    b.lmax = std::max(b.lmax, I.rank);
  }
  b.R = row0;
  b.lmax = (b.lmax + 15) / 16 * 16;  // 16-byte aligned rows of U and F
  b.nblk = b.R / BLK;
  b.gstride = (int64_t)b.mmax * b.mmax;
  std::vector<int> blk_inst(b.nblk), ch_inst(nchunks);
  std::vector<int2> gitems;  // Gram work items (instance, chunk), largest instances first
  for (int i = 0; i < count; ++i) {
    const int64_t first = b.h[i].row0 / BLK, nb = (b.h[i].n + BROWS - 1) / BROWS * (BROWS / BLK);
    for (int64_t q = 0; q < nb; ++q) blk_inst[first + q] = i;
    for (int g = 0; g < b.h[i].nch; ++g) ch_inst[b.h[i].ch0 + g] = i;
  }
  {
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b.h[x].n > b.h[y].n; });
    for (int i : order)
      for (int g = 0; g < b.h[i].gnch; ++g) gitems.push_back(make_int2(i, g));
  }
  const int ngitems = (int)gitems.size();
  b.ngitems = ngitems;
  const int64_t R = b.R, B = count;
  const int64_t ncol = B * s;
  const int cbs = (b.mmax + 63) / 64;

  // ---- scratch (one reservation; every buffer below is carved from it)
  size_t need = 0;
  auto add = [&](size_t bytes) { need += ((bytes + 255) & ~(size_t)255) + 256; };
  add(B * sizeof(BInst));
  add(b.nblk * sizeof(int));
  add(nchunks * sizeof(int));
  add(ngitems * sizeof(int2));
  add((size_t)ngpart * b.gstride * 8);
  add(R * BDX * 4);
  add(R * b.mmax * 8);
  add(R * b.mmax * 8);
  add(R * b.mmax * 4);
  add(R * b.mmax * 4);
  for (int q = 0; q < 3; ++q) add(B * b.gstride * 8);
  add(B * b.mmax * 8);
  add(B * 2 * (int64_t)b.mmax * b.mmax * 8);
  add(B * 4);
  add(B * 4);
  add(R * b.lmax * 8);
  add(R * b.lmax * 8);
  add(R * b.lmax * 4);
  add(R * 8);
  add(R * 8);
  add(R * 4);
  add(B * 8);
  for (int q = 0; q < 6; ++q) add(R * s * 4);
  for (int q = 0; q < 3; ++q) add(b.nblk * s * 8);
  for (int q = 0; q < 3; ++q) add(ncol * 8);
  add(B * b.lmax * s * 8);
  add((size_t)nchunks * b.lmax * s * 8);
  add((size_t)(7 * ncol + 4 * J * ncol + J) * 8);
  add((size_t)(J * ncol + ncol + 2) * 4);
  add(B * 4);
  add(2 * 8);
  add((size_t)(ncol + 4 * B) * 8);
  add(b.nblk * (size_t)cbs * sizeof(BItem));  // product work items: sketch
  // solver: the autotuner's candidate shapes (at most four, each at most
  // one item per 64-row block and 16 columns)
  for (int q = 0; q < 4; ++q) add(b.nblk * (size_t)((s + 15) / 16) * sizeof(BItem));
  if (sym_form(s, flags)) add(sym_scratch_bytes(b));
  ctx->arena.reset();
  LD_TRY(ctx->arena.reserve(need));
  Arena& ar = ctx->arena;
  auto tk = [&](size_t bytes) { return ar.take(bytes); };
  b.d_inst = (BInst*)tk(B * sizeof(BInst));
  b.d_blk_inst = (int*)tk(b.nblk * sizeof(int));
  int* d_ch_inst = (int*)tk(nchunks * sizeof(int));
  b.d_gitems = (int2*)tk(ngitems * sizeof(int2));
  b.gpart = (double*)tk((size_t)ngpart * b.gstride * 8);
  b.X32 = (float*)tk(R * BDX * 4);
  Bufs f{};
  f.Q = (double*)tk(R * b.mmax * 8);
  f.Y = (double*)tk(R * b.mmax * 8);
  f.V32 = (float*)tk(R * b.mmax * 4);
  f.Y32 = (float*)tk(R * b.mmax * 4);
  f.G = (double*)tk(B * b.gstride * 8);
  f.Rinv = (double*)tk(B * b.gstride * 8);
  f.evecs = (double*)tk(B * b.gstride * 8);
  f.evals = (double*)tk(B * b.mmax * 8);
  f.jwork = (double*)tk(B * 2 * (int64_t)b.mmax * b.mmax * 8);
  f.fail = (int*)tk(B * 4);
  f.jstat = (int*)tk(B * 4);
  f.U = (double*)tk(R * b.lmax * 8);
  f.F64 = (double*)tk(R * b.lmax * 8);
  f.F32 = (float*)tk(R * b.lmax * 4);
  f.D = (double*)tk(R * 8);
  f.Dinv64 = (double*)tk(R * 8);
  f.Dinv32 = (float*)tk(R * 4);
  f.ldP = (double*)tk(B * 8);
  float* Z = (float*)tk(R * s * 4);
  float* r = (float*)tk(R * s * 4);
  float* u = (float*)tk(R * s * 4);
  float* p = (float*)tk(R * s * 4);
  float* w = (float*)tk(R * s * 4);
  float* q = (float*)tk(R * s * 4);
  double* dwq = (double*)tk(b.nblk * s * 8);
  double* d1 = (double*)tk(b.nblk * s * 8);
  double* d2 = (double*)tk(b.nblk * s * 8);
  double* sg1 = (double*)tk(ncol * 8);
  double* sg2 = (double*)tk(ncol * 8);
  double* sgw = (double*)tk(ncol * 8);
  double* tl = (double*)tk(B * b.lmax * s * 8);
  double* tpart = (double*)tk((size_t)nchunks * b.lmax * s * 8);
  double* scal = (double*)tk((size_t)(7 * ncol + 4 * J * ncol + J) * 8);
  int* iscal = (int*)tk((size_t)(J * ncol + ncol + 2) * 4);
  int* iact = (int*)tk(B * 4);
  double* tacc = (double*)tk(2 * 8);
  double* hut = (double*)tk((size_t)(ncol + 4 * count) * 8);  // per-probe values, statistics
  if (!tacc) return fail(LD_ENOMEM, "batch: scratch arena too small");

  // the graph form runs on a side stream that joins the context stream
  const bool use_graph = (flags & LD_BATCH_GRAPH) != 0;
  hipStream_t st = ctx->stream;
  if (use_graph) {
    if (!ctx->side) LD_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    if (!ctx->ev_join) LD_HIP(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    LD_HIP(hipEventRecord(ctx->ev_join, ctx->stream));
    LD_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_join, 0));
    st = ctx->side;
  }
  // On any return after this point the side stream is joined back first.
  auto join = [&]() {
    if (use_graph && hipEventRecord(ctx->ev_join, st) == hipSuccess)
      (void)hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0);
  };
  struct Joiner {
    std::function<void()> fn;
    ~Joiner() { fn(); }
  } joiner{join};

  const auto t0 = std::chrono::steady_clock::now();
  LD_HIP(hipMemcpyAsync(b.d_inst, b.h.data(), B * sizeof(BInst), hipMemcpyHostToDevice, st));
  LD_HIP(hipMemcpyAsync(b.d_blk_inst, blk_inst.data(), b.nblk * sizeof(int), hipMemcpyHostToDevice, st));
  LD_HIP(hipMemcpyAsync(d_ch_inst, ch_inst.data(), nchunks * sizeof(int), hipMemcpyHostToDevice, st));
  LD_HIP(hipMemcpyAsync(b.d_gitems, gitems.data(), ngitems * sizeof(int2), hipMemcpyHostToDevice, st));
  LD_HIP(hipMemsetAsync(f.fail, 0, B * 4, st));
  LD_HIP(hipMemsetAsync(f.jstat, 0, B * 4, st));
  hipLaunchKernelGGL(k_bx32, dim3(grid1(R * BDX)), dim3(256), 0, st, b.d_inst, b.d_blk_inst, R, b.X32);

  // ---- preconditioners (range finder, Rayleigh-Ritz, Woodbury factors)
  ProductPlan sketch;
  LD_TRY(with_stream(ctx, st, b, b.mmax, 0, &sketch));
  hipLaunchKernelGGL(k_bomega, dim3(grid1(R * b.mmax)), dim3(256), 0, st, b.d_inst, b.d_blk_inst, R,
                     b.mmax, f.Q);
  b_apply(st, b, f, sketch, f.Q, f.Y);
  double* Qb = nullptr;
  b_orth(st, b, f, f.Y, f.Q, power_iters == 0 ? 3 : 2, &Qb);
  for (int it = 0; it < power_iters; ++it) {
    double* other = Qb == f.Q ? f.Y : f.Q;
    b_apply(st, b, f, sketch, Qb, other);
    b_orth(st, b, f, other, Qb, it + 1 == power_iters ? 3 : 2, &Qb);
  }
  double* MQ = Qb == f.Q ? f.Y : f.Q;
  b_apply(st, b, f, sketch, Qb, MQ);
  const int tiles = (b.mmax + 63) / 64;
  hipLaunchKernelGGL(k_bgram, dim3(tiles, tiles, b.ngitems), dim3(256), 0, st, b.d_inst, b.d_gitems, 0,
                     Qb, b.mmax, MQ, b.mmax, (const double*)nullptr, f.G, b.gpart, b.gstride, 0);
  hipLaunchKernelGGL(k_bgram_sum, dim3(B, gsum_rows(b)), dim3(256), 0, st, b.d_inst, 0, b.gpart, f.G,
                     b.gstride);
  hipLaunchKernelGGL(k_beigh, dim3(B), dim3(1024), 0, st, b.d_inst, f.G, b.gstride, f.jwork,
                     2 * (int64_t)b.mmax * b.mmax, f.evals, b.mmax, f.evecs, f.jstat);
  LD_HIP(hipGetLastError());
  {
    std::vector<int> h;
    LD_TRY(read_ints(ctx, st, f.fail, count, h));
    for (int i = 0; i < count; ++i)
      if (h[i]) return fail(LD_ENOTSPD, "batch: CholeskyQR breakdown in instance " + std::to_string(i));
    LD_TRY(read_ints(ctx, st, f.jstat, count, h));
    for (int i = 0; i < count; ++i)
      if (h[i])
        return fail(LD_ENOCONV, "batch: eigen-solver did not converge in instance " + std::to_string(i));
    LD_TRY(ensure_pinned(ctx, (size_t)B * b.mmax + 8));
    LD_HIP(hipMemcpyAsync(ctx->pinned, f.evals, B * b.mmax * 8, hipMemcpyDeviceToHost, st));
    LD_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < count; ++i)
      for (int j = 0; j < b.h[i].rank; ++j) {
        const double v = ctx->pinned[(int64_t)i * b.mmax + j];
        if (!(v > 0.0) || !std::isfinite(v))
          return fail(LD_ENOTSPD, "batch: non-positive kept eigenvalue in instance " + std::to_string(i));
      }
    if (lambda_out)
      for (int i = 0; i < count; ++i)
        for (int j = 0; j < lambda_stride; ++j)
          lambda_out[(int64_t)i * lambda_stride + j] =
              j < b.h[i].rank ? ctx->pinned[(int64_t)i * b.mmax + j] : 0.0;
  }
  // U = Q V_l;  D;  C = diag(1/lam) + U^T D^-1 U = R^T R;  log det P;  F = D^-1 U R^-1
  hipLaunchKernelGGL(k_bgemm, gemm_grid(b, b.lmax), dim3(256), 0, st, b.d_inst, 0, 1, Qb, b.mmax,
                     f.evecs, b.gstride, 1, (const double*)nullptr, f.U, b.lmax);
  hipLaunchKernelGGL(k_bd, dim3(grid1(R)), dim3(256), 0, st, b.d_inst, b.d_blk_inst, R, f.U, b.lmax,
                     f.evals, b.mmax, f.D, f.Dinv64);
  const int ltiles = (b.lmax + 63) / 64;
  hipLaunchKernelGGL(k_bgram, dim3(ltiles, ltiles, b.ngitems), dim3(256), 0, st, b.d_inst, b.d_gitems,
                     1, f.U, b.lmax, f.U, b.lmax, f.Dinv64, f.G, b.gpart, b.gstride, 1);
  hipLaunchKernelGGL(k_bgram_sum, dim3(B, gsum_rows(b)), dim3(256), 0, st, b.d_inst, 1, b.gpart, f.G,
                     b.gstride);
  hipLaunchKernelGGL(k_bcapdiag, dim3(B), dim3(256), 0, st, b.d_inst, f.G, b.gstride, f.evals, b.mmax);
  LD_HIP(hipMemsetAsync(f.fail, 0, B * 4, st));
  hipLaunchKernelGGL(k_bchol, dim3(B), dim3(dev::CT), 0, st, b.d_inst, 1, f.G, b.gstride, f.fail);
  hipLaunchKernelGGL(k_blogdet, dim3(B), dim3(256), 0, st, b.d_inst, f.D, f.evals, b.mmax, f.G,
                     b.gstride, f.ldP);
  hipLaunchKernelGGL(k_btrinv, dim3(B), dim3(dev::CT), 0, st, b.d_inst, 1, f.G, f.Rinv, b.gstride);
  hipLaunchKernelGGL(k_bgemm, gemm_grid(b, b.lmax), dim3(256), 0, st, b.d_inst, 1, 1, f.U, b.lmax,
                     f.Rinv, b.gstride, 0, f.Dinv64, f.F64, b.lmax);
  launch_convert_f64_to_f32(st, f.F64, f.F32, R * b.lmax);
  launch_convert_f64_to_f32(st, f.Dinv64, f.Dinv32, R);
  LD_HIP(hipGetLastError());
  std::vector<double> logdetP(count);
  {
    std::vector<int> h;
    LD_TRY(read_ints(ctx, st, f.fail, count, h));
    for (int i = 0; i < count; ++i)
      if (h[i])
        return fail(LD_ENOTSPD, "batch: capacitance Cholesky breakdown in instance " + std::to_string(i));
    LD_HIP(hipMemcpyAsync(ctx->pinned, f.ldP, B * 8, hipMemcpyDeviceToHost, st));
    LD_HIP(hipStreamSynchronize(st));
    std::copy(ctx->pinned, ctx->pinned + count, logdetP.begin());
    for (int i = 0; i < count; ++i)
      if (!std::isfinite(logdetP[i]))
        return fail(LD_ENOTSPD, "batch: log det P is not finite in instance " + std::to_string(i));
  }
  auto t1 = std::chrono::steady_clock::now();
  const double precond_s = std::chrono::duration<double>(t1 - t0).count();
  if (flags & LD_BATCH_PRECOND_ONLY) {
    for (int i = 0; i < count; ++i) {
      ld_result& o = out[i];
      o = ld_result{};
      o.seconds_precond = precond_s;
      o.logdet_P = logdetP[i];
      o.logdet = logdetP[i];
      o.k = J;
      o.num_probes = s;
    }
    return LD_OK;
  }

  // ---- multi-shift CG over every (instance, probe) column
  Scal S;
  S.rho = scal;
  S.rho0 = scal + ncol;
  S.alpha = scal + 2 * ncol;
  S.beta = scal + 3 * ncol;
  S.alpha_prev = scal + 4 * ncol;
  S.beta_prev = scal + 5 * ncol;
  S.ztz = scal + 6 * ncol;
  S.zeta = scal + 7 * ncol;
  S.zeta_prev = S.zeta + J * ncol;
  S.ztp = S.zeta_prev + J * ncol;
  S.ztx = S.ztp + J * ncol;
  double* delta = S.ztx + J * ncol;
  S.frozen = iscal;
  S.active = iscal + J * ncol;
  S.status = iscal + J * ncol + ncol;
  LD_TRY(ensure_pinned(ctx, (size_t)(J * ncol + 3 * ncol + 4 * count + 16)));
  for (int j = 0; j < J; ++j) ctx->pinned[j] = shifts[j] - shifts[0];
  LD_HIP(hipMemcpyAsync(delta, ctx->pinned, J * sizeof(double), hipMemcpyHostToDevice, st));
  LD_HIP(hipMemsetAsync(S.status, 0, 2 * sizeof(int), st));
  LD_HIP(hipStreamSynchronize(st));

  hipLaunchKernelGGL(k_bprobes, dim3(grid1(R * s)), dim3(256), 0, st, b.d_inst, b.d_blk_inst, R, s, Z);
  const int64_t vec = R * s;
  auto woodbury = [&](const float* rin, float* uout, const int* act) {
    hipLaunchKernelGGL(k_bft, dim3(nchunks), dim3(256), 0, st, b.d_inst, d_ch_inst, f.F32, b.lmax,
                       rin, s, b.lmax, tpart, act);
    hipLaunchKernelGGL(k_bft_sum, dim3(B, (unsigned)((b.lmax * s + 63) / 64)), dim3(64), 0, st,
                       b.d_inst, s, b.lmax, tpart, tl, act);
#define LD_BWOUT(CT)                                                                          \
  hipLaunchKernelGGL((k_bwout<CT>), dim3((unsigned)b.nblk), dim3(256), 0, st, b.d_inst,        \
                     b.d_blk_inst, f.F32, b.lmax, f.Dinv32, tl, b.lmax, rin, s, uout, Z, d1, d2, \
                     act)
    switch ((s + 15) / 16) {
      case 1: LD_BWOUT(1); break;
      case 2: LD_BWOUT(2); break;
      case 3: LD_BWOUT(3); break;
      default: LD_BWOUT(4); break;
    }
#undef LD_BWOUT
  };
  hipLaunchKernelGGL(k_bcopy2, dim3(grid1(vec)), dim3(256), 0, st, Z, r, p, vec);
  woodbury(r, u, nullptr);
  hipLaunchKernelGGL(k_bcopy2, dim3(grid1(vec)), dim3(256), 0, st, u, w, (float*)nullptr, vec);
  hipLaunchKernelGGL(k_bsegsum, dim3(B), dim3(256), 0, st, b.d_inst, s, d1, sg1);
  hipLaunchKernelGGL(k_bsegsum, dim3(B), dim3(256), 0, st, b.d_inst, s, d2, sg2);
  launch_scal_init(st, S, sg1, sg2, 1, ncol, J);
  hipLaunchKernelGGL(k_binst_active, dim3((count + 255) / 256), dim3(256), 0, st, count, s,
                     S.active, iact);
  LD_HIP(hipGetLastError());

  // product tile shape (autotuner): every candidate shape for s columns is
  // timed once per context (or on request) on this batch's first product,
  // and the fastest is kept; the symmetric form, where it applies, replaces it
  const bool use_sym = sym_form(s, flags);
  const int nshape = (int)product_shapes(s).size();
  ProductPlan pv[5];
  for (int v = 0; v < nshape + (use_sym ? 1 : 0); ++v)
    LD_TRY(with_stream(ctx, st, b, s, v, &pv[v]));
  if (!use_sym && (ctx->bvariant < 0 || ctx->bvariant_cols != s || (flags & LD_BATCH_RETUNE))) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LD_HIP(hipEventCreate(&e0));
    LD_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int pick = 0;
    for (int v = 0; v < nshape; ++v) {
      float tot = 0.f;
      for (int rep = 0; rep < 3; ++rep) {
        float ms = 0.f;
        (void)hipEventRecord(e0, st);
        launch_product(st, b, pv[v], w, s, q, p, (float)shifts[0], dwq, nullptr);
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) tot += ms;  // the first launch warms up
      }
      if (tot < best) {
        best = tot;
        pick = v;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    LD_HIP(hipGetLastError());
    ctx->bvariant = pick;
    ctx->bvariant_cols = s;
  }
  const ProductPlan& pp = pv[use_sym ? nshape : ctx->bvariant];
  // Instrumentation (ctx->timing, eager form only): events around every
  // product launch and the launch's algorithmic work summed on the device.
  const bool timed = ctx->timing && !use_graph;
  if (timed) LD_HIP(hipMemsetAsync(tacc, 0, 2 * 8, st));

  auto body = [&]() -> ld_status {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
      hipLaunchKernelGGL(k_bwork, dim3(1), dim3(256), 0, st, b.d_inst, iact, count, s, tacc);
      LD_TRY(timing_pair(ctx, &e0, &e1, 0.0, 0.0));
      LD_HIP(hipEventRecord(e0, st));
    }
    launch_product(st, b, pp, w, s, q, p, (float)shifts[0], dwq, iact);
    if (timed) LD_HIP(hipEventRecord(e1, st));
    hipLaunchKernelGGL(k_bsegsum, dim3(B), dim3(256), 0, st, b.d_inst, s, dwq, sgw);
    launch_scal_alpha(st, S, sgw, 1, ncol);
    hipLaunchKernelGGL(k_bupdate_r, dim3(grid1(vec)), dim3(256), 0, st, b.d_inst, b.d_blk_inst, R,
                       s, r, q, S.alpha, iact);
    woodbury(r, u, iact);
    hipLaunchKernelGGL(k_bsegsum, dim3(B), dim3(256), 0, st, b.d_inst, s, d1, sg1);
    hipLaunchKernelGGL(k_bsegsum, dim3(B), dim3(256), 0, st, b.d_inst, s, d2, sg2);
    launch_scal_beta(st, S, sg1, sg2, 1, ncol, J, delta, tol);
    hipLaunchKernelGGL(k_bupdate_pw, dim3(grid1(vec)), dim3(256), 0, st, b.d_inst, b.d_blk_inst, R,
                       s, p, w, r, u, S.beta, S.active, iact);
    hipLaunchKernelGGL(k_binst_active, dim3((count + 255) / 256), dim3(256), 0, st, count, s,
                       S.active, iact);
    return LD_OK;
  };

  hipGraphExec_t exec = nullptr;
  if (use_graph) {
    hipGraph_t graph = nullptr;
    LD_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    ld_status cs = LD_OK;
    for (int kk = 0; kk < kChunk && cs == LD_OK; ++kk) cs = body();
    const hipError_t ce = hipStreamEndCapture(st, &graph);
    if (cs != LD_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return cs;
    }
    if (ce != hipSuccess) return fail(LD_EHIP, std::string("graph capture: ") + hipGetErrorString(ce));
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess)
      return fail(LD_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
  }
  int it = 0, active = (int)ncol;
  bool breakdown = false;
  ld_status st_ = LD_OK;
  while (it < max_iters && active > 0 && st_ == LD_OK) {
    if (use_graph && it + kChunk <= max_iters) {
      if (hipGraphLaunch(exec, st) != hipSuccess) {
        st_ = fail(LD_EHIP, "graph launch failed");
        break;
      }
      it += kChunk;
    } else {
      const int todo = std::min(kChunk, max_iters - it);
      for (int kk = 0; kk < todo && st_ == LD_OK; ++kk) st_ = body();
      it += todo;
    }
    if (st_ != LD_OK) break;
    if (hipMemcpyAsync(ctx->pinned, S.status, 2 * sizeof(int), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      st_ = fail(LD_EHIP, "status readback failed");
      break;
    }
    if (timed) timing_collect(ctx);
    active = ((const int*)ctx->pinned)[0];
    if (((const int*)ctx->pinned)[1]) breakdown = true;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  LD_TRY(st_);
  if (timed) {
    LD_HIP(hipMemcpyAsync(ctx->pinned, tacc, 2 * 8, hipMemcpyDeviceToHost, st));
    LD_HIP(hipStreamSynchronize(st));
    ctx->mm_flops += ctx->pinned[0];
    ctx->mm_bytes += ctx->pinned[1];
  }

  // ---- the Hutchinson combination of every instance on the device (FP64),
  // then the per-probe values and per-instance statistics read back
  BCoef bc{};
  bc.b = bcoef;
  bc.J = J;
  for (int j = 0; j < J; ++j) bc.c[j] = ccoef[j];
  hipLaunchKernelGGL(k_bhutchinson, dim3(count), dim3(64), 0, st, s, ncol, bc, S.ztx, S.ztz,
                     S.rho, S.rho0, tol, hut, hut + ncol);
  LD_HIP(hipGetLastError());
  double* hp = ctx->pinned;
  LD_HIP(hipMemcpyAsync(hp, hut, (size_t)(ncol + 4 * count) * 8, hipMemcpyDeviceToHost, st));
  LD_HIP(hipStreamSynchronize(st));
  const double solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
  int unconverged = 0;
  for (int i = 0; i < count; ++i) {
    const double* sv = hp + ncol + 4 * i;
    const int conv = (int)sv[3];
    ld_result& o = out[i];
    o.logdet_P = logdetP[i];
    o.trace_term = sv[0];
    o.logdet = logdetP[i] + sv[0];
    o.std_err = sv[1];
    o.rel_resid = sv[2];
    o.seconds_solve = solve_s;
    o.seconds_precond = precond_s;
    o.iterations = std::min(it, max_iters);
    o.converged_cols = conv;
    o.k = J;
    o.num_probes = s;
    if (per_probe) std::copy(hp + (int64_t)i * s, hp + (int64_t)(i + 1) * s, per_probe + (int64_t)i * s);
    if (conv < s) ++unconverged;
  }
  if (breakdown) return fail(LD_ENOTSPD, "batch: non-positive curvature or residual in the solver");
  if (unconverged) return fail(LD_ENOCONV, "batch: max_iters reached before every probe converged");
  return LD_OK;
}

}  // namespace ld
