// Learned surrogate of the trace term: an ensemble of small MLPs that maps
// 38 features of a problem (kernel kind and hyperparameters, n, d, and a
// histogram of the preconditioner's eigenvalues) to tr log(M P^-1) / n.
//
// Network (per member): 38 -> 256 -> 256 -> 256 -> 1, GELU (erf form) after
// each of the first three layers.  Inputs are standardised by stored means
// and standard deviations, the target by a stored mean and standard
// deviation.  Training: FP32 forward and backward passes (tiled FP32 GEMMs),
// MSE loss, Adam; all members step together (members along the grid's z).
// Inference: BF16 weights and activations on BF16 matrix cores
// (v_mfma_f32_32x32x16_bf16) with FP32 accumulation, bias and GELU.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ld_common.hpp"
#include "rng_dev.hpp"

// Layout of one member's parameters (FP32, offsets in floats; every tensor
// starts on a 64-float boundary).  W_l is in x out, row-major.
namespace ld {
namespace mlp {

constexpr int NF = LD_SUR_FEATURES;  // input features
constexpr int W = LD_SUR_WIDTH;      // hidden width
constexpr int KP1 = 48;              // input features padded for the BF16 k-steps
constexpr int64_t al64(int64_t x) { return (x + 63) / 64 * 64; }
constexpr int64_t OFF_W1 = 0;
constexpr int64_t OFF_B1 = al64(OFF_W1 + (int64_t)NF * W);
constexpr int64_t OFF_W2 = al64(OFF_B1 + W);
constexpr int64_t OFF_B2 = al64(OFF_W2 + (int64_t)W * W);
constexpr int64_t OFF_W3 = al64(OFF_B2 + W);
constexpr int64_t OFF_B3 = al64(OFF_W3 + (int64_t)W * W);
constexpr int64_t OFF_W4 = al64(OFF_B3 + W);
constexpr int64_t OFF_B4 = al64(OFF_W4 + W);
constexpr int64_t PSTRIDE = al64(OFF_B4 + 1);  // floats per member
// BF16 inference copy (transposed: out x in_padded)
constexpr int64_t Q_W1 = 0;
constexpr int64_t Q_W2 = Q_W1 + (int64_t)W * KP1;
constexpr int64_t Q_W3 = Q_W2 + (int64_t)W * W;
constexpr int64_t Q_W4 = Q_W3 + (int64_t)W * W;
constexpr int64_t QSTRIDE = Q_W4 + W;  // bf16 per member

}  // namespace mlp
}  // namespace ld

struct ld_surrogate {
  int device = 0;
  int members = 0;
  int64_t step = 0;             // Adam steps taken
  float* params = nullptr;      // members x PSTRIDE
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* grad = nullptr;
  float* xmean = nullptr;       // NF (device)
  float* xstd = nullptr;        // NF (device)
  double ymean = 0.0, ystd = 1.0;
  __bf16* q = nullptr;          // members x QSTRIDE
  bool q_dirty = true;
  void* block = nullptr;
};

namespace ld {
namespace {

using namespace mlp;

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  return cdf + z * pdf;
}

// ------------------------------------------------------------ FP32 GEMM --
// C[z] (M x N, leading dimension ldc) = A[z] B[z] (+ bias[z]) with A(i, k) at
// A[i sa_i + k sa_k], B(k, j) at B[k sb_k + j sb_j] (any transposition by
// strides); if Act != nullptr, Act = gelu(C) as well.  64 x 64 tiles, k
// staged 16 at a time in LDS, 4 x 4 outputs per thread; member z along
// blockIdx.z with per-member strides.
struct GemmArgs {
  int M, N, K;
  const float* A;
  int64_t sa_i, sa_k, sa_z;
  const float* B;
  int64_t sb_k, sb_j, sb_z;
  const float* bias;
  int64_t sbias_z;
  float* C;
  int64_t ldc, sc_z;
  float* Act;
};

__global__ __launch_bounds__(256) void k_sgemm(GemmArgs g) {
  __shared__ float As[16][65];
  __shared__ float Bs[16][65];
  const int z = blockIdx.z;
  const float* A = g.A + z * g.sa_z;
  const float* B = g.B + z * g.sb_z;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const int tid = threadIdx.x, ti = tid / 16, tj = tid % 16;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    __syncthreads();
    for (int e = tid; e < 16 * 64; e += 256) {
      const int kk = e / 64, c = e % 64;
      const int i = i0 + c, k = k0 + kk, j = j0 + c;
      As[kk][c] = (i < g.M && k < g.K) ? A[i * g.sa_i + k * g.sa_k] : 0.f;
      Bs[kk][c] = (j < g.N && k < g.K) ? B[k * g.sb_k + j * g.sb_j] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ti + 16 * q];
        b[q] = Bs[kk][tj + 16 * q];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_fmaf(a[x], b[y], acc[x][y]);
    }
  }
  float* C = g.C + z * g.sc_z;
  float* Act = g.Act ? g.Act + z * g.sc_z : nullptr;
  const float* bias = g.bias ? g.bias + z * g.sbias_z : nullptr;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = i0 + ti + 16 * x, j = j0 + tj + 16 * y;
      if (i < g.M && j < g.N) {
        float v = acc[x][y];
        if (bias) v += bias[j];
        C[(int64_t)i * g.ldc + j] = v;
        if (Act) Act[(int64_t)i * g.ldc + j] = gelu(v);
      }
    }
}

void sgemm(hipStream_t st, int members, const GemmArgs& g) {
  const dim3 grid((unsigned)((g.M + 63) / 64), (unsigned)((g.N + 63) / 64), (unsigned)members);
  hipLaunchKernelGGL(k_sgemm, grid, dim3(256), 0, st, g);
}

// ------------------------------------------------------ small kernels --
// standardised features: Xs (B x NF) = (X - mean) / std
__global__ void k_standardize(const float* __restrict__ X, int64_t rows, const float* __restrict__ mean,
                              const float* __restrict__ sd, float* __restrict__ Xs) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < rows * NF;
       e += (int64_t)gridDim.x * 256) {
    const int f = (int)(e % NF);
    Xs[e] = (X[e] - mean[f]) / sd[f];
  }
}

// dy = 2 (y - t') / B with t' the standardised target; loss partials (FP64)
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, int64_t B,
                                              const float* __restrict__ t, double ymean, double ystd,
                                              float* __restrict__ dy, double* __restrict__ loss) {
  __shared__ double red[256];
  const int z = blockIdx.x;
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < B; b += 256) {
    const double tt = ((double)t[b] - ymean) / ystd;
    const double r = (double)y[z * B + b] - tt;
    acc += r * r;
    dy[z * B + b] = (float)(2.0 * r / (double)B);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[z] = red[0] / (double)B;
}

// dZ = dH .* gelu'(Z), all members (count elements)
__global__ void k_gelu_back(const float* __restrict__ dH, const float* __restrict__ Z,
                            float* __restrict__ dZ, int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * 256)
    dZ[e] = dH[e] * gelu_grad(Z[e]);
}

// db (N) = column sums of dZ (B x N) for each member (blockIdx.y), in FP64
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ dZ, int64_t B, int N,
                                                int64_t sz_z, float* __restrict__ out,
                                                int64_t so_z) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int z = blockIdx.y;
  if (j >= N) return;
  double acc = 0.0;
  for (int64_t b = 0; b < B; ++b) acc += (double)dZ[z * sz_z + b * N + j];
  out[z * so_z + j] = (float)acc;
}

// Adam (bias-corrected): p -= lr mhat / (sqrt(vhat) + eps)
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t count, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * 256) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.0f - b1) * gg;
    const float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// initial weights: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from the counter
// stream 3 of seed + member (index = offset within the member); biases 0
__global__ void k_init(float* __restrict__ params, int members, uint64_t seed) {
  const int64_t total = (int64_t)members * PSTRIDE;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int z = (int)(e / PSTRIDE);
    const int64_t o = e % PSTRIDE;
    float bound = 0.f;
    if (o < OFF_W1 + (int64_t)NF * W)
      bound = 1.0f / sqrtf((float)NF);
    else if ((o >= OFF_W2 && o < OFF_W2 + (int64_t)W * W) || (o >= OFF_W3 && o < OFF_W3 + (int64_t)W * W) ||
             (o >= OFF_W4 && o < OFF_W4 + W))
      bound = 1.0f / sqrtf((float)W);
    float val = 0.f;
    if (bound > 0.f) {
      // key of stream 3 for seed + z, as in the host-side key derivation
      uint64_t zz = (seed + (uint64_t)z) + 0x9E3779B97F4A7C15ull * 4ull;
      zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ull;
      zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBull;
      const uint64_t key = zz ^ (zz >> 31);
      const double u = dev::rng_uniform(dev::rng_bits(key, (uint64_t)o));
      val = (float)((2.0 * u - 1.0) * bound);
    }
    params[e] = val;
  }
}

// FP32 master weights -> BF16, transposed (out x in_padded) for inference
__global__ void k_quantize(const float* __restrict__ params, int members, __bf16* __restrict__ q) {
  const int64_t total = (int64_t)members * QSTRIDE;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int z = (int)(e / QSTRIDE);
    const int64_t o = e % QSTRIDE;
    const float* P = params + (int64_t)z * PSTRIDE;
    float v = 0.f;
    if (o < Q_W2) {  // W1^T: 256 x 48
      const int j = (int)(o / KP1), k = (int)(o % KP1);
      v = k < NF ? P[OFF_W1 + (int64_t)k * W + j] : 0.f;
    } else if (o < Q_W3) {
      const int64_t r = o - Q_W2;
      const int j = (int)(r / W), k = (int)(r % W);
      v = P[OFF_W2 + (int64_t)k * W + j];
    } else if (o < Q_W4) {
      const int64_t r = o - Q_W3;
      const int j = (int)(r / W), k = (int)(r % W);
      v = P[OFF_W3 + (int64_t)k * W + j];
    } else {
      v = P[OFF_W4 + (o - Q_W4)];
    }
    q[e] = (__bf16)v;
  }
}

// ------------------------------------------------------- BF16 inference --
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// standardised features -> BF16, padded to KP1 columns
__global__ void k_features_bf16(const float* __restrict__ X, int64_t rows, const float* __restrict__ mean,
                                const float* __restrict__ sd, __bf16* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < rows * KP1;
       e += (int64_t)gridDim.x * 256) {
    const int f = (int)(e % KP1);
    const int64_t r = e / KP1;
    out[e] = f < NF ? (__bf16)((X[r * NF + f] - mean[f]) / sd[f]) : (__bf16)0.f;
  }
}

// H_out[z] (rows x 256, BF16) = gelu(H_in[z] (rows x K, BF16) W^T[z] + b[z]).
// Workgroup: 4 waves, 128 rows x 64 columns; wave w: rows 32 w .. 32 w + 31,
// two 32-column MFMA blocks.  In k-step q lane half h supplies k = 16 q + 8 h
// + j (j < 8) for both operands: A from the activation row li, B from the
// transposed weight row (output column) li, 16 bytes each.
__global__ __launch_bounds__(256) void k_layer_bf16(const __bf16* __restrict__ Hin, int64_t rows, int K,
                                                    int64_t sin_z, const __bf16* __restrict__ q,
                                                    int64_t qoff, const float* __restrict__ params,
                                                    int64_t boff, __bf16* __restrict__ Hout,
                                                    int64_t sout_z) {
  const int z = blockIdx.z;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, lh = lane >> 5;
  const int64_t row = (int64_t)blockIdx.x * 128 + 32 * wave + li;  // A row of this lane
  const int c0 = blockIdx.y * 64;
  const __bf16* A = Hin + z * sin_z;
  const __bf16* Wt = q + z * QSTRIDE + qoff;
  f32x16 acc[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x8 a;
    if (row < rows)
      a = *(const bf16x8*)&A[row * K + k0 + 8 * lh];
    else
      for (int j = 0; j < 8; ++j) a[j] = (__bf16)0.f;
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const bf16x8 b = *(const bf16x8*)&Wt[(int64_t)(c0 + 32 * nb + li) * K + k0 + 8 * lh];
      acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[nb], 0, 0, 0);
    }
  }
  const float* bias = params + z * PSTRIDE + boff;
  __bf16* O = Hout + z * sout_z;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t orow = (int64_t)blockIdx.x * 128 + 32 * wave + 8 * (r >> 2) + 4 * lh + (r & 3);
      const int col = c0 + 32 * nb + li;
      if (orow < rows) O[orow * W + col] = (__bf16)gelu(acc[nb][r] + bias[col]);
    }
}

// last layer and ensemble statistics: per row, y_z = H3_z . w4_z + b4_z (FP32
// from BF16), de-standardised; mean and standard deviation over members
__global__ __launch_bounds__(256) void k_head(const __bf16* __restrict__ H3, int64_t rows, int64_t s_z,
                                              const __bf16* __restrict__ q, const float* __restrict__ params,
                                              int members, double ymean, double ystd,
                                              float* __restrict__ mean, float* __restrict__ sdev) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  double s1 = 0.0, s2 = 0.0;
  for (int z = 0; z < members; ++z) {
    const __bf16* h = H3 + z * s_z + row * W;
    const __bf16* w4 = q + z * QSTRIDE + Q_W4;
    float acc = 0.f;
    for (int k = lane; k < W; k += 64) acc = __builtin_fmaf((float)h[k], (float)w4[k], acc);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    const double y = ymean + ystd * ((double)acc + (double)params[z * PSTRIDE + OFF_B4]);
    s1 += y;
    s2 += y * y;
  }
  if (lane == 0) {
    const double m = s1 / members;
    const double var = members > 1 ? (s2 - members * m * m) / (members - 1) : 0.0;
    mean[row] = (float)m;
    sdev[row] = (float)sqrt(var > 0.0 ? var : 0.0);
  }
}

int grid1(int64_t count) {
  int64_t b = (count + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

ld_status check_sur(ld_ctx* ctx, const ld_surrogate* S) {
  if (!ctx || !S) return fail(LD_EINVAL, "context or surrogate is NULL");
  if (S->device != ctx->device) return fail(LD_EINVAL, "surrogate and context are on different devices");
  LD_HIP(hipSetDevice(ctx->device));
  return LD_OK;
}

// Forward and backward pass of every member on one minibatch; gradients in S->grad.
ld_status forward_backward(ld_ctx* ctx, ld_surrogate* S, const float* X, const float* t, int B,
                           double* loss_host) {
  hipStream_t st = ctx->stream;
  const int E = S->members;
  const int64_t bw = (int64_t)B * W;
  size_t need = 0;
  auto add = [&](size_t b) { need += ((b + 255) & ~(size_t)255) + 256; };
  add((size_t)B * NF * 4);
  for (int q = 0; q < 8; ++q) add((size_t)E * bw * 4);
  add((size_t)E * B * 4 * 2);
  add((size_t)E * 8);
  ctx->arena.reset();
  LD_TRY(ctx->arena.reserve(need));
  Arena& ar = ctx->arena;
  float* Xs = (float*)ar.take((size_t)B * NF * 4);
  float* Z1 = (float*)ar.take((size_t)E * bw * 4);
  float* H1 = (float*)ar.take((size_t)E * bw * 4);
  float* Z2 = (float*)ar.take((size_t)E * bw * 4);
  float* H2 = (float*)ar.take((size_t)E * bw * 4);
  float* Z3 = (float*)ar.take((size_t)E * bw * 4);
  float* H3 = (float*)ar.take((size_t)E * bw * 4);
  float* dH = (float*)ar.take((size_t)E * bw * 4);
  float* dZ = (float*)ar.take((size_t)E * bw * 4);
  float* y = (float*)ar.take((size_t)E * B * 4);
  float* dy = (float*)ar.take((size_t)E * B * 4);
  double* loss = (double*)ar.take((size_t)E * 8);
  if (!loss) return fail(LD_ENOMEM, "surrogate: scratch arena too small");
  float* P = S->params;
  float* G = S->grad;
  const int64_t PS = PSTRIDE;

  hipLaunchKernelGGL(k_standardize, dim3(grid1((int64_t)B * NF)), dim3(256), 0, st, X, (int64_t)B,
                     S->xmean, S->xstd, Xs);
  // forward
  sgemm(st, E, GemmArgs{B, W, NF, Xs, NF, 1, 0, P + OFF_W1, W, 1, PS, P + OFF_B1, PS, Z1, W, bw, H1});
  sgemm(st, E, GemmArgs{B, W, W, H1, W, 1, bw, P + OFF_W2, W, 1, PS, P + OFF_B2, PS, Z2, W, bw, H2});
  sgemm(st, E, GemmArgs{B, W, W, H2, W, 1, bw, P + OFF_W3, W, 1, PS, P + OFF_B3, PS, Z3, W, bw, H3});
  sgemm(st, E, GemmArgs{B, 1, W, H3, W, 1, bw, P + OFF_W4, 1, 0, PS, P + OFF_B4, PS, y, 1, B, nullptr});
  hipLaunchKernelGGL(k_loss, dim3(E), dim3(256), 0, st, y, (int64_t)B, t, S->ymean, S->ystd, dy, loss);
  // backward
  sgemm(st, E, GemmArgs{W, 1, B, H3, 1, W, bw, dy, 1, 0, B, nullptr, 0, G + OFF_W4, 1, PS, nullptr});
  hipLaunchKernelGGL(k_colsum, dim3(1, E), dim3(256), 0, st, dy, (int64_t)B, 1, (int64_t)B, G + OFF_B4, PS);
  sgemm(st, E, GemmArgs{B, W, 1, dy, 1, 0, B, P + OFF_W4, 0, 1, PS, nullptr, 0, dH, W, bw, nullptr});
  hipLaunchKernelGGL(k_gelu_back, dim3(grid1(E * bw)), dim3(256), 0, st, dH, Z3, dZ, E * bw);
  sgemm(st, E, GemmArgs{W, W, B, H2, 1, W, bw, dZ, W, 1, bw, nullptr, 0, G + OFF_W3, W, PS, nullptr});
  hipLaunchKernelGGL(k_colsum, dim3(1, E), dim3(256), 0, st, dZ, (int64_t)B, W, bw, G + OFF_B3, PS);
  sgemm(st, E, GemmArgs{B, W, W, dZ, W, 1, bw, P + OFF_W3, 1, W, PS, nullptr, 0, dH, W, bw, nullptr});
  hipLaunchKernelGGL(k_gelu_back, dim3(grid1(E * bw)), dim3(256), 0, st, dH, Z2, dZ, E * bw);
  sgemm(st, E, GemmArgs{W, W, B, H1, 1, W, bw, dZ, W, 1, bw, nullptr, 0, G + OFF_W2, W, PS, nullptr});
  hipLaunchKernelGGL(k_colsum, dim3(1, E), dim3(256), 0, st, dZ, (int64_t)B, W, bw, G + OFF_B2, PS);
  sgemm(st, E, GemmArgs{B, W, W, dZ, W, 1, bw, P + OFF_W2, 1, W, PS, nullptr, 0, dH, W, bw, nullptr});
  hipLaunchKernelGGL(k_gelu_back, dim3(grid1(E * bw)), dim3(256), 0, st, dH, Z1, dZ, E * bw);
  sgemm(st, E, GemmArgs{NF, W, B, Xs, 1, NF, 0, dZ, W, 1, bw, nullptr, 0, G + OFF_W1, W, PS, nullptr});
  hipLaunchKernelGGL(k_colsum, dim3(1, E), dim3(256), 0, st, dZ, (int64_t)B, W, bw, G + OFF_B1, PS);
  LD_HIP(hipGetLastError());
  if (loss_host) {
    LD_TRY(ensure_pinned(ctx, (size_t)E + 8));
    LD_HIP(hipMemcpyAsync(ctx->pinned, loss, (size_t)E * 8, hipMemcpyDeviceToHost, st));
    LD_HIP(hipStreamSynchronize(st));
    std::memcpy(loss_host, ctx->pinned, (size_t)E * 8);
  }
  return LD_OK;
}

}  // namespace
}  // namespace ld

using namespace ld;
using namespace ld::mlp;

extern "C" {

int64_t ld_surrogate_param_count(void) { return OFF_B4 + 1; }

ld_status ld_surrogate_features(const double* lambda, int32_t rank, int32_t kind, double lengthscale,
                                double variance, double noise, int64_t n, int32_t d,
                                const double* edges, float* out) {
  if (!lambda || !edges || !out) return fail(LD_EINVAL, "null pointer");
  if (rank < 1 || n < 1 || d < 1) return fail(LD_EINVAL, "rank, n and d must be >= 1");
  if (!(lengthscale > 0.0) || !(variance > 0.0) || !(noise > 0.0))
    return fail(LD_EINVAL, "lengthscale, variance and noise must be > 0");
  if (!(edges[LD_SUR_BINS] > edges[0])) return fail(LD_EINVAL, "edges must increase");
  out[0] = (float)kind;
  out[1] = (float)std::log(lengthscale);
  out[2] = (float)std::log(variance);
  out[3] = (float)std::log(noise);
  out[4] = (float)std::log((double)n);
  out[5] = (float)d;
  std::vector<double> h(LD_SUR_BINS, 0.0);
  const double lo = edges[0], width = (edges[LD_SUR_BINS] - edges[0]) / LD_SUR_BINS;
  for (int j = 0; j < rank; ++j) {
    if (!(lambda[j] > 0.0)) return fail(LD_EINVAL, "eigenvalues must be > 0");
    const double x = std::log(lambda[j] / (double)n);
    int b = (int)std::floor((x - lo) / width);
    b = b < 0 ? 0 : (b >= LD_SUR_BINS ? LD_SUR_BINS - 1 : b);
    h[b] += 1.0;
  }
  for (int b = 0; b < LD_SUR_BINS; ++b) out[6 + b] = (float)(h[b] / rank);
  return LD_OK;
}

ld_status ld_surrogate_create(ld_ctx* ctx, int32_t members, uint64_t seed, ld_surrogate** out) {
  if (!ctx || !out) return fail(LD_EINVAL, "context or out is NULL");
  if (members < 1 || members > 64) return fail(LD_EINVAL, "members must be in 1..64");
  LD_HIP(hipSetDevice(ctx->device));
  ld_surrogate* S = new ld_surrogate();
  S->device = ctx->device;
  S->members = members;
  const size_t pbytes = (size_t)members * PSTRIDE * 4;
  const size_t qbytes = ((size_t)members * QSTRIDE * 2 + 255) & ~(size_t)255;
  const size_t total = 4 * pbytes + 2 * 256 + qbytes;
  if (hipMalloc(&S->block, total) != hipSuccess) {
    (void)hipGetLastError();
    delete S;
    return fail(LD_ENOMEM, "surrogate allocation failed");
  }
  char* c = (char*)S->block;
  S->params = (float*)c; c += pbytes;
  S->adam_m = (float*)c; c += pbytes;
  S->adam_v = (float*)c; c += pbytes;
  S->grad = (float*)c; c += pbytes;
  S->xmean = (float*)c; c += 256;
  S->xstd = (float*)c; c += 256;
  S->q = (__bf16*)c;
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_init, dim3(grid1((int64_t)members * PSTRIDE)), dim3(256), 0, st, S->params,
                     members, seed);
  std::vector<float> ones(NF, 1.0f);
  if (hipMemsetAsync(S->adam_m, 0, 3 * pbytes, st) != hipSuccess ||  // m, v, grad
      hipMemsetAsync(S->xmean, 0, NF * 4, st) != hipSuccess ||
      hipMemcpy(S->xstd, ones.data(), NF * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    (void)hipFree(S->block);
    delete S;
    return fail(LD_EHIP, "surrogate initialisation failed");
  }
  *out = S;
  return LD_OK;
}

void ld_surrogate_free(ld_surrogate* S) {
  if (!S) return;
  (void)hipSetDevice(S->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(S->block);
  delete S;
}

ld_status ld_surrogate_set_scaling(ld_ctx* ctx, ld_surrogate* S, const float* x_mean, const float* x_std,
                                   double y_mean, double y_std) {
  LD_TRY(check_sur(ctx, S));
  if (!x_mean || !x_std) return fail(LD_EINVAL, "scaling arrays are NULL");
  for (int f = 0; f < NF; ++f)
    if (!(x_std[f] > 0.f) || !std::isfinite(x_std[f]) || !std::isfinite(x_mean[f]))
      return fail(LD_EINVAL, "feature scales must be finite with std > 0");
  if (!(y_std > 0.0) || !std::isfinite(y_std) || !std::isfinite(y_mean))
    return fail(LD_EINVAL, "target scale must be finite with std > 0");
  LD_HIP(hipMemcpyAsync(S->xmean, x_mean, NF * 4, hipMemcpyHostToDevice, ctx->stream));
  LD_HIP(hipMemcpyAsync(S->xstd, x_std, NF * 4, hipMemcpyHostToDevice, ctx->stream));
  LD_HIP(hipStreamSynchronize(ctx->stream));
  S->ymean = y_mean;
  S->ystd = y_std;
  return LD_OK;
}

ld_status ld_surrogate_params(ld_ctx* ctx, ld_surrogate* S, int32_t member, float* out, const float* in) {
  LD_TRY(check_sur(ctx, S));
  if (member < 0 || member >= S->members) return fail(LD_EINVAL, "member out of range");
  float* P = S->params + (int64_t)member * PSTRIDE;
  const size_t bytes = (size_t)ld_surrogate_param_count() * 4;
  if (out) LD_HIP(hipMemcpyAsync(out, P, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  if (in) {
    LD_HIP(hipMemcpyAsync(P, in, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    S->q_dirty = true;
  }
  return LD_OK;
}

ld_status ld_surrogate_gradient(ld_ctx* ctx, ld_surrogate* S, int32_t member, const float* X,
                                const float* y, int32_t B, float* grad, double* loss) {
  LD_TRY(check_sur(ctx, S));
  if (member < 0 || member >= S->members) return fail(LD_EINVAL, "member out of range");
  if (!X || !y || B < 1) return fail(LD_EINVAL, "bad minibatch");
  std::vector<double> l(S->members);
  LD_TRY(forward_backward(ctx, S, X, y, B, l.data()));
  if (grad)
    LD_HIP(hipMemcpyAsync(grad, S->grad + (int64_t)member * PSTRIDE,
                          (size_t)ld_surrogate_param_count() * 4, hipMemcpyDeviceToDevice, ctx->stream));
  LD_HIP(hipStreamSynchronize(ctx->stream));
  if (loss) *loss = l[member];
  return LD_OK;
}

ld_status ld_surrogate_train_step(ld_ctx* ctx, ld_surrogate* S, const float* X, const float* y,
                                  int32_t B, float lr, double* loss) {
  LD_TRY(check_sur(ctx, S));
  if (!X || !y || B < 1) return fail(LD_EINVAL, "bad minibatch");
  if (!(lr > 0.f) || !std::isfinite(lr)) return fail(LD_EINVAL, "lr must be finite and > 0");
  LD_TRY(forward_backward(ctx, S, X, y, B, loss));
  S->step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)S->step));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)S->step));
  const int64_t count = (int64_t)S->members * PSTRIDE;
  hipLaunchKernelGGL(k_adam, dim3(grid1(count)), dim3(256), 0, ctx->stream, S->params, S->adam_m,
                     S->adam_v, S->grad, count, lr, b1, b2, eps, c1, c2);
  LD_HIP(hipGetLastError());
  S->q_dirty = true;
  return LD_OK;
}

ld_status ld_surrogate_predict(ld_ctx* ctx, ld_surrogate* S, const float* X, int64_t N, float* mean,
                               float* stddev) {
  LD_TRY(check_sur(ctx, S));
  if (!X || !mean || !stddev || N < 1) return fail(LD_EINVAL, "bad prediction arguments");
  hipStream_t st = ctx->stream;
  const int E = S->members;
  if (S->q_dirty) {
    hipLaunchKernelGGL(k_quantize, dim3(grid1((int64_t)E * QSTRIDE)), dim3(256), 0, st, S->params, E, S->q);
    S->q_dirty = false;
  }
  const int64_t rows = (N + 127) / 128 * 128;
  const int64_t hs = rows * W;
  ctx->arena.reset();
  LD_TRY(ctx->arena.reserve((size_t)rows * KP1 * 2 + 2 * (size_t)E * hs * 2 + 1024));
  __bf16* X0 = (__bf16*)ctx->arena.take((size_t)rows * KP1 * 2);
  __bf16* Ha = (__bf16*)ctx->arena.take((size_t)E * hs * 2);
  __bf16* Hb = (__bf16*)ctx->arena.take((size_t)E * hs * 2);
  if (!Hb) return fail(LD_ENOMEM, "surrogate: scratch arena too small");
  hipLaunchKernelGGL(k_features_bf16, dim3(grid1(N * KP1)), dim3(256), 0, st, X, N, S->xmean, S->xstd, X0);
  const dim3 grid((unsigned)(rows / 128), W / 64, (unsigned)E);
  hipLaunchKernelGGL(k_layer_bf16, grid, dim3(256), 0, st, X0, N, KP1, (int64_t)0, S->q, Q_W1,
                     S->params, OFF_B1, Ha, hs);
  hipLaunchKernelGGL(k_layer_bf16, grid, dim3(256), 0, st, Ha, N, W, hs, S->q, Q_W2, S->params,
                     OFF_B2, Hb, hs);
  hipLaunchKernelGGL(k_layer_bf16, grid, dim3(256), 0, st, Hb, N, W, hs, S->q, Q_W3, S->params,
                     OFF_B3, Ha, hs);
  hipLaunchKernelGGL(k_head, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, st, Ha, N, hs, S->q,
                     S->params, E, S->ymean, S->ystd, mean, stddev);
  LD_HIP(hipGetLastError());
  return LD_OK;
}

}  // extern "C"
