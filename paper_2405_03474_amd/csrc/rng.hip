// Counter-based random blocks: Rademacher probes (Algorithm 1 step 1) and the
// Gaussian test matrix of the randomized range finder (Section 2).
//
// bits(i) = mix(key + G * (i + 1)) with mix the SplitMix64 finalizer and
// key = mix(seed + G * (stream + 1)) derived on the host.  Rademacher takes
// bit 63 (0 -> +1); uniforms are ((bits >> 11) + 1/2) * 2^-53; a normal is
// sqrt(-2 ln u(2i)) cos(2 pi u(2i+1)).
#include "ld_common.hpp"

namespace ld {
namespace {

__device__ __forceinline__ uint64_t dmix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t dbits(uint64_t key, uint64_t idx) {
  return dmix(key + kGolden * (idx + 1ull));
}

__device__ __forceinline__ double duniform(uint64_t b) {
  return ((double)(b >> 11) + 0.5) * 0x1.0p-53;
}

template <typename T>
__global__ void k_rademacher(uint64_t key, int64_t total, T* __restrict__ Z) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < total; i += stride) {
    uint64_t b = dbits(key, (uint64_t)i);
    Z[i] = (b >> 63) ? T(-1) : T(1);
  }
}

__global__ void k_gaussian(uint64_t key, int64_t total, double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const double two_pi = 2.0 * 3.141592653589793;
  for (; i < total; i += stride) {
    double u1 = duniform(dbits(key, 2ull * (uint64_t)i));
    double u2 = duniform(dbits(key, 2ull * (uint64_t)i + 1ull));
    out[i] = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
  }
}

int grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

void launch_fill_rademacher(hipStream_t st, uint64_t key, int64_t n, int64_t s, bool f64, void* Z) {
  int64_t total = n * s;
  if (total <= 0) return;
  if (f64)
    hipLaunchKernelGGL(k_rademacher<double>, dim3(grid_for(total)), dim3(256), 0, st, key, total,
                       (double*)Z);
  else
    hipLaunchKernelGGL(k_rademacher<float>, dim3(grid_for(total)), dim3(256), 0, st, key, total,
                       (float*)Z);
}

void launch_fill_gaussian(hipStream_t st, uint64_t key, int64_t rows, int64_t cols, double* out) {
  int64_t total = rows * cols;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_gaussian, dim3(grid_for(total)), dim3(256), 0, st, key, total, out);
}

}  // namespace ld
