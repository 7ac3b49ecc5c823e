// Counter-based random blocks: Rademacher probes (Algorithm 1 step 1) and the
// Gaussian test matrix of the randomized range finder (Section 2).  The
// generator itself is in rng_dev.hpp.
#include "ld_common.hpp"
#include "rng_dev.hpp"

namespace ld {
namespace {

template <typename T>
__global__ void k_rademacher(uint64_t key, int64_t total, T* __restrict__ Z) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < total; i += stride) Z[i] = (T)dev::rng_rademacher(key, (uint64_t)i);
}

__global__ void k_gaussian(uint64_t key, int64_t total, double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < total; i += stride) out[i] = dev::rng_gaussian(key, (uint64_t)i);
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
