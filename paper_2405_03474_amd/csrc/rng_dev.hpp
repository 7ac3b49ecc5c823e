// Device side of the counter-based random stream (probe vectors of
// Algorithm 1 step 1; Gaussian test matrix of the range finder, Section 2).
// bits(i) = mix(key + G (i + 1)) with mix the SplitMix64 finalizer and
// key = mix(seed + G (stream + 1)) derived on the host.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ld {
namespace dev {

__device__ __forceinline__ uint64_t rng_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t rng_bits(uint64_t key, uint64_t idx) {
  return rng_mix(key + 0x9E3779B97F4A7C15ull * (idx + 1ull));
}

// ((bits >> 11) + 1/2) 2^-53, strictly inside (0, 1)
__device__ __forceinline__ double rng_uniform(uint64_t b) {
  return ((double)(b >> 11) + 0.5) * 0x1.0p-53;
}

// bit 63 clear -> +1, set -> -1
__device__ __forceinline__ float rng_rademacher(uint64_t key, uint64_t idx) {
  return (rng_bits(key, idx) >> 63) ? -1.f : 1.f;
}

// sqrt(-2 ln u(2i)) cos(2 pi u(2i + 1))
__device__ __forceinline__ double rng_gaussian(uint64_t key, uint64_t idx) {
  const double u1 = rng_uniform(rng_bits(key, 2ull * idx));
  const double u2 = rng_uniform(rng_bits(key, 2ull * idx + 1ull));
  return sqrt(-2.0 * log(u1)) * cos((2.0 * 3.141592653589793) * u2);
}

}  // namespace dev
}  // namespace ld
