// Covariance-kernel values (Section 3 kernels: RBF and Matern-5/2 in their
// textbook forms): FP32 for the on-the-fly products, FP64 for the FP64 path
// and the preconditioner builds.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "logdet.h"

namespace ld {
namespace dev {

constexpr float kLog2eF = 1.4426950408889634f;

// FP32 kernel values with the constants folded into base-2 exponents and
// into the points: the FP32 points are stored times
//   RBF     sqrt(c), c = log2(e) / (2 l^2):  r2 = c r^2 (scaled), v = log2(variance),
//           value 2^(v - r2)
//   Matern  c = sqrt(5) log2(e) / l:  u = sqrt(r2) = c r (= t log2 e, t = sqrt5 r / l),
//           v = variance, value variance (1 + t + t^2/3) e^-t
//           = (v + u v / log2e + u^2 v / (3 log2e^2)) 2^-u
template <int KIND>
__device__ __forceinline__ float kval32s(float r2, float v) {
  if (KIND == LD_RBF) return __builtin_amdgcn_exp2f(v - r2);
  const float u = __builtin_amdgcn_sqrtf(r2);
  const float p = __builtin_fmaf(
      u, __builtin_fmaf(u, v * (1.0f / (3.0f * kLog2eF * kLog2eF)), v * (1.0f / kLog2eF)), v);
  return p * __builtin_amdgcn_exp2f(-u);
}

// Derivatives of the kernels with respect to the lengthscale l, as further
// FP64 kernel kinds (gradient of log det): with the same c as the kernel,
//   RBF     dk/dl = (variance / l^3) r^2 exp(-r^2 c)
//   Matern  dk/dl = (variance / (3 l)) t^2 (1 + t) exp(-t),  t = sqrt(r^2) c
// (the factor in brackets is passed as `var`).
constexpr int kKindRbfDl = 2;
constexpr int kKindMaternDl = 3;

// FP64 values: RBF c = 1 / (2 l^2);  Matern-5/2 c = sqrt(5) / l
template <int KIND>
__device__ __forceinline__ double kval64(double r2, double var, double c) {
  if (KIND == LD_RBF) return var * exp(-r2 * c);
  if (KIND == kKindRbfDl) return var * r2 * exp(-r2 * c);
  const double t = sqrt(r2) * c;
  if (KIND == kKindMaternDl) return var * t * t * (1.0 + t) * exp(-t);
  return var * (1.0 + t + t * t * (1.0 / 3.0)) * exp(-t);
}

}  // namespace dev
}  // namespace ld
