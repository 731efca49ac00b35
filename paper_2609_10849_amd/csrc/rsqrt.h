// Reciprocal square root from the hardware estimate.
#pragma once
#include <hip/hip_runtime.h>

#include <cfloat>

// 1 / sqrt(x) for x > 0: the estimate refined by two Newton steps y <- y (3/2 - x y^2 / 2), each of
// which squares the relative error, to within rounding of FP64.
__device__ __forceinline__ double rsqrt_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * (1.5 - h * y * y);
  y = y * (1.5 - h * y * y);
  return y;
}
