// Reciprocal and reciprocal square root from the hardware estimates.
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

// 1 / x for finite, nonzero x whose reciprocal is a normal number: the estimate refined by two
// Newton steps y <- y + y (1 - x y) (fused), each of which squares the relative error, to within
// rounding of FP64.  It replaces the scaled, correctly rounded division sequence (two scalings, a
// fix-up and a special-value pass) where the operand is known to be an ordinary positive or
// negative number.
__device__ __forceinline__ double rcp_refined(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}
