// Device logarithm used by the entropy-conservative flux.
#pragma once
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

// Natural logarithm of the EC flux variables: x = m 2^k with m in [sqrt(1/2), sqrt(2)), and
// log m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...) with s = (m - 1) / (m + 1), |s| < 0.1716; the
// series is summed to s^21 (relative truncation below 3e-18) and k ln 2 is added in two parts (the
// leading part holds 32 significant bits, so k times it is exact; the two constants are the public
// ln2_hi / ln2_lo split of Sun's freely distributable fdlibm).  Within 2 ulp of the correctly
// rounded logarithm over the whole double range, with about a third of the
// library function's instructions.  Special arguments as the library: log 0 = -inf, log inf = inf,
// NaN for negative and NaN arguments.
__device__ __forceinline__ double log_ec(double x) {
  int k;
  double m = frexp(x, &k);  // m in [1/2, 1)
  const bool lo = m < 0.70710678118654752440;
  m = lo ? 2.0 * m : m;
  k = lo ? k - 1 : k;
  const double s = (m - 1.0) / (m + 1.0), z = s * s;
  double p = 1.0 / 21.0;
  p = fma(p, z, 1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  const double s2 = 2.0 * s, kd = (double)k;
  const double LN2_HI = 6.93147180369123816490e-01, LN2_LO = 1.90821492927058770002e-10;
  const double r = fma(kd, LN2_HI, s2 + fma(s2 * z, p, kd * LN2_LO));
  return x > 0.0 ? (x <= DBL_MAX ? r : x) : (x == 0.0 ? -HUGE_VAL : __builtin_nan(""));
}
