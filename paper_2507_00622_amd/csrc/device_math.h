// device_math.h -- small device helpers of the HIP path.
#pragma once
#include <hip/hip_runtime.h>

namespace chx {

// Yoshida (1990) fourth-order triple jump S(w1 h) S(w0 h) S(w1 h) of the
// kick-drift-kick leapfrog S(h): w1 = 1/(2 - 2^(1/3)),
// w0 = -2^(1/3)/(2 - 2^(1/3)), as the nearest binary64 values.
constexpr double YOSHIDA_W1 = 1.3512071919596575;
constexpr double YOSHIDA_W0 = -1.7024143839193153;

// 1/sqrt(a) for a > 0 to about one ulp: the hardware estimate refined by
// two Newton steps y <- y + y (1 - a y^2) / 2.
__device__ __forceinline__ double rsqrt_nr(double a) {
  double y = __builtin_amdgcn_rsq(a);
  double e = __builtin_fma(-a * y, y, 1.0);
  y = __builtin_fma(0.5 * y, e, y);
  e = __builtin_fma(-a * y, y, 1.0);
  return __builtin_fma(0.5 * y, e, y);
}

// sqrt(a) for a >= 0, relative error a few 1e-16: s = a y with y the
// refined reciprocal root estimate (Goldschmidt step, then a Newton
// correction of s).  a is floored at 1e-300 so that a = 0 gives 1e-150,
// which no sum of O(1) terms can see.
__device__ __forceinline__ double sqrt_nr(double a) {
  a = __builtin_fmax(a, 1e-300);
  double y = __builtin_amdgcn_rsq(a);
  double s = a * y;
  double h = 0.5 * y;
  double r = __builtin_fma(-s, h, 0.5);
  s = __builtin_fma(s, r, s);
  h = __builtin_fma(h, r, h);
  r = __builtin_fma(-s, s, a);
  return __builtin_fma(r, h, s);
}

// Keep a growth product as mantissa * 2^exponent: multiply the mantissa by
// f and move its binary exponent into e.
__device__ __forceinline__ void grow(double &m, int &e, double f) {
  m *= f;
  int k = __builtin_amdgcn_frexp_exp(m);
  m = __builtin_amdgcn_frexp_mant(m);
  e += k;
}

}  // namespace chx
