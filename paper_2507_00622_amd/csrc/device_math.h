// device_math.h -- small device helpers of the HIP path.
#pragma once
#include <hip/hip_runtime.h>

namespace chx {

// Yoshida (1990) fourth-order triple jump S(w1 h) S(w0 h) S(w1 h) of the
// kick-drift-kick leapfrog S(h): w1 = 1/(2 - 2^(1/3)),
// w0 = -2^(1/3)/(2 - 2^(1/3)), as the nearest binary64 values.
constexpr double YOSHIDA_W1 = 1.3512071919596575;
constexpr double YOSHIDA_W0 = -1.7024143839193153;

// 1/sqrt(a) for a > 0, relative error below 1e-14: the hardware estimate
// (relative error up to about 5e-8 on gfx950) refined by one Newton step
// y <- y + y (1 - a y^2) / 2, which leaves 1.5 e^2.  Used to rescale
// deviation vectors; the growth accounting takes |w|^2 itself, so a
// rescaled vector off unit length by 1e-14 only moves the next norm.
__device__ __forceinline__ double rsqrt_nr(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  const double e = __builtin_fma(-a * y, y, 1.0);
  return __builtin_fma(0.5 * y, e, y);
}

// sqrt(|a|) for the Lagrangian-descriptor integrand, relative error below
// 1e-14: one Goldschmidt step from the hardware reciprocal-root estimate
// (error 1.5 e^2 for an estimate with relative error e; e <= 5.3e-8 was
// measured over 2^20 arguments spanning 1e-13..1e13 on gfx950, giving
// 4e-15).  |a| is
// offset by 1e-300 -- invisible for |a| > 1e-284 -- so that a = 0 gives
// 1e-150 instead of 0 * inf.
__device__ __forceinline__ double sqrt_ld(double a) {
  a = __builtin_fabs(a) + 1e-300;
  const double y = __builtin_amdgcn_rsq(a);
  const double s = a * y;
  const double h = 0.5 * y;
  const double r = __builtin_fma(-s, h, 0.5);
  return __builtin_fma(s, r, s);
}

// Step coefficients of one launch.
struct StepCoef {
  double c0, c1, hk0, hk1, hkm, hdt;
  __device__ explicit StepCoef(double dt)
      : c0(YOSHIDA_W1 * dt), c1(YOSHIDA_W0 * dt), hk0((0.5 * YOSHIDA_W1) * dt),
        hk1((0.5 * (YOSHIDA_W1 + YOSHIDA_W0)) * dt), hkm(2.0 * ((0.5 * YOSHIDA_W1) * dt)),
        hdt(0.5 * dt) {}
};

// Keep a growth product as mantissa * 2^exponent: multiply the mantissa by
// f and move its binary exponent into e.
__device__ __forceinline__ void grow(double &m, int &e, double f) {
  m *= f;
  int k = __builtin_amdgcn_frexp_exp(m);
  m = __builtin_amdgcn_frexp_mant(m);
  e += k;
}

// Loads and stores of orbit state that a wavefront on another XCD may read
// or write in another launch (the persistent kernel moves orbits between
// wavefronts): with CO they are agent-scope relaxed atomics, which the
// XCDs' L2 caches keep coherent; otherwise plain accesses.
template <bool CO, class T>
__device__ __forceinline__ T gld(const T *p) {
  if constexpr (CO)
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *p;
}
template <bool CO, class T>
__device__ __forceinline__ void gst(T *p, T v) {
  if constexpr (CO)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}

}  // namespace chx
