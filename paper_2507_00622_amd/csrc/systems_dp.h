// systems_dp.h -- the dimensionless double pendulum, a Hamiltonian that is
// not separable, for the Runge-Kutta lane kernels and the set-up kernel.
//
// Examples section (its Hamiltonian in matrix form and Hamilton's
// equations): x = (theta_1, theta_2, p_1, p_2), parameters {alpha, sigma}
// (length and mass ratios),
//   H = p^T B^{-1}(c) p / 2 - alpha (1 + sigma) cos theta_1 - cos theta_2,
//   c = cos(theta_1 - theta_2),
//   B^{-1}(c) = [[1/alpha^2, -c/alpha], [-c/alpha, 1 + sigma]] / (1 + sigma - c^2).
// With D = 1 + sigma - c^2 and Q = p_1^2/alpha^2 - 2 c p_1 p_2/alpha +
// (1 + sigma) p_2^2 the kinetic part is Q / (2D), and
//   theta' = B^{-1}(c) p,
//   p_1' = s dT/dc - alpha (1 + sigma) sin theta_1,
//   p_2' = -s dT/dc - sin theta_2,
// s = sin(theta_1 - theta_2), dT/dc = (c Q - p_1 p_2 D / alpha) / D^2, which
// is the printed (s/2) p^T C p with C = dB^{-1}/dc.
//
// The field is written once over T = double (the vector field) and T = Dual
// (value + derivative part): evaluated at x + e dx it gives f(x) + e Df(x) dx,
// the right-hand side of the variational equations.  The state's stage
// evaluation leaves a record (sin and cos of both angles, both momenta) from
// which a deviation vector's stage builds its dual numbers without calling
// the trigonometric functions again.
#pragma once
#include <hip/hip_runtime.h>

namespace chx {

struct Dual {
  double v, d;  // value, derivative part
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) {
  return {a.v * b.v, __builtin_fma(a.v, b.d, a.d * b.v)};
}
__device__ __forceinline__ Dual operator*(double k, Dual a) { return {k * a.v, k * a.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dual operator-(double k, Dual a) { return {k - a.v, -a.d}; }

struct SysDP {
  static constexpr int N = 2;
  static constexpr int NREC = 6;  // stage record: sin t1, cos t1, sin t2, cos t2, p1, p2
  template <class T>
  __device__ static inline void field(const T &s1t, const T &c1t, const T &s2t, const T &c2t,
                                      const T &p1, const T &p2, T *f, const double *prm) {
    const double al = prm[0], sg = prm[1];
    const double ia = 1.0 / al, ia2 = ia * ia, s1 = 1.0 + sg;
    // sin and cos of theta_1 - theta_2 from those of the angles
    const T s = s1t * c2t - c1t * s2t, c = c1t * c2t + s1t * s2t;
    const T D = s1 - c * c;
    const T cp2 = c * p2, cp1 = c * p1;
    f[0] = (ia2 * p1 - ia * cp2) / D;
    f[1] = (s1 * p2 - ia * cp1) / D;
    const T p12 = p1 * p2;
    const T Q = (ia2 * (p1 * p1) - (2.0 * ia) * (c * p12)) + s1 * (p2 * p2);
    const T dTdc = (c * Q - ia * (p12 * D)) / (D * D);
    const T sd = s * dTdc;
    f[2] = sd - (al * s1) * s1t;
    f[3] = (0.0 - sd) - s2t;
  }
  // f = f(x) and the stage record of x
  __device__ static inline void rhs_rec(const double *x, double *f, double *rec,
                                        const double *prm) {
    sincos(x[0], &rec[0], &rec[1]);
    sincos(x[1], &rec[2], &rec[3]);
    rec[4] = x[2];
    rec[5] = x[3];
    field(rec[0], rec[1], rec[2], rec[3], rec[4], rec[5], f, prm);
  }
  // df = Df(x) dx from the stage record of x
  __device__ static inline void jvp(const double *rec, const double *dx, double *df,
                                    const double *prm) {
    const Dual s1t{rec[0], rec[1] * dx[0]}, c1t{rec[1], -rec[0] * dx[0]};
    const Dual s2t{rec[2], rec[3] * dx[1]}, c2t{rec[3], -rec[2] * dx[1]};
    const Dual p1{rec[4], dx[2]}, p2{rec[5], dx[3]};
    Dual f[4];
    field(s1t, c1t, s2t, c2t, p1, p2, f, prm);
#pragma unroll
    for (int c = 0; c < 4; ++c) df[c] = f[c].d;
  }
  __device__ static inline double hamiltonian(const double *x, const double *prm) {
    const double al = prm[0], sg = prm[1];
    const double c = cos(x[0] - x[1]);
    const double D = 1.0 + sg - c * c;
    const double p1 = x[2], p2 = x[3];
    const double Q = p1 * p1 / (al * al) - 2.0 * c * p1 * p2 / al + (1.0 + sg) * p2 * p2;
    return Q / (2.0 * D) - al * (1.0 + sg) * cos(x[0]) - cos(x[1]);
  }
};

}  // namespace chx
