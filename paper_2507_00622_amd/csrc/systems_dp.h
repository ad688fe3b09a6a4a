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
// The field is written once over T = double (the vector field) and T =
// MDual<M> (a value and M derivative parts): evaluated at x + sum_v e_v dx_v
// it gives f(x) and Df(x) dx_v for every v, the right-hand sides of the
// variational equations, with the value parts computed once for all M.  A
// state stage evaluated alone leaves a record (sin and cos of both angles,
// both momenta) from which a deviation vector's stage later builds its dual
// numbers without calling the trigonometric functions again.
#pragma once
#include <hip/hip_runtime.h>

namespace chx {

template <int M>
struct MDual {
  double v;     // value
  double d[M];  // derivative parts
};
template <int M>
__device__ __forceinline__ MDual<M> operator+(const MDual<M> &a, const MDual<M> &b) {
  MDual<M> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int M>
__device__ __forceinline__ MDual<M> operator-(const MDual<M> &a, const MDual<M> &b) {
  MDual<M> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int M>
__device__ __forceinline__ MDual<M> operator*(const MDual<M> &a, const MDual<M> &b) {
  MDual<M> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = __builtin_fma(a.v, b.d[i], a.d[i] * b.v);
  return r;
}
template <int M>
__device__ __forceinline__ MDual<M> operator*(double k, const MDual<M> &a) {
  MDual<M> r;
  r.v = k * a.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = k * a.d[i];
  return r;
}
template <int M>
__device__ __forceinline__ MDual<M> operator-(double k, const MDual<M> &a) {
  MDual<M> r;
  r.v = k - a.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = -a.d[i];
  return r;
}
// 1 / a: one division for the value, d(1/a) = -da / a^2
template <int M>
__device__ __forceinline__ MDual<M> inv(const MDual<M> &a) {
  MDual<M> r;
  r.v = 1.0 / a.v;
  const double q2 = -(r.v * r.v);
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = q2 * a.d[i];
  return r;
}
__device__ __forceinline__ double inv(double a) { return 1.0 / a; }

// The rest of the arithmetic a general field written over T may use (the
// run-time compiled user systems write theirs this way): mixed operands,
// negation, quotients and the elementary functions, each with its
// derivative parts by the chain rule.
template <int M>
__device__ __forceinline__ MDual<M> operator-(const MDual<M> &a) {
  return 0.0 - a;
}
template <int M>
__device__ __forceinline__ MDual<M> operator*(const MDual<M> &a, double k) {
  return k * a;
}
template <int M>
__device__ __forceinline__ MDual<M> operator+(const MDual<M> &a, double k) {
  MDual<M> r = a;
  r.v = a.v + k;
  return r;
}
template <int M>
__device__ __forceinline__ MDual<M> operator+(double k, const MDual<M> &a) {
  return a + k;
}
template <int M>
__device__ __forceinline__ MDual<M> operator-(const MDual<M> &a, double k) {
  return a + (-k);
}
template <int M>
__device__ __forceinline__ MDual<M> operator/(const MDual<M> &a, const MDual<M> &b) {
  return a * inv(b);
}
template <int M>
__device__ __forceinline__ MDual<M> operator/(const MDual<M> &a, double k) {
  return (1.0 / k) * a;
}
template <int M>
__device__ __forceinline__ MDual<M> operator/(double k, const MDual<M> &b) {
  return k * inv(b);
}
// (the library's double functions stay visible beside these overloads)
using ::cos;
using ::exp;
using ::log;
using ::pow;
using ::sin;
using ::sqrt;
// f(a) with value fv and derivative dv at a.v
template <int M>
__device__ __forceinline__ MDual<M> chain(const MDual<M> &a, double fv, double dv) {
  MDual<M> r;
  r.v = fv;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = dv * a.d[i];
  return r;
}
template <int M>
__device__ __forceinline__ MDual<M> sin(const MDual<M> &a) {
  return chain(a, ::sin(a.v), ::cos(a.v));
}
template <int M>
__device__ __forceinline__ MDual<M> cos(const MDual<M> &a) {
  return chain(a, ::cos(a.v), -::sin(a.v));
}
template <int M>
__device__ __forceinline__ MDual<M> exp(const MDual<M> &a) {
  const double e = ::exp(a.v);
  return chain(a, e, e);
}
template <int M>
__device__ __forceinline__ MDual<M> log(const MDual<M> &a) {
  return chain(a, ::log(a.v), 1.0 / a.v);
}
template <int M>
__device__ __forceinline__ MDual<M> sqrt(const MDual<M> &a) {
  const double r = ::sqrt(a.v);
  return chain(a, r, 0.5 / r);
}
template <int M>
__device__ __forceinline__ MDual<M> pow(const MDual<M> &a, double k) {
  const double r = ::pow(a.v, k);
  return chain(a, r, k * ::pow(a.v, k - 1.0));
}

// sin and cos of an angle x with |x| < 2^32 (NaN beyond): Cody-Waite
// reduction x = k pi/2 + r + dr, k = rint(2x/pi), with pi/2 split into five
// heads of at most 20 significant bits (each k * head exact for |k| < 2^32)
// and a 53-bit tail, the subtraction of the second and third heads carried
// exactly (Knuth's two-sum) into dr; then the Taylor series of sin and cos on
// |r| <= pi/4 through r^17 and r^16 (truncation below 3e-18 relative),
// first-order corrections for dr, and the quadrant k mod 4.  Straight-line
// code: a wide-range reduction with a table (or a call) would hold many
// registers across the integrator's stage loop.
__host__ __device__ __forceinline__ void sincos_cw(double x, double &s, double &c) {
  const double k = __builtin_rint(x * 0x1.45f306dc9c883p-1);
  // t - k (P2 + P3) = r2 + e1 + e2 exactly (two two-sums), the rest of
  // k pi/2 (below 2^-28 |k| ... 2^-60 |k|) subtracted in the low part
  const double t = __builtin_fma(-k, 0x1.921fa00000000p+0, x);  // exact
  const double p2 = k * 0x1.5444200000000p-20;                    // exact
  const double p3 = k * 0x1.a308c00000000p-41;                    // exact
  const double r1 = t - p2, b1 = r1 - t;
  const double e1 = (t - (r1 - b1)) - (p2 + b1);
  const double r2 = r1 - p3, b2 = r2 - r1;
  const double e2 = (r1 - (r2 - b2)) - (p3 + b2);
  const double tail = __builtin_fma(k, 0x1.3131800000000p-61,
                                    __builtin_fma(k, 0x1.8a2e000000000p-81,
                                                  k * 0x1.b839a252049c1p-104));
  const double lo = (e1 + e2) - tail;
  const double r = r2 + lo;
  const double dr = lo - (r - r2);
  const double z = r * r;
  double ps = 0x1.952c77030ad4ap-49;  // 1/17!
  ps = __builtin_fma(ps, z, -0x1.ae7f3e733b81fp-41);
  ps = __builtin_fma(ps, z, 0x1.6124613a86d09p-33);
  ps = __builtin_fma(ps, z, -0x1.ae64567f544e4p-26);
  ps = __builtin_fma(ps, z, 0x1.71de3a556c734p-19);
  ps = __builtin_fma(ps, z, -0x1.a01a01a01a01ap-13);
  ps = __builtin_fma(ps, z, 0x1.1111111111111p-7);
  ps = __builtin_fma(ps, z, -0x1.5555555555555p-3);
  double pc = 0x1.ae7f3e733b81fp-45;  // 1/16!
  pc = __builtin_fma(pc, z, -0x1.93974a8c07c9dp-37);
  pc = __builtin_fma(pc, z, 0x1.1eed8eff8d898p-29);
  pc = __builtin_fma(pc, z, -0x1.27e4fb7789f5cp-22);
  pc = __builtin_fma(pc, z, 0x1.a01a01a01a01ap-16);
  pc = __builtin_fma(pc, z, -0x1.6c16c16c16c17p-10);
  pc = __builtin_fma(pc, z, 0x1.5555555555555p-5);
  // sin(r + dr) = r + (r z ps + dr (1 - z/2)); cos(r + dr) = 1 - z/2 +
  // (z^2 pc - r dr), with the rounding of 1 - z/2 carried along
  const double hz = 0.5 * z, wz = 1.0 - hz;
  const double sr = r + __builtin_fma(r * z, ps, dr * wz);
  const double cr = wz + ((((1.0 - wz) - hz) + (z * z) * pc) - r * dr);
  const long long kq = (__builtin_fabs(k) < 0x1p32) ? (long long)k : 0;
  const int q = (int)(kq & 3);
  const double a = (q & 1) ? cr : sr, b = (q & 1) ? sr : cr;
  const bool ok = __builtin_fabs(x) < 0x1p32;
  s = ok ? ((q & 2) ? -a : a) : __builtin_nan("");
  c = ok ? (((q + 1) & 2) ? -b : b) : __builtin_nan("");
}

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
    const T iD = inv(D);
    const T cp2 = c * p2, cp1 = c * p1;
    f[0] = (ia2 * p1 - ia * cp2) * iD;
    f[1] = (s1 * p2 - ia * cp1) * iD;
    const T p12 = p1 * p2;
    const T Q = (ia2 * (p1 * p1) - (2.0 * ia) * (c * p12)) + s1 * (p2 * p2);
    const T dTdc = (c * Q - ia * (p12 * D)) * (iD * iD);
    const T sd = s * dTdc;
    f[2] = sd - (al * s1) * s1t;
    f[3] = (0.0 - sd) - s2t;
  }
  // f = f(x) and the stage record of x
  __device__ static inline void rhs_rec(const double *x, double *f, double *rec,
                                        const double *prm) {
    sincos_cw(x[0], rec[0], rec[1]);
    sincos_cw(x[1], rec[2], rec[3]);
    rec[4] = x[2];
    rec[5] = x[3];
    field(rec[0], rec[1], rec[2], rec[3], rec[4], rec[5], f, prm);
  }
  // df = Df(x) dx from the stage record of x
  __device__ static inline void jvp(const double *rec, const double *dx, double *df,
                                    const double *prm) {
    const MDual<1> s1t{rec[0], {rec[1] * dx[0]}}, c1t{rec[1], {-rec[0] * dx[0]}};
    const MDual<1> s2t{rec[2], {rec[3] * dx[1]}}, c2t{rec[3], {-rec[2] * dx[1]}};
    const MDual<1> p1{rec[4], {dx[2]}}, p2{rec[5], {dx[3]}};
    MDual<1> f[4];
    field(s1t, c1t, s2t, c2t, p1, p2, f, prm);
#pragma unroll
    for (int c = 0; c < 4; ++c) df[c] = f[c].d[0];
  }
  // f = f(x) and df[v] = Df(x) dx[v] for M directions, in one evaluation
  template <int M>
  __device__ static inline void rhs_multi(const double *x, const double (&dx)[M][4],
                                          double *f, double (&df)[M][4], const double *prm) {
    double sa, ca, sb, cb;
    sincos_cw(x[0], sa, ca);
    sincos_cw(x[1], sb, cb);
    MDual<M> s1t, c1t, s2t, c2t, p1, p2;
    s1t.v = sa;
    c1t.v = ca;
    s2t.v = sb;
    c2t.v = cb;
    p1.v = x[2];
    p2.v = x[3];
#pragma unroll
    for (int v = 0; v < M; ++v) {
      s1t.d[v] = ca * dx[v][0];
      c1t.d[v] = -sa * dx[v][0];
      s2t.d[v] = cb * dx[v][1];
      c2t.d[v] = -sb * dx[v][1];
      p1.d[v] = dx[v][2];
      p2.d[v] = dx[v][3];
    }
    MDual<M> F[4];
    field(s1t, c1t, s2t, c2t, p1, p2, F, prm);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      f[c] = F[c].v;
#pragma unroll
      for (int v = 0; v < M; ++v) df[v][c] = F[c].d[v];
    }
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
