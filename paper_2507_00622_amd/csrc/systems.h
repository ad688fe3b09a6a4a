// systems.h -- potentials, forces and Hessians of the built-in systems for
// the lane-per-orbit kernel.  Each system gives, at a configuration q:
//   force(q, F):            F = grad V(q)                      (N values)
//   hess_scaled(q, h, Hs):  Hs = h Hess V(q), packed upper triangle,
//                           Hs[hidx(i, j)] for i <= j
// in registers.  The kernels use them for the kick of the state
// (p -= h F) and of every deviation vector (dp -= h Hess V dq); the step
// size h is folded into the Hessian's coefficients where the system allows,
// so a kick costs no separate rescaling.
#pragma once
#include <hip/hip_runtime.h>

#include "chx_internal.h"

namespace chx {

__host__ __device__ constexpr int hidx(int N, int i, int j) {
  return (i <= j) ? i * N - (i * (i - 1)) / 2 + (j - i) : j * N - (j * (j - 1)) / 2 + (i - j);
}

// Henon-Heiles (Examples section): V = (x^2 + y^2)/2 + x^2 y - y^3/3,
// dV/dx = x (1 + 2y), dV/dy = y - y^2 + x^2; Hessian [[1+2y, 2x], [2x, 1-2y]].
struct SysHH {
  static constexpr int N = 2;
  static constexpr int NH = 3;
  static constexpr bool diag_only = false;
  __device__ static inline void force(const double *q, double *F, const double *) {
    const double x = q[0], y = q[1];
    F[0] = __builtin_fma(x + x, y, x);
    F[1] = __builtin_fma(x, x, __builtin_fma(-y, y, y));
  }
  __device__ static inline void hess_scaled(const double *q, double h, double *Hs,
                                            const double *) {
    const double h2 = h + h;
    Hs[0] = __builtin_fma(h2, q[1], h);
    Hs[1] = h2 * q[0];
    Hs[2] = __builtin_fma(-h2, q[1], h);
  }
  __device__ static inline double potential(const double *q, const double *) {
    const double x = q[0], y = q[1];
    const double r2 = __builtin_fma(x, x, y * y);
    return __builtin_fma(0.5, r2, y * __builtin_fma(x, x, (-1.0 / 3.0) * y * y));
  }
};

// Coupled quartic oscillator: V = sum q_i^4/4 + eps sum_{i<j} q_i^2 q_j^2.
// With S = |q|^2: dV/dq_i = q_i ((1 - 2 eps) q_i^2 + 2 eps S),
// H_ii = (3 - 2 eps) q_i^2 + 2 eps S, H_ij = 4 eps q_i q_j.
template <int NN>
struct SysQuartic {
  static constexpr int N = NN;
  static constexpr int NH = NN * (NN + 1) / 2;
  static constexpr bool diag_only = false;
  __device__ static inline void force(const double *q, double *F, const double *prm) {
    const double eps = prm[0];
    double S = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) S = __builtin_fma(q[i], q[i], S);
    const double te = 2.0 * eps * S, a1 = 1.0 - 2.0 * eps;
#pragma unroll
    for (int i = 0; i < N; ++i) F[i] = q[i] * __builtin_fma(a1, q[i] * q[i], te);
  }
  __device__ static inline void hess_scaled(const double *q, double h, double *Hs,
                                            const double *prm) {
    const double eps = prm[0];
    double S = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) S = __builtin_fma(q[i], q[i], S);
    const double hte = (2.0 * eps * h) * S, ha3 = (3.0 - 2.0 * eps) * h, he4 = 4.0 * eps * h;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      Hs[hidx(N, i, i)] = __builtin_fma(ha3, q[i] * q[i], hte);
#pragma unroll
      for (int j = i + 1; j < N; ++j) Hs[hidx(N, i, j)] = (he4 * q[i]) * q[j];
    }
  }
  __device__ static inline void force_hess(const double *q, double *F, double *H,
                                           const double *prm) {
    force(q, F, prm);
    hess_scaled(q, 1.0, H, prm);
  }
  __device__ static inline double potential(const double *q, const double *prm) {
    const double eps = prm[0];
    double v = 0.0, c = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double qi2 = q[i] * q[i];
      v = __builtin_fma(0.25 * qi2, qi2, v);
#pragma unroll
      for (int j = i + 1; j < N; ++j) c = __builtin_fma(qi2, q[j] * q[j], c);
    }
    return __builtin_fma(eps, c, v);
  }
};

// Uncoupled harmonic oscillators: V = sum omega_i^2 q_i^2 / 2 (prm = omega).
template <int NN>
struct SysHarmonic {
  static constexpr int N = NN;
  static constexpr int NH = NN * (NN + 1) / 2;
  static constexpr bool diag_only = true;
  __device__ static inline void force(const double *q, double *F, const double *prm) {
#pragma unroll
    for (int i = 0; i < N; ++i) F[i] = (prm[i] * prm[i]) * q[i];
  }
  __device__ static inline void hess_scaled(const double *, double h, double *Hs,
                                            const double *prm) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      Hs[hidx(N, i, i)] = h * (prm[i] * prm[i]);
#pragma unroll
      for (int j = i + 1; j < N; ++j) Hs[hidx(N, i, j)] = 0.0;
    }
  }
  __device__ static inline double potential(const double *q, const double *prm) {
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double a = prm[i] * q[i];
      v = __builtin_fma(0.5 * a, a, v);
    }
    return v;
  }
};

}  // namespace chx
