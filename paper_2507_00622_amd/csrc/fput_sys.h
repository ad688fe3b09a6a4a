// fput_sys.h -- Fermi-Pasta-Ulam chain with fixed ends (Examples section):
// masses i = 1..N, springs j = 1..N+1 with extension d_j = q_j - q_{j-1}
// and q_0 = q_{N+1} = 0 (the boundary condition printed with the equations
// of motion, which contain the wall springs):
//   V = sum_j [k d_j^2/2 + alpha d_j^3/3 + beta d_j^4/4],
//   dV/dq_i = phi'(d_i) - phi'(d_{i+1}),  phi'(d) = d (k + d (alpha + beta d)),
//   Hessian tridiagonal with kappa_j = phi''(d_j) = k + d_j (2 alpha + 3 beta d_j):
//   H_ii = kappa_i + kappa_{i+1},  H_{i,i+1} = -kappa_{i+1}.
// Generic (non-hot) device helpers used for set-up and output.
#pragma once
#include <hip/hip_runtime.h>

namespace chx {

__device__ inline double fput_qw(const double *q, int N, int j) {
  return (j <= 0 || j > N) ? 0.0 : q[j - 1];
}

__device__ inline double fput_potential(const double *q, int N, const double *prm) {
  const double k = prm[0], al = prm[1], be = prm[2];
  double v = 0.0;
  for (int j = 1; j <= N + 1; ++j) {
    const double d = fput_qw(q, N, j) - fput_qw(q, N, j - 1);
    const double d2 = d * d;
    v += d2 * __builtin_fma(d, __builtin_fma(0.25 * be, d, al * (1.0 / 3.0)), 0.5 * k);
  }
  return v;
}

__device__ inline double fput_dphi(double d, const double *prm) {
  return d * __builtin_fma(d, __builtin_fma(prm[2], d, prm[1]), prm[0]);
}

__device__ inline void fput_force(const double *q, int N, const double *prm, double *F) {
  for (int i = 1; i <= N; ++i) {
    const double dl = fput_qw(q, N, i) - fput_qw(q, N, i - 1);
    const double dr = fput_qw(q, N, i + 1) - fput_qw(q, N, i);
    F[i - 1] = fput_dphi(dl, prm) - fput_dphi(dr, prm);
  }
}

}  // namespace chx
