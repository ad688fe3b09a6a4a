// lane_kernel.h -- one lane per orbit: the integration kernel for systems of
// 1-3 degrees of freedom (Henon-Heiles, coupled quartic, harmonic).
//
// Each lane keeps its orbit -- state, force, Hessian, the M deviation
// vectors and every accumulator -- in VGPRs for a whole launch; HBM is read
// once at the start and written once at the end (structure-of-arrays
// columns, so a wavefront's accesses are fully coalesced).  The work is
// FP64 FMA throughput bound (see the roofline model of the benchmark).
//
// Step (Yoshida-4 triple jump of kick-drift-kick leapfrog; the tangent map
// is its exact Jacobian):
//   K(d0) D(c0) K(d1) D(c1) K(d2) D(c2) K(d3),  c = (w1, w0, w1) dt,
//   d = (w1/2, (w1+w0)/2, (w1+w0)/2, w1/2) dt,
// with K: p -= d F(q), dp -= d H(q) dq;  D: q += c p, dq += c dp.
// The force and Hessian after each drift are reused by the next kick (3
// evaluations per step).  Kicks commute, so between two steps inside a
// checkpoint block K(d3) K(d0) of the deviation vectors is applied as one
// kick K(w1 dt); the state keeps both kicks because the Lagrangian
// descriptor needs p at every step endpoint.
//
// Checkpoint every K steps and at the last step (time t = s dt):
// non-finite and escape checks, renormalisation of the SALI/GALI set, SALI,
// modified Gram-Schmidt of the Lyapunov set, energy error, early exit.
#pragma once
#include "chx_internal.h"
#include "device_math.h"
#include "systems.h"

namespace chx {

template <class S, int M, bool GP>
__global__ void __launch_bounds__(256) lane_kernel(const StepArgs a) {
  constexpr int N = S::N, D = 2 * N, MM = (M > 0 ? M : 1);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t P = a.pitch;
  int st = a.st[i];
  if (st != CHX_ORBIT_OK) return;

  double x[D];
#pragma unroll
  for (int c = 0; c < D; ++c) x[c] = a.x[c * P + i];
  double w[MM][D];
  double gm[MM];
  int ge[MM];
#pragma unroll
  for (int v = 0; v < M; ++v) {
#pragma unroll
    for (int c = 0; c < D; ++c) w[v][c] = a.w[((int64_t)v * D + c) * P + i];
    gm[v] = a.gm[v * P + i];
    ge[v] = a.ge[v * P + i];
  }
  double ld = a.sc[SC_LD * P + i], gprev = a.sc[SC_GPREV * P + i];
  double smin2 = a.sc[SC_SALI_MIN2 * P + i], slast2 = a.sc[SC_SALI_LAST2 * P + i];
  double tch = a.sc[SC_T_CHAOS * P + i], eerr = a.sc[SC_EERR * P + i];
  const double H0 = a.sc[SC_H0 * P + i];
  double tend = a.sc[SC_T_END * P + i];

  const double dt = a.dt;
  const double c0 = YOSHIDA_W1 * dt, c1 = YOSHIDA_W0 * dt;
  const double hk0 = (0.5 * YOSHIDA_W1) * dt;
  const double hk1 = (0.5 * (YOSHIDA_W1 + YOSHIDA_W0)) * dt;
  const double hkm = 2.0 * hk0;
  const double hdt = 0.5 * dt;
  const bool do_ld = (a.ind & CHX_IND_LD) != 0;
  const bool do_sali = (a.ind & CHX_IND_SALI) && a.m_s >= 2;
  const bool do_energy = (a.ind & CHX_IND_ENERGY) != 0;
  const int m_s = a.m_s;

  double F[N], H[S::NH], Hp[S::NH];
  S::force_hess(x, F, H, a.prm);

  auto kick_vectors = [&](double hk) {
#pragma unroll
    for (int k = 0; k < S::NH; ++k) Hp[k] = hk * H[k];
#pragma unroll
    for (int v = 0; v < M; ++v) {
      double dq[N];
#pragma unroll
      for (int r = 0; r < N; ++r) dq[r] = w[v][r];
#pragma unroll
      for (int r = 0; r < N; ++r) {
        double acc = w[v][N + r];
        if (S::diag_only) {
          acc = __builtin_fma(-Hp[hidx(N, r, r)], dq[r], acc);
        } else {
#pragma unroll
          for (int cc = 0; cc < N; ++cc) acc = __builtin_fma(-Hp[hidx(N, r, cc)], dq[cc], acc);
        }
        w[v][N + r] = acc;
      }
    }
  };
  auto kick_state = [&](double hk) {
#pragma unroll
    for (int r = 0; r < N; ++r) x[N + r] = __builtin_fma(-hk, F[r], x[N + r]);
  };
  auto drift = [&](double c) {
#pragma unroll
    for (int r = 0; r < N; ++r) x[r] = __builtin_fma(c, x[N + r], x[r]);
#pragma unroll
    for (int v = 0; v < M; ++v) {
#pragma unroll
      for (int r = 0; r < N; ++r) w[v][r] = __builtin_fma(c, w[v][N + r], w[v][r]);
    }
  };
  auto ld_term = [&](double u) {
    if constexpr (GP)
      return pow(__builtin_fabs(u), a.ld_p);
    else
      return sqrt_nr(__builtin_fabs(u));
  };

  int64_t s = a.s_begin;
  const int64_t K = a.K;
  while (s < a.s_end) {
    int64_t next = (s / K + 1) * K;
    if (next > a.n_total) next = a.n_total;
    const int blk = (int)(next - s);
    kick_state(hk0);
    kick_vectors(hk0);
    for (int k = 0; k < blk; ++k) {
      drift(c0);
      S::force_hess(x, F, H, a.prm);
      kick_state(hk1);
      kick_vectors(hk1);
      drift(c1);
      S::force_hess(x, F, H, a.prm);
      kick_state(hk1);
      kick_vectors(hk1);
      drift(c0);
      S::force_hess(x, F, H, a.prm);
      kick_state(hk0);  // p at the step endpoint
      if (do_ld) {
        double g = 0.0;
#pragma unroll
        for (int r = 0; r < N; ++r) g += ld_term(x[N + r]) + ld_term(F[r]);
        ld = __builtin_fma(hdt, gprev + g, ld);
        gprev = g;
      }
      if (k + 1 < blk) {
        kick_state(hk0);  // first kick of the next step
        kick_vectors(hkm);
      } else {
        kick_vectors(hk0);
      }
    }
    s = next;

    // ---- checkpoint at t = s dt ----
    const double t = (double)s * dt;
    tend = t;
    bool finite = true;
#pragma unroll
    for (int c = 0; c < D; ++c) finite = finite && __builtin_isfinite(x[c]);
    if (!finite) {
      st = CHX_ORBIT_NONFINITE;
      break;
    }
    bool escaped = false;
    if (a.escape_r2 > 0.0) {
      double r2 = 0.0;
#pragma unroll
      for (int r = 0; r < N; ++r) r2 = __builtin_fma(x[r], x[r], r2);
      escaped = r2 > a.escape_r2;
    }
    // SALI/GALI set: each vector back to unit length
#pragma unroll
    for (int v = 0; v < M; ++v) {
      if (v < m_s) {
        double r2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) r2 = __builtin_fma(w[v][c], w[v][c], r2);
        const double inv = rsqrt_nr(r2);
#pragma unroll
        for (int c = 0; c < D; ++c) w[v][c] *= inv;
        grow(gm[v], ge[v], r2);
      }
    }
    double s2 = 0.0;
    if (do_sali) {
      double sp = 0.0, sm = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double ap = w[0][c] + w[MM > 1 ? 1 : 0][c];
        const double am = w[0][c] - w[MM > 1 ? 1 : 0][c];
        sp = __builtin_fma(ap, ap, sp);
        sm = __builtin_fma(am, am, sm);
      }
      s2 = __builtin_fmin(sp, sm);
      slast2 = s2;
      smin2 = __builtin_fmin(smin2, s2);
      if (s2 < a.thr2 && __builtin_isnan(tch)) tch = t;
    }
    // Lyapunov set: modified Gram-Schmidt in vector order
#pragma unroll
    for (int j = 0; j < M; ++j) {
      if (j >= m_s) {
#pragma unroll
        for (int l = 0; l < j; ++l) {
          if (l >= m_s) {
            double d = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) d = __builtin_fma(w[l][c], w[j][c], d);
#pragma unroll
            for (int c = 0; c < D; ++c) w[j][c] = __builtin_fma(-d, w[l][c], w[j][c]);
          }
        }
        double r2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) r2 = __builtin_fma(w[j][c], w[j][c], r2);
        const double inv = rsqrt_nr(r2);
#pragma unroll
        for (int c = 0; c < D; ++c) w[j][c] *= inv;
        grow(gm[j], ge[j], r2);
      }
    }
    if (do_energy) {
      double kin = 0.0;
#pragma unroll
      for (int r = 0; r < N; ++r) kin = __builtin_fma(x[N + r], x[N + r], kin);
      const double e = __builtin_fabs(__builtin_fma(0.5, kin, S::potential(x, a.prm)) - H0);
      eerr = __builtin_fmax(eerr, e);
    }
    if (escaped) {
      st = CHX_ORBIT_ESCAPED;
      break;
    }
    if (a.early_exit && do_sali && s2 < a.thr2) {
      st = CHX_ORBIT_EXITED;
      break;
    }
  }

#pragma unroll
  for (int c = 0; c < D; ++c) a.x[c * P + i] = x[c];
#pragma unroll
  for (int v = 0; v < M; ++v) {
#pragma unroll
    for (int c = 0; c < D; ++c) a.w[((int64_t)v * D + c) * P + i] = w[v][c];
    a.gm[v * P + i] = gm[v];
    a.ge[v * P + i] = ge[v];
  }
  a.sc[SC_LD * P + i] = ld;
  a.sc[SC_GPREV * P + i] = gprev;
  a.sc[SC_SALI_MIN2 * P + i] = smin2;
  a.sc[SC_SALI_LAST2 * P + i] = slast2;
  a.sc[SC_T_CHAOS * P + i] = tch;
  a.sc[SC_EERR * P + i] = eerr;
  a.sc[SC_T_END * P + i] = tend;
  a.st[i] = st;
}

// Dispatch over the vector count for one system; the LD exponent 1/2 takes
// the square-root kernel, any other exponent the pow() kernel.
template <class S, int M>
struct LaneDispatch {
  static hipError_t go(int m, const StepArgs &a, int block, hipStream_t s) {
    if (m == M) {
      const int64_t grid = (a.n + block - 1) / block;
      const bool gp = (a.ind & CHX_IND_LD) && a.ld_p != 0.5;
      if (gp)
        hipLaunchKernelGGL((lane_kernel<S, M, true>), dim3((unsigned)grid), dim3(block), 0, s, a);
      else
        hipLaunchKernelGGL((lane_kernel<S, M, false>), dim3((unsigned)grid), dim3(block), 0, s, a);
      return hipGetLastError();
    }
    return LaneDispatch<S, M - 1>::go(m, a, block, s);
  }
};
template <class S>
struct LaneDispatch<S, -1> {
  static hipError_t go(int, const StepArgs &, int, hipStream_t) {
    return hipErrorInvalidValue;
  }
};

}  // namespace chx
