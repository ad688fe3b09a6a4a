// lane_kernel.h -- one lane per orbit (or OPL orbits per lane): the
// integration kernel for systems of 1-3 degrees of freedom (Henon-Heiles,
// coupled quartic, harmonic).
//
// Each lane keeps its orbits -- state, force, the M deviation vectors and
// every accumulator -- in VGPRs for a whole launch; HBM is read once at the
// start and written once at the end (structure-of-arrays columns, so a
// wavefront's accesses are fully coalesced).  The work is FP64 FMA
// throughput bound.  With OPL = 2 a lane interleaves two independent
// orbits, doubling the instruction-level parallelism of the latency-bound
// parts (the Gram-Schmidt chains at checkpoints).
//
// Step (Yoshida-4 triple jump of kick-drift-kick leapfrog; the tangent map
// is its exact Jacobian):
//   K(d0) D(c0) K(d1) D(c1) K(d2) D(c2) K(d3),  c = (w1, w0, w1) dt,
//   d = (w1/2, (w1+w0)/2, (w1+w0)/2, w1/2) dt,
// with K: p -= d F(q), dp -= d H(q) dq;  D: q += c p, dq += c dp.
// The force after each drift serves the next kick (3 evaluations per
// step).  Kicks commute, so between two steps inside a checkpoint block
// K(d3) K(d0) of the deviation vectors is applied as one kick K(w1 dt); the
// state keeps both kicks because the Lagrangian descriptor needs p at every
// step endpoint.
//
// Checkpoint every K steps and at the last step (time t = s dt):
// non-finite and escape checks, renormalisation of the SALI/GALI set, SALI,
// modified Gram-Schmidt of the Lyapunov set, energy error, early exit.  An
// orbit that stops (escape, non-finite state, early exit) is written back
// at once and no longer updated.
#pragma once
#include "chx_internal.h"
#include "device_math.h"
#include "systems.h"

namespace chx {

template <class S, int M, bool GP, int OPL>
__global__ void __launch_bounds__(256) lane_kernel(const StepArgs a) {
  constexpr int N = S::N, D = 2 * N, MM = (M > 0 ? M : 1);
  const int64_t P = a.pitch;
  int64_t idx[OPL];
  bool act[OPL];
  bool any = false;
#pragma unroll
  for (int j = 0; j < OPL; ++j) {
    idx[j] = (int64_t)blockIdx.x * blockDim.x * OPL + (int64_t)j * blockDim.x + threadIdx.x;
    act[j] = idx[j] < a.n && a.st[idx[j]] == CHX_ORBIT_OK;
    any = any || act[j];
  }
  if (!any) return;

  double x[OPL][D], w[OPL][MM][D], gm[OPL][MM];
  int ge[OPL][MM];
  double ld[OPL], gprev[OPL], smin2[OPL], slast2[OPL], tch[OPL], eerr[OPL], H0[OPL],
      tend[OPL];
  int st[OPL];
#pragma unroll
  for (int j = 0; j < OPL; ++j) {
    const int64_t i = act[j] ? idx[j] : 0;  // inactive slots compute on a copy
#pragma unroll
    for (int c = 0; c < D; ++c) x[j][c] = a.x[c * P + i];
#pragma unroll
    for (int v = 0; v < M; ++v) {
#pragma unroll
      for (int c = 0; c < D; ++c) w[j][v][c] = a.w[((int64_t)v * D + c) * P + i];
      gm[j][v] = a.gm[v * P + i];
      ge[j][v] = a.ge[v * P + i];
    }
    ld[j] = a.sc[SC_LD * P + i];
    gprev[j] = a.sc[SC_GPREV * P + i];
    smin2[j] = a.sc[SC_SALI_MIN2 * P + i];
    slast2[j] = a.sc[SC_SALI_LAST2 * P + i];
    tch[j] = a.sc[SC_T_CHAOS * P + i];
    eerr[j] = a.sc[SC_EERR * P + i];
    H0[j] = a.sc[SC_H0 * P + i];
    tend[j] = a.sc[SC_T_END * P + i];
    st[j] = CHX_ORBIT_OK;
  }

  auto store = [&](int j) {
    const int64_t i = idx[j];
#pragma unroll
    for (int c = 0; c < D; ++c) a.x[c * P + i] = x[j][c];
#pragma unroll
    for (int v = 0; v < M; ++v) {
#pragma unroll
      for (int c = 0; c < D; ++c) a.w[((int64_t)v * D + c) * P + i] = w[j][v][c];
      a.gm[v * P + i] = gm[j][v];
      a.ge[v * P + i] = ge[j][v];
    }
    a.sc[SC_LD * P + i] = ld[j];
    a.sc[SC_GPREV * P + i] = gprev[j];
    a.sc[SC_SALI_MIN2 * P + i] = smin2[j];
    a.sc[SC_SALI_LAST2 * P + i] = slast2[j];
    a.sc[SC_T_CHAOS * P + i] = tch[j];
    a.sc[SC_EERR * P + i] = eerr[j];
    a.sc[SC_T_END * P + i] = tend[j];
    a.st[i] = st[j];
  };

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

  double F[OPL][N];
#pragma unroll
  for (int j = 0; j < OPL; ++j) S::force(x[j], F[j], a.prm);

  auto kick_vectors = [&](double hk) {
#pragma unroll
    for (int j = 0; j < OPL; ++j) {
      double Hs[S::NH];
      S::hess_scaled(x[j], hk, Hs, a.prm);
#pragma unroll
      for (int v = 0; v < M; ++v) {
        double dq[N];
#pragma unroll
        for (int r = 0; r < N; ++r) dq[r] = w[j][v][r];
#pragma unroll
        for (int r = 0; r < N; ++r) {
          double acc = w[j][v][N + r];
          if (S::diag_only) {
            acc = __builtin_fma(-Hs[hidx(N, r, r)], dq[r], acc);
          } else {
#pragma unroll
            for (int cc = 0; cc < N; ++cc)
              acc = __builtin_fma(-Hs[hidx(N, r, cc)], dq[cc], acc);
          }
          w[j][v][N + r] = acc;
        }
      }
    }
  };
  auto kick_state = [&](double hk) {
#pragma unroll
    for (int j = 0; j < OPL; ++j)
#pragma unroll
      for (int r = 0; r < N; ++r) x[j][N + r] = __builtin_fma(-hk, F[j][r], x[j][N + r]);
  };
  auto drift = [&](double c) {
#pragma unroll
    for (int j = 0; j < OPL; ++j) {
#pragma unroll
      for (int r = 0; r < N; ++r) x[j][r] = __builtin_fma(c, x[j][N + r], x[j][r]);
#pragma unroll
      for (int v = 0; v < M; ++v)
#pragma unroll
        for (int r = 0; r < N; ++r) w[j][v][r] = __builtin_fma(c, w[j][v][N + r], w[j][v][r]);
    }
  };
  auto force = [&]() {
#pragma unroll
    for (int j = 0; j < OPL; ++j) S::force(x[j], F[j], a.prm);
  };
  auto ld_term = [&](double u) {
    if constexpr (GP)
      return pow(__builtin_fabs(u), a.ld_p);
    else
      return sqrt_ld(u);
  };
  // One step without its closing kicks: the state gets K(d3) (the LD needs
  // p at the endpoint), the vectors wait for the merged kick.
  auto step_body = [&]() {
    drift(c0);
    force();
    kick_state(hk1);
    kick_vectors(hk1);
    drift(c1);
    force();
    kick_state(hk1);
    kick_vectors(hk1);
    drift(c0);
    force();
    kick_state(hk0);  // p at the step endpoint
    if (do_ld) {
#pragma unroll
      for (int j = 0; j < OPL; ++j) {
        double g = 0.0;
#pragma unroll
        for (int r = 0; r < N; ++r) g += ld_term(x[j][N + r]) + ld_term(F[j][r]);
        ld[j] = __builtin_fma(hdt, gprev[j] + g, ld[j]);
        gprev[j] = g;
      }
    }
  };

  // Checkpoint of orbit j at time t; returns false when the orbit stops.
  auto checkpoint = [&](int j, double t) {
    tend[j] = t;
    bool finite = true;
#pragma unroll
    for (int c = 0; c < D; ++c) finite = finite && __builtin_isfinite(x[j][c]);
    if (!finite) {
      st[j] = CHX_ORBIT_NONFINITE;
      return false;
    }
    bool escaped = false;
    if (a.escape_r2 > 0.0) {
      double r2 = 0.0;
#pragma unroll
      for (int r = 0; r < N; ++r) r2 = __builtin_fma(x[j][r], x[j][r], r2);
      escaped = r2 > a.escape_r2;
    }
    // SALI/GALI set: each vector back to unit length
#pragma unroll
    for (int v = 0; v < M; ++v) {
      if (v < m_s) {
        double r2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) r2 = __builtin_fma(w[j][v][c], w[j][v][c], r2);
        const double inv = rsqrt_nr(r2);
#pragma unroll
        for (int c = 0; c < D; ++c) w[j][v][c] *= inv;
        grow(gm[j][v], ge[j][v], r2);
      }
    }
    double s2 = 0.0;
    if (do_sali) {
      double sp = 0.0, sm = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double ap = w[j][0][c] + w[j][MM > 1 ? 1 : 0][c];
        const double am = w[j][0][c] - w[j][MM > 1 ? 1 : 0][c];
        sp = __builtin_fma(ap, ap, sp);
        sm = __builtin_fma(am, am, sm);
      }
      s2 = __builtin_fmin(sp, sm);
      slast2[j] = s2;
      smin2[j] = __builtin_fmin(smin2[j], s2);
      if (s2 < a.thr2 && __builtin_isnan(tch[j])) tch[j] = t;
    }
    // Lyapunov set: modified Gram-Schmidt in vector order
#pragma unroll
    for (int q = 0; q < M; ++q) {
      if (q >= m_s) {
#pragma unroll
        for (int l = 0; l < q; ++l) {
          if (l >= m_s) {
            double d = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) d = __builtin_fma(w[j][l][c], w[j][q][c], d);
#pragma unroll
            for (int c = 0; c < D; ++c) w[j][q][c] = __builtin_fma(-d, w[j][l][c], w[j][q][c]);
          }
        }
        double r2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) r2 = __builtin_fma(w[j][q][c], w[j][q][c], r2);
        const double inv = rsqrt_nr(r2);
#pragma unroll
        for (int c = 0; c < D; ++c) w[j][q][c] *= inv;
        grow(gm[j][q], ge[j][q], r2);
      }
    }
    if (do_energy) {
      double kin = 0.0;
#pragma unroll
      for (int r = 0; r < N; ++r) kin = __builtin_fma(x[j][N + r], x[j][N + r], kin);
      const double e = __builtin_fabs(__builtin_fma(0.5, kin, S::potential(x[j], a.prm)) - H0[j]);
      eerr[j] = __builtin_fmax(eerr[j], e);
    }
    if (escaped) {
      st[j] = CHX_ORBIT_ESCAPED;
      return false;
    }
    if (a.early_exit && do_sali && s2 < a.thr2) {
      st[j] = CHX_ORBIT_EXITED;
      return false;
    }
    return true;
  };

  int64_t s = a.s_begin;
  const int64_t K = a.K;
  while (s < a.s_end) {
    int64_t next = (s / K + 1) * K;
    if (next > a.n_total) next = a.n_total;
    const int blk = (int)(next - s);
    kick_state(hk0);
    kick_vectors(hk0);
    for (int k = 0; k + 1 < blk; ++k) {
      step_body();
      kick_state(hk0);  // first kick of the next step
      kick_vectors(hkm);
    }
    step_body();
    kick_vectors(hk0);
    s = next;
    const double t = (double)s * dt;
    if constexpr (OPL == 1) {
      // a stopped orbit leaves the loop; the write-back happens once, after
      // it (keeps the store addresses out of the loop's registers)
      if (!checkpoint(0, t)) break;
    } else {
      bool alive = false;
#pragma unroll
      for (int j = 0; j < OPL; ++j) {
        if (act[j]) {
          if (!checkpoint(j, t)) {
            store(j);
            act[j] = false;
          }
        }
        alive = alive || act[j];
      }
      if (!alive) break;
    }
  }
  if constexpr (OPL == 1) {
    store(0);
  } else {
#pragma unroll
    for (int j = 0; j < OPL; ++j)
      if (act[j]) store(j);
  }
}

// Dispatch over the vector count for one system; the LD exponent 1/2 takes
// the square-root kernel, any other exponent the pow() kernel.
template <class S, int M, int OPL>
struct LaneDispatch {
  static hipError_t go(int m, const StepArgs &a, int block, hipStream_t s) {
    if (m == M) {
      const bool gp = (a.ind & CHX_IND_LD) && a.ld_p != 0.5;
      if (gp) {
        const int64_t grid = (a.n + block - 1) / block;
        hipLaunchKernelGGL((lane_kernel<S, M, true, 1>), dim3((unsigned)grid), dim3(block), 0, s,
                           a);
      } else {
        const int64_t per = (int64_t)block * OPL;
        const int64_t grid = (a.n + per - 1) / per;
        hipLaunchKernelGGL((lane_kernel<S, M, false, OPL>), dim3((unsigned)grid), dim3(block), 0,
                           s, a);
      }
      return hipGetLastError();
    }
    return LaneDispatch<S, M - 1, OPL>::go(m, a, block, s);
  }
};
template <class S, int OPL>
struct LaneDispatch<S, -1, OPL> {
  static hipError_t go(int, const StepArgs &, int, hipStream_t) {
    return hipErrorInvalidValue;
  }
};

}  // namespace chx
