// lane_kernel.h -- one lane per orbit: the integration kernel for systems of
// 1-3 degrees of freedom (Henon-Heiles, coupled quartic, harmonic).
//
// Each lane keeps its orbit -- state, force, the M deviation vectors and
// every accumulator -- in VGPRs for a whole launch; HBM is read once at the
// start and written once at the end (structure-of-arrays columns, so a
// wavefront's accesses are fully coalesced).  The work is FP64 FMA
// throughput bound.
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
// modified Gram-Schmidt of the Lyapunov set, energy error, early exit.
//
// The per-orbit work lives in LaneOrbit so that the plain kernel below and
// the persistent batched kernel run the same arithmetic.
#pragma once
#include <type_traits>

#include "chx_internal.h"
#include "device_math.h"
#include "systems.h"

namespace chx {

// Systems whose Hamiltonian is not of the form |p|^2/2 + V(q) provide
// hamiltonian(x, prm) and a general right-hand side (systems_dp.h); only
// the Runge-Kutta kernels integrate them.
template <class S, class = void>
struct has_hamiltonian : std::false_type {};
template <class S>
struct has_hamiltonian<S, std::void_t<decltype(&S::hamiltonian)>> : std::true_type {};

// MS >= 0 fixes the size of the SALI/GALI set at compile time (the rest of
// the M vectors are the Lyapunov set), so the checkpoint has no branches on
// it; MS = -1 reads it from the launch arguments.
// CO: coherent loads and stores of the orbit's state (gld/gst), for the
// persistent kernel.
template <class S, int M, bool GP, int MS = -1, bool CO = false>
struct LaneOrbit {
  static constexpr int N = S::N, D = 2 * N, MM = (M > 0 ? M : 1);
  static constexpr int UNROLL = (N == 2 && M >= 4) ? 2 : 1;
  double x[D], w[MM][D], gm[MM];
  int ge[MM];
  double ld, gprev, smin2, slast2, tch, eerr, H0, tend;
  int st;
  double F[N];

  __device__ void load(const StepArgs &a, int64_t i) {
    const int64_t P = a.pitch;
#pragma unroll
    for (int c = 0; c < D; ++c) x[c] = gld<CO>(&a.x[c * P + i]);
#pragma unroll
    for (int v = 0; v < M; ++v) {
#pragma unroll
      for (int c = 0; c < D; ++c) w[v][c] = gld<CO>(&a.w[((int64_t)v * D + c) * P + i]);
      gm[v] = gld<CO>(&a.gm[v * P + i]);
      ge[v] = gld<CO>(&a.ge[v * P + i]);
    }
    ld = gld<CO>(&a.sc[SC_LD * P + i]);
    gprev = gld<CO>(&a.sc[SC_GPREV * P + i]);
    smin2 = gld<CO>(&a.sc[SC_SALI_MIN2 * P + i]);
    slast2 = gld<CO>(&a.sc[SC_SALI_LAST2 * P + i]);
    tch = gld<CO>(&a.sc[SC_T_CHAOS * P + i]);
    eerr = gld<CO>(&a.sc[SC_EERR * P + i]);
    H0 = gld<CO>(&a.sc[SC_H0 * P + i]);
    tend = gld<CO>(&a.sc[SC_T_END * P + i]);
    st = gld<CO>(&a.st[i]);
    if constexpr (!has_hamiltonian<S>::value) S::force(x, F, a.prm);
  }

  __device__ void store(const StepArgs &a, int64_t i) const {
    const int64_t P = a.pitch;
#pragma unroll
    for (int c = 0; c < D; ++c) gst<CO>(&a.x[c * P + i], x[c]);
#pragma unroll
    for (int v = 0; v < M; ++v) {
#pragma unroll
      for (int c = 0; c < D; ++c) gst<CO>(&a.w[((int64_t)v * D + c) * P + i], w[v][c]);
      gst<CO>(&a.gm[v * P + i], gm[v]);
      gst<CO>(&a.ge[v * P + i], ge[v]);
    }
    gst<CO>(&a.sc[SC_LD * P + i], ld);
    gst<CO>(&a.sc[SC_GPREV * P + i], gprev);
    gst<CO>(&a.sc[SC_SALI_MIN2 * P + i], smin2);
    gst<CO>(&a.sc[SC_SALI_LAST2 * P + i], slast2);
    gst<CO>(&a.sc[SC_T_CHAOS * P + i], tch);
    gst<CO>(&a.sc[SC_EERR * P + i], eerr);
    gst<CO>(&a.sc[SC_T_END * P + i], tend);
    gst<CO>(&a.st[i], st);
  }

  __device__ __forceinline__ void kick_vectors(const StepArgs &a, double hk) {
    double Hs[S::NH];
    S::hess_scaled(x, hk, Hs, a.prm);
#pragma unroll
    for (int v = 0; v < M; ++v) {
      double dq[N];
#pragma unroll
      for (int r = 0; r < N; ++r) dq[r] = w[v][r];
#pragma unroll
      for (int r = 0; r < N; ++r) {
        double acc = w[v][N + r];
        if (S::diag_only) {
          acc = __builtin_fma(-Hs[hidx(N, r, r)], dq[r], acc);
        } else {
#pragma unroll
          for (int cc = 0; cc < N; ++cc) acc = __builtin_fma(-Hs[hidx(N, r, cc)], dq[cc], acc);
        }
        w[v][N + r] = acc;
      }
    }
  }
  __device__ __forceinline__ void kick_state(double hk) {
#pragma unroll
    for (int r = 0; r < N; ++r) x[N + r] = __builtin_fma(-hk, F[r], x[N + r]);
  }
  __device__ __forceinline__ void drift(double c) {
#pragma unroll
    for (int r = 0; r < N; ++r) x[r] = __builtin_fma(c, x[N + r], x[r]);
#pragma unroll
    for (int v = 0; v < M; ++v)
#pragma unroll
      for (int r = 0; r < N; ++r) w[v][r] = __builtin_fma(c, w[v][N + r], w[v][r]);
  }
  __device__ __forceinline__ double ld_term(const StepArgs &a, double u) const {
    if constexpr (GP)
      return pow(__builtin_fabs(u), a.ld_p);
    else
      return sqrt_ld(u);
  }
  // One step without its closing kicks: the state gets K(d3) (the LD needs
  // p at the endpoint), the vectors wait for the merged kick.
  __device__ __forceinline__ void step_body(const StepArgs &a, const StepCoef &k, bool do_ld) {
    drift(k.c0);
    S::force(x, F, a.prm);
    kick_state(k.hk1);
    kick_vectors(a, k.hk1);
    drift(k.c1);
    S::force(x, F, a.prm);
    kick_state(k.hk1);
    kick_vectors(a, k.hk1);
    drift(k.c0);
    S::force(x, F, a.prm);
    kick_state(k.hk0);  // p at the step endpoint
    if (do_ld) {
      double g = 0.0;
#pragma unroll
      for (int r = 0; r < N; ++r) g += ld_term(a, x[N + r]) + ld_term(a, F[r]);
      ld = __builtin_fma(k.hdt, gprev + g, ld);
      gprev = g;
    }
  }
  // blk whole steps from one checkpoint to the next
  __device__ void block(const StepArgs &a, const StepCoef &k, int blk) {
    const bool do_ld = (a.ind & CHX_IND_LD) != 0;
    kick_state(k.hk0);
    kick_vectors(a, k.hk0);
    // two steps per iteration saves register moves of the loop-carried
    // values for 2-dof systems with several vectors; elsewhere it costs
    // occupancy
#pragma unroll(UNROLL)
    for (int s = 0; s + 1 < blk; ++s) {
      step_body(a, k, do_ld);
      kick_state(k.hk0);  // first kick of the next step
      kick_vectors(a, k.hkm);
    }
    step_body(a, k, do_ld);
    kick_vectors(a, k.hk0);
  }

  // Checkpoint at time t; returns false when the orbit stops (status set).
  __device__ bool checkpoint(const StepArgs &a, double t) {
    const int m_s = MS >= 0 ? MS : a.m_s;
    const bool do_sali = (a.ind & CHX_IND_SALI) && m_s >= 2;
    tend = t;
    bool finite = true;
#pragma unroll
    for (int c = 0; c < D; ++c) finite = finite && __builtin_isfinite(x[c]);
    if (!finite) {
      st = CHX_ORBIT_NONFINITE;
      return false;
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
    for (int q = 0; q < M; ++q) {
      if (q >= m_s) {
#pragma unroll
        for (int l = 0; l < q; ++l) {
          if (l >= m_s) {
            double d = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) d = __builtin_fma(w[l][c], w[q][c], d);
#pragma unroll
            for (int c = 0; c < D; ++c) w[q][c] = __builtin_fma(-d, w[l][c], w[q][c]);
          }
        }
        double r2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) r2 = __builtin_fma(w[q][c], w[q][c], r2);
        const double inv = rsqrt_nr(r2);
#pragma unroll
        for (int c = 0; c < D; ++c) w[q][c] *= inv;
        grow(gm[q], ge[q], r2);
      }
    }
    if (a.ind & CHX_IND_ENERGY) {
      double e;
      if constexpr (has_hamiltonian<S>::value) {
        e = __builtin_fabs(S::hamiltonian(x, a.prm) - H0);
      } else {
        double kin = 0.0;
#pragma unroll
        for (int r = 0; r < N; ++r) kin = __builtin_fma(x[N + r], x[N + r], kin);
        e = __builtin_fabs(__builtin_fma(0.5, kin, S::potential(x, a.prm)) - H0);
      }
      eerr = __builtin_fmax(eerr, e);
    }
    if (escaped) {
      st = CHX_ORBIT_ESCAPED;
      return false;
    }
    if (a.early_exit && do_sali && s2 < a.thr2) {
      st = CHX_ORBIT_EXITED;
      return false;
    }
    return true;
  }
};

template <class S, int M, bool GP, int MS>
__global__ void __launch_bounds__(256) lane_kernel(const StepArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  if (a.st[i] != CHX_ORBIT_OK) return;
  LaneOrbit<S, M, GP, MS> o;
  o.load(a, i);
  const StepCoef k(a.dt);
  int64_t s = a.s_begin;
  const int64_t K = a.K;
  while (s < a.s_end) {
    int64_t next = (s / K + 1) * K;
    if (next > a.n_total) next = a.n_total;
    o.block(a, k, (int)(next - s));
    s = next;
    // a stopped orbit leaves the loop; the write-back happens once, after it
    if (!o.checkpoint(a, (double)s * a.dt)) break;
  }
  // Hide the index from the optimiser so that the store addresses are formed
  // here rather than kept in registers from the loads across the whole loop.
  int64_t j = i;
  asm volatile("" : "+v"(j));
  o.store(a, j);
}

// Dispatch over the vector count for one system; the LD exponent 1/2 takes
// the square-root kernel, any other exponent the pow() kernel.
template <class S, int M>
struct LaneDispatch {
  static hipError_t go(int m, const StepArgs &a, int block, hipStream_t s) {
    if (m == M) {
      const bool gp = (a.ind & CHX_IND_LD) && a.ld_p != 0.5;
      const int64_t grid = (a.n + block - 1) / block;
      if (gp)
        hipLaunchKernelGGL((lane_kernel<S, M, true, -1>), dim3((unsigned)grid), dim3(block), 0, s,
                           a);
      else if (M >= 2 && a.m_s == 2)  // the SALI pair (+ Lyapunov vectors)
        hipLaunchKernelGGL((lane_kernel<S, M, false, (M >= 2 ? 2 : -1)>), dim3((unsigned)grid),
                           dim3(block), 0, s, a);
      else
        hipLaunchKernelGGL((lane_kernel<S, M, false, -1>), dim3((unsigned)grid), dim3(block), 0,
                           s, a);
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
