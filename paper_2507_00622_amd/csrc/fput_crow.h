// fput_crow.h -- Fermi-Pasta-Ulam chains with few deviation vectors: one
// 16-lane row per orbit, lane l holding component l of the state AND of
// every deviation vector ("component row").
//
// With M = 1..4 vectors a vector-per-lane layout would leave most of the row
// idle; here every lane works on its own component: drifts and the state
// kick are lane-local, the springs read the neighbours' q through
// row_shr/row_shl DPP (bound_ctrl zero = the walls q_0 = q_{N+1} = 0, ghost
// lanes N..15 hold zeros), and each tangent kick reads dq_{l-1}, dq_{l+1}
// the same way:
//   dp_l -= h [(kappa_l + kappa_{l+1}) dq_l - kappa_l dq_{l-1} - kappa_{l+1} dq_{l+1}].
// Norms, dot products, the LD integrand and the energy are row sums
// (quad_perm / half-mirror / mirror butterfly, identical bits in all 16
// lanes), so all per-orbit decisions are row-uniform.  Few registers per
// lane (state, 2M vector components), so the kernel runs at high
// occupancy; this is also the FPU path of the persistent batched kernel.
#pragma once
#include "chx_internal.h"
#include "device_math.h"
#include "fput_row.h"

namespace chx {

// CO: coherent loads and stores of the orbit's state (gld/gst), for the
// persistent kernel.
template <int N, int M, bool CO = false>
struct CRowOrbit {
  static constexpr int MM = (M > 0 ? M : 1);
  double q, p, F, kl, kr;
  double dq[MM], dp[MM], gm[MM];
  int ge[MM];
  double ld, gprev, smin2, slast2, tch, eerr, H0, tend;
  int st;
  bool mass;
  int lane, row;

  __device__ void init_lane() {
    lane = threadIdx.x & 15;
    row = (threadIdx.x & 63) >> 4;
    mass = lane < N;
  }

  __device__ void load(const StepArgs &a, int64_t o) {
    init_lane();
    const int64_t P = a.pitch;
    q = mass ? gld<CO>(&a.x[lane * P + o]) : 0.0;
    p = mass ? gld<CO>(&a.x[(N + lane) * P + o]) : 0.0;
#pragma unroll
    for (int v = 0; v < M; ++v) {
      dq[v] = mass ? gld<CO>(&a.w[((int64_t)v * 2 * N + lane) * P + o]) : 0.0;
      dp[v] = mass ? gld<CO>(&a.w[((int64_t)v * 2 * N + N + lane) * P + o]) : 0.0;
      gm[v] = gld<CO>(&a.gm[v * P + o]);
      ge[v] = gld<CO>(&a.ge[v * P + o]);
    }
    ld = gld<CO>(&a.sc[SC_LD * P + o]);
    gprev = gld<CO>(&a.sc[SC_GPREV * P + o]);
    smin2 = gld<CO>(&a.sc[SC_SALI_MIN2 * P + o]);
    slast2 = gld<CO>(&a.sc[SC_SALI_LAST2 * P + o]);
    tch = gld<CO>(&a.sc[SC_T_CHAOS * P + o]);
    eerr = gld<CO>(&a.sc[SC_EERR * P + o]);
    H0 = gld<CO>(&a.sc[SC_H0 * P + o]);
    tend = gld<CO>(&a.sc[SC_T_END * P + o]);
    st = gld<CO>(&a.st[o]);
    springs(a);
  }

  __device__ void store(const StepArgs &a, int64_t o) const {
    const int64_t P = a.pitch;
    if (mass) {
      gst<CO>(&a.x[lane * P + o], q);
      gst<CO>(&a.x[(N + lane) * P + o], p);
#pragma unroll
      for (int v = 0; v < M; ++v) {
        gst<CO>(&a.w[((int64_t)v * 2 * N + lane) * P + o], dq[v]);
        gst<CO>(&a.w[((int64_t)v * 2 * N + N + lane) * P + o], dp[v]);
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int v = 0; v < M; ++v) {
        gst<CO>(&a.gm[v * P + o], gm[v]);
        gst<CO>(&a.ge[v * P + o], ge[v]);
      }
      gst<CO>(&a.sc[SC_LD * P + o], ld);
      gst<CO>(&a.sc[SC_GPREV * P + o], gprev);
      gst<CO>(&a.sc[SC_SALI_MIN2 * P + o], smin2);
      gst<CO>(&a.sc[SC_SALI_LAST2 * P + o], slast2);
      gst<CO>(&a.sc[SC_T_CHAOS * P + o], tch);
      gst<CO>(&a.sc[SC_EERR * P + o], eerr);
      gst<CO>(&a.sc[SC_T_END * P + o], tend);
      gst<CO>(&a.st[o], st);
    }
  }

  // Net spring force F = V'(d_l) - V'(d_{l+1}) on the mass of this lane at
  // positions y (one per lane, ghosts zero), and the stiffnesses
  // kl = V''(d_l), kr = V''(d_{l+1}) of its two springs; zero on ghosts.
  __device__ __forceinline__ static void spring_terms(const StepArgs &a, double y, bool mass,
                                                      double &F, double &kl, double &kr) {
    using namespace fputrow;
    const double kk = a.prm[0], al = a.prm[1], be = a.prm[2];
    const double ql = dpp<0x111>(y);  // row_shr:1
    const double qr = dpp<0x101>(y);  // row_shl:1
    const double dl = y - ql, dr = qr - y;
    const double fl = dl * __builtin_fma(dl, __builtin_fma(be, dl, al), kk);
    const double fr = dr * __builtin_fma(dr, __builtin_fma(be, dr, al), kk);
    F = mass ? fl - fr : 0.0;
    const double twoal = 2.0 * al, threebe = 3.0 * be;
    kl = mass ? __builtin_fma(dl, __builtin_fma(threebe, dl, twoal), kk) : 0.0;
    kr = mass ? __builtin_fma(dr, __builtin_fma(threebe, dr, twoal), kk) : 0.0;
  }
  __device__ __forceinline__ void springs(const StepArgs &a) { spring_terms(a, q, mass, F, kl, kr); }
  __device__ __forceinline__ void kick_state(double h) { p = __builtin_fma(-h, F, p); }
  __device__ __forceinline__ void drift(double c) {
    q = __builtin_fma(c, p, q);
#pragma unroll
    for (int v = 0; v < M; ++v) dq[v] = __builtin_fma(c, dp[v], dq[v]);
  }
  __device__ __forceinline__ void kick_vectors(double h) {
    using namespace fputrow;
    const double hd = h * (kl + kr), hl = h * kl, hr = h * kr;
#pragma unroll
    for (int v = 0; v < M; ++v) {
      const double ql = dpp<0x111>(dq[v]);
      const double qr = dpp<0x101>(dq[v]);
      double acc = __builtin_fma(-hd, dq[v], dp[v]);
      acc = __builtin_fma(hl, ql, acc);
      dp[v] = __builtin_fma(hr, qr, acc);
    }
  }
  __device__ __forceinline__ void step_body(const StepArgs &a, const StepCoef &k, bool do_ld) {
    using namespace fputrow;
    drift(k.c0);
    springs(a);
    kick_state(k.hk1);
    kick_vectors(k.hk1);
    drift(k.c1);
    springs(a);
    kick_state(k.hk1);
    kick_vectors(k.hk1);
    drift(k.c0);
    springs(a);
    kick_state(k.hk0);
    if (do_ld) {
      const double g = row_sum(mass ? sqrt_ld(p) + sqrt_ld(F) : 0.0);
      ld = __builtin_fma(k.hdt, gprev + g, ld);
      gprev = g;
    }
  }
  __device__ void block(const StepArgs &a, const StepCoef &k, int blk) {
    const bool do_ld = (a.ind & CHX_IND_LD) != 0;
    kick_state(k.hk0);
    kick_vectors(k.hk0);
    for (int s = 0; s + 1 < blk; ++s) {
      step_body(a, k, do_ld);
      kick_state(k.hk0);
      kick_vectors(k.hkm);
    }
    step_body(a, k, do_ld);
    kick_vectors(k.hk0);
  }

  // Checkpoint at t; returns false when the orbit stops.  Decisions use
  // row sums, identical in every lane of the row.
  __device__ bool checkpoint(const StepArgs &a, double t) {
    using namespace fputrow;
    const int m_s = a.m_s;
    const bool do_sali = (a.ind & CHX_IND_SALI) && m_s >= 2;
    tend = t;
    const bool bad = !(__builtin_isfinite(q) && __builtin_isfinite(p));
    if ((__ballot(bad) >> (16 * row)) & 0xFFFFull) {
      st = CHX_ORBIT_NONFINITE;
      return false;
    }
    bool escaped = false;
    if (a.escape_r2 > 0.0) escaped = row_sum(q * q) > a.escape_r2;
#pragma unroll
    for (int v = 0; v < M; ++v) {
      if (v < m_s) {
        const double r2 = row_sum(__builtin_fma(dq[v], dq[v], dp[v] * dp[v]));
        const double inv = rsqrt_nr(r2);
        dq[v] *= inv;
        dp[v] *= inv;
        grow(gm[v], ge[v], r2);
      }
    }
    double s2 = 0.0;
    if (do_sali) {
      const double aq = dq[0] + dq[MM > 1 ? 1 : 0], ap = dp[0] + dp[MM > 1 ? 1 : 0];
      const double bq = dq[0] - dq[MM > 1 ? 1 : 0], bp = dp[0] - dp[MM > 1 ? 1 : 0];
      const double sp = row_sum(__builtin_fma(aq, aq, ap * ap));
      const double sm = row_sum(__builtin_fma(bq, bq, bp * bp));
      s2 = __builtin_fmin(sp, sm);
      slast2 = s2;
      smin2 = __builtin_fmin(smin2, s2);
      if (s2 < a.thr2 && __builtin_isnan(tch)) tch = t;
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
      if (j >= m_s) {
#pragma unroll
        for (int l = 0; l < j; ++l) {
          if (l >= m_s) {
            const double d = row_sum(__builtin_fma(dq[l], dq[j], dp[l] * dp[j]));
            dq[j] = __builtin_fma(-d, dq[l], dq[j]);
            dp[j] = __builtin_fma(-d, dp[l], dp[j]);
          }
        }
        const double r2 = row_sum(__builtin_fma(dq[j], dq[j], dp[j] * dp[j]));
        const double inv = rsqrt_nr(r2);
        dq[j] *= inv;
        dp[j] *= inv;
        grow(gm[j], ge[j], r2);
      }
    }
    if (a.ind & CHX_IND_ENERGY) {
      const double kk = a.prm[0], al = a.prm[1], be = a.prm[2];
      const double ql = dpp<0x111>(q);
      const double qr = dpp<0x101>(q);
      const double dl = q - ql, dr = qr - q;
      auto spring = [&](double d) {
        const double d2 = d * d;
        return d2 * __builtin_fma(d, __builtin_fma(0.25 * be, d, al * (1.0 / 3.0)), 0.5 * kk);
      };
      double e = (lane <= N) ? spring(dl) : 0.0;
      if (mass) e = __builtin_fma(0.5 * p, p, e);
      if (N == 16 && lane == 15) e += spring(dr);
      eerr = __builtin_fmax(eerr, __builtin_fabs(row_sum(e) - H0));
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

template <int N, int M>
__global__ void __launch_bounds__(256) fput_crow_kernel(const StepArgs a) {
  const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  // rows beyond the ensemble or already stopped do nothing; all lanes of a
  // row take the same branch
  if (o >= a.n) return;
  if (a.st[o] != CHX_ORBIT_OK) return;
  CRowOrbit<N, M> r;
  r.load(a, o);
  const StepCoef k(a.dt);
  int64_t s = a.s_begin;
  const int64_t K = a.K;
  while (s < a.s_end) {
    int64_t next = (s / K + 1) * K;
    if (next > a.n_total) next = a.n_total;
    r.block(a, k, (int)(next - s));
    s = next;
    if (!r.checkpoint(a, (double)s * a.dt)) break;
  }
  r.store(a, o);
}

}  // namespace chx
