// fput_row.h -- Fermi-Pasta-Ulam chains: one 16-lane row per orbit.
//
// A wavefront carries four orbits, one per 16-lane DPP row, in a block of
// one wavefront.  Lane l of a row holds
//   - the state component l (q_l, p_l) of its orbit, for l < N; lanes
//     N..15 are ghost masses held at q = p = 0, so the last mass's right
//     neighbour reads 0, which is the fixed wall q_{N+1} = 0;
//   - V whole deviation vectors (2N components each): vector position
//     pos = s*16 + l for slot s.  Positions 0..n_l-1 are the Lyapunov set,
//     n_l..n_l+m_s-1 the SALI/GALI set, the rest unused.
// Kicks need the tridiagonal Hessian of the chain (Examples section, FPU
// equations of motion): with spring stiffness kappa(d) = k + d (2 alpha +
// 3 beta d), (H dq)_i = (kappa_i + kappa_{i+1}) dq_i - kappa_i dq_{i-1}
// - kappa_{i+1} dq_{i+1}.  Each lane computes the coefficients of its own
// component from its neighbours (row_shr/row_shl DPP), then every lane gets
// them by row_newbcast (one v_mov_b64_dpp per coefficient, shared by the
// lane's V vectors) -- no LDS, no readlane, no scalar memory.
//
// At checkpoints the Lyapunov set is orthonormalised by modified
// Gram-Schmidt: the pivot's owner lane normalises it and stages it in LDS
// (one 2N-double buffer per row), then every lane projects it out of its
// own later vectors.  Row sums (energy, LD, escape radius) use a
// quad_perm / half-mirror / mirror butterfly, so all 16 lanes hold the
// same bits.
#pragma once
#include <type_traits>

#include "chx_internal.h"
#include "device_math.h"

namespace chx {

namespace fputrow {

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, CTRL, 0xf, 0xf, true);
}
// row_newbcast:i -- lane i of each row to the whole row.  Every lane is
// written from a lane of its own row, so the old value is dead; asking for
// bound_ctrl lets the compiler skip initialising it.
template <int I>
__device__ __forceinline__ double bcast(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + I, 0xf, 0xf, true);
}
// compile-time loop: f(std::integral_constant<int, I>{}) for I = B..E-1
template <int I, int E, class Fn>
__device__ __forceinline__ void static_for(Fn &&f) {
  if constexpr (I < E) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, E>(f);
  }
}

// sum over the 16 lanes of a row, identical in every lane
__device__ __forceinline__ double row_sum(double s) {
  s += dpp<0xB1>(s);   // quad_perm [1,0,3,2]
  s += dpp<0x4E>(s);   // quad_perm [2,3,0,1]
  s += dpp<0x141>(s);  // row_half_mirror
  s += dpp<0x140>(s);  // row_mirror
  return s;
}

}  // namespace fputrow

template <int N, int V>
__global__ void __launch_bounds__(64) fput_row_kernel(const StepArgs a) {
  using namespace fputrow;
  constexpr int D = 2 * N;
  __shared__ double piv[4][D];
  const int lane = threadIdx.x & 15, row = threadIdx.x >> 4;
  const int64_t o = (int64_t)blockIdx.x * 4 + row;
  const int64_t P = a.pitch;
  bool act = (o < a.n) && (a.st[o] == CHX_ORBIT_OK);
  const int64_t oo = act ? o : 0;  // inactive rows compute on a copy
  const bool mass = lane < N;
  const int n_l = a.n_l, m_s = a.m_s, M = n_l + m_s;
  const double kk = a.prm[0], al = a.prm[1], be = a.prm[2];

  double q = mass ? a.x[lane * P + oo] : 0.0;
  double p = mass ? a.x[(N + lane) * P + oo] : 0.0;
  double w[V][D], gm[V];
  int ge[V];
  int vk[V];  // vector index in the ensemble layout, -1 = unused slot
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const int pos = s * 16 + lane;
    vk[s] = pos < n_l ? m_s + pos : (pos < M ? pos - n_l : -1);
    const int64_t k = vk[s] < 0 ? 0 : vk[s];
#pragma unroll
    for (int c = 0; c < D; ++c) w[s][c] = vk[s] < 0 ? 0.0 : a.w[(k * D + c) * P + oo];
    gm[s] = vk[s] < 0 ? 1.0 : a.gm[k * P + oo];
    ge[s] = vk[s] < 0 ? 0 : a.ge[k * P + oo];
  }
  double ld = a.sc[SC_LD * P + oo], gprev = a.sc[SC_GPREV * P + oo];
  double smin2 = a.sc[SC_SALI_MIN2 * P + oo], slast2 = a.sc[SC_SALI_LAST2 * P + oo];
  double tch = a.sc[SC_T_CHAOS * P + oo], eerr = a.sc[SC_EERR * P + oo];
  const double H0 = a.sc[SC_H0 * P + oo];
  double tend = a.sc[SC_T_END * P + oo];
  int st = CHX_ORBIT_OK;

  const double dt = a.dt;
  const double c0 = YOSHIDA_W1 * dt, c1 = YOSHIDA_W0 * dt;
  const double hk0 = (0.5 * YOSHIDA_W1) * dt;
  const double hk1 = (0.5 * (YOSHIDA_W1 + YOSHIDA_W0)) * dt;
  const double hkm = 2.0 * hk0;
  const double hdt = 0.5 * dt;
  const bool do_ld = (a.ind & CHX_IND_LD) != 0;
  const bool do_sali = (a.ind & CHX_IND_SALI) && m_s >= 2;
  const bool do_energy = (a.ind & CHX_IND_ENERGY) != 0;

  // After every drift: the two springs of lane l (left extension
  // d_l = q_l - q_{l-1}, right d_{l+1} = q_{l+1} - q_l), the force and the
  // stiffnesses kappa of both springs.
  double F = 0.0, kl = 0.0, kr = 0.0;
  const double twoal = 2.0 * al, threebe = 3.0 * be;
  auto springs = [&]() {
    const double ql = dpp<0x111>(q);  // row_shr:1, lane 0 reads the wall
    const double qr = dpp<0x101>(q);  // row_shl:1, lane 15 reads the wall
    const double dl = q - ql, dr = qr - q;
    const double fl = dl * __builtin_fma(dl, __builtin_fma(be, dl, al), kk);
    const double fr = dr * __builtin_fma(dr, __builtin_fma(be, dr, al), kk);
    F = mass ? fl - fr : 0.0;
    kl = __builtin_fma(dl, __builtin_fma(threebe, dl, twoal), kk);
    kr = __builtin_fma(dr, __builtin_fma(threebe, dr, twoal), kk);
  };
  auto kick_state = [&](double h) { p = __builtin_fma(-h, F, p); };
  auto drift = [&](double c) {
    q = __builtin_fma(c, p, q);
#pragma unroll
    for (int s = 0; s < V; ++s)
#pragma unroll
      for (int i = 0; i < N; ++i) w[s][i] = __builtin_fma(c, w[s][N + i], w[s][i]);
  };
  // dp_i -= h [(kappa_i + kappa_{i+1}) dq_i - kappa_i dq_{i-1} - kappa_{i+1} dq_{i+1}]
  auto kick_vectors = [&](double h) {
    const double hdiag = h * (kl + kr), hleft = h * kl;
    // component by component: the diagonal coefficient of component i and
    // the coupling to component i+1 come from lanes i and i+1
    double Kcur = 0.0;
    static_for<0, N>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const double Ai = bcast<i>(hdiag);
      double Knext = 0.0;
      if constexpr (i + 1 < N) Knext = bcast<i + 1>(hleft);
#pragma unroll
      for (int s = 0; s < V; ++s) {
        double acc = __builtin_fma(-Ai, w[s][i], w[s][N + i]);
        if constexpr (i > 0) acc = __builtin_fma(Kcur, w[s][i - 1], acc);
        if constexpr (i + 1 < N) acc = __builtin_fma(Knext, w[s][i + 1], acc);
        w[s][N + i] = acc;
      }
      Kcur = Knext;
    });
  };
  auto ld_integrand = [&]() {
    const double g = mass ? sqrt_ld(p) + sqrt_ld(F) : 0.0;
    return row_sum(g);
  };
  auto step_body = [&]() {
    drift(c0);
    springs();
    kick_state(hk1);
    kick_vectors(hk1);
    drift(c1);
    springs();
    kick_state(hk1);
    kick_vectors(hk1);
    drift(c0);
    springs();
    kick_state(hk0);  // p at the step endpoint
    if (do_ld) {
      const double g = ld_integrand();
      ld = __builtin_fma(hdt, gprev + g, ld);
      gprev = g;
    }
  };

  // Checkpoint at t; returns false when the orbit stops.  Every decision is
  // taken on row-uniform values.
  auto checkpoint = [&](double t) {
    tend = t;
    const bool bad = !(__builtin_isfinite(q) && __builtin_isfinite(p));
    const uint64_t bb = __ballot(bad);
    if ((bb >> (16 * row)) & 0xFFFFull) {
      st = CHX_ORBIT_NONFINITE;
      return false;
    }
    bool escaped = false;
    if (a.escape_r2 > 0.0) escaped = row_sum(q * q) > a.escape_r2;
    // SALI/GALI set: each vector back to unit length (lane-local)
#pragma unroll
    for (int s = 0; s < V; ++s) {
      const int pos = s * 16 + lane;
      if (pos >= n_l && pos < M) {
        double r2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) r2 = __builtin_fma(w[s][c], w[s][c], r2);
        const double inv = rsqrt_nr(r2);
#pragma unroll
        for (int c = 0; c < D; ++c) w[s][c] *= inv;
        grow(gm[s], ge[s], r2);
      }
    }
    double s2 = 0.0;
    if (do_sali) {
      // the SALI pair sits at positions n_l and n_l + 1 (lanes 0 and 1 of
      // slot n_l / 16; the launcher requires n_l % 16 == 0)
      const int s0 = n_l / 16;
      double sp = 0.0, sm = 0.0;
#pragma unroll
      for (int s = 0; s < V; ++s) {
        if (s == s0) {
#pragma unroll
          for (int c = 0; c < D; ++c) {
            const double other = bcast<1>(w[s][c]);
            const double ap = w[s][c] + other, am = w[s][c] - other;
            sp = __builtin_fma(ap, ap, sp);
            sm = __builtin_fma(am, am, sm);
          }
        }
      }
      s2 = bcast<0>(__builtin_fmin(sp, sm));
      slast2 = s2;
      smin2 = __builtin_fmin(smin2, s2);
      if (s2 < a.thr2 && __builtin_isnan(tch)) tch = t;
    }
    // Lyapunov set: modified Gram-Schmidt in vector order; the pivot's owner
    // normalises it and stages it in LDS, every lane projects it out of its
    // own later vectors.
#pragma unroll
    for (int j = 0; j < 16 * V; ++j) {
      if (j < n_l) {
        const int sj = j / 16, lj = j % 16;
        if (lane == lj) {
#pragma unroll
          for (int s = 0; s < V; ++s) {
            if (s == sj) {
              double r2 = 0.0;
#pragma unroll
              for (int c = 0; c < D; ++c) r2 = __builtin_fma(w[s][c], w[s][c], r2);
              const double inv = rsqrt_nr(r2);
#pragma unroll
              for (int c = 0; c < D; ++c) {
                w[s][c] *= inv;
                piv[row][c] = w[s][c];
              }
              grow(gm[s], ge[s], r2);
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int s = 0; s < V; ++s) {
          if (s >= sj && s * 16 < n_l) {
            const int pos = s * 16 + lane;
            if (pos > j && pos < n_l) {
              double d = 0.0;
#pragma unroll
              for (int c = 0; c < D; ++c) d = __builtin_fma(piv[row][c], w[s][c], d);
#pragma unroll
              for (int c = 0; c < D; ++c) w[s][c] = __builtin_fma(-d, piv[row][c], w[s][c]);
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    if (do_energy) {
      const double ql = dpp<0x111>(q);
      const double qr = dpp<0x101>(q);
      const double dl = q - ql, dr = qr - q;
      auto spring = [&](double d) {
        const double d2 = d * d;
        return d2 * __builtin_fma(d, __builtin_fma(0.25 * be, d, al * (1.0 / 3.0)), 0.5 * kk);
      };
      // each lane: its kinetic energy and its left spring; the wall spring
      // of the last mass comes from ghost lane N, or from lane 15 itself
      // when N = 16
      double e = (lane <= N) ? spring(dl) : 0.0;
      if (mass) e = __builtin_fma(0.5 * p, p, e);
      if (N == 16 && lane == 15) e += spring(dr);
      const double Hs = row_sum(e);
      eerr = __builtin_fmax(eerr, __builtin_fabs(Hs - H0));
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
  };

  auto store = [&]() {
    if (mass) {
      a.x[lane * P + o] = q;
      a.x[(N + lane) * P + o] = p;
    }
#pragma unroll
    for (int s = 0; s < V; ++s) {
      if (vk[s] >= 0) {
        const int64_t k = vk[s];
#pragma unroll
        for (int c = 0; c < D; ++c) a.w[(k * D + c) * P + o] = w[s][c];
        a.gm[k * P + o] = gm[s];
        a.ge[k * P + o] = ge[s];
      }
    }
    if (lane == 0) {
      a.sc[SC_LD * P + o] = ld;
      a.sc[SC_GPREV * P + o] = gprev;
      a.sc[SC_SALI_MIN2 * P + o] = smin2;
      a.sc[SC_SALI_LAST2 * P + o] = slast2;
      a.sc[SC_T_CHAOS * P + o] = tch;
      a.sc[SC_EERR * P + o] = eerr;
      a.sc[SC_T_END * P + o] = tend;
      a.st[o] = st;
    }
  };

  springs();
  int64_t s = a.s_begin;
  const int64_t K = a.K;
  // a row that stops leaves the loop; all rows write back once, after it
  while (act && s < a.s_end) {
    int64_t next = (s / K + 1) * K;
    if (next > a.n_total) next = a.n_total;
    const int blk = (int)(next - s);
    kick_state(hk0);
    kick_vectors(hk0);
    for (int k = 0; k + 1 < blk; ++k) {
      step_body();
      kick_state(hk0);
      kick_vectors(hkm);
    }
    step_body();
    kick_vectors(hk0);
    s = next;
    if (!checkpoint((double)s * dt)) break;
  }
  if (o < a.n && a.st[o] == CHX_ORBIT_OK) store();
}

}  // namespace chx
