// fput_row2.h -- Fermi-Pasta-Ulam chains of N = 8 masses with 17..24
// deviation vectors: two orbits per 16-lane row, eight per wavefront.
//
// The one-orbit-per-row form (fput_row.h) gives each orbit 16 lanes, one
// whole vector per lane and slot; 3N = 24 vectors at N = 8 then fill 24 of
// 32 slot positions.  Here a row holds two orbits, lanes 8g..8g+7 serving
// orbit g of the wavefront: lane c of the group holds
//   - the state component c (q_c, p_c) -- every lane is a mass;
//   - V = 3 whole deviation vectors (2N components each): vector position
//     pos = s*8 + c for slot s, so 24 vectors fill every position.
// Positions 0..n_l-1 are the Lyapunov set, n_l..n_l+m_s-1 the SALI/GALI
// set (the SALI pair at lanes 0 and 1 of slot n_l / 8).
//
// A row_newbcast operand takes one source lane for all 16 lanes of a row,
// so one instruction cannot serve both orbits of a row.  The two kinds of
// cross-lane traffic take different routes:
//   - each tangent kick: lane c stores the two coefficients of component c,
//     -h (kappa_c + kappa_{c+1}) and h kappa_c, in the orbit's LDS region
//     and every lane of the group reads all N pairs (a broadcast read:
//     the group's lanes read the same addresses); the kick is then 3 plain
//     FMAs per component and vector.  LDS accesses of one wavefront execute
//     in program order, so a lane reads what another lane stored before;
//   - each Gram-Schmidt pivot comes straight from the owner's registers
//     through the FMA's row_newbcast operand, issued once per half row with
//     the DPP bank mask choosing the lanes written (lanes 0-7 from the
//     pivot lane of the first group, lanes 8-15 from that of the second).
// The springs read the neighbours' q through row_shr/row_shl DPP; at the
// group edges the other orbit's lane is replaced by the wall q = 0.  Sums
// over an orbit (norms, energy, escape radius, the LD at checkpoints) use a
// quad_perm / half-mirror butterfly inside the 8-lane group, identical bits
// in all its lanes.
#pragma once
#include "fput_row.h"

namespace chx {

namespace fputrow2 {

using fputrow::dpp;
using fputrow::norm2_4;
using fputrow::static_for;

// acc += coef(lane I of the row) * x, written to lanes 0-7 (fmac_lo) or
// 8-15 (fmac_hi) of each row only: v_fmac_f64 with its first source read
// through row_newbcast:I and the DPP bank mask (a bank = 4 lanes of a row)
// selecting the lanes written; kept in program order
template <int I>
__device__ __forceinline__ void fmac_lo(double &acc, double coef, double x) {
  asm volatile("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0x3"
               : "+v"(acc)
               : "v"(coef), "v"(x), "n"(I));
}
template <int I>
__device__ __forceinline__ void fmac_hi(double &acc, double coef, double x) {
  asm volatile("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xc"
               : "+v"(acc)
               : "v"(coef), "v"(x), "n"(I));
}
// lane I of each group of 8 to the whole group: row_newbcast:I into lanes
// 0-7 of the row, row_newbcast:(8 + I) into lanes 8-15
template <int I>
__device__ __forceinline__ double bcast_halves(double v) {
  double r = 0.0;
  asm volatile(
      "v_mov_b64_dpp %0, %1 row_newbcast:%2 row_mask:0xf bank_mask:0x3\n\t"
      "v_mov_b64_dpp %0, %1 row_newbcast:%3 row_mask:0xf bank_mask:0xc"
      : "+v"(r)
      : "v"(v), "n"(I), "n"(8 + I));
  return r;
}

// sum over the 8 lanes of a group, identical in all of them
__device__ __forceinline__ double grp_sum(double s) {
  s += dpp<0xB1>(s);   // quad_perm [1,0,3,2]
  s += dpp<0x4E>(s);   // quad_perm [2,3,0,1]
  s += dpp<0x141>(s);  // row_half_mirror
  return s;
}

}  // namespace fputrow2

template <int N, int V>
__global__ void __launch_bounds__(64, 2) fput_row2_kernel(const StepArgs a) {
  using namespace fputrow2;
  static_assert(N == 8, "two orbits per 16-lane row");
  constexpr int D = 2 * N;
  constexpr int G = N;        // lanes per orbit
  constexpr int OPW = 64 / G;  // orbits per wavefront
  // per orbit: the kick coefficients of its N components
  __shared__ __align__(16) double cf[OPW][N][2];
  const int g = threadIdx.x / G, c = threadIdx.x % G;
  const int64_t o = (int64_t)blockIdx.x * OPW + g;
  const int64_t P = a.pitch;
  const bool act = (o < a.n) && (a.st[o] == CHX_ORBIT_OK);
  const int64_t oo = act ? o : 0;  // inactive groups compute on a copy
  const int n_l = a.n_l, m_s = a.m_s, M = n_l + m_s;
  const double kk = a.prm[0], al = a.prm[1], be = a.prm[2];

  // vector index in the ensemble layout of slot s, -1 = unused slot
  auto vk_of = [&](int s) {
    const int pos = s * G + c;
    return pos < n_l ? m_s + pos : (pos < M ? pos - n_l : -1);
  };

  double q = a.x[c * P + oo];
  double p = a.x[(N + c) * P + oo];
  double w[V][D], gm[V];
  int ge[V];
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const int vk = vk_of(s);
    const int64_t k = vk < 0 ? 0 : vk;
#pragma unroll
    for (int i = 0; i < D; ++i) w[s][i] = vk < 0 ? 0.0 : a.w[(k * D + i) * P + oo];
    gm[s] = vk < 0 ? 1.0 : a.gm[k * P + oo];
    ge[s] = vk < 0 ? 0 : a.ge[k * P + oo];
  }
  // LD: each lane accumulates its components' part of the trapezoid sums
  // (ldl, with gpl its last integrand); every checkpoint adds the group's
  // sum to ld and hands the group's last integrand to lane 0, so that a
  // launch boundary (always at a checkpoint) changes nothing
  double ld = a.sc[SC_LD * P + oo], gprev = a.sc[SC_GPREV * P + oo];
  double ldl = 0.0, gpl = c == 0 ? gprev : 0.0;
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

  auto wave_sync = []() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  // neighbours' positions, the walls at the group's ends
  auto left = [&](double v) {
    const double u = dpp<0x111>(v);  // row_shr:1
    return c == 0 ? 0.0 : u;
  };
  auto right = [&](double v) {
    const double u = dpp<0x101>(v);  // row_shl:1
    return c == G - 1 ? 0.0 : u;
  };

  // After every drift: the springs of mass c (left extension
  // d_c = q_c - q_{c-1}, right d_{c+1} = q_{c+1} - q_c), the force and the
  // stiffnesses kappa(d) = k + d (2 alpha + 3 beta d) of both springs.
  double F = 0.0, kl = 0.0, kr = 0.0;
  const double twoal = 2.0 * al, threebe = 3.0 * be;
  auto springs = [&]() {
    const double dl = q - left(q), dr = right(q) - q;
    const double fl = dl * __builtin_fma(dl, __builtin_fma(be, dl, al), kk);
    const double fr = dr * __builtin_fma(dr, __builtin_fma(be, dr, al), kk);
    F = fl - fr;
    kl = __builtin_fma(dl, __builtin_fma(threebe, dl, twoal), kk);
    kr = __builtin_fma(dr, __builtin_fma(threebe, dr, twoal), kk);
  };
  auto kick_state = [&](double h) { p = __builtin_fma(-h, F, p); };
  auto drift = [&](double cc) {
    q = __builtin_fma(cc, p, q);
#pragma unroll
    for (int s = 0; s < V; ++s)
#pragma unroll
      for (int i = 0; i < N; ++i) w[s][i] = __builtin_fma(cc, w[s][N + i], w[s][i]);
  };
  // dp_i -= h [(kappa_i + kappa_{i+1}) dq_i - kappa_i dq_{i-1} - kappa_{i+1} dq_{i+1}]
  auto kick_vectors = [&](double h) {
    cf[g][c][0] = -(h * (kl + kr));
    cf[g][c][1] = h * kl;
    wave_sync();
    double cn[N], cl[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double2 v = *(const double2 *)&cf[g][i][0];
      cn[i] = v.x;
      cl[i] = v.y;
    }
    wave_sync();  // every read above before the next kick's stores
#pragma unroll
    for (int s = 0; s < V; ++s)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double acc = __builtin_fma(cn[i], w[s][i], w[s][N + i]);
        if (i > 0) acc = __builtin_fma(cl[i], w[s][i - 1], acc);
        if (i + 1 < N) acc = __builtin_fma(cl[i + 1], w[s][i + 1], acc);
        w[s][N + i] = acc;
      }
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
      const double gl = sqrt_ld(p) + sqrt_ld(F);
      ldl = __builtin_fma(hdt, gpl + gl, ldl);
      gpl = gl;
    }
  };

  // Checkpoint at t; returns false when the orbit stops.  Every decision is
  // taken on values that are identical in all lanes of the group.
  auto checkpoint = [&](double t) {
    tend = t;
    if (do_ld) {
      ld += grp_sum(ldl);
      ldl = 0.0;
      gprev = grp_sum(gpl);
      gpl = c == 0 ? gprev : 0.0;
    }
    const bool bad = !(__builtin_isfinite(q) && __builtin_isfinite(p));
    const uint64_t bb = __ballot(bad);
    if ((bb >> (G * g)) & ((1ull << G) - 1ull)) {
      st = CHX_ORBIT_NONFINITE;
      return false;
    }
    bool escaped = false;
    if (a.escape_r2 > 0.0) escaped = grp_sum(q * q) > a.escape_r2;
    // SALI/GALI set: each vector back to unit length (lane-local)
#pragma unroll
    for (int s = 0; s < V; ++s) {
      const int pos = s * G + c;
      if (pos >= n_l && pos < M) {
        const double r2 = norm2_4<D>(w[s]);
        const double inv = rsqrt_nr(r2);
#pragma unroll
        for (int i = 0; i < D; ++i) w[s][i] *= inv;
        grow(gm[s], ge[s], r2);
      }
    }
    double s2 = 0.0;
    if (do_sali) {
      // the SALI pair: positions n_l and n_l + 1, lanes 0 and 1 of slot
      // n_l / 8 (the launcher requires n_l % 8 == 0); lane 0 takes lane 1's
      // vector through quad_perm [1,1,1,1]
      const int s0 = n_l / G;
      double sp[2] = {0.0, 0.0}, sm[2] = {0.0, 0.0};
#pragma unroll
      for (int s = 0; s < V; ++s) {
        if (s == s0) {
#pragma unroll
          for (int i = 0; i < D; ++i) {
            const double other = dpp<0x55>(w[s][i]);
            const double ap = w[s][i] + other, am = w[s][i] - other;
            sp[i & 1] = __builtin_fma(ap, ap, sp[i & 1]);
            sm[i & 1] = __builtin_fma(am, am, sm[i & 1]);
          }
        }
      }
      s2 = __builtin_fmin(sp[0] + sp[1], sm[0] + sm[1]);
      s2 = grp_sum(c == 0 ? s2 : 0.0);  // lane 0's value in every lane
      slast2 = s2;
      smin2 = __builtin_fmin(smin2, s2);
      if (s2 < a.thr2 && __builtin_isnan(tch)) tch = t;
    }
    // Lyapunov set: modified Gram-Schmidt in vector order.  Pivot j sits
    // in slot j / 8 at lane j % 8 of every group.  The dot products and the
    // updates take its components straight from the owner's registers
    // through the FMA's row_newbcast operand, once per half row (bank_mask
    // 0x3 writes lanes 0-7 of a row from lane j % 8, bank_mask 0xc lanes
    // 8-15 from lane 8 + j % 8), so no pivot goes through memory and no
    // wait is exposed; pivots are unrolled (the lane is an immediate).  Per
    // pivot: dot products of every later vector with it (four partial
    // sums), |w_j|^2 from the owner's own dot product, the
    // coefficients, then w_k -= (w_j . w_k / |w_j|^2) w_j.  The owner's
    // coefficient is zero, so its source registers keep their values
    // during its pass.  Ordering: each update pass writes a register that
    // the other half's pass then reads through DPP, so all updates of one
    // half come before those of the other (at least 16 instructions apart,
    // past the two wait states a DPP read needs after a VALU write), and
    // the later slots before the pivots' own.  The owner keeps |w_j|^2 of
    // its slot; growth and normalisation follow the last pivot.
    double own2[V];
#pragma unroll
    for (int s = 0; s < V; ++s) own2[s] = 1.0;
    constexpr int NLS_MAX = (2 * N + G - 1) / G < V ? (2 * N + G - 1) / G : V;
    // n_l taken afresh here, so that the compiler forms the pivots'
    // comparisons with it in each checkpoint instead of keeping sixteen of
    // them in scalar registers through the step loop
    int nlg = n_l;
    asm volatile("" : "+s"(nlg));
    const int nls = (nlg + G - 1) / G;  // slots holding Lyapunov vectors
    static_for<0, NLS_MAX>([&](auto jc) {
      constexpr int sj = decltype(jc)::value;  // the pivots' slot
      if (sj * G < nlg) {
        // slots sj..L-1 hold Lyapunov vectors (code per possible L, chosen
        // by a uniform branch)
        auto group = [&](auto lc) {
          constexpr int L = decltype(lc)::value;
          static_for<0, G>([&](auto ljc) {
            constexpr int lj = decltype(ljc)::value;  // the pivot's lane
            // the last lane's pivot has no later vector in its own slot:
            // that slot takes no dot products or updates, and |w_j|^2 is the
            // owner's own norm
            constexpr int s1 = lj == G - 1 ? sj + 1 : sj;
            const int pj = sj * G + lj;
            if (pj < nlg) {
              // two wait states before the first DPP read of w[sj]
              asm volatile("s_nop 1" : "+v"(w[sj][0]), "+v"(w[sj][1]));
              // four partial sums per vector; the first half row's pass
              // writes lanes 0-7 of them, the second's (16 or more
              // instructions later) lanes 8-15
              double d[V][4];
#pragma unroll
              for (int s = 0; s < V; ++s) d[s][0] = d[s][1] = d[s][2] = d[s][3] = 0.0;
              static_for<0, D>([&](auto cc) {
                constexpr int i = decltype(cc)::value;
#pragma unroll
                for (int s = s1; s < L; ++s) fmac_lo<lj>(d[s][i & 3], w[sj][i], w[s][i]);
              });
              static_for<0, D>([&](auto cc) {
                constexpr int i = decltype(cc)::value;
#pragma unroll
                for (int s = s1; s < L; ++s) fmac_hi<G + lj>(d[s][i & 3], w[sj][i], w[s][i]);
              });
              double t[V];
#pragma unroll
              for (int s = s1; s < L; ++s) t[s] = (d[s][0] + d[s][1]) + (d[s][2] + d[s][3]);
              if constexpr (s1 != sj) t[sj] = norm2_4<D>(w[sj]);
              // |w_j|^2: the owner's own dot product, to its group
              double r2 = t[sj];
              asm volatile("s_nop 1" : "+v"(r2));
              r2 = bcast_halves<lj>(r2);
              own2[sj] = c == lj ? r2 : own2[sj];
              const double inv = rsqrt_nr(r2);
              double ni2 = -(inv * inv);
              // computed once for all lanes, not under the per-lane select
              asm volatile("" : "+v"(ni2));
              double nd[V];
#pragma unroll
              for (int s = s1; s < L; ++s) {
                const int pos = s * G + c;
                nd[s] = (pos > pj && pos < nlg) ? t[s] * ni2 : 0.0;
              }
              static_for<0, D>([&](auto cc) {
                constexpr int i = decltype(cc)::value;
#pragma unroll
                for (int s = sj + 1; s < L; ++s) fmac_lo<lj>(w[s][i], w[sj][i], nd[s]);
              });
              static_for<0, D>([&](auto cc) {
                constexpr int i = decltype(cc)::value;
#pragma unroll
                for (int s = sj + 1; s < L; ++s) fmac_hi<G + lj>(w[s][i], w[sj][i], nd[s]);
              });
              if constexpr (s1 == sj) {
                static_for<0, D>([&](auto cc) {
                  constexpr int i = decltype(cc)::value;
                  fmac_lo<lj>(w[sj][i], w[sj][i], nd[sj]);
                });
                static_for<0, D>([&](auto cc) {
                  constexpr int i = decltype(cc)::value;
                  fmac_hi<G + lj>(w[sj][i], w[sj][i], nd[sj]);
                });
              }
            }
          });
        };
        static_for<sj + 1, NLS_MAX + 1>([&](auto lc) {
          if (nls == decltype(lc)::value) group(lc);
        });
      }
    });
#pragma unroll
    for (int s = 0; s < V; ++s) {
      if (s * G + c < n_l) {
        const double inv = rsqrt_nr(own2[s]);
        grow(gm[s], ge[s], own2[s]);
#pragma unroll
        for (int i = 0; i < D; ++i) w[s][i] *= inv;
      }
    }
    if (do_energy) {
      const double dl = q - left(q), dr = right(q) - q;
      auto spring = [&](double d) {
        const double d2 = d * d;
        return d2 * __builtin_fma(d, __builtin_fma(0.25 * be, d, al * (1.0 / 3.0)), 0.5 * kk);
      };
      // each lane: its kinetic energy and its left spring; the last mass
      // also its spring to the right wall
      double e = __builtin_fma(0.5 * p, p, spring(dl));
      if (c == G - 1) e += spring(dr);
      const double Hs = grp_sum(e);
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

  auto store = [&](int64_t ob) {
    a.x[c * P + ob] = q;
    a.x[(N + c) * P + ob] = p;
#pragma unroll
    for (int s = 0; s < V; ++s) {
      const int vk = vk_of(s);
      if (vk >= 0) {
        const int64_t k = vk;
#pragma unroll
        for (int i = 0; i < D; ++i) a.w[(k * D + i) * P + ob] = w[s][i];
        a.gm[k * P + ob] = gm[s];
        a.ge[k * P + ob] = ge[s];
      }
    }
    if (c == 0) {
      a.sc[SC_LD * P + ob] = ld;
      a.sc[SC_GPREV * P + ob] = gprev;
      a.sc[SC_SALI_MIN2 * P + ob] = smin2;
      a.sc[SC_SALI_LAST2 * P + ob] = slast2;
      a.sc[SC_T_CHAOS * P + ob] = tch;
      a.sc[SC_EERR * P + ob] = eerr;
      a.sc[SC_T_END * P + ob] = tend;
      a.st[ob] = st;
    }
  };

  springs();
  int64_t s = a.s_begin;
  const int64_t K = a.K;
  // an orbit that stops leaves the loop; all orbits write back once, after it
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
  // the store addresses are formed here, not kept from the loads
  int64_t ob = o;
  asm volatile("" : "+v"(ob));
  if (act) store(ob);
}

}  // namespace chx
