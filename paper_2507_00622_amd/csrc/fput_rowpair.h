// fput_rowpair.h -- Fermi-Pasta-Ulam chains of N = 8 masses with up to 2N
// Lyapunov vectors and up to N SALI/GALI vectors: two orbits per 16-lane
// row, eight per wavefront, each orbit's Lyapunov set filling a whole slot.
//
// Row r of the wavefront serves orbits A = 2r and B = 2r + 1 of the block.
// Lane l of the row (c = l % 8, its half h = l / 8) holds
//   - the state component c of orbit A (h = 0) or B (h = 1);
//   - slot 0: orbit A's Lyapunov vector l (l < n_l);
//   - slot 1: orbit B's Lyapunov vector l (l < n_l);
//   - slot 2: SALI/GALI vector c (c < m_s) of its own orbit (A or B).
// With the configuration's 2N + N = 24 vectors per orbit every slot
// position is used, and each orbit's Lyapunov set spans all 16 lanes of one
// slot, so one row_newbcast operand serves a whole Gram-Schmidt pass.
//
// Cross-lane traffic:
//   - kicks of slots 0 and 1: the coupling of component i comes straight
//     from the state lane of the slot's orbit (lane i for A, 8 + i for B)
//     through the FMA's row_newbcast operand, 3 FMAs per component;
//   - kicks of slot 2 (each half its own orbit): lane c stores its two
//     coefficients, -h (kappa_c + kappa_{c+1}) and h kappa_c, in the orbit's
//     LDS region and every lane of the group reads the N pairs (broadcast
//     reads; LDS accesses of one wavefront execute in program order);
//   - Gram-Schmidt: pivot j of A is lane j of slot 0, of B lane j of slot 1;
//     the dot products and updates read it by row_newbcast:j, A's and B's
//     passes interleaved (independent chains);
//   - springs: row_shr/row_shl DPP, the other orbit's lane at the group
//     edges replaced by the wall q = 0; orbit sums: butterflies inside the
//     8-lane group.
// An orbit's data spans both halves of its row, so a row runs until both of
// its orbits have stopped: an orbit that stops is written back at once (by
// the whole row) and then keeps computing values that are never stored,
// which touch only its own data.
#pragma once
#include "fput_row.h"

namespace chx {

namespace fputpair {

// sum over the 8 lanes of a group, identical in all of them
__device__ __forceinline__ double grp_sum(double s) {
  using fputrow::dpp;
  s += dpp<0xB1>(s);   // quad_perm [1,0,3,2]
  s += dpp<0x4E>(s);   // quad_perm [2,3,0,1]
  s += dpp<0x141>(s);  // row_half_mirror
  return s;
}

}  // namespace fputpair

template <int N>
__global__ void __launch_bounds__(64, 2) fput_rowpair_kernel(const StepArgs a) {
  using namespace fputpair;
  using fputrow::bcast;
  using fputrow::dpp;
  using fputrow::norm2_4;
  using fputrow::static_for;
  using fputrow::fmac_bcast;
  using fputrow::fmac_bcast_ordered;
  static_assert(N == 8, "two orbits per 16-lane row");
  constexpr int D = 2 * N;
  constexpr int G = N;         // lanes per orbit
  constexpr int OPW = 64 / G;  // orbits per wavefront
  __shared__ __align__(16) double cf[OPW][N][2];  // slot-2 kick coefficients per orbit
  const int l = threadIdx.x & 15, row = threadIdx.x >> 4;
  const int h = l / G, c = l % G, g = threadIdx.x / G;  // g: the lane's own orbit in the wavefront
  const int64_t oA = (int64_t)blockIdx.x * OPW + 2 * row, oB = oA + 1;
  const int64_t oOwn = h ? oB : oA;
  const int64_t P = a.pitch;
  const bool actA = (oA < a.n) && (a.st[oA] == CHX_ORBIT_OK);
  const bool actB = (oB < a.n) && (a.st[oB] == CHX_ORBIT_OK);
  const int64_t ooA = actA ? oA : 0, ooB = actB ? oB : 0;  // inactive orbits: a copy
  const int64_t ooOwn = h ? ooB : ooA;
  const int n_l = a.n_l, m_s = a.m_s;
  const double kk = a.prm[0], al = a.prm[1], be = a.prm[2];

  // vector index in the ensemble layout of slot s and the orbit it belongs
  // to; -1 = unused position
  auto vk_of = [&](int s) {
    if (s < 2) return l < n_l ? m_s + l : -1;
    return c < m_s ? c : -1;
  };
  auto oo_of = [&](int s) { return s == 0 ? ooA : (s == 1 ? ooB : ooOwn); };

  double q = a.x[c * P + ooOwn];
  double p = a.x[(N + c) * P + ooOwn];
  double w[3][D], gm[3];
  int ge[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int vk = vk_of(s);
    const int64_t k = vk < 0 ? 0 : vk, ob = oo_of(s);
#pragma unroll
    for (int i = 0; i < D; ++i) w[s][i] = vk < 0 ? 0.0 : a.w[(k * D + i) * P + ob];
    gm[s] = vk < 0 ? 1.0 : a.gm[k * P + ob];
    ge[s] = vk < 0 ? 0 : a.ge[k * P + ob];
  }
  // LD: each lane accumulates its components' part of the trapezoid sums
  // (ldl, with gpl its last integrand); every checkpoint adds the group's
  // sum to ld and hands the group's last integrand to lane 0, so that a
  // launch boundary (always at a checkpoint) changes nothing
  double ld = a.sc[SC_LD * P + ooOwn], gprev = a.sc[SC_GPREV * P + ooOwn];
  double ldl = 0.0, gpl = c == 0 ? gprev : 0.0;
  double smin2 = a.sc[SC_SALI_MIN2 * P + ooOwn], slast2 = a.sc[SC_SALI_LAST2 * P + ooOwn];
  double tch = a.sc[SC_T_CHAOS * P + ooOwn], eerr = a.sc[SC_EERR * P + ooOwn];
  const double H0 = a.sc[SC_H0 * P + ooOwn];
  double tend = a.sc[SC_T_END * P + ooOwn];
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
  auto left = [&](double v) {
    const double u = dpp<0x111>(v);  // row_shr:1
    return c == 0 ? 0.0 : u;
  };
  auto right = [&](double v) {
    const double u = dpp<0x101>(v);  // row_shl:1
    return c == G - 1 ? 0.0 : u;
  };

  // After every drift: the springs of mass c, the force and the
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
  auto kick_state = [&](double hh) { p = __builtin_fma(-hh, F, p); };
  auto drift = [&](double cc) {
    q = __builtin_fma(cc, p, q);
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int i = 0; i < N; ++i) w[s][i] = __builtin_fma(cc, w[s][N + i], w[s][i]);
  };
  // dp_i -= h [(kappa_i + kappa_{i+1}) dq_i - kappa_i dq_{i-1} - kappa_{i+1} dq_{i+1}]
  auto kick_vectors = [&](double hh) {
    double nhd = -(hh * (kl + kr)), hl = hh * kl;
    cf[g][c][0] = nhd;
    cf[g][c][1] = hl;
    // two wait states between the VALU writes of nhd, hl and their DPP reads
    asm volatile("s_nop 1" : "+v"(nhd), "+v"(hl));
    // slots 0 and 1: orbit A's coefficients from lanes i, B's from 8 + i
    static_for<0, N>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      double a0 = w[0][N + i], a1 = w[1][N + i];
      fmac_bcast<i>(a0, nhd, w[0][i]);
      fmac_bcast<G + i>(a1, nhd, w[1][i]);
      if constexpr (i > 0) {
        fmac_bcast<i>(a0, hl, w[0][i - 1]);
        fmac_bcast<G + i>(a1, hl, w[1][i - 1]);
      }
      if constexpr (i + 1 < N) {
        fmac_bcast<i + 1>(a0, hl, w[0][i + 1]);
        fmac_bcast<G + i + 1>(a1, hl, w[1][i + 1]);
      }
      w[0][N + i] = a0;
      w[1][N + i] = a1;
    });
    // slot 2: each half its own orbit's coefficients, through LDS
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
    for (int i = 0; i < N; ++i) {
      double acc = __builtin_fma(cn[i], w[2][i], w[2][N + i]);
      if (i > 0) acc = __builtin_fma(cl[i], w[2][i - 1], acc);
      if (i + 1 < N) acc = __builtin_fma(cl[i + 1], w[2][i + 1], acc);
      w[2][N + i] = acc;
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

  // Write back orbit A (stA), orbit B (stB): row-uniform flags; every lane
  // stores what it holds of them.
  auto store = [&](bool stA, bool stB) {
    int64_t obA = oA, obB = oB;
    asm volatile("" : "+v"(obA), "+v"(obB));  // addresses formed here
    const bool own = h ? stB : stA;
    const int64_t obOwn = h ? obB : obA;
    if (own) {
      a.x[c * P + obOwn] = q;
      a.x[(N + c) * P + obOwn] = p;
    }
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const bool st_s = s == 0 ? stA : (s == 1 ? stB : own);
      const int vk = vk_of(s);
      if (st_s && vk >= 0) {
        const int64_t k = vk, ob = s == 0 ? obA : (s == 1 ? obB : obOwn);
#pragma unroll
        for (int i = 0; i < D; ++i) a.w[(k * D + i) * P + ob] = w[s][i];
        a.gm[k * P + ob] = gm[s];
        a.ge[k * P + ob] = ge[s];
      }
    }
    if (own && c == 0) {
      a.sc[SC_LD * P + obOwn] = ld;
      a.sc[SC_GPREV * P + obOwn] = gprev;
      a.sc[SC_SALI_MIN2 * P + obOwn] = smin2;
      a.sc[SC_SALI_LAST2 * P + obOwn] = slast2;
      a.sc[SC_T_CHAOS * P + obOwn] = tch;
      a.sc[SC_EERR * P + obOwn] = eerr;
      a.sc[SC_T_END * P + obOwn] = tend;
      a.st[obOwn] = st;
    }
  };
  // flags of the row's two orbits from a per-group condition (the same in
  // all lanes of the group)
  auto row_flags = [&](bool f, bool &fA, bool &fB) {
    const uint64_t b = __ballot(f && c == 0);
    fA = (b >> (16 * row)) & 1ull;
    fB = (b >> (16 * row + G)) & 1ull;
  };

  // Gram-Schmidt of both orbits' Lyapunov sets (slot 0: A, slot 1: B) in
  // vector order, the two passes interleaved.  Pivot j is lane j of its
  // slot; the dot products and updates read it by row_newbcast:j (pivots
  // unrolled).  Per pivot: dot products of every vector with it (four
  // partial sums), |w_j|^2 from the owner's own dot product, the
  // coefficients (zero for vectors not after the pivot and outside the
  // set), then w_k -= (w_j . w_k / |w_j|^2) w_j.  The owner's coefficient
  // is zero, so its source register keeps its value through the pass, and
  // a component's update comes at least 16 instructions before the next
  // pivot reads it.  The last lane's pivot has no later vector: only its
  // norm.  Growth and normalisation follow the last pivot.
  auto gram_schmidt = [&]() {
    double own2[2] = {1.0, 1.0};
    int nlg = n_l;  // formed afresh per checkpoint (not kept in SGPRs)
    asm volatile("" : "+s"(nlg));
    static_for<0, 2 * N>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      if (j < nlg) {
        double t0, t1;
        if constexpr (j < 2 * N - 1) {
          asm volatile("s_nop 1" : "+v"(w[0][0]), "+v"(w[1][0]));
          double d0[4] = {0.0, 0.0, 0.0, 0.0}, d1[4] = {0.0, 0.0, 0.0, 0.0};
          static_for<0, D>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            fmac_bcast_ordered<j>(d0[i & 3], w[0][i], w[0][i]);
            fmac_bcast_ordered<j>(d1[i & 3], w[1][i], w[1][i]);
          });
          t0 = (d0[0] + d0[1]) + (d0[2] + d0[3]);
          t1 = (d1[0] + d1[1]) + (d1[2] + d1[3]);
        } else {
          t0 = norm2_4<D>(w[0]);
          t1 = norm2_4<D>(w[1]);
        }
        asm volatile("s_nop 1" : "+v"(t0), "+v"(t1));
        const double r0 = bcast<j>(t0), r1 = bcast<j>(t1);
        own2[0] = l == j ? r0 : own2[0];
        own2[1] = l == j ? r1 : own2[1];
        if constexpr (j < 2 * N - 1) {
          const double i0 = rsqrt_nr(r0), i1 = rsqrt_nr(r1);
          double n0 = -(i0 * i0), n1 = -(i1 * i1);
          asm volatile("" : "+v"(n0), "+v"(n1));
          const bool later = l > j && l < nlg;
          const double nd0 = later ? t0 * n0 : 0.0, nd1 = later ? t1 * n1 : 0.0;
          static_for<0, D>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            fmac_bcast_ordered<j>(w[0][i], w[0][i], nd0);
            fmac_bcast_ordered<j>(w[1][i], w[1][i], nd1);
          });
        }
      }
    });
    if (l < nlg) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const double inv = rsqrt_nr(own2[s]);
        grow(gm[s], ge[s], own2[s]);
#pragma unroll
        for (int i = 0; i < D; ++i) w[s][i] *= inv;
      }
    }
  };

  springs();
  int64_t s = a.s_begin;
  const int64_t K = a.K;
  bool aliveA = actA, aliveB = actB;  // row-uniform
  while ((aliveA || aliveB) && s < a.s_end) {
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
    // checkpoint at t; every per-orbit decision is taken on values
    // identical in all lanes of the orbit's group
    const double t = (double)s * dt;
    const bool alive = h ? aliveB : aliveA;
    if (alive) tend = t;
    if (do_ld) {
      ld += grp_sum(ldl);
      ldl = 0.0;
      gprev = grp_sum(gpl);
      gpl = c == 0 ? gprev : 0.0;
    }
    const bool bad = !(__builtin_isfinite(q) && __builtin_isfinite(p));
    const uint64_t bb = __ballot(bad);
    const bool badOwn = alive && ((bb >> (G * g)) & ((1ull << G) - 1ull));
    if (badOwn) st = CHX_ORBIT_NONFINITE;
    bool bA, bB;
    row_flags(badOwn, bA, bB);
    if (bA || bB) {
      store(bA, bB);
      aliveA = aliveA && !bA;
      aliveB = aliveB && !bB;
    }
    bool escaped = false;
    if (a.escape_r2 > 0.0) escaped = grp_sum(q * q) > a.escape_r2;
    // SALI/GALI set (slot 2): back to unit length (lane-local)
    if (c < m_s) {
      const double r2 = norm2_4<D>(w[2]);
      const double inv = rsqrt_nr(r2);
#pragma unroll
      for (int i = 0; i < D; ++i) w[2][i] *= inv;
      grow(gm[2], ge[2], r2);
    }
    double s2 = 0.0;
    if (do_sali) {
      // the pair at lanes 0 and 1 of each group's slot 2: lane 0 takes
      // lane 1's vector through quad_perm [1,1,1,1]
      double sp[2] = {0.0, 0.0}, sm[2] = {0.0, 0.0};
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const double other = dpp<0x55>(w[2][i]);
        const double ap = w[2][i] + other, am = w[2][i] - other;
        sp[i & 1] = __builtin_fma(ap, ap, sp[i & 1]);
        sm[i & 1] = __builtin_fma(am, am, sm[i & 1]);
      }
      s2 = __builtin_fmin(sp[0] + sp[1], sm[0] + sm[1]);
      s2 = grp_sum(c == 0 ? s2 : 0.0);  // lane 0's value in every lane
      slast2 = s2;
      smin2 = __builtin_fmin(smin2, s2);
      if (s2 < a.thr2 && __builtin_isnan(tch)) tch = t;
    }
    gram_schmidt();
    if (do_energy) {
      const double dl = q - left(q), dr = right(q) - q;
      auto spring = [&](double d) {
        const double d2 = d * d;
        return d2 * __builtin_fma(d, __builtin_fma(0.25 * be, d, al * (1.0 / 3.0)), 0.5 * kk);
      };
      double e = __builtin_fma(0.5 * p, p, spring(dl));
      if (c == G - 1) e += spring(dr);
      const double Hs = grp_sum(e);
      eerr = __builtin_fmax(eerr, __builtin_fabs(Hs - H0));
    }
    bool stopOwn = false;
    if (alive && !badOwn) {
      if (escaped) {
        st = CHX_ORBIT_ESCAPED;
        stopOwn = true;
      } else if (a.early_exit && do_sali && s2 < a.thr2) {
        st = CHX_ORBIT_EXITED;
        stopOwn = true;
      }
    }
    bool sA, sB;
    row_flags(stopOwn, sA, sB);
    if (sA || sB) {
      store(sA, sB);
      aliveA = aliveA && !sA;
      aliveB = aliveB && !sB;
    }
  }
  store(aliveA, aliveB);
}

}  // namespace chx
