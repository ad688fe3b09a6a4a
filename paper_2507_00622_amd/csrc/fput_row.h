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
// Gram-Schmidt.  With one row per orbit every lane takes the pivot's
// components straight from the owner lane's registers through the FMA's
// row_newbcast operand (pivots unrolled, no LDS); with two rows per orbit
// the owner stages the pivot in LDS, each lane reads one or two of its
// components and spreads them by row_newbcast.  Row sums (energy, LD,
// escape radius) use a quad_perm / half-mirror / mirror butterfly, so all
// 16 lanes hold the same bits.
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

// acc += coef(lane I of the row) * x in one instruction: v_fmac_f64 with
// its first source read through row_newbcast:I (DPP on 64-bit operands
// exists for this broadcast only)
template <int I>
__device__ __forceinline__ void fmac_bcast(double &acc, double coef, double x) {
  asm("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
      : "+v"(acc)
      : "v"(coef), "v"(x), "n"(I));
}

// the same, kept in program order with the other ordered ones (the
// Gram-Schmidt sweeps: left free, the scheduler interleaves them into far
// more live registers than the sweep needs)
template <int I>
__device__ __forceinline__ void fmac_bcast_ordered(double &acc, double coef, double x) {
  asm volatile("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
               : "+v"(acc)
               : "v"(coef), "v"(x), "n"(I));
}

// |v|^2 over D components with four partial sums, so that the FMAs are not
// one dependent chain
template <int D>
__device__ __forceinline__ double norm2_4(const double *v) {
  double p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < D; ++c) p[c & 3] = __builtin_fma(v[c], v[c], p[c & 3]);
  return (p[0] + p[1]) + (p[2] + p[3]);
}

// sum over the 16 lanes of a row, identical in every lane
__device__ __forceinline__ double row_sum(double s) {
  s += dpp<0xB1>(s);   // quad_perm [1,0,3,2]
  s += dpp<0x4E>(s);   // quad_perm [2,3,0,1]
  s += dpp<0x141>(s);  // row_half_mirror
  s += dpp<0x140>(s);  // row_mirror
  return s;
}

// Values that only checkpoints touch (SALI minimum and last value, time of
// chaos, energy error, H0, end time, growth mantissas and exponents): in
// registers, or (S) in LDS between checkpoints, [field][lane] of the 64
// lanes, read and written with volatile accesses so that the compiler does
// not carry them in registers through the step loop anyway.
template <bool S, int V>
struct CkptVals {
  enum { SMIN2, SLAST2, TCH, EERR, H0, TEND, GM, ND = GM + V };
  volatile double *d;  // LDS [ND][64] when S
  volatile int *e;     // LDS [V][64] when S
  double rd[S ? 1 : ND];
  int re[S ? 1 : V];
  int t;
  __device__ __forceinline__ double get(int f) const {
    if constexpr (S) return d[f * 64 + t];
    else return rd[f];
  }
  __device__ __forceinline__ void set(int f, double v) {
    if constexpr (S) d[f * 64 + t] = v;
    else rd[f] = v;
  }
  __device__ __forceinline__ int gete(int s) const {
    if constexpr (S) return e[s * 64 + t];
    else return re[s];
  }
  __device__ __forceinline__ void sete(int s, int v) {
    if constexpr (S) e[s * 64 + t] = v;
    else re[s] = v;
  }
  // growth of slot s's vector by the squared norm r2
  __device__ __forceinline__ void grow_slot(int s, double r2) {
    double m = get(GM + s);
    int x = gete(s);
    grow(m, x, r2);
    set(GM + s, m);
    sete(s, x);
  }
};

}  // namespace fputrow

// R rows per orbit (R = 1: four orbits per wavefront; R = 2: two).  Every
// row of an orbit holds the whole state (the rows execute the same
// instructions, so the copy costs nothing) and V vector slots per lane:
// slot s of lane l in row r of the orbit is vector position
// pos = (s R + r) 16 + l -- the rows interleave, so the Lyapunov set (the
// first positions) is spread over all rows of the orbit.
// B: Gram-Schmidt pivots per round (one-row layouts).
// STASH: N = 16 with three slots keeps the checkpoint-only values in LDS,
// which lets two wavefronts share a SIMD (the vectors alone are 192 VGPRs).
template <int N, int V, int R, int B = 1,
          bool STASH = (N == 16 && V == 3 && R == 1)>
__global__ void __launch_bounds__(64, STASH ? 2 : 1) fput_row_kernel(const StepArgs a) {
  using namespace fputrow;
  constexpr int D = 2 * N;
  constexpr int OPW = 4 / R;  // orbits per wavefront
  constexpr int CPL = (D + 15) / 16;  // pivot components per lane
  __shared__ __align__(16) double piv[R == 1 ? 1 : OPW][16][CPL];
  using CV = CkptVals<STASH, V>;
  __shared__ double cvd[STASH ? (int)CV::ND : 1][64];
  __shared__ int cve[STASH ? V : 1][64];
  CV cv;
  cv.d = &cvd[0][0];
  cv.e = &cve[0][0];
  cv.t = threadIdx.x;
  const int lane = threadIdx.x & 15, row = threadIdx.x >> 4;
  const int ow = row / R, ro = row % R;
  const int64_t o = (int64_t)blockIdx.x * OPW + ow;
  const int64_t P = a.pitch;
  bool act = (o < a.n) && (a.st[o] == CHX_ORBIT_OK);
  const int64_t oo = act ? o : 0;  // inactive rows compute on a copy
  const bool mass = lane < N;
  const int n_l = a.n_l, m_s = a.m_s, M = n_l + m_s;
  const double kk = a.prm[0], al = a.prm[1], be = a.prm[2];

  // vector index in the ensemble layout of slot s, -1 = unused slot
  auto vk_of = [&](int s) {
    const int pos = (s * R + ro) * 16 + lane;
    return pos < n_l ? m_s + pos : (pos < M ? pos - n_l : -1);
  };
  double q = mass ? a.x[lane * P + oo] : 0.0;
  double p = mass ? a.x[(N + lane) * P + oo] : 0.0;
  double w[V][D];
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const int vk = vk_of(s);
    const int64_t k = vk < 0 ? 0 : vk;
#pragma unroll
    for (int c = 0; c < D; ++c) w[s][c] = vk < 0 ? 0.0 : a.w[(k * D + c) * P + oo];
    cv.set(CV::GM + s, vk < 0 ? 1.0 : a.gm[k * P + oo]);
    cv.sete(s, vk < 0 ? 0 : a.ge[k * P + oo]);
  }
  double ld = a.sc[SC_LD * P + oo], gprev = a.sc[SC_GPREV * P + oo];
  cv.set(CV::SMIN2, a.sc[SC_SALI_MIN2 * P + oo]);
  cv.set(CV::SLAST2, a.sc[SC_SALI_LAST2 * P + oo]);
  cv.set(CV::TCH, a.sc[SC_T_CHAOS * P + oo]);
  cv.set(CV::EERR, a.sc[SC_EERR * P + oo]);
  cv.set(CV::H0, a.sc[SC_H0 * P + oo]);
  cv.set(CV::TEND, a.sc[SC_T_END * P + oo]);
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
    // Per lane: -h (kappa_l + kappa_{l+1}) and h kappa_l.  Every coupling of
    // component i is taken from lane i or i+1 by the FMA itself
    // (v_fmac_f64 with a row_newbcast source), so no broadcast moves.  The
    // s_nop covers the two wait states a DPP read needs after the VALU
    // write of its source.
    double nhd = -(h * (kl + kr)), hl = h * kl;
    asm volatile("s_nop 1" : "+v"(nhd), "+v"(hl));
    // components in groups, the three FMAs of each component in stages,
    // so that consecutive FMAs do not feed each other
    constexpr int GS = V >= 2 ? 2 : 3;
    static_for<0, (N + GS - 1) / GS>([&](auto gc) {
      constexpr int i0 = decltype(gc)::value * GS;
      double acc[GS][V];
      static_for<0, GS>([&](auto jc) {
        constexpr int j = decltype(jc)::value, i = i0 + j;
        if constexpr (i < N) {
#pragma unroll
          for (int s = 0; s < V; ++s) {
            acc[j][s] = w[s][N + i];
            fmac_bcast<i>(acc[j][s], nhd, w[s][i]);
          }
        }
      });
      static_for<0, GS>([&](auto jc) {
        constexpr int j = decltype(jc)::value, i = i0 + j;
        if constexpr (i < N && i > 0) {
#pragma unroll
          for (int s = 0; s < V; ++s) fmac_bcast<i>(acc[j][s], hl, w[s][i - 1]);
        }
      });
      static_for<0, GS>([&](auto jc) {
        constexpr int j = decltype(jc)::value, i = i0 + j;
        if constexpr (i + 1 < N) {
#pragma unroll
          for (int s = 0; s < V; ++s) fmac_bcast<(i + 1 < N ? i + 1 : 0)>(acc[j][s], hl, w[s][i + 1]);
        }
      });
      static_for<0, GS>([&](auto jc) {
        constexpr int j = decltype(jc)::value, i = i0 + j;
        if constexpr (i < N) {
#pragma unroll
          for (int s = 0; s < V; ++s) w[s][N + i] = acc[j][s];
        }
      });
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
  auto wave_sync = []() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };

  // Checkpoint at t; returns false when the orbit stops.  Every decision is
  // taken on values that are identical in all lanes of the orbit's rows.
  auto checkpoint = [&](double t) {
    cv.set(CV::TEND, t);
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
      const int pos = (s * R + ro) * 16 + lane;
      if (pos >= n_l && pos < M) {
        const double r2 = norm2_4<D>(w[s]);
        const double inv = rsqrt_nr(r2);
#pragma unroll
        for (int c = 0; c < D; ++c) w[s][c] *= inv;
        cv.grow_slot(s, r2);
      }
    }
    double s2 = 0.0;
    if (do_sali) {
      // the SALI pair sits at positions n_l and n_l + 1: lanes 0 and 1 of
      // group n_l / 16 (the launcher requires n_l % 16 == 0), which is slot
      // (n_l / 16) / R of the orbit's row (n_l / 16) % R
      const int g0 = n_l / 16, r0 = g0 % R, s0 = g0 / R;
      double sp[2] = {0.0, 0.0}, sm[2] = {0.0, 0.0};
#pragma unroll
      for (int s = 0; s < V; ++s) {
        if (s == s0) {
#pragma unroll
          for (int c = 0; c < D; ++c) {
            const double other = bcast<1>(w[s][c]);
            const double ap = w[s][c] + other, am = w[s][c] - other;
            sp[c & 1] = __builtin_fma(ap, ap, sp[c & 1]);
            sm[c & 1] = __builtin_fma(am, am, sm[c & 1]);
          }
        }
      }
      s2 = __builtin_fmin(sp[0] + sp[1], sm[0] + sm[1]);
      if constexpr (R == 1) {
        s2 = bcast<0>(s2);
      } else {
        // lane 0 of the pair's row to every lane of the orbit
        s2 = __shfl(s2, (ow * R + r0) * 16, 64);
      }
      cv.set(CV::SLAST2, s2);
      cv.set(CV::SMIN2, __builtin_fmin(cv.get(CV::SMIN2), s2));
      if (s2 < a.thr2 && __builtin_isnan(cv.get(CV::TCH))) cv.set(CV::TCH, t);
    }
    // Lyapunov set: modified Gram-Schmidt in vector order.  The pivot's
    // owner stages the vector as it stands (orthogonal to the earlier
    // pivots, not yet normalised) in LDS, spread over the lanes: lane i of
    // every row of the orbit reads components i and i + 16.  Its squared
    // norm is a row sum (the same bits in every lane of the orbit), and the
    // dot products and updates take component c through the FMA's
    // row_newbcast operand from lane c % 16, so the pivot costs one LDS
    // read per lane.  w_k -= (w_j . w_k / |w_j|^2) w_j is the projection on
    // the normalised pivot.  The owner keeps |w_j|^2 of its own slot; the
    // growth and the normalisation of every Lyapunov slot follow the last
    // pivot.  Pivots come in groups of 16 (group G = slot G / R of row
    // G % R); the group is a compile-time index and the 16 pivots of a
    // group are a runtime loop.
    double own2[V];  // |w|^2 of this lane's slot when it was the pivot
#pragma unroll
    for (int s = 0; s < V; ++s) own2[s] = 1.0;
    // n_l taken afresh here, so that the compiler forms the pivots'
    // comparisons with it in each checkpoint instead of keeping them in
    // scalar registers through the step loop (where they spill)
    int nlg = n_l;
    asm volatile("" : "+s"(nlg));
    const int nls = (nlg + 16 * R - 1) / (16 * R);  // slots holding Lyapunov vectors
    if constexpr (R == 1) {
      // One row per orbit: the pivots are read straight from their owners'
      // registers.  The dot products and the updates take component c of
      // pivot j from lane j % 16 through the FMA's row_newbcast operand, so
      // the pivots are unrolled (the lane is an immediate) and nothing is
      // staged in LDS.  Pivots go B at a time (modified Gram-Schmidt
      // regrouped): one pass of dot products of every later vector with
      // the B pivots as they stand (B independent accumulators); the B x B
      // Gram matrix G of the pivots from their owners' own dot products;
      // its Cholesky factor L in every lane (L_nn is the norm of pivot n
      // after projecting out pivots 0..n-1, as in modified Gram-Schmidt);
      // then one pass of updates w <- w - P y with y = G^-1 (P^T w), the
      // projection out of the pivots' span -- for the owner of pivot n the
      // same solves cut to pivots 0..n-1, which leaves its vector's part
      // orthogonal to them, of norm L_nn (kept for the growth and the
      // normalisation after the last pivot).  Slots from nls on hold no
      // Lyapunov vector (the set has at most 2N vectors, so at most
      // ceil(2N / 16) slots).
      //
      // Ordering: the owners' coefficients for their own and later pivots
      // are zero, so a source lane is unchanged until every pivot it owns
      // has been applied.  In the pivots' own slot the updates go pivot by
      // pivot in decreasing order (an owner is written only by the pivots
      // before its own), each over all components, so no DPP read follows
      // the write of its source register closely.
      constexpr int NLS_MAX = (2 * N + 15) / 16 < V ? (2 * N + 15) / 16 : V;
      constexpr int PS = B >= 4 ? 1 : 4 / B;  // partial sums per dot product
      static_for<0, NLS_MAX>([&](auto gc) {
        constexpr int sj = decltype(gc)::value;  // the pivots' slot
        if (sj * 16 < nlg) {
          auto group = [&](auto lc) {
            constexpr int L = decltype(lc)::value;  // slots sj..L-1 hold Lyapunov vectors
            static_for<0, 16 / B>([&](auto jc) {
              constexpr int l0 = decltype(jc)::value * B;  // the first pivot's lane
              const int j0 = sj * 16 + l0;
              if (j0 < nlg) {
                const int nb = nlg - j0 < B ? nlg - j0 : B;  // pivots in this round
                // two wait states before the first DPP read of w[sj]
                asm volatile("s_nop 1" : "+v"(w[sj][0]), "+v"(w[sj][1]));
                double d[V][B][PS];
#pragma unroll
                for (int s = 0; s < V; ++s)
#pragma unroll
                  for (int m = 0; m < B; ++m)
#pragma unroll
                    for (int k = 0; k < PS; ++k) d[s][m][k] = 0.0;
                static_for<0, D>([&](auto cc) {
                  constexpr int c = decltype(cc)::value;
                  static_for<0, B>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
#pragma unroll
                    for (int s = sj; s < L; ++s)
                      fmac_bcast_ordered<l0 + m>(d[s][m][c % PS], w[sj][c], w[s][c]);
                  });
                });
                double t[V][B];
#pragma unroll
                for (int s = sj; s < L; ++s)
#pragma unroll
                  for (int m = 0; m < B; ++m) {
                    double v = d[s][m][0];
#pragma unroll
                    for (int k = 1; k < PS; ++k) v += d[s][m][k];
                    t[s][m] = v;
                  }
                if constexpr (B == 1)
                  asm volatile("s_nop 1" : "+v"(t[sj][0]));
                else if constexpr (B == 2)
                  asm volatile("s_nop 1" : "+v"(t[sj][0]), "+v"(t[sj][1]));
                else
                  asm volatile("s_nop 1" : "+v"(t[sj][0]), "+v"(t[sj][1]), "+v"(t[sj][2]), "+v"(t[sj][3]));
                // Gram matrix (upper triangle): G_mn = p_m . p_n, from the
                // owner of p_n; identity rows past the last pivot
                double G[B][B];
                static_for<0, B>([&](auto nc) {
                  constexpr int n = decltype(nc)::value;
                  static_for<0, n + 1>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    const double g = bcast<l0 + n>(t[sj][m]);
                    G[m][n] = n < nb ? g : (m == n ? 1.0 : 0.0);
                  });
                });
                double Lm[B][B], rr[B], iv[B];
#pragma unroll
                for (int n = 0; n < B; ++n) {
                  double r = G[n][n];
#pragma unroll
                  for (int k = 0; k < n; ++k) r = __builtin_fma(-Lm[n][k], Lm[n][k], r);
                  rr[n] = r;
                  iv[n] = rsqrt_nr(r);
#pragma unroll
                  for (int m = n + 1; m < B; ++m) {
                    double v = G[n][m];
#pragma unroll
                    for (int k = 0; k < n; ++k) v = __builtin_fma(-Lm[m][k], Lm[n][k], v);
                    Lm[m][n] = v * iv[n];
                  }
                }
                // coefficients -y, with y = G^-1 (P^T w) cut to the first
                // ne pivots: ne = nb for later Lyapunov vectors, the pivot's
                // index for its owner, 0 before the pivots and outside the set
                double ny[V][B];
#pragma unroll
                for (int s = sj; s < L; ++s) {
                  const int pos = s * 16 + lane;
                  int ne = pos < nlg ? nb : 0;
                  if (s == sj) ne = lane < l0 ? 0 : (lane < l0 + nb ? lane - l0 : ne);
                  double z[B], y[B];
#pragma unroll
                  for (int m = 0; m < B; ++m) {
                    double v = t[s][m];
#pragma unroll
                    for (int k = 0; k < m; ++k) v = __builtin_fma(-Lm[m][k], z[k], v);
                    z[m] = m < ne ? v * iv[m] : 0.0;
                  }
#pragma unroll
                  for (int m = B - 1; m >= 0; --m) {
                    double v = z[m];
#pragma unroll
                    for (int k = m + 1; k < B; ++k) v = __builtin_fma(-Lm[k][m], y[k], v);
                    y[m] = v * iv[m];
                    ny[s][m] = -y[m];
                  }
                }
                {
                  double o2 = own2[sj];
#pragma unroll
                  for (int m = 0; m < B; ++m) o2 = (lane == l0 + m && m < nb) ? rr[m] : o2;
                  own2[sj] = o2;
                }
                // later slots: any order (they are no pivot's source)
                static_for<0, D>([&](auto cc) {
                  constexpr int c = decltype(cc)::value;
                  static_for<0, B>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
#pragma unroll
                    for (int s = sj + 1; s < L; ++s)
                      fmac_bcast_ordered<l0 + m>(w[s][c], w[sj][c], ny[s][m]);
                  });
                });
                // the pivots' slot: pivot by pivot, last first
                static_for<0, B>([&](auto mc) {
                  constexpr int m = B - 1 - decltype(mc)::value;
                  static_for<0, D>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    fmac_bcast_ordered<l0 + m>(w[sj][c], w[sj][c], ny[sj][m]);
                  });
                });
              }
            });
          };
          static_for<sj + 1, NLS_MAX + 1>([&](auto lc) {
            if (nls == decltype(lc)::value) group(lc);
          });
        }
      });
    } else
    static_for<0, V * R>([&](auto gc) {
      constexpr int G = decltype(gc)::value;
      constexpr int rj = G % R, sj = G / R;
      int jend = n_l - G * 16;
      if (jend > 16) jend = 16;
      for (int lj = 0; lj < jend; ++lj) {
        const bool owner = ro == rj && lane == lj;
        if (owner) {
#pragma unroll
          for (int i = 0; i < 16; ++i)
#pragma unroll
            for (int k = 0; k < CPL; ++k)
              piv[ow][i][k] = k * 16 + i < D ? w[sj][k * 16 + i] : 0.0;
        }
        wave_sync();
        double pc[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) pc[k] = piv[ow][lane][k];
        // DPP reads of pc follow; keep two wait states after its load
        if constexpr (CPL == 2)
          asm volatile("s_nop 1" : "+v"(pc[0]), "+v"(pc[1]));
        else
          asm volatile("s_nop 1" : "+v"(pc[0]));
        double r2 = pc[0] * pc[0];
        if constexpr (CPL == 2) r2 = __builtin_fma(pc[1], pc[1], r2);
        // Slot s of this lane is after the pivot if its position is, and
        // holds a Lyapunov vector if its position is below n_l.  Slots
        // before sj never are (no code for them), and slots from nls on
        // hold no Lyapunov vector: the projection is instantiated for each
        // possible nls and one is chosen by a uniform branch.  Slots that
        // are not after the pivot take a zero coefficient.
        const int pj = G * 16 + lj;
        auto project = [&](auto lc) {
          constexpr int L = decltype(lc)::value;
          constexpr int PS = 4;  // partial sums per dot product
          double d[V][PS];
#pragma unroll
          for (int s = 0; s < V; ++s)
#pragma unroll
            for (int k = 0; k < PS; ++k) d[s][k] = 0.0;
          static_for<0, D>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
#pragma unroll
            for (int s = sj; s < L; ++s) fmac_bcast_ordered<c % 16>(d[s][c % PS], pc[c / 16], w[s][c]);
          });
          r2 = row_sum(r2);
          own2[sj] = owner ? r2 : own2[sj];
          const double inv = rsqrt_nr(r2);
          const double ni2 = -(inv * inv);
          double nd[V];
#pragma unroll
          for (int s = sj; s < L; ++s) {
            const int pos = (s * R + ro) * 16 + lane;
            const double t = (d[s][0] + d[s][1]) + (d[s][2] + d[s][3]);
            nd[s] = (pos > pj && pos < n_l) ? t * ni2 : 0.0;
          }
          static_for<0, D>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
#pragma unroll
            for (int s = sj; s < L; ++s) fmac_bcast_ordered<c % 16>(w[s][c], pc[c / 16], nd[s]);
          });
        };
        static_for<sj + 1, V + 1>([&](auto lc) {
          if (nls == decltype(lc)::value) project(lc);
        });
        wave_sync();
      }
    });
#pragma unroll
    for (int s = 0; s < V; ++s) {
      if ((s * R + ro) * 16 + lane < n_l) {
        const double inv = rsqrt_nr(own2[s]);
        cv.grow_slot(s, own2[s]);
#pragma unroll
        for (int c = 0; c < D; ++c) w[s][c] *= inv;
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
      cv.set(CV::EERR, __builtin_fmax(cv.get(CV::EERR), __builtin_fabs(Hs - cv.get(CV::H0))));
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
    if (mass && ro == 0) {
      a.x[lane * P + ob] = q;
      a.x[(N + lane) * P + ob] = p;
    }
#pragma unroll
    for (int s = 0; s < V; ++s) {
      const int vk = vk_of(s);
      if (vk >= 0) {
        const int64_t k = vk;
#pragma unroll
        for (int c = 0; c < D; ++c) a.w[(k * D + c) * P + ob] = w[s][c];
        a.gm[k * P + ob] = cv.get(CV::GM + s);
        a.ge[k * P + ob] = cv.gete(s);
      }
    }
    if (lane == 0 && ro == 0) {
      a.sc[SC_LD * P + ob] = ld;
      a.sc[SC_GPREV * P + ob] = gprev;
      a.sc[SC_SALI_MIN2 * P + ob] = cv.get(CV::SMIN2);
      a.sc[SC_SALI_LAST2 * P + ob] = cv.get(CV::SLAST2);
      a.sc[SC_T_CHAOS * P + ob] = cv.get(CV::TCH);
      a.sc[SC_EERR * P + ob] = cv.get(CV::EERR);
      a.sc[SC_T_END * P + ob] = cv.get(CV::TEND);
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
