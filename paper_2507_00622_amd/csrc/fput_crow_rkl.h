// fput_crow_rkl.h -- DOP853 (fixed step and adaptive DOP8(5)) for FPU chains
// with more than four deviation vectors, up to the full Lyapunov set and a
// GALI set: component rows as in fput_crow_rk.h (one 16-lane row per orbit,
// lane l holding component l of the state and of every vector, ghost lanes
// N..15 zero), with the vectors in LDS instead of registers.
//
// A step is the state's 12 stages (positions, forces and the two spring
// stiffnesses of each stage kept in registers), then one pass per vector in
// a runtime loop: the vector's two components of this lane come from LDS,
// its 12 stages are built from the stage stiffnesses (the tridiagonal
// Hessian couples each component to its neighbours, read through row DPP),
// and the new components go back.  Only one vector's stage derivatives are
// live at a time, so the register count does not grow with the number of
// vectors.  The adaptive solver writes the attempted vectors to a second
// LDS buffer and swaps the two on acceptance.
//
// LDS of a 64-thread block (four orbits, one per row), per buffer:
//   vec[(2 v + c) * 64 + threadIdx.x], c = 0: dq, c = 1: dp,
// so the 64 lanes of a wavefront read 64 consecutive doubles.  The growth
// products of vector v (identical in every lane of the orbit) are held by
// lane v % 16 of the row, slot v / 16.
//
// Checkpoints follow the order of the component-row kernels: the SALI/GALI
// set back to unit length, SALI from its first two vectors, modified
// Gram-Schmidt on the Lyapunov set (vector j minus its projections on the
// normalised earlier ones, then normalised), the energy; dot products and
// norms are row sums, identical in all 16 lanes, so every decision is
// row-uniform.
#pragma once
#include "fput_crow_rk.h"

namespace chx {

namespace rkl {

constexpr int MAX_VEC = 64;  // 4N at N = 16
constexpr int GSLOTS = MAX_VEC / 16;

// LDS bytes of one block: M vectors x 2 components x 64 lanes, doubled for
// the adaptive solver's attempted vectors
inline size_t lds_bytes(int M, bool adaptive) {
  return (size_t)M * 2 * 64 * sizeof(double) * (adaptive ? 2 : 1);
}

// One vector's 12 stages from the state's stage stiffnesses (the same
// arithmetic as the register form in fput_crow_rk.h).
__device__ __forceinline__ void vec_stages(const double (&skl)[12], const double (&skr)[12],
                                           double h, double dq, double dp, double (&kq)[12][1],
                                           double (&kp)[12][1]) {
  using namespace fputrow;
  dop853::static_for<0, 12>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    const double Yq = dq + dop853::stage_sum<I>(kq, 0);
    const double Yp = dp + dop853::stage_sum<I>(kp, 0);
    const double ql = dpp<0x111>(Yq);  // row_shr:1
    const double qr = dpp<0x101>(Yq);  // row_shl:1
    double hq = (skl[I] + skr[I]) * Yq;
    hq = __builtin_fma(-skl[I], ql, hq);
    hq = __builtin_fma(-skr[I], qr, hq);
    kq[I][0] = h * Yp;
    kp[I][0] = -h * hq;
  });
}

}  // namespace rkl

template <int N>
struct CRowRKL : CRowRK<N, 0> {
  using B = CRowRK<N, 0>;
  using B::eerr;
  using B::gprev;
  using B::H0;
  using B::lane;
  using B::ld;
  using B::mass;
  using B::p;
  using B::q;
  using B::row;
  using B::skl;
  using B::skr;
  using B::slast2;
  using B::smin2;
  using B::st;
  using B::tch;
  using B::tend;

  double *vec, *vnew;  // this block's vector buffers (vnew: adaptive only)
  int tid, M;
  double gmr[rkl::GSLOTS];  // growth products of vectors lane + 16 s
  int ger[rkl::GSLOTS];

  __device__ double &cq(double *b, int v) const { return b[(2 * v) * 64 + tid]; }
  __device__ double &cp(double *b, int v) const { return b[(2 * v + 1) * 64 + tid]; }

  __device__ void setup(double *lds, int m, bool adaptive) {
    tid = threadIdx.x & 63;
    M = m;
    vec = lds;
    vnew = adaptive ? lds + (size_t)M * 2 * 64 : lds;
  }

  __device__ void load_vectors(const StepArgs &a, int64_t o) {
    const int64_t P = a.pitch;
    for (int v = 0; v < M; ++v) {
      cq(vec, v) = mass ? a.w[((int64_t)v * 2 * N + lane) * P + o] : 0.0;
      cp(vec, v) = mass ? a.w[((int64_t)v * 2 * N + N + lane) * P + o] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < rkl::GSLOTS; ++s) {
      const int v = lane + 16 * s;
      gmr[s] = v < M ? a.gm[(int64_t)v * P + o] : 1.0;
      ger[s] = v < M ? a.ge[(int64_t)v * P + o] : 0;
    }
  }

  __device__ void store_vectors(const StepArgs &a, int64_t o) const {
    const int64_t P = a.pitch;
    if (mass)
      for (int v = 0; v < M; ++v) {
        a.w[((int64_t)v * 2 * N + lane) * P + o] = cq(vec, v);
        a.w[((int64_t)v * 2 * N + N + lane) * P + o] = cp(vec, v);
      }
#pragma unroll
    for (int s = 0; s < rkl::GSLOTS; ++s) {
      const int v = lane + 16 * s;
      if (v < M) {
        a.gm[(int64_t)v * P + o] = gmr[s];
        a.ge[(int64_t)v * P + o] = ger[s];
      }
    }
  }

  // growth of vector v by the factor f (row-uniform): kept by lane v % 16
  __device__ void grow_vec(int v, double f) {
#pragma unroll
    for (int s = 0; s < rkl::GSLOTS; ++s)
      if (lane + 16 * s == v) grow(gmr[s], ger[s], f);
  }

  // one fixed DOP853 step of size h
  __device__ void rk_step(const StepArgs &a, double h, bool do_ld) {
    {
      double kq[12][1], kp[12][1], g = 0.0;
      B::state_pass(a, h, do_ld, kq, kp, g);
      q += dop853::final_sum(kq, 0);
      p += dop853::final_sum(kp, 0);
      if (do_ld) ld = __builtin_fma(h, fputrow::row_sum(g), ld);
    }
    for (int v = 0; v < M; ++v) {
      double kq[12][1], kp[12][1];
      const double dq = cq(vec, v), dp = cp(vec, v);
      rkl::vec_stages(skl, skr, h, dq, dp, kq, kp);
      cq(vec, v) = dq + dop853::final_sum(kq, 0);
      cp(vec, v) = dp + dop853::final_sum(kp, 0);
    }
  }

  // One attempted step of size h: the new state and LD in qn, pn, ldn, the
  // new vectors in vnew; returns DOP853's scaled error estimate over the
  // state and the vectors (the LD left out), err = e5 / sqrt(n (e5 + 0.01
  // e3)), n = 2N (1 + M), from row sums of the mass lanes' error terms.
  __device__ double rk_attempt(const StepArgs &a, double h, bool do_ld, double &qn, double &pn,
                               double &ldn) {
    double e5 = 0.0, e3 = 0.0;
    {
      double kq[12][1], kp[12][1], g = 0.0;
      B::state_pass(a, h, do_ld, kq, kp, g);
      const double sq = dop853::final_sum(kq, 0), sp = dop853::final_sum(kp, 0);
      qn = q + sq;
      pn = p + sp;
      if (mass) {
        dop853::err_terms(kq, 0, q, qn, sq, a.rtol, a.atol, e5, e3);
        dop853::err_terms(kp, 0, p, pn, sp, a.rtol, a.atol, e5, e3);
      }
      ldn = do_ld ? __builtin_fma(h, fputrow::row_sum(g), ld) : ld;
    }
    for (int v = 0; v < M; ++v) {
      double kq[12][1], kp[12][1];
      const double dq = cq(vec, v), dp = cp(vec, v);
      rkl::vec_stages(skl, skr, h, dq, dp, kq, kp);
      const double sq = dop853::final_sum(kq, 0), sp = dop853::final_sum(kp, 0);
      const double dqn = dq + sq, dpn = dp + sp;
      if (mass) {
        dop853::err_terms(kq, 0, dq, dqn, sq, a.rtol, a.atol, e5, e3);
        dop853::err_terms(kp, 0, dp, dpn, sp, a.rtol, a.atol, e5, e3);
      }
      cq(vnew, v) = dqn;
      cp(vnew, v) = dpn;
    }
    e5 = fputrow::row_sum(e5);
    e3 = fputrow::row_sum(e3);
    const double deno = __builtin_fma(0.01, e3, e5);
    if (!(deno > 0.0)) return deno == 0.0 ? 0.0 : deno;  // NaN stays NaN
    return e5 / sqrt((double)(2 * N * (1 + M)) * deno);
  }

  __device__ void accept_vectors() {
    double *t = vec;
    vec = vnew;
    vnew = t;
  }

  // Checkpoint at t; returns false when the orbit stops.
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
    for (int v = 0; v < m_s; ++v) {
      const double dq = cq(vec, v), dp = cp(vec, v);
      const double r2 = row_sum(__builtin_fma(dq, dq, dp * dp));
      const double inv = rsqrt_nr(r2);
      cq(vec, v) = dq * inv;
      cp(vec, v) = dp * inv;
      grow_vec(v, r2);
    }
    double s2 = 0.0;
    if (do_sali) {
      const double q0 = cq(vec, 0), p0 = cp(vec, 0), q1 = cq(vec, 1), p1 = cp(vec, 1);
      const double aq = q0 + q1, ap = p0 + p1, bq = q0 - q1, bp = p0 - p1;
      const double sp = row_sum(__builtin_fma(aq, aq, ap * ap));
      const double sm = row_sum(__builtin_fma(bq, bq, bp * bp));
      s2 = __builtin_fmin(sp, sm);
      slast2 = s2;
      smin2 = __builtin_fmin(smin2, s2);
      if (s2 < a.thr2 && __builtin_isnan(tch)) tch = t;
    }
    for (int j = m_s; j < M; ++j) {
      double wq = cq(vec, j), wp = cp(vec, j);
      for (int l = m_s; l < j; ++l) {
        const double lq = cq(vec, l), lp = cp(vec, l);
        const double d = row_sum(__builtin_fma(lq, wq, lp * wp));
        wq = __builtin_fma(-d, lq, wq);
        wp = __builtin_fma(-d, lp, wp);
      }
      const double r2 = row_sum(__builtin_fma(wq, wq, wp * wp));
      const double inv = rsqrt_nr(r2);
      cq(vec, j) = wq * inv;
      cp(vec, j) = wp * inv;
      grow_vec(j, r2);
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

extern __shared__ double fput_rkl_lds[];

template <int N>
__global__ void __launch_bounds__(64) fput_crow_rkl_kernel(const StepArgs a) {
  const int64_t o = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 4);
  // rows beyond the ensemble or already stopped do nothing; every lane of a
  // row takes the same branch, and a row only touches its own lanes' LDS
  if (o >= a.n) return;
  if (a.st[o] != CHX_ORBIT_OK) return;
  CRowRKL<N> r;
  r.setup(fput_rkl_lds, a.m_s + a.n_l, false);
  r.load(a, o);
  r.load_vectors(a, o);
  const bool do_ld = (a.ind & CHX_IND_LD) != 0;
  int64_t s = a.s_begin;
  const int64_t K = a.K;
  while (s < a.s_end) {
    int64_t next = (s / K + 1) * K;
    if (next > a.n_total) next = a.n_total;
    for (int64_t j = s; j < next; ++j) r.rk_step(a, a.dt, do_ld);
    s = next;
    if (!r.checkpoint(a, (double)s * a.dt)) break;
  }
  r.store(a, o);
  r.store_vectors(a, o);
}

// The adaptive DOP8(5) solver: the checkpoint schedule, controller and
// landing rule of the other adaptive kernels, one step loop per row.
template <int N>
__global__ void __launch_bounds__(64) fput_crow_rkla_kernel(const StepArgs a) {
  const int64_t o = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 4);
  if (o >= a.n) return;
  if (a.st[o] != CHX_ORBIT_OK) return;
  CRowRKL<N> r;
  r.setup(fput_rkl_lds, a.m_s + a.n_l, true);
  r.load(a, o);
  r.load_vectors(a, o);
  const int64_t P = a.pitch;
  double h = a.sc[SC_H * P + o];
  if (!(h > 0.0)) h = a.dt;  // the first step
  bool rej = a.sc[SC_REJ * P + o] != 0.0;
  double nacc = a.sc[SC_NACC * P + o], nrej = a.sc[SC_NREJ * P + o];
  double emax = a.sc[SC_ERR_MAX * P + o], elast = a.sc[SC_ERR_LAST * P + o];
  const bool do_ld = (a.ind & CHX_IND_LD) != 0;
  int64_t s = a.s_begin;
  const int64_t K = a.K;
  while (s < a.s_end) {
    int64_t next = (s / K + 1) * K;
    if (next > a.n_total) next = a.n_total;
    double t = (double)s * a.dt;
    const double tb = (double)next * a.dt;
    int attempts = 0, fail = CHX_ORBIT_OK;
    while (t < tb) {
      double hh = h;
      bool last = false;
      if (t + 1.01 * hh >= tb) {
        hh = tb - t;
        last = true;
      }
      double qn, pn, ldn;
      const double err = r.rk_attempt(a, hh, do_ld, qn, pn, ldn);
      const bool lane_bad = !(__builtin_isfinite(qn) && __builtin_isfinite(pn));
      const bool bad = ((__ballot(lane_bad) >> (16 * r.row)) & 0xFFFFull) != 0;
      if (bad || !__builtin_isfinite(err) || !__builtin_isfinite(ldn)) {
        fail = CHX_ORBIT_NONFINITE;
        break;
      }
      if (++attempts > dop853::MAX_ATTEMPTS) {
        fail = CHX_ORBIT_STEP_FAILED;
        break;
      }
      const double qf = sqrt(sqrt(sqrt(err)));
      double fac = qf / dop853::SAFE;
      if (fac > dop853::FACC1) fac = dop853::FACC1;
      if (err <= 1.0) {
        if (fac < dop853::FACC2) fac = dop853::FACC2;
        double hnew = hh / fac;
        if (rej && hnew > hh) hnew = hh;
        rej = false;
        h = hnew;
        nacc += 1.0;
        emax = fmax(emax, err);
        elast = err;
        r.q = qn;
        r.p = pn;
        r.accept_vectors();
        r.ld = ldn;
        t = last ? tb : t + hh;
      } else {
        h = hh / fac;
        rej = true;
        nrej += 1.0;
      }
    }
    if (fail != CHX_ORBIT_OK) {
      r.st = fail;
      break;
    }
    s = next;
    if (!r.checkpoint(a, tb)) break;
  }
  r.store(a, o);
  r.store_vectors(a, o);
  if (r.lane == 0) {
    a.sc[SC_H * P + o] = h;
    a.sc[SC_REJ * P + o] = rej ? 1.0 : 0.0;
    a.sc[SC_NACC * P + o] = nacc;
    a.sc[SC_NREJ * P + o] = nrej;
    a.sc[SC_ERR_MAX * P + o] = emax;
    a.sc[SC_ERR_LAST * P + o] = elast;
  }
}

}  // namespace chx
