// fput_crow_rk.h -- DOP853 (fixed step and adaptive DOP8(5)) for FPU chains
// on the component rows: one 16-lane row per orbit, lane l holding q_l, p_l
// of the state and of each of the M <= 4 deviation vectors (ghost lanes
// N..15 zero), as in the Yoshida-4 component-row kernel.
//
// The extended system of every orbit (Functionalities section: the solvers
// build on DOP853, with the variational equations and the LD):
//   dq_l/dt = p_l,   dp_l/dt = -F_l(q),
//   d(dq_l)/dt = dp_l,
//   d(dp_l)/dt = -[(kl_l + kr_l) dq_l - kl_l dq_{l-1} - kr_l dq_{l+1}],
//   dM/dt = sum_l |p_l|^(1/2) + |F_l|^(1/2),
// with F_l the net spring force and kl_l, kr_l the stiffnesses of the
// springs left and right of mass l at the stage positions (neighbours
// through row DPP, the walls as zero ghosts).  A step is two passes: the
// state's 12 stages, keeping each stage's two stiffnesses in registers (24
// doubles per lane), then each vector's 12 stages from them.  Every lane
// carries its own components' stage derivatives (12 x 2 doubles per pass);
// the LD integrand and the error estimate are row sums, identical in all
// 16 lanes, so every decision (accept, reject, stop) is row-uniform.
#pragma once
#include "dop853.h"
#include "fput_crow.h"

namespace chx {

template <int N, int M>
struct CRowRK : CRowOrbit<N, M> {
  using B = CRowOrbit<N, M>;
  using B::dp;
  using B::dq;
  using B::ld;
  using B::mass;
  using B::p;
  using B::q;
  static constexpr int MM = B::MM;

  double skl[12], skr[12];  // stiffnesses at the state's stages

  // the state's 12 stages: k = h f at Y = x + sum a_ij k_j; g += the LD
  // integrand of this lane's components at the weighted stages
  __device__ __forceinline__ void state_pass(const StepArgs &a, double h, bool do_ld,
                                             double (&kq)[12][1], double (&kp)[12][1],
                                             double &g) {
    dop853::static_for<0, 12>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      const double Yq = q + dop853::stage_sum<I>(kq, 0);
      const double Yp = p + dop853::stage_sum<I>(kp, 0);
      double F, kl, kr;
      B::spring_terms(a, Yq, mass, F, kl, kr);
      skl[I] = kl;
      skr[I] = kr;
      if constexpr (dop853::B[I] != 0.0) {
        if (do_ld) g = __builtin_fma(dop853::B[I], mass ? sqrt_ld(Yp) + sqrt_ld(F) : 0.0, g);
      }
      kq[I][0] = h * Yp;
      kp[I][0] = -h * F;
    });
  }

  // vector v's 12 stages from the state's stiffnesses
  template <int V>
  __device__ __forceinline__ void vector_pass(double h, double (&kq)[12][1],
                                              double (&kp)[12][1]) {
    using namespace fputrow;
    dop853::static_for<0, 12>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      const double Yq = dq[V] + dop853::stage_sum<I>(kq, 0);
      const double Yp = dp[V] + dop853::stage_sum<I>(kp, 0);
      const double ql = dpp<0x111>(Yq);  // row_shr:1
      const double qr = dpp<0x101>(Yq);  // row_shl:1
      double hq = (skl[I] + skr[I]) * Yq;
      hq = __builtin_fma(-skl[I], ql, hq);
      hq = __builtin_fma(-skr[I], qr, hq);
      kq[I][0] = h * Yp;
      kp[I][0] = -h * hq;
    });
  }

  // one fixed DOP853 step of size h
  __device__ __forceinline__ void rk_step(const StepArgs &a, double h, bool do_ld) {
    {
      double kq[12][1], kp[12][1], g = 0.0;
      state_pass(a, h, do_ld, kq, kp, g);
      q += dop853::final_sum(kq, 0);
      p += dop853::final_sum(kp, 0);
      if (do_ld) ld = __builtin_fma(h, fputrow::row_sum(g), ld);
    }
    __builtin_amdgcn_sched_barrier(0);
    dop853::static_for<0, M>([&](auto vc) {
      constexpr int V = decltype(vc)::value;
      double kq[12][1], kp[12][1];
      vector_pass<V>(h, kq, kp);
      dq[V] += dop853::final_sum(kq, 0);
      dp[V] += dop853::final_sum(kp, 0);
      __builtin_amdgcn_sched_barrier(0);
    });
  }

  // One attempted step of size h: the new state, vectors and LD in qn, pn,
  // dqn, dpn, ldn; returns DOP853's scaled error estimate over the state and
  // the vectors, err = e5 / sqrt(n (e5 + 0.01 e3)), n = 2N (1 + M), from
  // the row sums of the lanes' error terms (the LD is left out of it).
  __device__ __forceinline__ double rk_attempt(const StepArgs &a, double h, bool do_ld,
                                               double &qn, double &pn, double (&dqn)[MM],
                                               double (&dpn)[MM], double &ldn) {
    double e5 = 0.0, e3 = 0.0;
    {
      double kq[12][1], kp[12][1], g = 0.0;
      state_pass(a, h, do_ld, kq, kp, g);
      const double sq = dop853::final_sum(kq, 0), sp = dop853::final_sum(kp, 0);
      qn = q + sq;
      pn = p + sp;
      if (mass) {  // ghost lanes are no components (0 / 0 when atol = 0)
        dop853::err_terms(kq, 0, q, qn, sq, a.rtol, a.atol, e5, e3);
        dop853::err_terms(kp, 0, p, pn, sp, a.rtol, a.atol, e5, e3);
      }
      ldn = do_ld ? __builtin_fma(h, fputrow::row_sum(g), ld) : ld;
    }
    __builtin_amdgcn_sched_barrier(0);
    dop853::static_for<0, M>([&](auto vc) {
      constexpr int V = decltype(vc)::value;
      double kq[12][1], kp[12][1];
      vector_pass<V>(h, kq, kp);
      const double sq = dop853::final_sum(kq, 0), sp = dop853::final_sum(kp, 0);
      dqn[V] = dq[V] + sq;
      dpn[V] = dp[V] + sp;
      if (mass) {
        dop853::err_terms(kq, 0, dq[V], dqn[V], sq, a.rtol, a.atol, e5, e3);
        dop853::err_terms(kp, 0, dp[V], dpn[V], sp, a.rtol, a.atol, e5, e3);
      }
      __builtin_amdgcn_sched_barrier(0);
    });
    e5 = fputrow::row_sum(e5);
    e3 = fputrow::row_sum(e3);
    const double deno = __builtin_fma(0.01, e3, e5);
    if (!(deno > 0.0)) return deno == 0.0 ? 0.0 : deno;  // NaN stays NaN
    return e5 / sqrt((double)(2 * N * (1 + M)) * deno);
  }
};

template <int N, int M>
__global__ void __launch_bounds__(256) fput_crow_rk_kernel(const StepArgs a) {
  const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  // rows beyond the ensemble or already stopped do nothing; all lanes of a
  // row take the same branch
  if (o >= a.n) return;
  if (a.st[o] != CHX_ORBIT_OK) return;
  CRowRK<N, M> r;
  r.load(a, o);
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
}

// The adaptive DOP8(5) solver on component rows: the checkpoint schedule,
// controller and landing rule of the lane-per-orbit adaptive kernel, with
// one step loop per row (its lanes agree on every decision).
template <int N, int M>
__global__ void __launch_bounds__(256) fput_crow_rka_kernel(const StepArgs a) {
  const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  if (o >= a.n) return;
  if (a.st[o] != CHX_ORBIT_OK) return;
  constexpr int MM = CRowRK<N, M>::MM;
  CRowRK<N, M> r;
  r.load(a, o);
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
      double qn, pn, dqn[MM], dpn[MM], ldn;
      const double err = r.rk_attempt(a, hh, do_ld, qn, pn, dqn, dpn, ldn);
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
#pragma unroll
        for (int v = 0; v < M; ++v) {
          r.dq[v] = dqn[v];
          r.dp[v] = dpn[v];
        }
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
