// lane_rk.h -- one lane per orbit with the fixed-step DOP853 integrator.
//
// The paper's solvers are built on DOP853, the explicit Runge-Kutta method
// of order 8 of Dormand and Prince (Functionalities section), with a fixed
// step (lane_rk_kernel) or with its embedded error estimate and step-size
// control (lane_rka_kernel), applied to one extended system per orbit:
//   dq/dt = p,  dp/dt = -grad V(q)                 (Hamilton's equations)
//   d(dq)/dt = dp,  d(dp)/dt = -Hess V(q) dq      (variational equations)
//   dM/dt = sum over the 2N components |dx_i/dt|^p (LD M-function)
// so the deviation vectors follow the exact Jacobian of the discrete step
// and the LD is integrated to the method's order.
//
// A step k_i = dt f(y + sum_{j<i} a_ij k_j), y <- y + sum_i b_i k_i is done
// in two passes to keep the live registers few: first the state (12 stages;
// a record of each stage goes to LDS), then each deviation vector on its
// own, whose stages need only the Hessian at the stage positions.  For a
// Hamiltonian that is not |p|^2/2 + V(q) (the double pendulum) a vector's
// stage derivative is the directional derivative of the vector field, by
// dual numbers: with one or two vectors the state and the vectors go
// through the stages together in one pass on multi-dual numbers (no
// records); with more, the record holds the stage's sines, cosines and
// momenta.  The stage derivatives a pass still needs are held in
// registers; with the method's zero pattern (stages 2 and 3 feed only
// stages 3..5, and the solution does not use stages 2..5) at most nine are
// live at once.  The stage records live in dynamic LDS, field-major
// (component f of thread t at f * blockDim + t).
//
// Load, store and the checkpoints (renormalisation, SALI, Gram-Schmidt,
// energy, escape, early exit) are those of the Yoshida-4 lane kernel.
#pragma once
#include <type_traits>

#include "dop853.h"
#include "lane_kernel.h"
#include "systems_dp.h"

namespace chx {



// LDS doubles per stage record: a general system's record, else the positions
template <class S, bool GEN>
constexpr int rec_width() {
  if constexpr (GEN)
    return S::NREC;
  else
    return S::N;
}

template <class S, int M, bool GP>
struct RKOrbit : LaneOrbit<S, M, GP, -1> {
  using Base = LaneOrbit<S, M, GP, -1>;
  using Base::N;
  using Base::D;
  using Base::x;
  using Base::w;
  using Base::ld;
  // A general Hamiltonian (not |p|^2/2 + V(q)) gives its vector field with
  // a stage record and, from that record, its directional derivative
  // (dual numbers); its stages keep the records in LDS, a separable one's
  // the positions.
  static constexpr bool GEN = has_hamiltonian<S>::value;
  static constexpr int QW = rec_width<S, GEN>();  // LDS doubles per stage and thread
  // With one or two vectors a general system integrates the state and the
  // vectors stage by stage in one pass: one evaluation on multi-dual
  // numbers gives the field and every vector's derivative (the values
  // shared), all stage derivatives stay in registers and no record goes
  // through LDS.  (The records' LDS would hold the kernel to one wavefront
  // per SIMD anyway, which leaves the register file to the pass.)
  static constexpr bool FUSED = GEN && M >= 1 && M <= 2;
  static constexpr int LDS_STAGE = FUSED ? 0 : QW;  // LDS doubles per stage and thread

  // Stage I of the state and the vectors together (FUSED): Y = x +
  // sum_j a_Ij k_j, dY_v = w_v + sum_j a_Ij kv_vj; k_I = h f(Y),
  // kv_vI = h Df(Y) dY_v; the LD integrand at weighted stages into g.
  template <int I>
  __device__ __forceinline__ void fused_stage(const StepArgs &a, double h, bool do_ld,
                                              double (&k)[12][D], double (&kv)[M][12][D],
                                              double &g) {
    double Y[D], dY[M][D], f[D], df[M][D];
#pragma unroll
    for (int c = 0; c < D; ++c) Y[c] = x[c] + dop853::stage_sum<I>(k, c);
#pragma unroll
    for (int v = 0; v < M; ++v)
#pragma unroll
      for (int c = 0; c < D; ++c) dY[v][c] = w[v][c] + dop853::stage_sum<I>(kv[v], c);
    S::template rhs_multi<M>(Y, dY, f, df, a.prm);
    if constexpr (dop853::B[I] != 0.0) {
      if (do_ld) {
        double gi = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) gi += this->ld_term(a, f[c]);
        g = __builtin_fma(dop853::B[I], gi, g);
      }
    }
#pragma unroll
    for (int c = 0; c < D; ++c) k[I][c] = h * f[c];
#pragma unroll
    for (int v = 0; v < M; ++v)
#pragma unroll
      for (int c = 0; c < D; ++c) kv[v][I][c] = h * df[v][c];
    // each stage's derivative parts finish inside the stage: left free, the
    // scheduler runs the value chain ahead through all twelve stages and
    // keeps every stage's dual-number intermediates live for the deferred
    // derivative parts, far beyond the register file
#pragma unroll
    for (int v = 0; v < M; ++v)
#pragma unroll
      for (int c = 0; c < D; ++c) asm volatile("" : "+v"(kv[v][I][c]));
#pragma unroll
    for (int c = 0; c < D; ++c) asm volatile("" : "+v"(k[I][c]));
    __builtin_amdgcn_sched_barrier(0);
  }

  // Stage I of the state: Y = x + sum_j a_Ij k_j; its LDS record; the LD
  // integrand sum |dY/dt|^p at weighted stages into g; k_I = h f(Y).
  template <int I>
  __device__ __forceinline__ void state_stage(const StepArgs &a, double h, bool do_ld,
                                              double *qs, int stride, double (&k)[12][D],
                                              double &g) {
    double Y[D], f[D];
#pragma unroll
    for (int c = 0; c < D; ++c) Y[c] = x[c] + dop853::stage_sum<I>(k, c);
    if constexpr (GEN) {
      double rec[QW];
      S::rhs_rec(Y, f, rec, a.prm);
      if constexpr (M > 0) {
#pragma unroll
        for (int r = 0; r < QW; ++r) qs[(I * QW + r) * stride] = rec[r];
      }
    } else {
      if constexpr (M > 0) {
#pragma unroll
        for (int r = 0; r < QW; ++r) qs[(I * QW + r) * stride] = Y[r];
      }
      double F[N];
      S::force(Y, F, a.prm);
#pragma unroll
      for (int r = 0; r < N; ++r) {
        f[r] = Y[N + r];
        f[N + r] = -F[r];
      }
    }
    if constexpr (dop853::B[I] != 0.0) {
      if (do_ld) {
        double gi = 0.0;
        if constexpr (GEN) {
#pragma unroll
          for (int c = 0; c < D; ++c) gi += this->ld_term(a, f[c]);
        } else {
#pragma unroll
          for (int r = 0; r < N; ++r) gi += this->ld_term(a, f[r]) + this->ld_term(a, f[N + r]);
        }
        g = __builtin_fma(dop853::B[I], gi, g);
      }
    }
#pragma unroll
    for (int c = 0; c < D; ++c) k[I][c] = h * f[c];
  }

  // Stage I of a deviation vector starting at w0: dY = w0 + sum_j a_Ij k_j,
  // k_I = h Df(Y_I) dY with Y_I the state's stage (from LDS).
  template <int I>
  __device__ __forceinline__ void vector_stage(const StepArgs &a, double h, const double *w0,
                                               const double *qs, int stride,
                                               double (&k)[12][D]) {
    double Y[D];
#pragma unroll
    for (int c = 0; c < D; ++c) Y[c] = w0[c] + dop853::stage_sum<I>(k, c);
    if constexpr (GEN) {
      // the records do not depend on the vector: with a plain LDS offset the
      // optimiser loads each stage's record once for all vectors and keeps
      // the twelve live; an offset it cannot see through keeps the loads in
      // each vector pass
      int off = I * QW * stride;
      asm volatile("" : "+v"(off));
      double rec[QW], f[D];
#pragma unroll
      for (int r = 0; r < QW; ++r) rec[r] = qs[off + r * stride];
      S::jvp(rec, Y, f, a.prm);
#pragma unroll
      for (int c = 0; c < D; ++c) k[I][c] = h * f[c];
    } else {
      double Hs[S::NH], q[N];
#pragma unroll
      for (int r = 0; r < N; ++r) q[r] = qs[(I * N + r) * stride];
      S::hess_scaled(q, h, Hs, a.prm);
#pragma unroll
      for (int r = 0; r < N; ++r) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) s = __builtin_fma(Hs[hidx(N, r, j)], Y[j], s);
        k[I][r] = h * Y[N + r];
        k[I][N + r] = -s;
      }
    }
  }

  // one fixed DOP853 step of size h of the state, the M vectors and the LD;
  // qs: this thread's stage records in LDS, component f at qs[f * stride]
  __device__ __forceinline__ void rk_step(const StepArgs &a, double h, bool do_ld, double *qs,
                                          int stride) {
    if constexpr (FUSED) {
      double k[12][D], kv[M][12][D];
      double g = 0.0;
      dop853::static_for<0, 12>([&](auto ic) {
        fused_stage<decltype(ic)::value>(a, h, do_ld, k, kv, g);
      });
#pragma unroll
      for (int c = 0; c < D; ++c) x[c] += dop853::final_sum(k, c);
#pragma unroll
      for (int v = 0; v < M; ++v)
#pragma unroll
        for (int c = 0; c < D; ++c) w[v][c] += dop853::final_sum(kv[v], c);
      if (do_ld) ld = __builtin_fma(h, g, ld);
      return;
    }
    {
      double k[12][D];  // h f(Y_i) of the state
      double g = 0.0;   // sum_i b_i (LD integrand at stage i)
      dop853::static_for<0, 12>([&](auto ic) {
        state_stage<decltype(ic)::value>(a, h, do_ld, qs, stride, k, g);
      });
#pragma unroll
      for (int c = 0; c < D; ++c) x[c] += dop853::final_sum(k, c);
      if (do_ld) ld = __builtin_fma(h, g, ld);
    }
    __builtin_amdgcn_sched_barrier(0);
    // (a compile-time loop: the vectors must stay in registers)
    dop853::static_for<0, M>([&](auto vc) {
      constexpr int v = decltype(vc)::value;
      double k[12][D];  // h f(dY_i) of vector v
      dop853::static_for<0, 12>([&](auto ic) {
        vector_stage<decltype(ic)::value>(a, h, w[v], qs, stride, k);
      });
#pragma unroll
      for (int c = 0; c < D; ++c) w[v][c] += dop853::final_sum(k, c);
      // one vector pass at a time: overlapped by the scheduler, two passes'
      // stage derivatives would be live together
      __builtin_amdgcn_sched_barrier(0);
    });
  }

  // One attempted step of size h for the adaptive solver: the new state in
  // xn, the new LD in ldn, the new vectors in LDS (component c of vector v at
  // wn[(v D + c) * stride]); returns DOP853's scaled error estimate over the
  // state and the vectors (the LD is left out of it):
  //   err = e5 / sqrt(n (e5 + 0.01 e3)) with the sums of err_terms over the
  //   n = 2N (1 + M) components, which equals |h| e5' / sqrt(n (e5' +
  //   0.01 e3')) for the sums e5', e3' of unscaled derivatives.
  __device__ __forceinline__ double rk_attempt(const StepArgs &a, double h, bool do_ld,
                                               double *qs, double *wn, int stride,
                                               double (&xn)[D], double &ldn) {
    double e5 = 0.0, e3 = 0.0;
    if constexpr (FUSED) {
      double k[12][D], kv[M][12][D];
      double g = 0.0;
      dop853::static_for<0, 12>([&](auto ic) {
        fused_stage<decltype(ic)::value>(a, h, do_ld, k, kv, g);
      });
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double sb = dop853::final_sum(k, c);
        xn[c] = x[c] + sb;
        dop853::err_terms(k, c, x[c], xn[c], sb, a.rtol, a.atol, e5, e3);
      }
      ldn = do_ld ? __builtin_fma(h, g, ld) : ld;
#pragma unroll
      for (int v = 0; v < M; ++v)
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const double sb = dop853::final_sum(kv[v], c);
          const double yn = w[v][c] + sb;
          wn[(v * D + c) * stride] = yn;
          dop853::err_terms(kv[v], c, w[v][c], yn, sb, a.rtol, a.atol, e5, e3);
        }
    } else {
      {
        double k[12][D];
        double g = 0.0;
        dop853::static_for<0, 12>([&](auto ic) {
          state_stage<decltype(ic)::value>(a, h, do_ld, qs, stride, k, g);
        });
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const double sb = dop853::final_sum(k, c);
          xn[c] = x[c] + sb;
          dop853::err_terms(k, c, x[c], xn[c], sb, a.rtol, a.atol, e5, e3);
        }
        ldn = do_ld ? __builtin_fma(h, g, ld) : ld;
      }
      __builtin_amdgcn_sched_barrier(0);
      dop853::static_for<0, M>([&](auto vc) {
        constexpr int v = decltype(vc)::value;
        double k[12][D];
        dop853::static_for<0, 12>([&](auto ic) {
          vector_stage<decltype(ic)::value>(a, h, w[v], qs, stride, k);
        });
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const double sb = dop853::final_sum(k, c);
          const double yn = w[v][c] + sb;
          wn[(v * D + c) * stride] = yn;
          dop853::err_terms(k, c, w[v][c], yn, sb, a.rtol, a.atol, e5, e3);
        }
        __builtin_amdgcn_sched_barrier(0);
      });
    }
    const double deno = __builtin_fma(0.01, e3, e5);
    if (!(deno > 0.0)) return deno == 0.0 ? 0.0 : deno;  // NaN stays NaN
    return e5 / sqrt((double)(D * (1 + M)) * deno);
  }
};

// Dynamic LDS of the DOP853 lane kernels: the stage records, 12 QW doubles
// per thread.
extern __shared__ double lane_rk_lds[];

template <class S, int M, bool GP>
__global__ void __launch_bounds__(256) lane_rk_kernel(const StepArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  if (a.st[i] != CHX_ORBIT_OK) return;
  RKOrbit<S, M, GP> o;
  o.load(a, i);
  const bool do_ld = (a.ind & CHX_IND_LD) != 0;
  const double h = a.dt;
  int64_t s = a.s_begin;
  const int64_t K = a.K;
  while (s < a.s_end) {
    int64_t next = (s / K + 1) * K;
    if (next > a.n_total) next = a.n_total;
    for (int64_t j = s; j < next; ++j) o.rk_step(a, h, do_ld, lane_rk_lds + threadIdx.x, blockDim.x);
    s = next;
    if (!o.checkpoint(a, (double)s * a.dt)) break;
  }
  // the store addresses are formed here, not kept from the loads
  int64_t ob = i;
  asm volatile("" : "+v"(ob));
  o.store(a, ob);
}

// The adaptive DOP8(5) solver: the checkpoint schedule of the fixed-step
// kernels (t = s dt for s a multiple of K or the last step); between two
// checkpoints each lane takes its own steps, sized by the error estimate of
// rk_attempt and the controller of Hairer-Norsett-Wanner's DOP853 (accept
// iff err <= 1; q = err^(1/8) by three square roots; accepted:
// h /= max(1/6, min(1/0.333, q / 0.9)), not growing right after a
// rejection; rejected: h /= min(1/0.333, q / 0.9)).  A step that would end
// within 1.01 h of the checkpoint ends on it exactly.  Each lane runs
// through its own checkpoints: one loop per lane in which every iteration
// is an attempted step, preceded by the lane's checkpoint once it has
// reached one, so the lanes of a wavefront meet only at the end of the
// launch (waiting at every checkpoint for the lane with the most steps in
// that interval would cost about a fifth of the time on the section grids).
// Every lane ends: every iteration attempts a step, which either moves the
// lane on or counts towards the limit of attempts.
// Dynamic LDS per thread: the 12 LDS_STAGE stage records, then the M D
// components of the attempted vectors.
template <class S, int M, bool GP>
__global__ void __launch_bounds__(256) lane_rka_kernel(const StepArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  if (a.st[i] != CHX_ORBIT_OK) return;
  constexpr int N = S::N, D = 2 * N;
  RKOrbit<S, M, GP> o;
  o.load(a, i);
  const int64_t P = a.pitch;
  double h = a.sc[SC_H * P + i];
  if (!(h > 0.0)) h = a.dt;  // the first step
  bool rej = a.sc[SC_REJ * P + i] != 0.0;
  double nacc = a.sc[SC_NACC * P + i], nrej = a.sc[SC_NREJ * P + i];
  double emax = a.sc[SC_ERR_MAX * P + i], elast = a.sc[SC_ERR_LAST * P + i];
  const int stride = blockDim.x;
  double *qs = lane_rk_lds + threadIdx.x;
  double *wn = lane_rk_lds + (size_t)12 * RKOrbit<S, M, GP>::LDS_STAGE * stride + threadIdx.x;
  const bool do_ld = (a.ind & CHX_IND_LD) != 0;
  const int64_t K = a.K;
  int64_t s = a.s_begin;
  int64_t next = (s / K + 1) * K;
  if (next > a.n_total) next = a.n_total;
  double t = (double)s * a.dt;
  double tb = (double)next * a.dt;
  int attempts = 0;
  while (s < a.s_end) {
    if (t >= tb) {
      // this lane's checkpoint, ahead of its next attempt in the same
      // iteration (as an iteration of its own it would cost the wavefront a
      // whole attempt while the other lanes step)
      s = next;
      if (!o.checkpoint(a, tb)) break;
      if (s >= a.s_end) break;
      next = (s / K + 1) * K;
      if (next > a.n_total) next = a.n_total;
      t = tb;
      tb = (double)next * a.dt;
      attempts = 0;
    }
    double hh = h;
    bool last = false;
    if (t + 1.01 * hh >= tb) {
      hh = tb - t;
      last = true;
    }
    double xn[D], ldn;
    const double err = o.rk_attempt(a, hh, do_ld, qs, wn, stride, xn, ldn);
    bool finite = __builtin_isfinite(err) && __builtin_isfinite(ldn);
#pragma unroll
    for (int c = 0; c < D; ++c) finite = finite && __builtin_isfinite(xn[c]);
    if (!finite) {
      o.st = CHX_ORBIT_NONFINITE;
      break;
    }
    if (++attempts > dop853::MAX_ATTEMPTS) {
      o.st = CHX_ORBIT_STEP_FAILED;
      break;
    }
    const double q = sqrt(sqrt(sqrt(err)));
    double fac = q / dop853::SAFE;
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
#pragma unroll
      for (int c = 0; c < D; ++c) o.x[c] = xn[c];
#pragma unroll
      for (int v = 0; v < M; ++v)
#pragma unroll
        for (int c = 0; c < D; ++c) o.w[v][c] = wn[(v * D + c) * stride];
      o.ld = ldn;
      t = last ? tb : t + hh;
    } else {
      h = hh / fac;
      rej = true;
      nrej += 1.0;
    }
  }
  int64_t ob = i;
  asm volatile("" : "+v"(ob));
  o.store(a, ob);
  a.sc[SC_H * P + ob] = h;
  a.sc[SC_REJ * P + ob] = rej ? 1.0 : 0.0;
  a.sc[SC_NACC * P + ob] = nacc;
  a.sc[SC_NREJ * P + ob] = nrej;
  a.sc[SC_ERR_MAX * P + ob] = emax;
  a.sc[SC_ERR_LAST * P + ob] = elast;
}

// Launch the fixed-step (ADAPT = false) or adaptive (true) kernel with M
// vectors; the two families are instantiated in separate source files.
template <class S, int M, bool ADAPT>
struct LaneRKDispatch {
  static hipError_t go(int m, const StepArgs &a, int block, hipStream_t s) {
    constexpr bool adaptive = ADAPT;
    if (m == M) {
      const bool gp = (a.ind & CHX_IND_LD) && a.ld_p != 0.5;
      // LDS per thread: stage records, and for the adaptive solver the
      // attempted vectors; at most 64 KB per block (smaller blocks where
      // needed)
      constexpr int QW = RKOrbit<S, M, false>::LDS_STAGE;
      const size_t per = M > 0 ? sizeof(double) * (12 * QW + (adaptive ? M * 2 * S::N : 0)) : 0;
      while (block > 64 && per * (size_t)block > 65536) block /= 2;
      const int64_t grid = (a.n + block - 1) / block;
      const size_t lds = per * (size_t)block;
      if constexpr (ADAPT) {
        if (gp)
          hipLaunchKernelGGL((lane_rka_kernel<S, M, true>), dim3((unsigned)grid), dim3(block),
                             lds, s, a);
        else
          hipLaunchKernelGGL((lane_rka_kernel<S, M, false>), dim3((unsigned)grid), dim3(block),
                             lds, s, a);
      } else {
        if (gp)
          hipLaunchKernelGGL((lane_rk_kernel<S, M, true>), dim3((unsigned)grid), dim3(block),
                             lds, s, a);
        else
          hipLaunchKernelGGL((lane_rk_kernel<S, M, false>), dim3((unsigned)grid), dim3(block),
                             lds, s, a);
      }
      return hipGetLastError();
    }
    return LaneRKDispatch<S, M - 1, ADAPT>::go(m, a, block, s);
  }
};
template <class S, bool ADAPT>
struct LaneRKDispatch<S, -1, ADAPT> {
  static hipError_t go(int, const StepArgs &, int, hipStream_t) { return hipErrorInvalidValue; }
};

}  // namespace chx
