// api.hip -- the C ABI of libchx (include/chx.h): argument validation, the
// resumable ensemble object, kernel selection and host<->device staging.
#include <math.h>
#include <string.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <type_traits>
#include <vector>

#include "chx_internal.h"
#include "ensemble.h"

using namespace chx;

namespace chx {
// DOP853 (fixed or adaptive) for FPU chains on the component rows
// (fput_crow_rk.hip, fput_crow_rka.hip).
hipError_t launch_fput_crow_rk(int ndof, int M, bool adaptive, const StepArgs &a,
                               hipStream_t s);
// LDS per block of four orbits of the DOP853 FPU kernels with more than four
// vectors (fput_crow_rkl.hip)
size_t fput_rkl_lds_bytes(int M, bool adaptive);

namespace host {

thread_local std::string g_err;

chx_status fail(chx_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

chx_status dev_fail(hipError_t e, const char *what) {
  if (e == hipErrorOutOfMemory)
    return fail(CHX_ERR_OUT_OF_MEMORY, "%s: out of device memory", what);
  return fail(CHX_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(expr, what)                         \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return dev_fail(e_, what); \
  } while (0)

int required_params(int kind, int ndof) {
  switch (kind) {
  case CHX_SYS_HENON_HEILES: return 0;
  case CHX_SYS_FPUT: return 3;
  case CHX_SYS_QUARTIC: return 1;
  case CHX_SYS_HARMONIC: return ndof;
  case CHX_SYS_DOUBLE_PENDULUM: return 2;
  case CHX_SYS_CUSTOM:
  case CHX_SYS_CUSTOM_GENERAL: return 0;
  }
  return -1;
}

chx_status check_system(const chx_system *sys) {
  if (!sys) return fail(CHX_ERR_INVALID_ARG, "system is NULL");
  const int k = sys->kind, N = sys->ndof;
  switch (k) {
  case CHX_SYS_HENON_HEILES:
    if (N != 2) return fail(CHX_ERR_INVALID_ARG, "Henon-Heiles needs ndof == 2 (got %d)", N);
    break;
  case CHX_SYS_FPUT:
    if (N < 2 || N > 16) return fail(CHX_ERR_INVALID_ARG, "FPUT needs 2 <= ndof <= 16 (got %d)", N);
    break;
  case CHX_SYS_QUARTIC:
  case CHX_SYS_HARMONIC:
    if (N < 1 || N > 3) return fail(CHX_ERR_INVALID_ARG, "ndof must be 1..3 (got %d)", N);
    break;
  case CHX_SYS_DOUBLE_PENDULUM:
    if (N != 2) return fail(CHX_ERR_INVALID_ARG, "the double pendulum needs ndof == 2 (got %d)", N);
    break;
  case CHX_SYS_CUSTOM:
  case CHX_SYS_CUSTOM_GENERAL:
    if (N < 1 || N > CHX_CUSTOM_MAX_NDOF)
      return fail(CHX_ERR_INVALID_ARG, "a custom system needs ndof 1..%d (got %d)", CHX_CUSTOM_MAX_NDOF, N);
    if (!sys->source || !sys->source[0]) return fail(CHX_ERR_INVALID_ARG, "a custom system needs its source");
    if (sys->nparams < 0 || sys->nparams > 16)
      return fail(CHX_ERR_INVALID_ARG, "a custom system takes 0..16 params (got %d)", sys->nparams);
    if (sys->nparams > 0 && !sys->params) return fail(CHX_ERR_INVALID_ARG, "system params is NULL");
    for (int i = 0; i < sys->nparams; ++i)
      if (!isfinite(sys->params[i])) return fail(CHX_ERR_INVALID_ARG, "system param %d is not finite", i);
    return CHX_OK;
  default: return fail(CHX_ERR_INVALID_ARG, "unknown system kind %d", k);
  }
  const int np = required_params(k, N);
  if (sys->nparams < np) return fail(CHX_ERR_INVALID_ARG, "system needs %d params (got %d)", np, sys->nparams);
  if (np > 0 && !sys->params) return fail(CHX_ERR_INVALID_ARG, "system params is NULL");
  for (int i = 0; i < np; ++i)
    if (!isfinite(sys->params[i])) return fail(CHX_ERR_INVALID_ARG, "system param %d is not finite", i);
  if (k == CHX_SYS_DOUBLE_PENDULUM && !(sys->params[0] > 0.0 && sys->params[1] > 0.0))
    return fail(CHX_ERR_INVALID_ARG, "the double pendulum needs alpha > 0 and sigma > 0");
  return CHX_OK;
}

chx_status make_plan(const chx_system *sys, const chx_options *opt, Plan *p) {
  if (!opt) return fail(CHX_ERR_INVALID_ARG, "options is NULL");
  chx_options o = *opt;
  const int N = sys->ndof;
  if (!(o.dt > 0.0) || !isfinite(o.dt)) return fail(CHX_ERR_INVALID_ARG, "dt must be finite and > 0");
  if (!(o.T > 0.0) || !isfinite(o.T)) return fail(CHX_ERR_INVALID_ARG, "T must be finite and > 0");
  const double r = o.T / o.dt;
  const double nr = nearbyint(r);
  if (nr < 1.0 || fabs(r - nr) > 1e-9 * nr || nr > 9.0e15)
    return fail(CHX_ERR_INVALID_ARG, "T/dt must be a positive integer to 1e-9 relative (T/dt = %.17g)", r);
  if (o.indicators & ~31u) return fail(CHX_ERR_INVALID_ARG, "unknown indicator bits 0x%x", o.indicators);
  if (o.renorm_every < 0) return fail(CHX_ERR_INVALID_ARG, "renorm_every must be >= 0");
  if (o.renorm_every == 0) o.renorm_every = 10;
  if (o.indicators & CHX_IND_LYAP) {
    if (o.n_lyap == 0) o.n_lyap = 2 * N;
    if (o.n_lyap < 1 || o.n_lyap > 2 * N)
      return fail(CHX_ERR_INVALID_ARG, "n_lyap must be 1..2N = %d (got %d)", 2 * N, o.n_lyap);
  } else {
    o.n_lyap = 0;
  }
  int kmax = 0;
  if (o.indicators & CHX_IND_GALI) {
    if (o.gali_kmax == 0) o.gali_kmax = 2;
    if (o.gali_kmax < 2 || o.gali_kmax > 2 * N)
      return fail(CHX_ERR_INVALID_ARG, "gali_kmax must be 2..2N = %d (got %d)", 2 * N, o.gali_kmax);
    kmax = o.gali_kmax;
  }
  if (o.ld_p == 0.0) o.ld_p = 0.5;
  if (!(o.ld_p > 0.0 && o.ld_p <= 1.0)) return fail(CHX_ERR_INVALID_ARG, "ld_p must be in (0, 1]");
  if (o.sali_threshold == 0.0) o.sali_threshold = 1e-8;
  if (!(o.sali_threshold > 0.0) || !isfinite(o.sali_threshold))
    return fail(CHX_ERR_INVALID_ARG, "sali_threshold must be finite and > 0");
  if (o.early_exit && !(o.indicators & CHX_IND_SALI))
    return fail(CHX_ERR_INVALID_ARG, "early_exit needs the SALI indicator");
  if (!(o.escape_r2 >= 0.0)) return fail(CHX_ERR_INVALID_ARG, "escape_r2 must be >= 0");
  if (o.steps_per_launch < 0) return fail(CHX_ERR_INVALID_ARG, "steps_per_launch must be >= 0");
  if (!(o.block_size == 0 || o.block_size == 64 || o.block_size == 128 || o.block_size == 256))
    return fail(CHX_ERR_INVALID_ARG, "block_size must be 0, 64, 128 or 256");
  if (o.flags & ~1u) return fail(CHX_ERR_INVALID_ARG, "unknown flags 0x%x", o.flags);
  if (o.integrator != CHX_INT_YOSHIDA4 && o.integrator != CHX_INT_DOP853 &&
      o.integrator != CHX_INT_DOP853_ADAPTIVE)
    return fail(CHX_ERR_INVALID_ARG, "unknown integrator %d", o.integrator);
  if (sys->kind == CHX_SYS_FPUT && (o.indicators & CHX_IND_LD) && o.ld_p != 0.5)
    return fail(CHX_ERR_UNSUPPORTED, "the FPU kernels compute the LD with p = 1/2 only");
  if (o.integrator == CHX_INT_YOSHIDA4 && sys->kind == CHX_SYS_DOUBLE_PENDULUM)
    return fail(CHX_ERR_UNSUPPORTED, "the double pendulum is not separable: integrate it with DOP853 (fixed or adaptive)");
  if (o.integrator == CHX_INT_YOSHIDA4 && sys->kind == CHX_SYS_CUSTOM_GENERAL)
    return fail(CHX_ERR_UNSUPPORTED, "a general custom system is not separable: integrate it with DOP853 (fixed or adaptive)");
  if (o.integrator == CHX_INT_DOP853_ADAPTIVE) {
    if (o.rtol == 0.0 && o.atol == 0.0) o.rtol = o.atol = 1e-10;
    if (!(o.rtol >= 0.0) || !(o.atol >= 0.0) || !isfinite(o.rtol) || !isfinite(o.atol))
      return fail(CHX_ERR_INVALID_ARG, "rtol and atol must be finite and >= 0");
  }
  int m_s = 0;
  if (o.indicators & CHX_IND_SALI) m_s = 2;
  if (kmax > m_s) m_s = kmax;
  p->o = o;
  p->N = N;
  p->D = 2 * N;
  p->m_s = m_s;
  p->n_l = o.n_lyap;
  p->M = m_s + o.n_lyap;
  p->K = o.renorm_every;
  p->kmax = kmax;
  p->n_total = (int64_t)nr;
  const int sk = sys->kind;
  const bool fput_rk = o.integrator != CHX_INT_YOSHIDA4 && sk == CHX_SYS_FPUT;
  if (fput_rk && p->M > 4) {
    // DOP853 for FPU chains with more than four vectors keeps them in LDS:
    // a block of four orbits needs 1 KB per vector (2 KB adaptive)
    const size_t need = fput_rkl_lds_bytes(p->M, o.integrator == CHX_INT_DOP853_ADAPTIVE);
    int dev = 0, lim = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        lim <= 0)
      lim = 65536;
    if (need > (size_t)lim)
      return fail(CHX_ERR_UNSUPPORTED, "DOP853 for FPU chains with %d deviation vectors needs %zu B of LDS per block of four orbits; the device allows %d", p->M, need, lim);
  }
  const bool ok = (sk == CHX_SYS_FPUT)
                      ? (fput_rk ? p->M <= 4 * N
                                 : fput_row_supported(N, p->M, p->n_l, (o.indicators & CHX_IND_SALI) != 0))
                      : lane_supported(sk, N, p->M);
  if (!ok)
    return fail(CHX_ERR_UNSUPPORTED, "system kind %d with ndof %d and %d deviation vectors is not supported", sk, N, p->M);
  if ((sk == CHX_SYS_CUSTOM || sk == CHX_SYS_CUSTOM_GENERAL) && o.integrator != CHX_INT_YOSHIDA4) {
    const size_t lds = custom_rk_lds_per_lane(sk == CHX_SYS_CUSTOM_GENERAL,
                                              o.integrator == CHX_INT_DOP853_ADAPTIVE, N, p->M);
    if (lds * 64 > 65536)
      return fail(CHX_ERR_UNSUPPORTED, "a custom system with ndof %d and %d deviation vectors needs %zu B of LDS per orbit for the DOP853 stages; at most 1024 B fit", N, p->M, lds);
  }
  return CHX_OK;
}

template <class T>
hipError_t dalloc(T **p, size_t count, hipStream_t s) {
  *p = nullptr;
  if (count == 0) return hipSuccess;
  return hipMallocAsync((void **)p, sizeof(T) * count, s);
}

void release(chx_ensemble *e) {
  if (!e) return;
  if (e->in_arena) {  // every buffer belongs to the caller's workspace
    delete e;
    return;
  }
  hipStream_t s = e->stream;
  if (e->x0) (void)hipFreeAsync(e->x0, s);
  if (e->mask) (void)hipFreeAsync(e->mask, s);
  if (e->idx) (void)hipFreeAsync(e->idx, s);
  if (e->state) (void)hipFreeAsync(e->state, s);
  if (e->istate) (void)hipFreeAsync(e->istate, s);
  (void)hipStreamSynchronize(s);
  delete e;
}

chx_status create(const chx_system *sys, const double *x0, const uint8_t *mask, int64_t n,
                  const chx_options *opt, chx_ensemble **out, Arena *arena) {
  if (!out) return fail(CHX_ERR_INVALID_ARG, "output handle pointer is NULL");
  *out = nullptr;
  chx_status st = check_system(sys);
  if (st) return st;
  Plan pl;
  st = make_plan(sys, opt, &pl);
  if (st) return st;
  if (n < 0) return fail(CHX_ERR_INVALID_ARG, "n must be >= 0");
  if (n > 0 && !x0) return fail(CHX_ERR_INVALID_ARG, "x0 is NULL");
  const bool device = pl.o.flags & CHX_PTR_DEVICE;
  const hipStream_t s = device ? (hipStream_t)pl.o.stream : nullptr;
  if (!device && pl.o.stream) return fail(CHX_ERR_INVALID_ARG, "stream given without CHX_PTR_DEVICE");
  if (arena && !device) return fail(CHX_ERR_INVALID_ARG, "a workspace needs device pointers");

  void *custom = nullptr;
  const bool is_custom = sys->kind == CHX_SYS_CUSTOM || sys->kind == CHX_SYS_CUSTOM_GENERAL;
  if (is_custom) {
    // compile before any device work, so that source errors come first
    st = custom_prepare(sys->source, sys->ndof, sys->kind == CHX_SYS_CUSTOM_GENERAL, pl, &custom);
    if (st) return st;
  }
  chx_ensemble *e = new chx_ensemble();
  e->kind = sys->kind;
  memset(e->prm, 0, sizeof e->prm);
  const int np = is_custom ? sys->nparams : required_params(sys->kind, sys->ndof);
  for (int i = 0; i < np; ++i) e->prm[i] = sys->params[i];
  if (is_custom) {
    e->custom_src = sys->source;
    e->custom = custom;
  }
  e->pl = pl;
  e->pl.o.w0 = nullptr;  // copied below, never retained
  e->n_all = n;
  e->stream = s;
  e->device = device;
  e->block = pl.o.block_size ? pl.o.block_size : 256;
  e->in_arena = arena != nullptr;
  const int D = pl.D, M = pl.M;
  const hipMemcpyKind kin = device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  double *w0 = nullptr;
  int64_t *scratch = nullptr, *count = nullptr;
  hipError_t he = hipSuccess;
  // buffers from the caller's workspace, else allocated on the stream
  auto get = [&](auto **p, size_t cnt) -> hipError_t {
    using T = std::remove_reference_t<decltype(**p)>;
    if (!arena) return dalloc(p, cnt, s);
    *p = arena->template take<T>(cnt);
    return (cnt == 0 || *p) ? hipSuccess : hipErrorOutOfMemory;
  };
  auto bail = [&](hipError_t err, const char *what) {
    if (!arena) {
      if (w0) (void)hipFreeAsync(w0, s);
      if (scratch) (void)hipFreeAsync(scratch, s);
      if (count) (void)hipFreeAsync(count, s);
    }
    release(e);
    return dev_fail(err, what);
  };
  if (n > 0) {
    if (arena) {
      // device inputs are read in place for the duration of the call
      e->x0 = const_cast<double *>(x0);
      e->mask = const_cast<uint8_t *>(mask);
      if (opt->w0 && pl.m_s > 0) w0 = const_cast<double *>(opt->w0);
    } else {
      if ((he = dalloc(&e->x0, (size_t)n * D, s))) return bail(he, "allocate x0");
      if ((he = hipMemcpyAsync(e->x0, x0, sizeof(double) * n * D, kin, s))) return bail(he, "copy x0");
      if (mask) {
        if ((he = dalloc(&e->mask, (size_t)n, s))) return bail(he, "allocate mask");
        if ((he = hipMemcpyAsync(e->mask, mask, n, kin, s))) return bail(he, "copy mask");
      }
      if (opt->w0 && pl.m_s > 0) {
        if ((he = dalloc(&w0, (size_t)n * pl.m_s * D, s))) return bail(he, "allocate w0");
        if ((he = hipMemcpyAsync(w0, opt->w0, sizeof(double) * n * pl.m_s * D, kin, s)))
          return bail(he, "copy w0");
      }
    }
    if ((he = get(&e->idx, (size_t)n))) return bail(he, "allocate index");
    if ((he = get(&scratch, (size_t)compact_scratch_len(n)))) return bail(he, "allocate scratch");
    if ((he = get(&count, 1))) return bail(he, "allocate count");
    if ((he = launch_compact(e->mask, n, e->idx, count, scratch, s))) return bail(he, "compact mask");
    int64_t hc = 0;
    if ((he = hipMemcpyAsync(&hc, count, sizeof hc, hipMemcpyDeviceToHost, s))) return bail(he, "read count");
    if ((he = hipStreamSynchronize(s))) return bail(he, "synchronise");
    e->n_active = hc;
  }
  const int64_t na = e->n_active;
  e->pitch = ((na + 63) / 64) * 64;
  if (e->pitch == 0) e->pitch = 64;
  const int64_t P = e->pitch;
  const size_t nd = (size_t)P * (D + (size_t)M * D + M + NSC);
  const size_t ni = (size_t)P * (M + 1);
  if ((he = get(&e->state, nd))) return bail(he, "allocate state");
  if ((he = get(&e->istate, ni))) return bail(he, "allocate state");
  StepArgs &a = e->args;
  a.x = e->state;
  a.w = a.x + (size_t)D * P;
  a.gm = a.w + (size_t)M * D * P;
  a.sc = a.gm + (size_t)M * P;
  a.ge = e->istate;
  a.st = a.ge + (size_t)M * P;
  a.n = na;
  a.pitch = P;
  a.n_total = pl.n_total;
  a.K = pl.K;
  a.m_s = pl.m_s;
  a.n_l = pl.n_l;
  a.ind = pl.o.indicators;
  a.early_exit = pl.o.early_exit ? 1 : 0;
  a.dt = pl.o.dt;
  a.thr2 = pl.o.sali_threshold * pl.o.sali_threshold;
  a.escape_r2 = pl.o.escape_r2;
  a.ld_p = pl.o.ld_p;
  a.rtol = pl.o.rtol;
  a.atol = pl.o.atol;
  memcpy(a.prm, e->prm, sizeof a.prm);
  if (na > 0) {
    InitArgs ia{};
    ia.x0 = e->x0;
    ia.idx = e->idx;
    ia.w0 = w0;
    ia.seed = pl.o.seed;
    ia.sys = sys->kind;
    ia.ndof = pl.N;
    ia.m_s = pl.m_s;
    ia.n_l = pl.n_l;
    ia.ind = pl.o.indicators;
    ia.ld_p = pl.o.ld_p;
    memcpy(ia.prm, e->prm, sizeof ia.prm);
    if ((he = launch_init(a, ia, s))) return bail(he, "initialise ensemble");
    if (e->custom && (he = custom_init(e->custom, a, s))) return bail(he, "initialise custom system");
  }
  // default launch granularity: about 5e10 orbit-steps per launch
  int64_t spl = pl.o.steps_per_launch;
  if (spl == 0) spl = (na > 0) ? (int64_t)(5.0e10 / (double)na) : pl.n_total;
  spl = (spl / pl.K) * pl.K;
  if (spl < pl.K) spl = pl.K;
  e->steps_per_launch = spl;
  if (!arena) {
    if (w0) (void)hipFreeAsync(w0, s);
    if (scratch) (void)hipFreeAsync(scratch, s);
    if (count) (void)hipFreeAsync(count, s);
  }
  if (!device) {
    if ((he = hipStreamSynchronize(s))) {
      release(e);
      return dev_fail(he, "synchronise");
    }
  }
  *out = e;
  return CHX_OK;
}

chx_status advance(chx_ensemble *e, int64_t s_end) {
  if (!e) return fail(CHX_ERR_INVALID_ARG, "ensemble is NULL");
  const Plan &pl = e->pl;
  if (s_end <= e->s_done || s_end > pl.n_total)
    return fail(CHX_ERR_INVALID_ARG, "s_end must be in (%lld, %lld] (got %lld)",
                (long long)e->s_done, (long long)pl.n_total, (long long)s_end);
  if (s_end % pl.K != 0 && s_end != pl.n_total)
    return fail(CHX_ERR_INVALID_ARG, "s_end must be a multiple of K = %d or the last step", pl.K);
  StepArgs a = e->args;
  while (e->s_done < s_end) {
    int64_t nxt = e->s_done + e->steps_per_launch;
    if (nxt > s_end) nxt = s_end;
    a.s_begin = e->s_done;
    a.s_end = nxt;
    if (a.n > 0) {
      hipError_t he = e->custom
                          ? custom_launch(e->custom, e->kind == CHX_SYS_CUSTOM_GENERAL, pl, a,
                                          e->block, e->stream)
                      : (e->kind == CHX_SYS_FPUT)
                          ? (pl.o.integrator != CHX_INT_YOSHIDA4
                                 ? launch_fput_crow_rk(pl.N, pl.M,
                                                       pl.o.integrator == CHX_INT_DOP853_ADAPTIVE,
                                                       a, e->stream)
                                 : launch_fput_row(pl.N, pl.M, a, e->stream))
                      : (pl.o.integrator != CHX_INT_YOSHIDA4)
                          ? launch_lane_rk(e->kind, pl.N, pl.M,
                                           pl.o.integrator == CHX_INT_DOP853_ADAPTIVE, a,
                                           e->block, e->stream)
                          : launch_lane(e->kind, pl.N, pl.M, a, e->block, e->stream);
      if (he != hipSuccess) return dev_fail(he, "integration kernel");
    }
    e->s_done = nxt;
  }
  if (!e->device) HIPCHK(hipStreamSynchronize(e->stream), "synchronise");
  return CHX_OK;
}

chx_status results(chx_ensemble *e, chx_result *res, double *gali_scratch) {
  if (!e) return fail(CHX_ERR_INVALID_ARG, "ensemble is NULL");
  if (!res) return fail(CHX_ERR_INVALID_ARG, "result is NULL");
  if (e->s_done == 0) return fail(CHX_ERR_INVALID_ARG, "no steps integrated yet");
  const Plan &pl = e->pl;
  const int64_t n = e->n_all;
  if (n == 0) return CHX_OK;
  const hipStream_t s = e->stream;
  const int D = pl.D;
  const int km1 = pl.kmax >= 2 ? pl.kmax - 1 : 0;
  OutArgs oa{};
  oa.idx = e->idx;
  oa.gali_kmax = pl.kmax;
  oa.sali = (pl.o.indicators & CHX_IND_SALI) ? 1 : 0;
  oa.thr = pl.o.sali_threshold;
  if (res->label && !oa.sali) return fail(CHX_ERR_INVALID_ARG, "label needs the SALI indicator");
  // which outputs make sense for the requested indicators
  chx_result r = *res;
  if (!(pl.o.indicators & CHX_IND_SALI)) r.sali_final = r.sali_min = r.t_chaos = nullptr;
  if (!(pl.o.indicators & CHX_IND_GALI)) r.gali = nullptr;
  if (!(pl.o.indicators & CHX_IND_LYAP)) r.lyap = nullptr;
  if (!(pl.o.indicators & CHX_IND_LD)) r.ld = nullptr;
  if (!(pl.o.indicators & CHX_IND_ENERGY)) r.energy_err = nullptr;
  if (pl.m_s == 0) r.ln_growth = nullptr;
  struct Out {
    void *host;
    void **dev;
    size_t bytes;
  };
  std::vector<Out> outs;
  chx_result d = r;
  if (!e->device) {
    outs = {{r.x_final, (void **)&d.x_final, sizeof(double) * n * D},
            {r.t_end, (void **)&d.t_end, sizeof(double) * n},
            {r.status, (void **)&d.status, sizeof(int32_t) * n},
            {r.label, (void **)&d.label, sizeof(int8_t) * n},
            {r.sali_final, (void **)&d.sali_final, sizeof(double) * n},
            {r.sali_min, (void **)&d.sali_min, sizeof(double) * n},
            {r.t_chaos, (void **)&d.t_chaos, sizeof(double) * n},
            {r.gali, (void **)&d.gali, sizeof(double) * n * km1},
            {r.lyap, (void **)&d.lyap, sizeof(double) * n * pl.n_l},
            {r.ld, (void **)&d.ld, sizeof(double) * n},
            {r.energy_err, (void **)&d.energy_err, sizeof(double) * n},
            {r.ln_growth, (void **)&d.ln_growth, sizeof(double) * n * pl.m_s},
            {r.steps, (void **)&d.steps, sizeof(int64_t) * n * 2},
            {r.step_err, (void **)&d.step_err, sizeof(double) * n * 2}};
    for (auto &o : outs) {
      *o.dev = nullptr;
      if (o.host && o.bytes) {
        hipError_t he = hipMallocAsync(o.dev, o.bytes, s);
        if (he != hipSuccess) {
          for (auto &q : outs)
            if (*q.dev) (void)hipFreeAsync(*q.dev, s);
          (void)hipStreamSynchronize(s);
          return dev_fail(he, "allocate outputs");
        }
      }
    }
  }
  oa.r = d;
  hipError_t he = launch_masked_fill(e->x0, e->mask, n, pl.N, oa, pl.m_s, pl.n_l, s);
  if (he == hipSuccess) he = launch_finalize(e->args, oa, pl.N, gali_scratch, s);
  if (!e->device) {
    for (auto &o : outs)
      if (*o.dev && he == hipSuccess) he = hipMemcpyAsync(o.host, *o.dev, o.bytes, hipMemcpyDeviceToHost, s);
    for (auto &o : outs)
      if (*o.dev) (void)hipFreeAsync(*o.dev, s);
    hipError_t h2 = hipStreamSynchronize(s);
    if (he == hipSuccess) he = h2;
  }
  if (he != hipSuccess) return dev_fail(he, "results");
  return CHX_OK;
}

// New ensemble holding the active orbits of e with keep[orbit] != 0 (keep
// on the device, indexed by caller orbit), in increasing orbit order, with
// their state, accumulators and step count; e is left unchanged.  The new
// ensemble's orbits are numbered 0..n2-1; *orbit_out (device, may be
// null) receives their caller indices in e.
chx_status subset(chx_ensemble *e, const uint8_t *keep, chx_ensemble **out, int64_t **orbit_out) {
  if (!out) return fail(CHX_ERR_INVALID_ARG, "output handle pointer is NULL");
  *out = nullptr;
  if (orbit_out) *orbit_out = nullptr;
  if (!e) return fail(CHX_ERR_INVALID_ARG, "ensemble is NULL");
  if (e->n_all > 0 && !keep) return fail(CHX_ERR_INVALID_ARG, "keep is NULL");
  const hipStream_t s = e->stream;
  const Plan &pl = e->pl;
  const int D = pl.D, M = pl.M;
  const int64_t na = e->n_active;
  uint8_t *flag = nullptr;
  int64_t *kpos = nullptr, *count = nullptr, *scratch = nullptr, *orbit = nullptr;
  chx_ensemble *e2 = new chx_ensemble();
  hipError_t he = hipSuccess;
  auto cleanup = [&]() {
    if (flag) (void)hipFreeAsync(flag, s);
    if (kpos) (void)hipFreeAsync(kpos, s);
    if (count) (void)hipFreeAsync(count, s);
    if (scratch) (void)hipFreeAsync(scratch, s);
  };
  auto bail = [&](hipError_t err, const char *what) {
    cleanup();
    if (orbit) (void)hipFreeAsync(orbit, s);
    release(e2);
    return dev_fail(err, what);
  };
  int64_t n2 = 0;
  if (na > 0) {
    if ((he = dalloc(&flag, (size_t)na, s))) return bail(he, "allocate flags");
    if ((he = dalloc(&kpos, (size_t)na, s))) return bail(he, "allocate positions");
    if ((he = dalloc(&count, 1, s))) return bail(he, "allocate count");
    if ((he = dalloc(&scratch, (size_t)compact_scratch_len(na), s))) return bail(he, "allocate scratch");
    if ((he = launch_keep_flags(keep, e->idx, na, flag, s))) return bail(he, "keep flags");
    if ((he = launch_compact(flag, na, kpos, count, scratch, s))) return bail(he, "compact");
    if ((he = hipMemcpyAsync(&n2, count, sizeof n2, hipMemcpyDeviceToHost, s))) return bail(he, "read count");
    if ((he = hipStreamSynchronize(s))) return bail(he, "synchronise");
  }
  e2->kind = e->kind;
  memcpy(e2->prm, e->prm, sizeof e2->prm);
  e2->custom_src = e->custom_src;
  e2->custom = e->custom;
  e2->pl = pl;
  e2->n_all = n2;
  e2->n_active = n2;
  e2->s_done = e->s_done;
  e2->stream = s;
  e2->device = e->device;
  e2->block = e->block;
  e2->pitch = n2 > 0 ? ((n2 + 63) / 64) * 64 : 64;
  const int64_t P = e->pitch, P2 = e2->pitch;
  const int rows_d = D + M * D + M + NSC, rows_i = M + 1;
  if ((he = dalloc(&e2->state, (size_t)P2 * rows_d, s))) return bail(he, "allocate state");
  if ((he = dalloc(&e2->istate, (size_t)P2 * rows_i, s))) return bail(he, "allocate state");
  if (n2 > 0) {
    if ((he = dalloc(&e2->x0, (size_t)n2 * D, s))) return bail(he, "allocate x0");
    if ((he = dalloc(&e2->idx, (size_t)n2, s))) return bail(he, "allocate index");
    if ((he = dalloc(&orbit, (size_t)n2, s))) return bail(he, "allocate orbit map");
    if ((he = launch_gather_x0(e->x0, D, e->idx, kpos, n2, e2->x0, orbit, s))) return bail(he, "gather x0");
    if ((he = launch_iota(e2->idx, n2, s))) return bail(he, "index");
    if ((he = launch_gather_columns(e->state, P, e2->state, P2, rows_d, kpos, n2, s)))
      return bail(he, "gather state");
    if ((he = launch_gather_columns_i(e->istate, P, e2->istate, P2, rows_i, kpos, n2, s)))
      return bail(he, "gather state");
  }
  StepArgs &a = e2->args;
  a = e->args;
  a.x = e2->state;
  a.w = a.x + (size_t)D * P2;
  a.gm = a.w + (size_t)M * D * P2;
  a.sc = a.gm + (size_t)M * P2;
  a.ge = e2->istate;
  a.st = a.ge + (size_t)M * P2;
  a.n = n2;
  a.pitch = P2;
  int64_t spl = pl.o.steps_per_launch;
  if (spl == 0) spl = (n2 > 0) ? (int64_t)(5.0e10 / (double)n2) : pl.n_total;
  spl = (spl / pl.K) * pl.K;
  if (spl < pl.K) spl = pl.K;
  e2->steps_per_launch = spl;
  cleanup();
  if (!e->device) {
    if ((he = hipStreamSynchronize(s))) {
      if (orbit) (void)hipFreeAsync(orbit, s);
      release(e2);
      return dev_fail(he, "synchronise");
    }
  }
  if (orbit_out) *orbit_out = orbit;
  else if (orbit) (void)hipFreeAsync(orbit, s);
  *out = e2;
  return CHX_OK;
}

chx_status run_once(const chx_system *sys, const double *x0, const uint8_t *mask, int64_t n,
                    const chx_options *opt, chx_result *res) {
  if (!res) return fail(CHX_ERR_INVALID_ARG, "result is NULL");
  chx_status st = check_system(sys);
  if (st) return st;
  Plan pl;
  st = make_plan(sys, opt, &pl);
  if (st) return st;
  if (res->label && !(pl.o.indicators & CHX_IND_SALI))
    return fail(CHX_ERR_INVALID_ARG, "label needs the SALI indicator");
  if (n < 0) return fail(CHX_ERR_INVALID_ARG, "n must be >= 0");
  if (n == 0) return CHX_OK;
  chx_ensemble *e = nullptr;
  st = create(sys, x0, mask, n, opt, &e);
  if (st) return st;
  st = advance(e, e->pl.n_total);
  if (!st) st = results(e, res);
  release(e);
  return st;
}

namespace {
hipStream_t stream_of(uint32_t flags, void *stream, chx_status *st) {
  *st = CHX_OK;
  if (flags & ~1u) *st = fail(CHX_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  else if (!(flags & CHX_PTR_DEVICE) && stream)
    *st = fail(CHX_ERR_INVALID_ARG, "stream given without CHX_PTR_DEVICE");
  return (flags & CHX_PTR_DEVICE) ? (hipStream_t)stream : nullptr;
}

// Host staging of inputs and outputs for the host-pointer variants.
struct Stage {
  bool device;
  hipStream_t s;
  std::vector<void *> allocs;
  hipError_t err = hipSuccess;
  template <class T>
  T *in(const T *p, size_t count) {
    if (device || !p || count == 0) return const_cast<T *>(p);
    T *d = nullptr;
    if (err == hipSuccess) err = hipMallocAsync((void **)&d, sizeof(T) * count, s);
    if (err == hipSuccess) {
      allocs.push_back(d);
      err = hipMemcpyAsync(d, p, sizeof(T) * count, hipMemcpyHostToDevice, s);
    }
    return d;
  }
  template <class T>
  T *out(size_t count) {
    T *d = nullptr;
    if (err == hipSuccess) err = hipMallocAsync((void **)&d, sizeof(T) * count, s);
    if (err == hipSuccess) allocs.push_back(d);
    return d;
  }
  template <class T>
  void back(T *host, const T *d, size_t count) {
    if (err == hipSuccess && count)
      err = hipMemcpyAsync(host, d, sizeof(T) * count, hipMemcpyDeviceToHost, s);
  }
  chx_status finish(const char *what) {
    for (void *p : allocs) (void)hipFreeAsync(p, s);
    if (!device) {
      hipError_t e = hipStreamSynchronize(s);
      if (err == hipSuccess) err = e;
    }
    if (err != hipSuccess) return dev_fail(err, what);
    return CHX_OK;
  }
};

}  // namespace

}  // namespace host
}  // namespace chx

using namespace chx::host;

extern "C" {

void chx_options_default(chx_options *o) {
  if (!o) return;
  memset(o, 0, sizeof *o);
  o->renorm_every = 10;
  o->ld_p = 0.5;
  o->sali_threshold = 1e-8;
}

const char *chx_last_error(void) { return g_err.c_str(); }
const char *chx_version(void) { return "libchx 0.1 (gfx950)"; }

chx_status chx_shutdown(void) {
  g_err.clear();
  const hipError_t e = custom_unload_all();
  if (e != hipSuccess) return dev_fail(e, "unload user-system code objects");
  return CHX_OK;
}

size_t chx_struct_size(int32_t which) {
  switch (which) {
  case 0: return sizeof(chx_system);
  case 1: return sizeof(chx_options);
  case 2: return sizeof(chx_result);
  case 3: return sizeof(chx_batch_item);
  case 4: return sizeof(chx_batch_stats);
  case 5: return sizeof(chx_gate_train_cfg);
  case 6: return sizeof(chx_gate_stats);
  case 7: return sizeof(chx_ldn_options);
  case 8: return sizeof(chx_ldn_result);
  }
  return 0;
}

chx_status chx_integrate_ensemble(const chx_system *sys, const double *x0, const uint8_t *mask,
                                  int64_t n, const chx_options *opt, chx_result *res) {
  g_err.clear();
  return run_once(sys, x0, mask, n, opt, res);
}

chx_status chx_ensemble_create(const chx_system *sys, const double *x0, const uint8_t *mask,
                               int64_t n, const chx_options *opt, chx_ensemble **out) {
  g_err.clear();
  return create(sys, x0, mask, n, opt, out);
}

chx_status chx_ensemble_advance(chx_ensemble *e, int64_t s_end) {
  g_err.clear();
  return advance(e, s_end);
}

chx_status chx_ensemble_results(chx_ensemble *e, chx_result *res) {
  g_err.clear();
  return results(e, res);
}

chx_status chx_ensemble_info(const chx_ensemble *e, int64_t *n_total, int64_t *s_done,
                             int64_t *n_active) {
  g_err.clear();
  if (!e) return fail(CHX_ERR_INVALID_ARG, "ensemble is NULL");
  if (n_total) *n_total = e->pl.n_total;
  if (s_done) *s_done = e->s_done;
  if (n_active) *n_active = e->n_active;
  return CHX_OK;
}

chx_status chx_ensemble_subset(chx_ensemble *e, const uint8_t *keep, chx_ensemble **out) {
  g_err.clear();
  if (!out) return fail(CHX_ERR_INVALID_ARG, "output handle pointer is NULL");
  *out = nullptr;
  if (!e) return fail(CHX_ERR_INVALID_ARG, "ensemble is NULL");
  if (e->n_all > 0 && !keep) return fail(CHX_ERR_INVALID_ARG, "keep is NULL");
  if (e->device || e->n_all == 0) return subset(e, keep, out, nullptr);
  uint8_t *dk = nullptr;
  hipError_t he = hipMallocAsync((void **)&dk, (size_t)e->n_all, e->stream);
  if (he == hipSuccess) he = hipMemcpyAsync(dk, keep, (size_t)e->n_all, hipMemcpyHostToDevice, e->stream);
  if (he != hipSuccess) {
    if (dk) (void)hipFreeAsync(dk, e->stream);
    (void)hipStreamSynchronize(e->stream);
    return dev_fail(he, "stage keep");
  }
  chx_status st = subset(e, dk, out, nullptr);
  (void)hipFreeAsync(dk, e->stream);
  he = hipStreamSynchronize(e->stream);
  if (st == CHX_OK && he != hipSuccess) {
    release(*out);
    *out = nullptr;
    return dev_fail(he, "synchronise");
  }
  return st;
}

void chx_ensemble_destroy(chx_ensemble *e) { release(e); }

static chx_status simple(const chx_system *sys, const double *x0, int64_t n, chx_options *o,
                         chx_result *r) {
  g_err.clear();
  return run_once(sys, x0, nullptr, n, o, r);
}

chx_status chx_sali(const chx_system *sys, const double *x0, int64_t n, double dt, double T,
                    uint64_t seed, double *sali_min_out, int8_t *label_out) {
  chx_options o;
  chx_options_default(&o);
  o.dt = dt;
  o.T = T;
  o.indicators = CHX_IND_SALI;
  o.seed = seed;
  chx_result r;
  memset(&r, 0, sizeof r);
  r.sali_min = sali_min_out;
  r.label = label_out;
  return simple(sys, x0, n, &o, &r);
}

chx_status chx_gali(const chx_system *sys, const double *x0, int64_t n, double dt, double T,
                    int32_t kmax, uint64_t seed, double *gali_out) {
  chx_options o;
  chx_options_default(&o);
  o.dt = dt;
  o.T = T;
  o.indicators = CHX_IND_GALI;
  o.gali_kmax = kmax;
  o.seed = seed;
  if (kmax < 2) {
    g_err.clear();
    return fail(CHX_ERR_INVALID_ARG, "kmax must be >= 2");
  }
  chx_result r;
  memset(&r, 0, sizeof r);
  r.gali = gali_out;
  return simple(sys, x0, n, &o, &r);
}

chx_status chx_lyap_spectrum(const chx_system *sys, const double *x0, int64_t n, double dt,
                             double T, int32_t n_exp, int32_t renorm_every, double *lyap_out) {
  chx_options o;
  chx_options_default(&o);
  o.dt = dt;
  o.T = T;
  o.indicators = CHX_IND_LYAP;
  o.n_lyap = n_exp;
  o.renorm_every = renorm_every;
  if (n_exp < 1) {
    g_err.clear();
    return fail(CHX_ERR_INVALID_ARG, "n_exp must be >= 1");
  }
  chx_result r;
  memset(&r, 0, sizeof r);
  r.lyap = lyap_out;
  return simple(sys, x0, n, &o, &r);
}

chx_status chx_ld(const chx_system *sys, const double *x0, int64_t n, double dt, double T,
                  double p, double *ld_out) {
  chx_options o;
  chx_options_default(&o);
  o.dt = dt;
  o.T = T;
  o.indicators = CHX_IND_LD;
  o.ld_p = p;
  if (!(p > 0.0)) {
    g_err.clear();
    return fail(CHX_ERR_INVALID_ARG, "p must be in (0, 1]");
  }
  chx_result r;
  memset(&r, 0, sizeof r);
  r.ld = ld_out;
  return simple(sys, x0, n, &o, &r);
}

chx_status chx_grid_hh_section(double E, double y0, double y1, int32_t ny, double py0,
                               double py1, int32_t npy, double *x0_out, uint8_t *mask_out,
                               uint32_t flags, void *stream) {
  g_err.clear();
  chx_status st;
  hipStream_t s = stream_of(flags, stream, &st);
  if (st) return st;
  if (ny < 0 || npy < 0) return fail(CHX_ERR_INVALID_ARG, "grid sizes must be >= 0");
  if (!isfinite(E) || !isfinite(y0) || !isfinite(y1) || !isfinite(py0) || !isfinite(py1))
    return fail(CHX_ERR_INVALID_ARG, "grid bounds and energy must be finite");
  const int64_t n = (int64_t)ny * npy;
  if (n == 0) return CHX_OK;
  if (!x0_out || !mask_out) return fail(CHX_ERR_INVALID_ARG, "output is NULL");
  Stage g{(flags & CHX_PTR_DEVICE) != 0, s};
  double *dx = g.device ? x0_out : g.out<double>(n * 4);
  uint8_t *dm = g.device ? mask_out : g.out<uint8_t>(n);
  if (g.err == hipSuccess) g.err = launch_hh_grid(E, y0, y1, ny, py0, py1, npy, dx, dm, s);
  if (!g.device) {
    g.back(x0_out, dx, n * 4);
    g.back(mask_out, dm, n);
  }
  return g.finish("section grid");
}

chx_status chx_hh_section_points(double E, const double *y, const double *py, int64_t n,
                                 double *x0_out, uint8_t *mask_out, uint32_t flags,
                                 void *stream) {
  g_err.clear();
  chx_status st;
  hipStream_t s = stream_of(flags, stream, &st);
  if (st) return st;
  if (n < 0) return fail(CHX_ERR_INVALID_ARG, "n must be >= 0");
  if (n == 0) return CHX_OK;
  if (!y || !py || !x0_out || !mask_out) return fail(CHX_ERR_INVALID_ARG, "NULL pointer");
  if (!isfinite(E)) return fail(CHX_ERR_INVALID_ARG, "E must be finite");
  Stage g{(flags & CHX_PTR_DEVICE) != 0, s};
  const double *dy = g.in(y, n), *dpy = g.in(py, n);
  double *dx = g.device ? x0_out : g.out<double>(n * 4);
  uint8_t *dm = g.device ? mask_out : g.out<uint8_t>(n);
  if (g.err == hipSuccess) g.err = launch_hh_points(E, dy, dpy, n, dx, dm, s);
  if (!g.device) {
    g.back(x0_out, dx, n * 4);
    g.back(mask_out, dm, n);
  }
  return g.finish("section points");
}

chx_status chx_ic_fput_modes(const chx_system *sys, const double *u, int64_t n, double *x0_out,
                             uint32_t flags, void *stream) {
  g_err.clear();
  chx_status st = check_system(sys);
  if (st) return st;
  if (sys->kind != CHX_SYS_FPUT) return fail(CHX_ERR_INVALID_ARG, "system must be FPUT");
  hipStream_t s = stream_of(flags, stream, &st);
  if (st) return st;
  if (n < 0) return fail(CHX_ERR_INVALID_ARG, "n must be >= 0");
  if (n == 0) return CHX_OK;
  if (!u || !x0_out) return fail(CHX_ERR_INVALID_ARG, "NULL pointer");
  if (!(sys->params[0] > 0.0) || sys->params[2] < 0.0)
    return fail(CHX_ERR_INVALID_ARG, "FPUT initial states need k > 0 and beta >= 0");
  const int D = 2 * sys->ndof;
  Stage g{(flags & CHX_PTR_DEVICE) != 0, s};
  const double *du = g.in(u, n * 5);
  double *dx = g.device ? x0_out : g.out<double>(n * D);
  if (g.err == hipSuccess) g.err = launch_fput_ic(sys->ndof, sys->params, du, n, dx, s);
  if (!g.device) g.back(x0_out, dx, n * D);
  return g.finish("FPUT initial states");
}

chx_status chx_ic_quartic(const chx_system *sys, const double *draws, int64_t n, double *x0_out,
                          uint32_t flags, void *stream) {
  g_err.clear();
  chx_status st = check_system(sys);
  if (st) return st;
  if (sys->kind != CHX_SYS_QUARTIC) return fail(CHX_ERR_INVALID_ARG, "system must be QUARTIC");
  hipStream_t s = stream_of(flags, stream, &st);
  if (st) return st;
  if (n < 0) return fail(CHX_ERR_INVALID_ARG, "n must be >= 0");
  if (n == 0) return CHX_OK;
  if (!draws || !x0_out) return fail(CHX_ERR_INVALID_ARG, "NULL pointer");
  if (!(sys->params[0] >= 0.0)) return fail(CHX_ERR_INVALID_ARG, "quartic initial states need eps >= 0");
  const int N = sys->ndof, D = 2 * N;
  Stage g{(flags & CHX_PTR_DEVICE) != 0, s};
  const double *dd = g.in(draws, n * (D + 1));
  double *dx = g.device ? x0_out : g.out<double>(n * D);
  if (g.err == hipSuccess) g.err = launch_quartic_ic(N, sys->params, dd, n, dx, s);
  if (!g.device) g.back(x0_out, dx, n * D);
  return g.finish("quartic initial states");
}

}  // extern "C"
