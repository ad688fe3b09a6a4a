// ldn.hip -- chaos indicators from the Lagrangian descriptors of
// neighbouring orbits (chx_ld_indicators): the member orbits of every
// initial condition (itself and its +/- sigma neighbours, each forward and
// momentum-reversed) are laid out by one kernel, integrated as one ensemble
// with the LD alone, and reduced to D, R, S by another.
#include <math.h>

#include <vector>

#include "chx_internal.h"
#include "ensemble.h"

namespace chx {
namespace {

// Member row r of the expanded ensemble: initial condition j = r / (nb nm),
// direction b = (r / nm) % nb (1: momenta reversed), member m = r % nm
// (0: x itself; 2i+1, 2i+2: x + sigma e_c, x - sigma e_c for the i-th set
// bit c of dirs).
__global__ void ldn_expand_kernel(const double *__restrict__ x0,
                                  const uint8_t *__restrict__ mask, int64_t n, int N,
                                  uint32_t dirs, double sigma, int nb, int nm,
                                  double *__restrict__ X, uint8_t *__restrict__ Xm) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rows = n * nb * nm;
  if (r >= rows) return;
  const int D = 2 * N;
  const int64_t j = r / (nb * nm);
  const int b = (int)((r / nm) % nb), m = (int)(r % nm);
  int cd = -1;
  if (m > 0) {
    int i = (m - 1) / 2;
    for (int c = 0; c < D; ++c)
      if (dirs & (1u << c)) {
        if (i == 0) {
          cd = c;
          break;
        }
        --i;
      }
  }
  const double dsg = (m % 2 == 1) ? sigma : -sigma;
  for (int c = 0; c < D; ++c) {
    double v = x0[j * D + c];
    if (c == cd) v = v + dsg;
    if (b == 1 && c >= N) v = -v;
    X[r * D + c] = v;
  }
  if (Xm) Xm[r] = mask[j];
}

__device__ inline int status_rank(int s) {
  return s == CHX_ORBIT_NONFINITE ? 3 : s == CHX_ORBIT_STEP_FAILED ? 2
       : s == CHX_ORBIT_ESCAPED   ? 1 : 0;
}

__global__ void ldn_combine_kernel(const double *__restrict__ ld,
                                   const int32_t *__restrict__ st, int64_t n, int nb, int nm,
                                   double *ld_out, double *D_out, double *R_out, double *S_out,
                                   int32_t *st_out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t base = j * nb * nm;
  int worst = CHX_ORBIT_OK;
  bool masked = false;
  for (int q = 0; q < nb * nm; ++q) {
    const int s = st[base + q];
    if (s == CHX_ORBIT_MASKED) masked = true;
    else if (status_rank(s) > status_rank(worst)) worst = s;
  }
  double L0 = NAN, dd = NAN, rr = NAN, ss = NAN;
  if (masked) {
    worst = CHX_ORBIT_MASKED;
  } else if (worst == CHX_ORBIT_OK) {
    // L of member m: the forward part plus (two-sided) the reversed one
    auto L = [&](int m) { return nb == 2 ? ld[base + m] + ld[base + nm + m] : ld[base + m]; };
    const int k = (nm - 1) / 2;
    const double c = L(0);
    double d = 0.0, r = 0.0, s2 = 0.0;
    for (int i = 0; i < k; ++i) {
      const double lp = L(2 * i + 1), lm = L(2 * i + 2);
      d += fabs(c - lp) + fabs(c - lm);
      r += lp + lm;
      s2 += fabs(lp - 2.0 * c + lm);
    }
    L0 = c;
    dd = d / (2 * k) / c;
    rr = fabs(1.0 - r / (2 * k) / c);
    ss = s2 / k / c;
  }
  if (ld_out) ld_out[j] = L0;
  if (D_out) D_out[j] = dd;
  if (R_out) R_out[j] = rr;
  if (S_out) S_out[j] = ss;
  if (st_out) st_out[j] = worst;
}

// Device staging for host-pointer calls (inputs uploaded, outputs
// downloaded), as in the other entry points.
struct Buf {
  bool device;
  hipStream_t s;
  std::vector<void *> allocs;
  hipError_t err = hipSuccess;
  template <class T>
  T *alloc(size_t count) {
    T *d = nullptr;
    if (err == hipSuccess && count) err = hipMallocAsync((void **)&d, sizeof(T) * count, s);
    if (err == hipSuccess && d) allocs.push_back(d);
    return d;
  }
  template <class T>
  const T *in(const T *p, size_t count) {
    if (device || !p || count == 0) return p;
    T *d = alloc<T>(count);
    if (err == hipSuccess) err = hipMemcpyAsync(d, p, sizeof(T) * count, hipMemcpyHostToDevice, s);
    return d;
  }
  template <class T>
  T *out(T *p, size_t count) {
    if (device || !p) return p;
    return alloc<T>(count);
  }
  template <class T>
  void back(T *host, const T *d, size_t count) {
    if (!device && host && err == hipSuccess && count)
      err = hipMemcpyAsync(host, d, sizeof(T) * count, hipMemcpyDeviceToHost, s);
  }
  hipError_t finish() {
    for (void *p : allocs) (void)hipFreeAsync(p, s);
    if (device) return err;
    hipError_t e = hipStreamSynchronize(s);
    return err != hipSuccess ? err : e;
  }
};

}  // namespace
}  // namespace chx

using namespace chx;
using namespace chx::host;

extern "C" chx_status chx_ld_indicators(const chx_system *sys, const double *x0,
                                        const uint8_t *mask, int64_t n,
                                        const chx_options *opt, const chx_ldn_options *lo,
                                        chx_ldn_result *res) {
  g_err.clear();
  chx_status st = check_system(sys);
  if (st) return st;
  if (!opt) return fail(CHX_ERR_INVALID_ARG, "options is NULL");
  if (!lo) return fail(CHX_ERR_INVALID_ARG, "LD-indicator options are NULL");
  if (!res) return fail(CHX_ERR_INVALID_ARG, "result is NULL");
  if (opt->flags & ~1u) return fail(CHX_ERR_INVALID_ARG, "unknown flags 0x%x", opt->flags);
  const bool device = (opt->flags & CHX_PTR_DEVICE) != 0;
  if (!device && opt->stream)
    return fail(CHX_ERR_INVALID_ARG, "stream given without CHX_PTR_DEVICE");
  if (opt->indicators & ~(uint32_t)CHX_IND_LD)
    return fail(CHX_ERR_INVALID_ARG, "the LD indicators integrate the LD alone: indicators must be 0 or CHX_IND_LD");
  if (opt->w0) return fail(CHX_ERR_INVALID_ARG, "w0 must be NULL (no deviation vectors)");
  if (opt->early_exit) return fail(CHX_ERR_INVALID_ARG, "early_exit needs the SALI indicator");
  const int N = sys->ndof, D = 2 * N;
  const uint32_t all = D >= 32 ? 0xffffffffu : ((1u << D) - 1u);
  const uint32_t dirs = lo->dirs ? lo->dirs : all;
  if (dirs & ~all)
    return fail(CHX_ERR_INVALID_ARG, "dirs has bits beyond the 2N = %d coordinates", D);
  if (!(lo->sigma > 0.0) || !isfinite(lo->sigma))
    return fail(CHX_ERR_INVALID_ARG, "sigma must be finite and > 0");
  // M- is taken as M+ of the momentum-reversed state, which is the backward
  // integral only when H is even in the momenta: true of every built-in
  // system and of separable user systems (p^2/2 + V), not of a general one.
  if (lo->two_sided && sys->kind == CHX_SYS_CUSTOM_GENERAL)
    return fail(CHX_ERR_UNSUPPORTED, "two-sided LD indicators need H even in the momenta: not available for a general custom system (set two_sided = 0)");
  chx_options o2 = *opt;
  o2.indicators = CHX_IND_LD;
  Plan pl;
  st = make_plan(sys, &o2, &pl);
  if (st) return st;
  if (n < 0) return fail(CHX_ERR_INVALID_ARG, "n must be >= 0");
  if (n == 0) return CHX_OK;
  if (!x0) return fail(CHX_ERR_INVALID_ARG, "x0 is NULL");
  const int nb = lo->two_sided ? 2 : 1;
  const int nm = 1 + 2 * __builtin_popcount(dirs);
  if (n > INT64_MAX / (nb * nm) / D) return fail(CHX_ERR_INVALID_ARG, "n is too large");
  const int64_t nx = n * nb * nm;
  hipStream_t s = device ? (hipStream_t)opt->stream : nullptr;
  Buf g{device, s};
  const double *dx0 = g.in(x0, (size_t)n * D);
  const uint8_t *dmask = g.in(mask, (size_t)n);
  double *X = g.alloc<double>((size_t)nx * D);
  uint8_t *Xm = mask ? g.alloc<uint8_t>((size_t)nx) : nullptr;
  double *LDx = g.alloc<double>((size_t)nx);
  int32_t *STx = g.alloc<int32_t>((size_t)nx);
  double *o_ld = g.out(res->ld, (size_t)n), *o_D = g.out(res->D, (size_t)n);
  double *o_R = g.out(res->R, (size_t)n), *o_S = g.out(res->S, (size_t)n);
  int32_t *o_st = g.out(res->status, (size_t)n);
  if (g.err == hipSuccess) {
    const unsigned blocks = (unsigned)((nx + 255) / 256);
    hipLaunchKernelGGL(ldn_expand_kernel, dim3(blocks), dim3(256), 0, s, dx0, dmask, n, N, dirs,
                       lo->sigma, nb, nm, X, Xm);
    g.err = hipGetLastError();
  }
  if (g.err != hipSuccess) {
    (void)g.finish();
    return dev_fail(g.err, "LD indicators: expand");
  }
  // the member orbits: one ensemble, LD only, on this stream
  o2.flags = CHX_PTR_DEVICE;
  o2.stream = (void *)s;
  chx_ensemble *e = nullptr;
  st = create(sys, X, Xm, nx, &o2, &e);
  if (!st) st = advance(e, e->pl.n_total);
  if (!st) {
    chx_result r{};
    r.ld = LDx;
    r.status = STx;
    st = results(e, &r);
  }
  if (e) release(e);
  if (st) {
    (void)g.finish();
    return st;
  }
  {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(ldn_combine_kernel, dim3(blocks), dim3(256), 0, s, LDx, STx, n, nb, nm,
                       o_ld, o_D, o_R, o_S, o_st);
    g.err = hipGetLastError();
  }
  g.back(res->ld, o_ld, (size_t)n);
  g.back(res->D, o_D, (size_t)n);
  g.back(res->R, o_R, (size_t)n);
  g.back(res->S, o_S, (size_t)n);
  g.back(res->status, o_st, (size_t)n);
  const hipError_t he = g.finish();
  if (he != hipSuccess) return dev_fail(he, "LD indicators");
  return CHX_OK;
}
