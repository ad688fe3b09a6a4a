// noalloc.hip -- chx_integrate_ensemble_noalloc: the whole-ensemble
// integration of chx_integrate_ensemble for callers that cannot allocate
// device memory.  Every buffer the call needs beyond the caller's inputs and
// outputs (active-orbit index, compaction counts, the ensemble's state in
// its structure-of-arrays layout, the GALI QR copies) is carved from one
// file-scope device array, `scratch`, of CHX_NOALLOC_MAX_BYTES.  Each GPU
// holds its own copy of the array, at its own address, from the loading of
// this code object until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: the
// device address is fetched once per device with hipGetSymbolAddress (with
// that device current) and only that address is handed to kernels.
//
// No buffer of the workspace is read before the call writes it (the set-up
// kernel writes every state row of every active orbit, the compaction
// writes its counts before scanning them), so nothing is cleared and a
// call never sees what the previous one left.  All calls on one GPU share
// its array: calls that overlap in time on the same GPU (two host threads,
// or two streams) race.
#include <mutex>
#include <vector>

#include "chx_internal.h"
#include "ensemble.h"

using namespace chx;
using namespace chx::host;

namespace {

__device__ __align__(256) char scratch[CHX_NOALLOC_MAX_BYTES];

std::mutex g_mu;
std::vector<char *> g_ptr;  // device address of `scratch`, per device

// The device address of this device's `scratch`; null (and *st set) if
// the runtime cannot give it.
char *scratch_of_current_device(chx_status *st) {
  *st = CHX_OK;
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) {
    *st = dev_fail(he, "current device");
    return nullptr;
  }
  std::lock_guard<std::mutex> g(g_mu);
  if ((int)g_ptr.size() <= dev) g_ptr.resize(dev + 1, nullptr);
  if (!g_ptr[dev]) {
    char *p = nullptr;
    he = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
    if (he != hipSuccess || !p) {
      *st = dev_fail(he != hipSuccess ? he : hipErrorInvalidSymbol, "workspace address");
      return nullptr;
    }
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

size_t round256(size_t b) { return ((b + 255) / 256) * 256; }

}  // namespace

extern "C" chx_status chx_integrate_ensemble_noalloc(const chx_system *sys, const double *x0,
                                                     const uint8_t *mask, int64_t n,
                                                     const chx_options *opt, chx_result *res) {
  g_err.clear();
  if (!res) return fail(CHX_ERR_INVALID_ARG, "result is NULL");
  chx_status st = check_system(sys);
  if (st) return st;
  if (sys->kind == CHX_SYS_CUSTOM || sys->kind == CHX_SYS_CUSTOM_GENERAL)
    return fail(CHX_ERR_UNSUPPORTED, "the allocation-free entry takes built-in systems only (a custom system compiles and loads code)");
  Plan pl;
  st = make_plan(sys, opt, &pl);
  if (st) return st;
  if (!(pl.o.flags & CHX_PTR_DEVICE))
    return fail(CHX_ERR_INVALID_ARG, "the allocation-free entry takes device pointers only (set CHX_PTR_DEVICE)");
  if (res->label && !(pl.o.indicators & CHX_IND_SALI))
    return fail(CHX_ERR_INVALID_ARG, "label needs the SALI indicator");
  if (n < 0) return fail(CHX_ERR_INVALID_ARG, "n must be >= 0");
  if (n == 0) return CHX_OK;
  if (!x0) return fail(CHX_ERR_INVALID_ARG, "x0 is NULL");
  // the workspace the call needs, with every orbit active (an upper bound)
  const int D = pl.D, M = pl.M;
  if (n > (int64_t)(CHX_NOALLOC_MAX_BYTES / 8))
    return fail(CHX_ERR_INVALID_ARG, "n = %lld initial conditions need more than the %llu-byte workspace of the allocation-free entry", (long long)n, (unsigned long long)CHX_NOALLOC_MAX_BYTES);
  const size_t P = (size_t)((n + 63) / 64) * 64;
  const bool gali = res->gali && (pl.o.indicators & CHX_IND_GALI) && pl.kmax >= 2;
  const size_t need = round256(sizeof(int64_t) * (size_t)n) +
                      round256(sizeof(int64_t) * (size_t)compact_scratch_len(n)) +
                      round256(sizeof(int64_t)) +
                      round256(sizeof(double) * P * (D + (size_t)M * D + M + NSC)) +
                      round256(sizeof(int) * P * (M + 1)) +
                      (gali ? round256(sizeof(double) * (size_t)n * pl.kmax * D) : 0);
  if (need > (size_t)CHX_NOALLOC_MAX_BYTES)
    return fail(CHX_ERR_INVALID_ARG, "this call needs %zu bytes of workspace; the allocation-free entry holds %llu per GPU (fewer initial conditions or deviation vectors)", need, (unsigned long long)CHX_NOALLOC_MAX_BYTES);
  char *base = scratch_of_current_device(&st);
  if (!base) return st;
  Arena ar;
  ar.base = base;
  ar.cap = CHX_NOALLOC_MAX_BYTES;
  chx_ensemble *e = nullptr;
  st = create(sys, x0, mask, n, opt, &e, &ar);
  if (st) return st;
  double *gq = nullptr;
  if (gali) {
    gq = ar.take<double>((size_t)e->n_active * pl.kmax * D);
    if (e->n_active > 0 && !gq) {
      release(e);
      return fail(CHX_ERR_INTERNAL, "workspace estimate too small");
    }
  }
  st = advance(e, e->pl.n_total);
  if (!st) st = results(e, res, gq);
  release(e);
  return st;
}
