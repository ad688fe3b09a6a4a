// ensemble.h -- host-side ensemble object shared by the C ABI (api.hip) and
// the batched launcher (batched_host.hip).
#pragma once
#include <string>

#include "chx_internal.h"

namespace chx {
namespace host {

// Options with defaults filled in, plus derived sizes.
struct Plan {
  chx_options o;
  int N, D, m_s, n_l, M, K, kmax;
  int64_t n_total;
};

// A device workspace handed in by the caller of create() / results(): their
// buffers are carved from it (256-byte aligned) instead of allocated, and
// nothing is freed (the allocation-free entry point, noalloc.hip).
struct Arena {
  char *base = nullptr;
  size_t cap = 0, used = 0;
  template <class T>
  T *take(size_t count) {
    const size_t bytes = ((sizeof(T) * count + 255) / 256) * 256;
    if (count == 0) return nullptr;
    if (used + bytes > cap) return nullptr;
    T *p = reinterpret_cast<T *>(base + used);
    used += bytes;
    return p;
  }
};

chx_status fail(chx_status st, const char *fmt, ...);
chx_status dev_fail(hipError_t e, const char *what);
chx_status check_system(const chx_system *sys);
chx_status make_plan(const chx_system *sys, const chx_options *opt, Plan *p);
extern thread_local std::string g_err;

}  // namespace host
}  // namespace chx

struct chx_ensemble {
  int kind;
  double prm[16];
  chx::host::Plan pl;
  int64_t n_all = 0, n_active = 0, pitch = 0, s_done = 0;
  hipStream_t stream = nullptr;
  bool device = false;
  double *x0 = nullptr;      // [n_all][D] own copy
  uint8_t *mask = nullptr;   // [n_all] own copy or null
  int64_t *idx = nullptr;    // [n_active]
  double *state = nullptr;   // x, w, gm, sc
  int *istate = nullptr;     // ge, st
  chx::StepArgs args{};
  std::string custom_src;  // CHX_SYS_CUSTOM: the caller's source
  void *custom = nullptr;  // its compiled program (process cache)
  int block = 256;
  int64_t steps_per_launch = 0;
  bool in_arena = false;   // buffers carved from a caller's workspace: not freed
};

namespace chx {
namespace host {
void release(chx_ensemble *e);
// With an arena (device pointers only) x0, mask and w0 are used in place
// and every other buffer comes from the arena.
chx_status create(const chx_system *sys, const double *x0, const uint8_t *mask, int64_t n,
                  const chx_options *opt, chx_ensemble **out, Arena *arena = nullptr);
chx_status advance(chx_ensemble *e, int64_t s_end);
// gali_scratch: n_active * gali_kmax * 2N doubles for the GALI QR, or null
// to allocate it
chx_status results(chx_ensemble *e, chx_result *res, double *gali_scratch = nullptr);
chx_status subset(chx_ensemble *e, const uint8_t *keep, chx_ensemble **out, int64_t **orbit_out);
// custom.hip: user systems compiled at run time
size_t custom_rk_lds_per_lane(bool general, bool adaptive, int N, int M);
chx_status custom_prepare(const std::string &src, int ndof, bool general, const Plan &pl,
                          void **handle);
hipError_t custom_init(void *handle, const chx::StepArgs &a, hipStream_t s);
hipError_t custom_launch(void *handle, bool general, const Plan &pl, const chx::StepArgs &a,
                         int block, hipStream_t s);
hipError_t custom_unload_all();
}  // namespace host
}  // namespace chx
