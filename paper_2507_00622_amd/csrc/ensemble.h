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
};

namespace chx {
namespace host {
void release(chx_ensemble *e);
chx_status create(const chx_system *sys, const double *x0, const uint8_t *mask, int64_t n,
                  const chx_options *opt, chx_ensemble **out);
chx_status advance(chx_ensemble *e, int64_t s_end);
chx_status results(chx_ensemble *e, chx_result *res);
chx_status subset(chx_ensemble *e, const uint8_t *keep, chx_ensemble **out, int64_t **orbit_out);
// custom.hip: user systems compiled at run time
size_t custom_rk_lds_per_lane(bool general, bool adaptive, int N, int M);
chx_status custom_prepare(const std::string &src, int ndof, bool general, const Plan &pl,
                          void **handle);
hipError_t custom_init(void *handle, const chx::StepArgs &a, hipStream_t s);
hipError_t custom_launch(void *handle, bool general, const Plan &pl, const chx::StepArgs &a,
                         int block, hipStream_t s);
}  // namespace host
}  // namespace chx
