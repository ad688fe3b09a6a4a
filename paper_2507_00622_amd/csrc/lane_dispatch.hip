// System dispatch of the lane-per-orbit kernels.
#include "chx_internal.h"

namespace chx {
hipError_t launch_lane_hh(int M, const StepArgs &a, int block, hipStream_t s);
hipError_t launch_lane_quartic1(int M, const StepArgs &a, int block, hipStream_t s);
hipError_t launch_lane_quartic2(int M, const StepArgs &a, int block, hipStream_t s);
hipError_t launch_lane_quartic3(int M, const StepArgs &a, int block, hipStream_t s);
hipError_t launch_lane_harmonic1(int M, const StepArgs &a, int block, hipStream_t s);
hipError_t launch_lane_harmonic2(int M, const StepArgs &a, int block, hipStream_t s);
hipError_t launch_lane_harmonic3(int M, const StepArgs &a, int block, hipStream_t s);

hipError_t launch_lane_rk_hh(int M, bool adaptive, const StepArgs &a, int block,
                            hipStream_t s);
hipError_t launch_lane_rk_quartic1(int M, bool adaptive, const StepArgs &a, int block,
                            hipStream_t s);
hipError_t launch_lane_rk_quartic2(int M, bool adaptive, const StepArgs &a, int block,
                            hipStream_t s);
hipError_t launch_lane_rk_quartic3(int M, bool adaptive, const StepArgs &a, int block,
                            hipStream_t s);
hipError_t launch_lane_rk_harmonic1(int M, bool adaptive, const StepArgs &a, int block,
                            hipStream_t s);
hipError_t launch_lane_rk_harmonic2(int M, bool adaptive, const StepArgs &a, int block,
                            hipStream_t s);
hipError_t launch_lane_rk_harmonic3(int M, bool adaptive, const StepArgs &a, int block,
                            hipStream_t s);
hipError_t launch_lane_rk_dp(int M, bool adaptive, const StepArgs &a, int block, hipStream_t s);

bool lane_supported(int sys, int ndof, int M) {
  if (M < 0 || M > 4 * ndof) return false;
  switch (sys) {
  case SYS_HH: return ndof == 2;
  case SYS_QUARTIC:
  case SYS_HARMONIC: return ndof >= 1 && ndof <= 3;
  case SYS_DP: return ndof == 2;  // DOP853 kernels only
  case CHX_SYS_CUSTOM:
  case CHX_SYS_CUSTOM_GENERAL: return ndof >= 1 && ndof <= CHX_CUSTOM_MAX_NDOF;  // compiled at run time
  }
  return false;
}

hipError_t launch_lane(int sys, int ndof, int M, const StepArgs &a, int block,
                       hipStream_t s) {
  if (!lane_supported(sys, ndof, M) || sys == SYS_DP || sys == CHX_SYS_CUSTOM ||
      sys == CHX_SYS_CUSTOM_GENERAL)
    return hipErrorInvalidValue;
  if (a.n == 0) return hipSuccess;
  switch (sys) {
  case SYS_HH: return launch_lane_hh(M, a, block, s);
  case SYS_QUARTIC:
    return ndof == 1 ? launch_lane_quartic1(M, a, block, s)
         : ndof == 2 ? launch_lane_quartic2(M, a, block, s)
                     : launch_lane_quartic3(M, a, block, s);
  case SYS_HARMONIC:
    return ndof == 1 ? launch_lane_harmonic1(M, a, block, s)
         : ndof == 2 ? launch_lane_harmonic2(M, a, block, s)
                     : launch_lane_harmonic3(M, a, block, s);
  }
  return hipErrorInvalidValue;
}

// The same systems and the double pendulum with the DOP853 kernels (fixed
// step or adaptive).
hipError_t launch_lane_rk(int sys, int ndof, int M, bool adaptive, const StepArgs &a,
                          int block, hipStream_t s) {
  if (!lane_supported(sys, ndof, M)) return hipErrorInvalidValue;
  if (a.n == 0) return hipSuccess;
  switch (sys) {
  case SYS_HH: return launch_lane_rk_hh(M, adaptive, a, block, s);
  case SYS_QUARTIC:
    return ndof == 1 ? launch_lane_rk_quartic1(M, adaptive, a, block, s)
         : ndof == 2 ? launch_lane_rk_quartic2(M, adaptive, a, block, s)
                     : launch_lane_rk_quartic3(M, adaptive, a, block, s);
  case SYS_HARMONIC:
    return ndof == 1 ? launch_lane_rk_harmonic1(M, adaptive, a, block, s)
         : ndof == 2 ? launch_lane_rk_harmonic2(M, adaptive, a, block, s)
                     : launch_lane_rk_harmonic3(M, adaptive, a, block, s);
  case SYS_DP: return launch_lane_rk_dp(M, adaptive, a, block, s);
  }
  return hipErrorInvalidValue;
}
}  // namespace chx
