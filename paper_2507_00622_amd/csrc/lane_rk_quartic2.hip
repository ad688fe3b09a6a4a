// DOP853 lane-per-orbit kernels (fixed step) for the coupled quartic oscillator
// with 2 degree(s) of freedom: up to 8 deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rka_quartic2(int M, const StepArgs &a, int block, hipStream_t s);

hipError_t launch_lane_rk_quartic2(int M, bool adaptive, const StepArgs &a, int block,
                                   hipStream_t s) {
  return adaptive ? launch_lane_rka_quartic2(M, a, block, s)
                  : LaneRKDispatch<SysQuartic<2>, 8, false>::go(M, a, block, s);
}
}  // namespace chx
