// DOP853 lane-per-orbit kernels (fixed step) for the coupled quartic oscillator
// with 3 degree(s) of freedom: up to 12 deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rka_quartic3(int M, const StepArgs &a, int block, hipStream_t s);

hipError_t launch_lane_rk_quartic3(int M, bool adaptive, const StepArgs &a, int block,
                                   hipStream_t s) {
  return adaptive ? launch_lane_rka_quartic3(M, a, block, s)
                  : LaneRKDispatch<SysQuartic<3>, 12, false>::go(M, a, block, s);
}
}  // namespace chx
