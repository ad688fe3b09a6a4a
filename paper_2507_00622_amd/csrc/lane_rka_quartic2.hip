// Adaptive DOP8(5) lane-per-orbit kernels for the coupled quartic oscillator
// with 2 degree(s) of freedom: up to 8 deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rka_quartic2(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneRKDispatch<SysQuartic<2>, 8, true>::go(M, a, block, s);
}
}  // namespace chx
