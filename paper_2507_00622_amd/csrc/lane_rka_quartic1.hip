// Adaptive DOP8(5) lane-per-orbit kernels for the coupled quartic oscillator
// with 1 degree(s) of freedom: up to 4 deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rka_quartic1(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneRKDispatch<SysQuartic<1>, 4, true>::go(M, a, block, s);
}
}  // namespace chx
