// Adaptive DOP8(5) lane-per-orbit kernels for the double pendulum: up to 8
// deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rka_dp(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneRKDispatch<SysDP, 8, true>::go(M, a, block, s);
}
}  // namespace chx
