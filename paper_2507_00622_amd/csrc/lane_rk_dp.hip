// DOP853 lane-per-orbit kernels (fixed step) for the double pendulum: up to
// 8 deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rka_dp(int M, const StepArgs &a, int block, hipStream_t s);

hipError_t launch_lane_rk_dp(int M, bool adaptive, const StepArgs &a, int block,
                             hipStream_t s) {
  return adaptive ? launch_lane_rka_dp(M, a, block, s)
                  : LaneRKDispatch<SysDP, 8, false>::go(M, a, block, s);
}
}  // namespace chx
