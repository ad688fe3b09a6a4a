// DOP853 lane-per-orbit kernels for the Henon-Heiles system: up to 8
// deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rk_hh(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneRKDispatch<SysHH, 8>::go(M, a, block, s);
}
}  // namespace chx
