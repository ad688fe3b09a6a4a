// Adaptive DOP8(5) lane-per-orbit kernels for the Henon-Heiles system: up to 8
// deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rka_hh(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneRKDispatch<SysHH, 8, true>::go(M, a, block, s);
}
}  // namespace chx
