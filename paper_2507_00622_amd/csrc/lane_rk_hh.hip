// DOP853 lane-per-orbit kernels (fixed step) for the Henon-Heiles system: up to
// 8 deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rka_hh(int M, const StepArgs &a, int block, hipStream_t s);

hipError_t launch_lane_rk_hh(int M, bool adaptive, const StepArgs &a, int block,
                             hipStream_t s) {
  return adaptive ? launch_lane_rka_hh(M, a, block, s)
                  : LaneRKDispatch<SysHH, 8, false>::go(M, a, block, s);
}
}  // namespace chx
