// Lane-per-orbit kernels for the Henon-Heiles system: up to 8 deviation
// vectors (2N SALI/GALI vectors + 2N Lyapunov vectors).
#include "lane_kernel.h"

namespace chx {
hipError_t launch_lane_hh(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneDispatch<SysHH, 8>::go(M, a, block, s);
}
}  // namespace chx
