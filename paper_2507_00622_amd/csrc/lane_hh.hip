// Lane-per-orbit kernels for the Henon-Heiles system: up to 8 deviation
// vectors (2N SALI/GALI vectors + 2N Lyapunov vectors).
#include "lane_kernel.h"

// Orbits per lane of the Henon-Heiles kernels.
#ifndef CHX_HH_OPL
#define CHX_HH_OPL 1
#endif

namespace chx {
hipError_t launch_lane_hh(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneDispatch<SysHH, 8, CHX_HH_OPL>::go(M, a, block, s);
}
}  // namespace chx
