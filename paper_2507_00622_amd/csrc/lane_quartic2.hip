// Lane-per-orbit kernels for the coupled quartic oscillator with 2
// degree(s) of freedom: up to 8 deviation vectors.
#include "lane_kernel.h"

namespace chx {
hipError_t launch_lane_quartic2(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneDispatch<SysQuartic<2>, 8>::go(M, a, block, s);
}
}  // namespace chx
