// Lane-per-orbit kernels for the coupled quartic oscillator with 1
// degree(s) of freedom: up to 4 deviation vectors.
#include "lane_kernel.h"

namespace chx {
hipError_t launch_lane_quartic1(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneDispatch<SysQuartic<1>, 4>::go(M, a, block, s);
}
}  // namespace chx
