// DOP853 lane-per-orbit kernels for the coupled quartic oscillator with 1 degree(s) of freedom:
// up to 4 deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rk_quartic1(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneRKDispatch<SysQuartic<1>, 4>::go(M, a, block, s);
}
}  // namespace chx
