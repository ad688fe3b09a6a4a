// Lane-per-orbit kernels for 1 uncoupled harmonic oscillator(s): up to
// 4 deviation vectors.
#include "lane_kernel.h"

namespace chx {
hipError_t launch_lane_harmonic1(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneDispatch<SysHarmonic<1>, 4>::go(M, a, block, s);
}
}  // namespace chx
