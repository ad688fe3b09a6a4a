// Lane-per-orbit kernels for 2 uncoupled harmonic oscillator(s): up to
// 8 deviation vectors.
#include "lane_kernel.h"

namespace chx {
hipError_t launch_lane_harmonic2(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneDispatch<SysHarmonic<2>, 8>::go(M, a, block, s);
}
}  // namespace chx
