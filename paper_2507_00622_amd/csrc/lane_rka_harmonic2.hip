// Adaptive DOP8(5) lane-per-orbit kernels for 2 uncoupled harmonic
// oscillator(s): up to 8 deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rka_harmonic2(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneRKDispatch<SysHarmonic<2>, 8, true>::go(M, a, block, s);
}
}  // namespace chx
