// Adaptive DOP8(5) lane-per-orbit kernels for 3 uncoupled harmonic
// oscillator(s): up to 12 deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rka_harmonic3(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneRKDispatch<SysHarmonic<3>, 12, true>::go(M, a, block, s);
}
}  // namespace chx
