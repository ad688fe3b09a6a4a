// Adaptive DOP8(5) lane-per-orbit kernels for 1 uncoupled harmonic
// oscillator(s): up to 4 deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rka_harmonic1(int M, const StepArgs &a, int block, hipStream_t s) {
  return LaneRKDispatch<SysHarmonic<1>, 4, true>::go(M, a, block, s);
}
}  // namespace chx
