// DOP853 lane-per-orbit kernels (fixed step) for 1 uncoupled harmonic
// oscillator(s): up to 4 deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rka_harmonic1(int M, const StepArgs &a, int block, hipStream_t s);

hipError_t launch_lane_rk_harmonic1(int M, bool adaptive, const StepArgs &a, int block,
                                    hipStream_t s) {
  return adaptive ? launch_lane_rka_harmonic1(M, a, block, s)
                  : LaneRKDispatch<SysHarmonic<1>, 4, false>::go(M, a, block, s);
}
}  // namespace chx
