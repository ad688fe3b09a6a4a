// DOP853 lane-per-orbit kernels (fixed step) for the coupled quartic oscillator
// with 1 degree(s) of freedom: up to 4 deviation vectors.
#include "lane_rk.h"

namespace chx {
hipError_t launch_lane_rka_quartic1(int M, const StepArgs &a, int block, hipStream_t s);

hipError_t launch_lane_rk_quartic1(int M, bool adaptive, const StepArgs &a, int block,
                                   hipStream_t s) {
  return adaptive ? launch_lane_rka_quartic1(M, a, block, s)
                  : LaneRKDispatch<SysQuartic<1>, 4, false>::go(M, a, block, s);
}
}  // namespace chx
