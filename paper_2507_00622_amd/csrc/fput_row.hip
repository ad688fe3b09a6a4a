// fput_row.hip -- FPU chains: one 16-lane row per orbit (not built yet).
#include "chx_internal.h"

namespace chx {
bool fput_row_supported(int, int) { return false; }
hipError_t launch_fput_row(int, int, const StepArgs &, hipStream_t) {
  return hipErrorInvalidValue;
}
}  // namespace chx
