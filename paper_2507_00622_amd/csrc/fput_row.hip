// fput_row.hip -- launcher of the row-per-orbit FPU kernels.
#include "fput_row.h"

namespace chx {

namespace {
template <int N>
hipError_t launch_n(int M, const StepArgs &a, hipStream_t s) {
  const unsigned grid = (unsigned)((a.n + 3) / 4);
  const int V = (M + 15) / 16;
  if (V <= 1)
    hipLaunchKernelGGL((fput_row_kernel<N, 1>), dim3(grid), dim3(64), 0, s, a);
  else if (V == 2)
    hipLaunchKernelGGL((fput_row_kernel<N, 2>), dim3(grid), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((fput_row_kernel<N, 3>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}
}  // namespace

bool fput_row_supported(int ndof, int M, int n_l, bool sali) {
  if (!(ndof == 2 || ndof == 4 || ndof == 8 || ndof == 16)) return false;
  if (M < 0 || M > 48) return false;
  if (sali && n_l % 16 != 0) return false;
  return true;
}

hipError_t launch_fput_row(int ndof, int M, const StepArgs &a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  switch (ndof) {
  case 2: return launch_n<2>(M, a, s);
  case 4: return launch_n<4>(M, a, s);
  case 8: return launch_n<8>(M, a, s);
  case 16: return launch_n<16>(M, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace chx
