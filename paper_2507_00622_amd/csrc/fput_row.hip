// fput_row.hip -- launchers of the FPU kernels: component rows for up to
// four deviation vectors, vector rows (up to 4N vectors) otherwise.
#include "fput_crow.h"
#include "fput_row.h"

namespace chx {

namespace {
template <int N>
hipError_t launch_n(int M, const StepArgs &a, hipStream_t s) {
  if (M <= 4) {
    // 16 rows (orbits) per 256-thread block
    const unsigned grid = (unsigned)((a.n + 15) / 16);
    switch (M) {
    case 0:
    case 1: hipLaunchKernelGGL((fput_crow_kernel<N, 1>), dim3(grid), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((fput_crow_kernel<N, 2>), dim3(grid), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((fput_crow_kernel<N, 3>), dim3(grid), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((fput_crow_kernel<N, 4>), dim3(grid), dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
  }
  // vector rows: V = ceil(M / 16) slots per lane and one row per orbit
  // while V N <= 32 (at most 64 doubles of vectors per lane); N = 16 with
  // more than 32 vectors takes two rows per orbit.  M <= 4N, so V <= 2.
  const int V = (M + 15) / 16;
  if (V * N <= 32) {
    const unsigned grid = (unsigned)((a.n + 3) / 4);
    if (V <= 1) {
      hipLaunchKernelGGL((fput_row_kernel<N, 1, 1>), dim3(grid), dim3(64), 0, s, a);
    } else {
      if constexpr (4 * N > 16)
        hipLaunchKernelGGL((fput_row_kernel<N, 2, 1>), dim3(grid), dim3(64), 0, s, a);
      else
        return hipErrorInvalidValue;
    }
  } else {
    if constexpr (N == 16) {
      const unsigned grid = (unsigned)((a.n + 1) / 2);
      hipLaunchKernelGGL((fput_row_kernel<N, 2, 2>), dim3(grid), dim3(64), 0, s, a);
    } else {
      return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}
}  // namespace

bool fput_row_supported(int ndof, int M, int n_l, bool sali) {
  if (!(ndof == 2 || ndof == 4 || ndof == 8 || ndof == 16)) return false;
  if (M < 0 || M > 4 * ndof) return false;
  // vector rows keep the SALI pair in lanes 0 and 1 of one slot
  if (M > 4 && sali && n_l % 16 != 0) return false;
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
