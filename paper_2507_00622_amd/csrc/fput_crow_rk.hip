// fput_crow_rk.hip -- launcher of the DOP853 component-row kernels for FPU
// chains (N = 2..16): up to four deviation vectors in registers here, more
// in LDS (fput_crow_rkl.hip).
#include "fput_crow_rk.h"

namespace chx {
hipError_t launch_fput_crow_rka(int ndof, int M, const StepArgs &a, hipStream_t s);
// more than four vectors: the vectors in LDS (fput_crow_rkl.hip)
hipError_t launch_fput_crow_rkl(int ndof, bool adaptive, const StepArgs &a, hipStream_t s);

namespace {
template <int N>
hipError_t launch_rk(int M, const StepArgs &a, hipStream_t s) {
  // 16 rows (orbits) per 256-thread block
  const unsigned grid = (unsigned)((a.n + 15) / 16);
  switch (M) {
  case 0: hipLaunchKernelGGL((fput_crow_rk_kernel<N, 0>), dim3(grid), dim3(256), 0, s, a); break;
  case 1: hipLaunchKernelGGL((fput_crow_rk_kernel<N, 1>), dim3(grid), dim3(256), 0, s, a); break;
  case 2: hipLaunchKernelGGL((fput_crow_rk_kernel<N, 2>), dim3(grid), dim3(256), 0, s, a); break;
  case 3: hipLaunchKernelGGL((fput_crow_rk_kernel<N, 3>), dim3(grid), dim3(256), 0, s, a); break;
  case 4: hipLaunchKernelGGL((fput_crow_rk_kernel<N, 4>), dim3(grid), dim3(256), 0, s, a); break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_fput_crow_rk(int ndof, int M, bool adaptive, const StepArgs &a,
                               hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  if (M > 4) return launch_fput_crow_rkl(ndof, adaptive, a, s);
  if (adaptive) return launch_fput_crow_rka(ndof, M, a, s);
  switch (ndof) {
  case 2: return launch_rk<2>(M, a, s);
  case 3: return launch_rk<3>(M, a, s);
  case 4: return launch_rk<4>(M, a, s);
  case 5: return launch_rk<5>(M, a, s);
  case 6: return launch_rk<6>(M, a, s);
  case 7: return launch_rk<7>(M, a, s);
  case 8: return launch_rk<8>(M, a, s);
  case 9: return launch_rk<9>(M, a, s);
  case 10: return launch_rk<10>(M, a, s);
  case 11: return launch_rk<11>(M, a, s);
  case 12: return launch_rk<12>(M, a, s);
  case 13: return launch_rk<13>(M, a, s);
  case 14: return launch_rk<14>(M, a, s);
  case 15: return launch_rk<15>(M, a, s);
  case 16: return launch_rk<16>(M, a, s);
  }
  return hipErrorInvalidValue;
}
}  // namespace chx
