// fput_crow_rkl.hip -- launchers of the DOP853 kernels (fixed step and
// adaptive) for FPU chains with more than four deviation vectors: component
// rows with the vectors in LDS (fput_crow_rkl.h).
#include "fput_crow_rkl.h"

namespace chx {

namespace {
template <int N>
hipError_t launch_rkl(bool adaptive, const StepArgs &a, hipStream_t s) {
  const int M = a.m_s + a.n_l;
  const size_t lds = rkl::lds_bytes(M, adaptive);
  // four orbits (rows) per 64-thread block
  const unsigned grid = (unsigned)((a.n + 3) / 4);
  const void *k = adaptive ? (const void *)fput_crow_rkla_kernel<N>
                           : (const void *)fput_crow_rkl_kernel<N>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (adaptive)
    hipLaunchKernelGGL((fput_crow_rkla_kernel<N>), dim3(grid), dim3(64), lds, s, a);
  else
    hipLaunchKernelGGL((fput_crow_rkl_kernel<N>), dim3(grid), dim3(64), lds, s, a);
  return hipGetLastError();
}
}  // namespace

size_t fput_rkl_lds_bytes(int M, bool adaptive) { return rkl::lds_bytes(M, adaptive); }

hipError_t launch_fput_crow_rkl(int ndof, bool adaptive, const StepArgs &a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  switch (ndof) {
  case 2: return launch_rkl<2>(adaptive, a, s);
  case 3: return launch_rkl<3>(adaptive, a, s);
  case 4: return launch_rkl<4>(adaptive, a, s);
  case 5: return launch_rkl<5>(adaptive, a, s);
  case 6: return launch_rkl<6>(adaptive, a, s);
  case 7: return launch_rkl<7>(adaptive, a, s);
  case 8: return launch_rkl<8>(adaptive, a, s);
  case 9: return launch_rkl<9>(adaptive, a, s);
  case 10: return launch_rkl<10>(adaptive, a, s);
  case 11: return launch_rkl<11>(adaptive, a, s);
  case 12: return launch_rkl<12>(adaptive, a, s);
  case 13: return launch_rkl<13>(adaptive, a, s);
  case 14: return launch_rkl<14>(adaptive, a, s);
  case 15: return launch_rkl<15>(adaptive, a, s);
  case 16: return launch_rkl<16>(adaptive, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace chx
