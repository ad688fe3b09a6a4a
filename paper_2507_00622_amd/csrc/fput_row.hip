// fput_row.hip -- launchers of the FPU kernels: component rows for up to
// four deviation vectors, vector rows (up to 4N vectors) otherwise.
#include "fput_crow.h"
#include "fput_row.h"
#include "fput_rowpair.h"

namespace chx {

namespace {
// Component rows: any N <= 16 (lanes N..15 of the row are zero ghosts, and
// the first ghost is the wall q_{N+1} = 0).
template <int N>
hipError_t launch_crow(int M, const StepArgs &a, hipStream_t s) {
  // 16 rows (orbits) per 256-thread block
  const unsigned grid = (unsigned)((a.n + 15) / 16);
  switch (M) {
  case 0: hipLaunchKernelGGL((fput_crow_kernel<N, 0>), dim3(grid), dim3(256), 0, s, a); break;
  case 1: hipLaunchKernelGGL((fput_crow_kernel<N, 1>), dim3(grid), dim3(256), 0, s, a); break;
  case 2: hipLaunchKernelGGL((fput_crow_kernel<N, 2>), dim3(grid), dim3(256), 0, s, a); break;
  case 3: hipLaunchKernelGGL((fput_crow_kernel<N, 3>), dim3(grid), dim3(256), 0, s, a); break;
  case 4: hipLaunchKernelGGL((fput_crow_kernel<N, 4>), dim3(grid), dim3(256), 0, s, a); break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N>
hipError_t launch_n(int M, const StepArgs &a, hipStream_t s) {
  if (M <= 4) return launch_crow<N>(M, a, s);
  // vector rows: V = ceil(M / 16) slots per lane and one row per orbit
  // while V N <= 32 (at most 64 doubles of vectors per lane), and for
  // N = 16 with 33..48 vectors (three slots, 96 doubles: the full Lyapunov
  // set and N GALI vectors with no slot position unused); N = 16 with more
  // than 48 vectors takes two rows per orbit; N = 8 with 17..24 vectors
  // of which at most N SALI/GALI (the full Lyapunov spectrum and N GALI
  // vectors) puts two orbits in a row, each orbit's Lyapunov set filling one
  // slot.  M <= 4N.
  const int V = (M + 15) / 16;
  if constexpr (N == 8) {
    if (M > 16 && M <= 24 && a.m_s <= 8) {
      const unsigned grid = (unsigned)((a.n + 7) / 8);
      hipLaunchKernelGGL((fput_rowpair_kernel<8>), dim3(grid), dim3(64), 0, s, a);
      return hipGetLastError();
    }
  }
  if constexpr (N == 16) {
    if (V == 3) {
      const unsigned grid = (unsigned)((a.n + 3) / 4);
      hipLaunchKernelGGL((fput_row_kernel<16, 3, 1>), dim3(grid), dim3(64), 0, s, a);
      return hipGetLastError();
    }
  }
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
  if (ndof < 2 || ndof > 16 || M < 0 || M > 4 * ndof) return false;
  // more than four vectors: vector rows, N a power of two
  if (M > 4 && !(ndof == 2 || ndof == 4 || ndof == 8 || ndof == 16)) return false;
  // vector rows keep the SALI pair in lanes 0 and 1 of one slot
  if (M > 4 && sali && n_l % 16 != 0) return false;
  return true;
}

hipError_t launch_fput_row(int ndof, int M, const StepArgs &a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  switch (ndof) {
  case 2: return launch_n<2>(M, a, s);
  case 3: return launch_crow<3>(M, a, s);
  case 4: return launch_n<4>(M, a, s);
  case 5: return launch_crow<5>(M, a, s);
  case 6: return launch_crow<6>(M, a, s);
  case 7: return launch_crow<7>(M, a, s);
  case 8: return launch_n<8>(M, a, s);
  case 9: return launch_crow<9>(M, a, s);
  case 10: return launch_crow<10>(M, a, s);
  case 11: return launch_crow<11>(M, a, s);
  case 12: return launch_crow<12>(M, a, s);
  case 13: return launch_crow<13>(M, a, s);
  case 14: return launch_crow<14>(M, a, s);
  case 15: return launch_crow<15>(M, a, s);
  case 16: return launch_n<16>(M, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace chx
