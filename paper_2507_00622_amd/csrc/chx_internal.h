// chx_internal.h -- declarations shared by the HIP sources of libchx.
//
// Device-resident ensemble layout (structure of arrays, one orbit per
// column, columns padded to a multiple of 64 so every wavefront reads whole
// 512-byte segments):
//   x   [2N][pitch]            phase-space state
//   w   [M][2N][pitch]         deviation vectors: the SALI/GALI set
//                              (m_s vectors) followed by the Lyapunov set
//                              (n_l vectors), M = m_s + n_l
//   gm  [M][pitch], ge [M][pitch]  growth product of squared norms kept as
//                              mantissa (double) and binary exponent (int):
//                              ln-growth = (ln gm + ge ln 2) / 2
//   sc  [NSC][pitch]           scalar accumulators (see Sc below)
//   st  [pitch]                orbit status (CHX_ORBIT_*)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/chx.h"

namespace chx {

enum Sc {
  SC_LD = 0,     // M-function accumulated so far
  SC_GPREV,      // LD integrand at the last step endpoint
  SC_SALI_MIN2,  // min over checkpoints of SALI^2
  SC_SALI_LAST2, // SALI^2 at the last checkpoint
  SC_T_CHAOS,    // first checkpoint time with SALI < threshold (NaN: none)
  SC_EERR,       // max |H - H0|
  SC_H0,         // H at t = 0
  SC_T_END,      // time of the last checkpoint reached
  SC_H,          // adaptive: the step the controller proposes next (0: dt)
  SC_REJ,        // adaptive: 1 if the last attempt was rejected
  SC_NACC,       // adaptive: accepted steps
  SC_NREJ,       // adaptive: rejected steps
  SC_ERR_MAX,    // adaptive: largest error estimate of an accepted step
  SC_ERR_LAST,   // adaptive: error estimate of the last accepted step
  NSC
};

enum SysKind { SYS_HH = 1, SYS_FPUT = 2, SYS_QUARTIC = 3, SYS_HARMONIC = 4, SYS_DP = 5 };

// Everything one integration launch needs (passed by value).
struct StepArgs {
  double *x;
  double *w;
  double *gm;
  int *ge;
  double *sc;
  int *st;
  int64_t n;        // orbits in the ensemble (columns in use)
  int64_t pitch;    // column stride (multiple of 64)
  int64_t s_begin;  // steps already done
  int64_t s_end;    // advance to this step (a checkpoint step)
  int64_t n_total;  // steps of the whole run
  int K;            // checkpoint period
  int m_s;          // SALI/GALI vectors (the first m_s of w)
  int n_l;          // Lyapunov vectors (the next n_l)
  uint32_t ind;     // CHX_IND_* bits
  int early_exit;
  double dt;
  double thr2;      // SALI threshold squared
  double escape_r2; // 0 = off
  double ld_p;      // LD exponent
  double rtol, atol; // adaptive DOP8(5) tolerances
  double prm[16];   // system parameters
};

// Launchers of the integration kernels (one per source file).
hipError_t launch_lane(int sys, int ndof, int M, const StepArgs &a, int block,
                       hipStream_t s);
// largest ndof of a system compiled at run time from the caller's source
#define CHX_CUSTOM_MAX_NDOF 8
bool lane_supported(int sys, int ndof, int M);
hipError_t launch_lane_rk(int sys, int ndof, int M, bool adaptive, const StepArgs &a,
                          int block, hipStream_t s);
hipError_t launch_fput_row(int ndof, int M, const StepArgs &a, hipStream_t s);
bool fput_row_supported(int ndof, int M, int n_l, bool sali);

// Preparation and output kernels (prep.hip).
struct InitArgs {
  const double *x0;     // [n_all][2N] caller layout
  const int64_t *idx;   // [n] active -> caller index
  const double *w0;     // [n_all][m_s][2N] or null
  uint64_t seed;
  int sys, ndof, m_s, n_l;
  uint32_t ind;
  double ld_p;
  double prm[16];
};
hipError_t launch_init(const StepArgs &a, const InitArgs &ia, hipStream_t s);

struct OutArgs {
  const int64_t *idx;   // active -> caller index
  chx_result r;         // caller outputs (device pointers)
  int gali_kmax;        // 0 = GALI not requested
  int sali;             // SALI requested
  double thr;
};
// scratch: a.n * gali_kmax * 2N doubles for the GALI QR when GALI is an
// output, or null to allocate them for the call.
hipError_t launch_finalize(const StepArgs &a, const OutArgs &oa, int ndof, double *scratch,
                           hipStream_t s);
hipError_t launch_masked_fill(const double *x0, const uint8_t *mask, int64_t n_all,
                              int ndof, const OutArgs &oa, int m_s, int n_l,
                              hipStream_t s);

// Stream compaction of the mask: writes idx[] (active caller indices, in
// order) and *count (device).  scratch must hold compact_scratch_len(n)
// int64 values.
int64_t compact_scratch_len(int64_t n);
hipError_t launch_compact(const uint8_t *mask, int64_t n, int64_t *idx,
                          int64_t *count, int64_t *scratch, hipStream_t s);

// Subsets of an ensemble (prep.hip): flag[k] = keep[idx[k]]; column
// gathers dst[r][j] = src[r][kpos[j]] for r < rows; x0 rows of the kept
// orbits and their caller indices; p[i] = i.
hipError_t launch_keep_flags(const uint8_t *keep, const int64_t *idx, int64_t n, uint8_t *flag,
                             hipStream_t s);
hipError_t launch_gather_columns(const double *src, int64_t ps, double *dst, int64_t pd, int rows,
                                 const int64_t *kpos, int64_t n2, hipStream_t s);
hipError_t launch_gather_columns_i(const int *src, int64_t ps, int *dst, int64_t pd, int rows,
                                   const int64_t *kpos, int64_t n2, hipStream_t s);
hipError_t launch_gather_x0(const double *x0, int D, const int64_t *idx, const int64_t *kpos,
                            int64_t n2, double *x0_out, int64_t *orbit_out, hipStream_t s);
hipError_t launch_iota(int64_t *p, int64_t n, hipStream_t s);

hipError_t launch_hh_grid(double E, double y0, double y1, int ny, double py0,
                          double py1, int npy, double *x0, uint8_t *mask,
                          hipStream_t s);
hipError_t launch_hh_points(double E, const double *y, const double *py, int64_t n,
                            double *x0, uint8_t *mask, hipStream_t s);
hipError_t launch_fput_ic(int ndof, const double *prm, const double *u, int64_t n,
                          double *x0, hipStream_t s);
hipError_t launch_quartic_ic(int ndof, const double *prm, const double *draws,
                             int64_t n, double *x0, hipStream_t s);

}  // namespace chx
