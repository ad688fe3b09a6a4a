// prep.hip -- set-up and output kernels of the ensemble: stream compaction
// of the mask, initial-condition assembly (Henon-Heiles section grid, FPU
// normal-mode states, quartic states), the t = 0 state of every orbit
// (deviation vectors, accumulators) and the final outputs.
//
// All of these run once per call and touch each orbit a handful of times;
// they are memory-latency bound and tiny next to the integration kernels.
#include <math.h>

#include "chx_internal.h"
#include "device_math.h"
#include "fput_sys.h"
#include "systems.h"
#include "systems_dp.h"

namespace chx {

namespace {

constexpr int TPB = 256;

inline unsigned blocks_for(int64_t n, int tpb = TPB) {
  return (unsigned)((n + tpb - 1) / tpb);
}

// ---- SplitMix64 (Steele, Lea, Flood 2014), counter based ----------------
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ inline uint64_t rng_key(uint64_t seed, uint64_t stream) {
  return mix64(seed ^ mix64(stream + 1));
}
__device__ inline double rng_uniform(uint64_t key, uint64_t k) {
  const uint64_t z = mix64(key + (k + 1) * 0x9E3779B97F4A7C15ull);
  return (double)(z >> 11) * 0x1.0p-53;
}
// Box-Muller, cosine branch (Box and Muller 1958).
__device__ inline double rng_normal(uint64_t key, uint64_t e) {
  const double u1 = rng_uniform(key, 2 * e), u2 = rng_uniform(key, 2 * e + 1);
  return sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * M_PI * u2);
}

// ---- system dispatch for the non-hot kernels ----------------------------
__device__ inline void sys_force(int sys, int N, const double *q, const double *prm,
                                 double *F) {
  switch (sys) {
  case SYS_HH: SysHH::force(q, F, prm); return;
  case SYS_FPUT: fput_force(q, N, prm, F); return;
  case SYS_QUARTIC:
    if (N == 1) SysQuartic<1>::force(q, F, prm);
    else if (N == 2) SysQuartic<2>::force(q, F, prm);
    else SysQuartic<3>::force(q, F, prm);
    return;
  case SYS_HARMONIC:
    if (N == 1) SysHarmonic<1>::force(q, F, prm);
    else if (N == 2) SysHarmonic<2>::force(q, F, prm);
    else SysHarmonic<3>::force(q, F, prm);
    return;
  }
}
__device__ inline double sys_potential(int sys, int N, const double *q, const double *prm) {
  switch (sys) {
  case SYS_HH: return SysHH::potential(q, prm);
  case SYS_FPUT: return fput_potential(q, N, prm);
  case SYS_QUARTIC:
    return N == 1 ? SysQuartic<1>::potential(q, prm)
         : N == 2 ? SysQuartic<2>::potential(q, prm) : SysQuartic<3>::potential(q, prm);
  case SYS_HARMONIC:
    return N == 1 ? SysHarmonic<1>::potential(q, prm)
         : N == 2 ? SysHarmonic<2>::potential(q, prm) : SysHarmonic<3>::potential(q, prm);
  }
  return NAN;
}

constexpr int MAXD = 32;  // 2N for N <= 16

// ---- t = 0 state ----------------------------------------------------------
__global__ void init_kernel(StepArgs a, InitArgs ia) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int N = ia.ndof, D = 2 * N;
  const int64_t P = a.pitch, j = ia.idx[i];
  double x[MAXD];
  bool finite = true;
  for (int c = 0; c < D; ++c) {
    x[c] = ia.x0[j * D + c];
    finite = finite && isfinite(x[c]);
    a.x[c * P + i] = x[c];
  }
  const int M = ia.m_s + ia.n_l;
  // SALI/GALI set: caller vectors or SplitMix64/Box-Muller normals drawn at
  // counter (j*m_s + v)*D + c of stream 0, normalised to unit length.
  const uint64_t key = rng_key(ia.seed, 0);
  for (int v = 0; v < ia.m_s; ++v) {
    double r2 = 0.0;
    for (int c = 0; c < D; ++c) {
      const double e = ia.w0 ? ia.w0[(j * ia.m_s + v) * D + c]
                             : rng_normal(key, (uint64_t)((j * ia.m_s + v) * D + c));
      a.w[((int64_t)v * D + c) * P + i] = e;
      r2 += e * e;
    }
    const double r = sqrt(r2);
    for (int c = 0; c < D; ++c) a.w[((int64_t)v * D + c) * P + i] /= r;
  }
  // Lyapunov set: canonical basis e_1..e_{n_l}.
  for (int v = 0; v < ia.n_l; ++v)
    for (int c = 0; c < D; ++c)
      a.w[((int64_t)(ia.m_s + v) * D + c) * P + i] = (c == v) ? 1.0 : 0.0;
  for (int v = 0; v < M; ++v) {
    a.gm[v * P + i] = 1.0;
    a.ge[v * P + i] = 0;
  }
  double gprev = 0.0, H0 = 0.0;
  if (finite && ia.sys == SYS_DP) {
    // not separable: H from its own formula, the LD integrand from the field
    double f[4], rec[SysDP::NREC];
    SysDP::rhs_rec(x, f, rec, ia.prm);
    H0 = SysDP::hamiltonian(x, ia.prm);
    if (ia.ind & CHX_IND_LD)
      for (int c = 0; c < 4; ++c)
        gprev += (ia.ld_p == 0.5) ? sqrt(fabs(f[c])) : pow(fabs(f[c]), ia.ld_p);
  } else if (finite) {
    double F[MAXD / 2];
    sys_force(ia.sys, N, x, ia.prm, F);
    double kin = 0.0;
    for (int r = 0; r < N; ++r) kin += x[N + r] * x[N + r];
    H0 = 0.5 * kin + sys_potential(ia.sys, N, x, ia.prm);
    if (ia.ind & CHX_IND_LD) {
      for (int r = 0; r < N; ++r) {
        gprev += (ia.ld_p == 0.5) ? sqrt(fabs(x[N + r])) : pow(fabs(x[N + r]), ia.ld_p);
        gprev += (ia.ld_p == 0.5) ? sqrt(fabs(F[r])) : pow(fabs(F[r]), ia.ld_p);
      }
    }
  }
  a.sc[SC_LD * P + i] = 0.0;
  a.sc[SC_GPREV * P + i] = gprev;
  a.sc[SC_SALI_MIN2 * P + i] = INFINITY;
  a.sc[SC_SALI_LAST2 * P + i] = NAN;
  a.sc[SC_T_CHAOS * P + i] = NAN;
  a.sc[SC_EERR * P + i] = 0.0;
  a.sc[SC_H0 * P + i] = H0;
  a.sc[SC_T_END * P + i] = 0.0;
  a.sc[SC_H * P + i] = 0.0;
  a.sc[SC_REJ * P + i] = 0.0;
  a.sc[SC_NACC * P + i] = 0.0;
  a.sc[SC_NREJ * P + i] = 0.0;
  a.sc[SC_ERR_MAX * P + i] = 0.0;
  a.sc[SC_ERR_LAST * P + i] = 0.0;
  a.st[i] = finite ? CHX_ORBIT_OK : CHX_ORBIT_NONFINITE;
}

// ---- outputs --------------------------------------------------------------
__global__ void finalize_kernel(StepArgs a, OutArgs o, int N, double *gscratch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int D = 2 * N;
  const int64_t P = a.pitch, j = o.idx[i];
  const int st = a.st[i];
  const bool bad = (st == CHX_ORBIT_NONFINITE || st == CHX_ORBIT_STEP_FAILED);
  const double te = a.sc[SC_T_END * P + i];
  const chx_result &r = o.r;
  if (r.x_final)
    for (int c = 0; c < D; ++c) r.x_final[j * D + c] = a.x[c * P + i];
  if (r.t_end) r.t_end[j] = te;
  if (r.status) r.status[j] = st;
  const double smin = sqrt(a.sc[SC_SALI_MIN2 * P + i]);
  if (r.label) {
    int8_t lb;
    if (st == CHX_ORBIT_NONFINITE || st == CHX_ORBIT_STEP_FAILED) lb = 3;
    else if (st == CHX_ORBIT_ESCAPED) lb = 2;
    else lb = (o.sali && smin < o.thr) ? 1 : 0;
    r.label[j] = lb;
  }
  if (r.sali_final) r.sali_final[j] = bad ? NAN : sqrt(a.sc[SC_SALI_LAST2 * P + i]);
  if (r.sali_min) r.sali_min[j] = bad ? NAN : smin;
  if (r.t_chaos) r.t_chaos[j] = bad ? NAN : a.sc[SC_T_CHAOS * P + i];
  if (r.ld) r.ld[j] = bad ? NAN : a.sc[SC_LD * P + i];
  if (r.energy_err) r.energy_err[j] = bad ? NAN : a.sc[SC_EERR * P + i];
  if (r.steps) {
    r.steps[2 * j] = (int64_t)a.sc[SC_NACC * P + i];
    r.steps[2 * j + 1] = (int64_t)a.sc[SC_NREJ * P + i];
  }
  if (r.step_err) {
    r.step_err[2 * j] = a.sc[SC_ERR_MAX * P + i];
    r.step_err[2 * j + 1] = a.sc[SC_ERR_LAST * P + i];
  }
  const double LN2 = 0.69314718055994530942;
  if (r.ln_growth)
    for (int v = 0; v < a.m_s; ++v)
      r.ln_growth[j * a.m_s + v] =
          bad ? NAN : 0.5 * (log(a.gm[v * P + i]) + (double)a.ge[v * P + i] * LN2);
  if (r.lyap)
    for (int v = 0; v < a.n_l; ++v) {
      const int k = a.m_s + v;
      const double g = 0.5 * (log(a.gm[k * P + i]) + (double)a.ge[k * P + i] * LN2);
      r.lyap[j * a.n_l + v] = (bad || !(te > 0.0)) ? NAN : g / te;
    }
  if (r.gali && o.gali_kmax >= 2) {
    const int km = o.gali_kmax;
    double *g = r.gali + j * (km - 1);
    if (bad) {
      for (int k = 2; k <= km; ++k) g[k - 2] = NAN;
      return;
    }
    // GALI_k = product of the diagonal of R in a modified Gram-Schmidt QR of
    // the k leading unit vectors (the volume the singular values give).
    double *u = gscratch + i * (int64_t)km * D;
    double prod = 1.0;
    for (int v = 0; v < km; ++v) {
      double r2 = 0.0;
      for (int c = 0; c < D; ++c) {
        const double e = a.w[((int64_t)v * D + c) * P + i];
        u[v * D + c] = e;
        r2 += e * e;
      }
      const double rn = sqrt(r2);
      for (int c = 0; c < D; ++c) u[v * D + c] /= rn;
      for (int l = 0; l < v; ++l) {
        double d = 0.0;
        for (int c = 0; c < D; ++c) d += u[l * D + c] * u[v * D + c];
        for (int c = 0; c < D; ++c) u[v * D + c] -= d * u[l * D + c];
      }
      double rr = 0.0;
      for (int c = 0; c < D; ++c) rr += u[v * D + c] * u[v * D + c];
      const double rj = sqrt(rr);
      for (int c = 0; c < D; ++c) u[v * D + c] /= rj;
      prod *= rj;
      if (v >= 1) g[v - 1] = prod;
    }
  }
}

__global__ void masked_fill_kernel(const double *x0, const uint8_t *mask, int64_t n, int N,
                                   OutArgs o, int m_s, int n_l) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || mask[j]) return;
  const int D = 2 * N;
  const chx_result &r = o.r;
  if (r.x_final)
    for (int c = 0; c < D; ++c) r.x_final[j * D + c] = x0[j * D + c];
  if (r.t_end) r.t_end[j] = 0.0;
  if (r.status) r.status[j] = CHX_ORBIT_MASKED;
  if (r.label) r.label[j] = -1;
  if (r.sali_final) r.sali_final[j] = NAN;
  if (r.sali_min) r.sali_min[j] = NAN;
  if (r.t_chaos) r.t_chaos[j] = NAN;
  if (r.ld) r.ld[j] = NAN;
  if (r.energy_err) r.energy_err[j] = NAN;
  if (r.steps) r.steps[2 * j] = r.steps[2 * j + 1] = 0;
  if (r.step_err) r.step_err[2 * j] = r.step_err[2 * j + 1] = NAN;
  if (r.ln_growth)
    for (int v = 0; v < m_s; ++v) r.ln_growth[j * m_s + v] = NAN;
  if (r.lyap)
    for (int v = 0; v < n_l; ++v) r.lyap[j * n_l + v] = NAN;
  if (r.gali && o.gali_kmax >= 2)
    for (int k = 0; k < o.gali_kmax - 1; ++k) r.gali[j * (o.gali_kmax - 1) + k] = NAN;
}

// ---- stream compaction -----------------------------------------------------
constexpr int CBLK = 1024;  // elements per compaction block (256 threads x 4)

__global__ void compact_count_kernel(const uint8_t *mask, int64_t n, int64_t *counts) {
  __shared__ int part[TPB / 64];
  const int64_t base = (int64_t)blockIdx.x * CBLK;
  int c = 0;
  for (int k = 0; k < 4; ++k) {
    const int64_t e = base + k * TPB + threadIdx.x;
    c += (e < n && (!mask || mask[e])) ? 1 : 0;
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < TPB / 64; ++w) t += part[w];
    counts[blockIdx.x] = t;
  }
}

// One block: exclusive scan of the per-block counts, total into *count.
__global__ void compact_scan_kernel(int64_t *counts, int64_t nb, int64_t *count) {
  __shared__ int64_t tot[TPB];
  const int64_t per = (nb + TPB - 1) / TPB;
  const int64_t lo = threadIdx.x * per, hi = (lo + per < nb) ? lo + per : nb;
  int64_t s = 0;
  for (int64_t b = lo; b < hi; ++b) s += counts[b];
  tot[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int t = 0; t < TPB; ++t) {
      const int64_t v = tot[t];
      tot[t] = run;
      run += v;
    }
    *count = run;
  }
  __syncthreads();
  int64_t run = tot[threadIdx.x];
  for (int64_t b = lo; b < hi; ++b) {
    const int64_t v = counts[b];
    counts[b] = run;
    run += v;
  }
}

__global__ void compact_scatter_kernel(const uint8_t *mask, int64_t n, const int64_t *offs,
                                       int64_t *idx) {
  __shared__ int wsum[4 * (TPB / 64)];
  const int64_t base = (int64_t)blockIdx.x * CBLK;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // element order inside the block: k-major (k = 0..3), then thread
  bool f[4];
  int wpre[4];
  for (int k = 0; k < 4; ++k) {
    const int64_t e = base + k * TPB + threadIdx.x;
    f[k] = (e < n && (!mask || mask[e]));
    const uint64_t b = __ballot(f[k]);
    wpre[k] = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[k * (TPB / 64) + wv] = __popcll(b);
  }
  __syncthreads();
  int64_t o = offs[blockIdx.x];
  for (int k = 0; k < 4; ++k) {
    int before = 0;
    for (int q = 0; q < k * (TPB / 64) + wv; ++q) before += wsum[q];
    if (f[k]) idx[o + before + wpre[k]] = base + k * TPB + threadIdx.x;
  }
}

// ---- subsets of an ensemble ------------------------------------------------
// flag[k] = keep[idx[k]] (k over the active columns)
__global__ void keep_flags_kernel(const uint8_t *keep, const int64_t *idx, int64_t n,
                                  uint8_t *flag) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) flag[k] = keep[idx[k]] ? 1 : 0;
}

// dst[r][j] = src[r][kpos[j]] for rows r (blockIdx.y) and new columns j
template <class T>
__global__ void gather_columns_kernel(const T *src, int64_t ps, T *dst, int64_t pd,
                                      const int64_t *kpos, int64_t n2) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (j < n2) dst[r * pd + j] = src[r * ps + kpos[j]];
}

// x0_out[j] = x0[idx[kpos[j]]] (rows of D values), orbit_out[j] = idx[kpos[j]]
__global__ void gather_x0_kernel(const double *x0, int D, const int64_t *idx,
                                 const int64_t *kpos, int64_t n2, double *x0_out,
                                 int64_t *orbit_out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n2) return;
  const int64_t o = idx[kpos[j]];
  for (int c = 0; c < D; ++c) x0_out[j * D + c] = x0[o * D + c];
  if (orbit_out) orbit_out[j] = o;
}

__global__ void iota_kernel(int64_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

// ---- initial conditions ----------------------------------------------------
// Henon-Heiles section x = 0: H = (px^2 + py^2)/2 + y^2/2 - y^3/3 there, so
// px^2 = 2E - py^2 - y^2 + 2 y^3/3; px >= 0; negative: inaccessible.
__device__ inline void hh_section_point(double E, double y, double py, double *x,
                                        uint8_t *m) {
  const double r = 2.0 * E - py * py - y * y + (2.0 / 3.0) * y * y * y;
  x[0] = 0.0;
  x[1] = y;
  x[3] = py;
  const bool ok = r >= 0.0;
  x[2] = ok ? sqrt(r) : 0.0;
  *m = ok ? 1 : 0;
}

__global__ void hh_grid_kernel(double E, double y0, double y1, int ny, double py0,
                               double py1, int npy, double *x0, uint8_t *mask) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= (int64_t)ny * npy) return;
  const int i = (int)(o % ny), j = (int)(o / ny);
  const double y = (ny > 1) ? y0 + (y1 - y0) * (double)i / (double)(ny - 1) : y0;
  const double py = (npy > 1) ? py0 + (py1 - py0) * (double)j / (double)(npy - 1) : py0;
  hh_section_point(E, y, py, x0 + 4 * o, mask + o);
}

__global__ void hh_points_kernel(double E, const double *y, const double *py, int64_t n,
                                 double *x0, uint8_t *mask) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  hh_section_point(E, y[o], py[o], x0 + 4 * o, mask + o);
}

struct Prm16 {
  double v[16];
};

// FPU chain, energy in the two lowest normal modes of the fixed-end linear
// chain: Q_k = a_k cos(phi_k)/omega_k, P_k = a_k sin(phi_k), k = 1, 2,
// omega_k = 2 sin(k pi / (2 (N+1))), mapped to (q, p) by the sine
// transform sqrt(2/(N+1)) sin(i k pi/(N+1)), then scaled by s with
// H(s q, s p) = E (s^2 H2 + s^3 H3 + s^4 H4 = E).
__global__ void fput_ic_kernel(int N, Prm16 prm, const double *u, int64_t n, double *x0) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const double *uu = u + 5 * o;
  const double E = 0.1 + 9.9 * uu[0];
  double Qm[2], Pm[2];
  for (int k = 1; k <= 2; ++k) {
    const double om = 2.0 * sin((double)k * M_PI / (2.0 * (double)(N + 1)));
    const double ph = 2.0 * M_PI * uu[k + 2];
    Qm[k - 1] = uu[k] * cos(ph) / om;
    Pm[k - 1] = uu[k] * sin(ph);
  }
  double *q = x0 + o * 2 * N, *p = q + N;
  const double nrm = sqrt(2.0 / (double)(N + 1));
  for (int i = 1; i <= N; ++i) {
    const double s1 = sin((double)i * M_PI / (double)(N + 1));
    const double s2 = sin((double)(2 * i) * M_PI / (double)(N + 1));
    q[i - 1] = nrm * (Qm[0] * s1 + Qm[1] * s2);
    p[i - 1] = nrm * (Pm[0] * s1 + Pm[1] * s2);
  }
  double h2 = 0.0, h3 = 0.0, h4 = 0.0;
  for (int i = 0; i < N; ++i) h2 += 0.5 * p[i] * p[i];
  for (int j = 1; j <= N + 1; ++j) {
    const double d = fput_qw(q, N, j) - fput_qw(q, N, j - 1);
    const double d2 = d * d;
    h2 += 0.5 * prm.v[0] * d2;
    h3 += (prm.v[1] / 3.0) * d2 * d;
    h4 += 0.25 * prm.v[2] * d2 * d2;
  }
  double s;
  if (h3 == 0.0 && h4 > 0.0) {
    s = sqrt(2.0 * E / (h2 + sqrt(h2 * h2 + 4.0 * h4 * E)));
  } else if (h3 == 0.0 && h4 == 0.0) {
    s = sqrt(E / h2);
  } else {
    s = sqrt(E / h2);
    for (int it = 0; it < 100; ++it) {
      const double f = s * s * (h2 + s * (h3 + s * h4)) - E;
      const double fp = s * (2.0 * h2 + s * (3.0 * h3 + 4.0 * s * h4));
      const double ds = f / fp;
      s -= ds;
      if (fabs(ds) <= 1e-16 * fabs(s)) break;
    }
  }
  for (int i = 0; i < N; ++i) {
    q[i] *= s;
    p[i] *= s;
  }
}

// Coupled quartic oscillator at H = 1: V is homogeneous of degree 4, so the
// point of potential f on the ray of the unit direction u is (f/V(u))^(1/4) u.
__global__ void quartic_ic_kernel(int N, Prm16 prm, const double *draws, int64_t n,
                                  double *x0) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const double *dr = draws + o * (2 * N + 1);
  double u[3], e[3], nu = 0.0, ne = 0.0;
  for (int i = 0; i < N; ++i) {
    nu += dr[i] * dr[i];
    ne += dr[N + i] * dr[N + i];
  }
  nu = sqrt(nu);
  ne = sqrt(ne);
  for (int i = 0; i < N; ++i) {
    u[i] = dr[i] / nu;
    e[i] = dr[N + i] / ne;
  }
  const double f = dr[2 * N];
  double V;
  if (N == 1) V = SysQuartic<1>::potential(u, prm.v);
  else if (N == 2) V = SysQuartic<2>::potential(u, prm.v);
  else V = SysQuartic<3>::potential(u, prm.v);
  const double s = sqrt(sqrt(f / V));
  const double pm = sqrt(2.0 * (1.0 - f));
  double *q = x0 + o * 2 * N, *p = q + N;
  for (int i = 0; i < N; ++i) {
    q[i] = s * u[i];
    p[i] = pm * e[i];
  }
}

}  // namespace

hipError_t launch_init(const StepArgs &a, const InitArgs &ia, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(init_kernel, dim3(blocks_for(a.n)), dim3(TPB), 0, s, a, ia);
  return hipGetLastError();
}

hipError_t launch_finalize(const StepArgs &a, const OutArgs &oa, int ndof, double *given,
                           hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  double *scratch = nullptr;
  hipError_t e;
  if (oa.r.gali && oa.gali_kmax >= 2) {
    if (given) {
      scratch = given;
    } else {
      e = hipMallocAsync((void **)&scratch,
                         sizeof(double) * (size_t)a.n * oa.gali_kmax * 2 * ndof, s);
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(finalize_kernel, dim3(blocks_for(a.n)), dim3(TPB), 0, s, a, oa, ndof,
                     scratch);
  e = hipGetLastError();
  if (scratch && scratch != given) {
    hipError_t e2 = hipFreeAsync(scratch, s);
    if (e == hipSuccess) e = e2;
  }
  return e;
}

hipError_t launch_masked_fill(const double *x0, const uint8_t *mask, int64_t n_all, int ndof,
                              const OutArgs &oa, int m_s, int n_l, hipStream_t s) {
  if (!mask || n_all == 0) return hipSuccess;
  hipLaunchKernelGGL(masked_fill_kernel, dim3(blocks_for(n_all)), dim3(TPB), 0, s, x0, mask,
                     n_all, ndof, oa, m_s, n_l);
  return hipGetLastError();
}

hipError_t launch_keep_flags(const uint8_t *keep, const int64_t *idx, int64_t n, uint8_t *flag,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(keep_flags_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, keep, idx, n, flag);
  return hipGetLastError();
}

hipError_t launch_gather_columns(const double *src, int64_t ps, double *dst, int64_t pd, int rows,
                                 const int64_t *kpos, int64_t n2, hipStream_t s) {
  if (n2 == 0 || rows == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_columns_kernel<double>, dim3(blocks_for(n2), (unsigned)rows),
                     dim3(TPB), 0, s, src, ps, dst, pd, kpos, n2);
  return hipGetLastError();
}

hipError_t launch_gather_columns_i(const int *src, int64_t ps, int *dst, int64_t pd, int rows,
                                   const int64_t *kpos, int64_t n2, hipStream_t s) {
  if (n2 == 0 || rows == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_columns_kernel<int>, dim3(blocks_for(n2), (unsigned)rows), dim3(TPB),
                     0, s, src, ps, dst, pd, kpos, n2);
  return hipGetLastError();
}

hipError_t launch_gather_x0(const double *x0, int D, const int64_t *idx, const int64_t *kpos,
                            int64_t n2, double *x0_out, int64_t *orbit_out, hipStream_t s) {
  if (n2 == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_x0_kernel, dim3(blocks_for(n2)), dim3(TPB), 0, s, x0, D, idx, kpos,
                     n2, x0_out, orbit_out);
  return hipGetLastError();
}

hipError_t launch_iota(int64_t *p, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(iota_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, p, n);
  return hipGetLastError();
}

int64_t compact_scratch_len(int64_t n) { return (n + CBLK - 1) / CBLK + 1; }

hipError_t launch_compact(const uint8_t *mask, int64_t n, int64_t *idx, int64_t *count,
                          int64_t *scratch, hipStream_t s) {
  const int64_t nb = (n + CBLK - 1) / CBLK;
  if (nb == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(compact_count_kernel, dim3((unsigned)nb), dim3(TPB), 0, s, mask, n,
                     scratch);
  hipLaunchKernelGGL(compact_scan_kernel, dim3(1), dim3(TPB), 0, s, scratch, nb, count);
  hipLaunchKernelGGL(compact_scatter_kernel, dim3((unsigned)nb), dim3(TPB), 0, s, mask, n,
                     scratch, idx);
  return hipGetLastError();
}

hipError_t launch_hh_grid(double E, double y0, double y1, int ny, double py0, double py1,
                          int npy, double *x0, uint8_t *mask, hipStream_t s) {
  const int64_t n = (int64_t)ny * npy;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(hh_grid_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, E, y0, y1, ny, py0,
                     py1, npy, x0, mask);
  return hipGetLastError();
}

hipError_t launch_hh_points(double E, const double *y, const double *py, int64_t n, double *x0,
                            uint8_t *mask, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(hh_points_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, E, y, py, n, x0,
                     mask);
  return hipGetLastError();
}

hipError_t launch_fput_ic(int ndof, const double *prm, const double *u, int64_t n, double *x0,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  Prm16 p{};
  for (int k = 0; k < 3; ++k) p.v[k] = prm[k];
  hipLaunchKernelGGL(fput_ic_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, ndof, p, u, n, x0);
  return hipGetLastError();
}

hipError_t launch_quartic_ic(int ndof, const double *prm, const double *draws, int64_t n,
                             double *x0, hipStream_t s) {
  if (n == 0) return hipSuccess;
  Prm16 p{};
  p.v[0] = prm[0];
  hipLaunchKernelGGL(quartic_ic_kernel, dim3(blocks_for(n)), dim3(TPB), 0, s, ndof, p, draws,
                     n, x0);
  return hipGetLastError();
}

}  // namespace chx
