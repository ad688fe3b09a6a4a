/*
 * chx_oracle.c -- the oracle (plain, slow, scalar FP64).  See chx_oracle.h.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, by the smoke check and by
 * the benchmark's CPU-baseline leg; never by the product path.
 *
 * Compiled with -O2 -ffp-contract=off: no fused multiply-add, operations in
 * the order written.  One initial condition at a time.
 */
#include "chx_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Systems                                                                 */
/* ---------------------------------------------------------------------- */

/* Henon-Heiles (Examples section, Henon-Heiles Hamiltonian):
 *   V(x, y) = (x^2 + y^2)/2 + x^2 y - y^3/3.
 * Its equations of motion give dp_x/dt = -x - 2xy, dp_y/dt = -y - x^2 + y^2,
 * i.e. dV/dx = x + 2xy and dV/dy = y + x^2 - y^2. */
static double hh_V(const double *q) {
  double x = q[0], y = q[1];
  return 0.5 * (x * x + y * y) + x * x * y - y * y * y / 3.0;
}
static void hh_grad(const double *q, double *g) {
  double x = q[0], y = q[1];
  g[0] = x + 2.0 * x * y;
  g[1] = y + x * x - y * y;
}
static void hh_hess(const double *q, double *h) {
  double x = q[0], y = q[1];
  h[0] = 1.0 + 2.0 * y; /* d2V/dx2  */
  h[1] = 2.0 * x;       /* d2V/dxdy */
  h[2] = 2.0 * x;
  h[3] = 1.0 - 2.0 * y; /* d2V/dy2  */
}

/* Fermi-Pasta-Ulam chain (Examples section, FPU Hamiltonian and equations
 * of motion, fixed ends q_0 = q_{N+1} = 0).  Masses i = 1..N, springs
 * j = 1..N+1 with extension d_j = q_j - q_{j-1}:
 *   V = sum_{j=1}^{N+1} [ k d_j^2/2 + alpha d_j^3/3 + beta d_j^4/4 ].
 * The printed potential sums j = 1..N over (q_{j+1} - q_j); the printed
 * equations of motion contain the wall spring d_1 = q_1 - q_0 as well, so the
 * sum here runs over all N+1 springs, consistent with the equations.
 *   dV/dq_i = phi'(d_i) - phi'(d_{i+1}),  phi'(d) = k d + alpha d^2 + beta d^3.
 * Arrays here are 0-based: q[i-1] is mass i. */
static double fput_qm(const double *q, int N, int j) { /* q_j with walls */
  if (j <= 0 || j >= N + 1) return 0.0;
  return q[j - 1];
}
static double fput_V(int N, const double *pr, const double *q) {
  double k = pr[0], a = pr[1], b = pr[2], v = 0.0;
  for (int j = 1; j <= N + 1; ++j) {
    double d = fput_qm(q, N, j) - fput_qm(q, N, j - 1);
    v += k * d * d / 2.0 + a * d * d * d / 3.0 + b * d * d * d * d / 4.0;
  }
  return v;
}
static double fput_dphi(const double *pr, double d) {
  return pr[0] * d + pr[1] * d * d + pr[2] * d * d * d;
}
static double fput_ddphi(const double *pr, double d) {
  return pr[0] + 2.0 * pr[1] * d + 3.0 * pr[2] * d * d;
}
static void fput_grad(int N, const double *pr, const double *q, double *g) {
  for (int i = 1; i <= N; ++i) {
    double dl = fput_qm(q, N, i) - fput_qm(q, N, i - 1);
    double dr = fput_qm(q, N, i + 1) - fput_qm(q, N, i);
    g[i - 1] = fput_dphi(pr, dl) - fput_dphi(pr, dr);
  }
}
static void fput_hess(int N, const double *pr, const double *q, double *h) {
  for (int i = 0; i < N * N; ++i) h[i] = 0.0;
  for (int i = 1; i <= N; ++i) {
    double dl = fput_qm(q, N, i) - fput_qm(q, N, i - 1);
    double dr = fput_qm(q, N, i + 1) - fput_qm(q, N, i);
    h[(i - 1) * N + (i - 1)] = fput_ddphi(pr, dl) + fput_ddphi(pr, dr);
    if (i < N) {
      h[(i - 1) * N + i] = -fput_ddphi(pr, dr);
      h[i * N + (i - 1)] = -fput_ddphi(pr, dr);
    }
  }
}

/* Coupled quartic oscillator: V = sum_i q_i^4/4 + eps sum_{i<j} q_i^2 q_j^2. */
static double quartic_V(int N, const double *pr, const double *q) {
  double eps = pr[0], v = 0.0;
  for (int i = 0; i < N; ++i) v += q[i] * q[i] * q[i] * q[i] / 4.0;
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j) v += eps * q[i] * q[i] * q[j] * q[j];
  return v;
}
static void quartic_grad(int N, const double *pr, const double *q, double *g) {
  double eps = pr[0];
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int j = 0; j < N; ++j)
      if (j != i) s += q[j] * q[j];
    g[i] = q[i] * q[i] * q[i] + 2.0 * eps * q[i] * s;
  }
}
static void quartic_hess(int N, const double *pr, const double *q, double *h) {
  double eps = pr[0];
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int j = 0; j < N; ++j)
      if (j != i) s += q[j] * q[j];
    for (int j = 0; j < N; ++j) {
      if (j == i)
        h[i * N + j] = 3.0 * q[i] * q[i] + 2.0 * eps * s;
      else
        h[i * N + j] = 4.0 * eps * q[i] * q[j];
    }
  }
}

/* Uncoupled harmonic oscillators: V = sum_i omega_i^2 q_i^2 / 2. */
static double harm_V(int N, const double *pr, const double *q) {
  double v = 0.0;
  for (int i = 0; i < N; ++i) v += pr[i] * pr[i] * q[i] * q[i] / 2.0;
  return v;
}
static void harm_grad(int N, const double *pr, const double *q, double *g) {
  for (int i = 0; i < N; ++i) g[i] = pr[i] * pr[i] * q[i];
}
static void harm_hess(int N, const double *pr, const double *q, double *h) {
  (void)q;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) h[i * N + j] = (i == j) ? pr[i] * pr[i] : 0.0;
}

double ora_potential(int kind, int N, const double *pr, const double *q) {
  switch (kind) {
  case ORA_SYS_HENON_HEILES: return hh_V(q);
  case ORA_SYS_FPUT: return fput_V(N, pr, q);
  case ORA_SYS_QUARTIC: return quartic_V(N, pr, q);
  case ORA_SYS_HARMONIC: return harm_V(N, pr, q);
  }
  return NAN;
}
void ora_grad(int kind, int N, const double *pr, const double *q, double *g) {
  switch (kind) {
  case ORA_SYS_HENON_HEILES: hh_grad(q, g); return;
  case ORA_SYS_FPUT: fput_grad(N, pr, q, g); return;
  case ORA_SYS_QUARTIC: quartic_grad(N, pr, q, g); return;
  case ORA_SYS_HARMONIC: harm_grad(N, pr, q, g); return;
  }
}
void ora_hess(int kind, int N, const double *pr, const double *q, double *h) {
  switch (kind) {
  case ORA_SYS_HENON_HEILES: hh_hess(q, h); return;
  case ORA_SYS_FPUT: fput_hess(N, pr, q, h); return;
  case ORA_SYS_QUARTIC: quartic_hess(N, pr, q, h); return;
  case ORA_SYS_HARMONIC: harm_hess(N, pr, q, h); return;
  }
}
double ora_hamiltonian(int kind, int N, const double *pr, const double *x) {
  double t = 0.0;
  for (int i = 0; i < N; ++i) t += x[N + i] * x[N + i];
  return t / 2.0 + ora_potential(kind, N, pr, x);
}

/* ---------------------------------------------------------------------- */
/* Integrator: Yoshida-4 triple jump of kick-drift-kick leapfrog           */
/* ---------------------------------------------------------------------- */

/* w1 = 1/(2 - 2^(1/3)), w0 = -2^(1/3)/(2 - 2^(1/3)), written as the binary64
 * values nearest to the exact real numbers. */
static const double YOSHIDA_W1 = 1.3512071919596575;
static const double YOSHIDA_W0 = -1.7024143839193153;

void ora_yoshida_coefficients(double c[3], double d[4]) {
  /* Composition S(w1 dt) S(w0 dt) S(w1 dt) of the leapfrog
   * S(h) = K(h/2) D(h) K(h/2): drifts w1, w0, w1; kicks w1/2, (w1+w0)/2,
   * (w0+w1)/2, w1/2. */
  c[0] = YOSHIDA_W1;
  c[1] = YOSHIDA_W0;
  c[2] = YOSHIDA_W1;
  d[0] = YOSHIDA_W1 / 2.0;
  d[1] = (YOSHIDA_W1 + YOSHIDA_W0) / 2.0;
  d[2] = (YOSHIDA_W0 + YOSHIDA_W1) / 2.0;
  d[3] = YOSHIDA_W1 / 2.0;
}

/* Kick: p -= h grad V(q); each tangent vector: dp -= h Hess V(q) dq.
 * Drift: q += h p; each tangent vector: dq += h dp.
 * The tangent updates are the exact Jacobian of the state updates, so the
 * deviation vectors follow the variational equations of the discrete map. */
#define ORA_MAX_DOF 64
void ora_step(int kind, int N, const double *pr, double dt, double *x, double *w,
              int m) {
  double c[3], d[4];
  double g[ORA_MAX_DOF], h[ORA_MAX_DOF * ORA_MAX_DOF], hv[ORA_MAX_DOF];
  ora_yoshida_coefficients(c, d);
  double *q = x, *p = x + N;
  for (int k = 0; k < 4; ++k) {
    double hk = d[k] * dt;
    ora_grad(kind, N, pr, q, g);
    ora_hess(kind, N, pr, q, h);
    for (int i = 0; i < N; ++i) p[i] = p[i] - hk * g[i];
    for (int v = 0; v < m; ++v) {
      double *dq = w + (int64_t)v * 2 * N, *dp = dq + N;
      for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int j = 0; j < N; ++j) s += h[i * N + j] * dq[j];
        hv[i] = s;
      }
      for (int i = 0; i < N; ++i) dp[i] = dp[i] - hk * hv[i];
    }
    if (k < 3) {
      double hd = c[k] * dt;
      for (int i = 0; i < N; ++i) q[i] = q[i] + hd * p[i];
      for (int v = 0; v < m; ++v) {
        double *dq = w + (int64_t)v * 2 * N, *dp = dq + N;
        for (int i = 0; i < N; ++i) dq[i] = dq[i] + hd * dp[i];
      }
    }
  }
}

/* ---------------------------------------------------------------------- */
/* Linear algebra                                                          */
/* ---------------------------------------------------------------------- */

static double dot(int n, const double *a, const double *b) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Modified Gram-Schmidt (the QR factorisation used for the Lyapunov
 * spectrum, Functionalities section): vectors processed in order; each
 * projection uses the current, partially orthogonalised vector. */
void ora_mgs(int dim, int m, double *w, double *rdiag) {
  for (int j = 0; j < m; ++j) {
    double *wj = w + (int64_t)j * dim;
    for (int i = 0; i < j; ++i) {
      const double *wi = w + (int64_t)i * dim;
      double r = dot(dim, wi, wj);
      for (int c = 0; c < dim; ++c) wj[c] = wj[c] - r * wi[c];
    }
    double r = sqrt(dot(dim, wj, wj));
    rdiag[j] = r;
    for (int c = 0; c < dim; ++c) wj[c] = wj[c] / r;
  }
}

/* GALI_k (Functionalities section: GALI through the singular values of the
 * matrix of k unit deviation vectors): the product of the k singular values
 * equals the k-volume of the parallelotope the vectors span, which is the
 * product of the diagonal of R in a QR factorisation.  Computed on a copy;
 * nested in k since R's leading block does not depend on later columns. */
void ora_gali(int dim, int m, const double *w, int kmax, double *gali_out) {
  double *cp = (double *)malloc(sizeof(double) * (size_t)dim * (size_t)m);
  double *rd = (double *)malloc(sizeof(double) * (size_t)m);
  memcpy(cp, w, sizeof(double) * (size_t)dim * (size_t)m);
  for (int v = 0; v < m; ++v) {
    double *u = cp + (int64_t)v * dim;
    double r = sqrt(dot(dim, u, u));
    for (int c = 0; c < dim; ++c) u[c] = u[c] / r;
  }
  ora_mgs(dim, m, cp, rd);
  double prod = 1.0;
  for (int k = 1; k <= kmax && k <= m; ++k) {
    prod = prod * rd[k - 1];
    if (k >= 2) gali_out[k - 2] = prod;
  }
  free(cp);
  free(rd);
}

/* ---------------------------------------------------------------------- */
/* Per-orbit state                                                         */
/* ---------------------------------------------------------------------- */

/* Layout of one orbit's state (doubles). */
enum {
  ST_LD = 0,     /* Lagrangian-descriptor M accumulated so far           */
  ST_GPREV,      /* LD integrand at the last step endpoint               */
  ST_SALI_MIN,   /* minimum SALI over checkpoints                        */
  ST_SALI_LAST,  /* SALI at the last checkpoint                          */
  ST_T_CHAOS,    /* first checkpoint time with SALI < threshold, or NaN  */
  ST_EERR,       /* max |H - H0| over checkpoints                        */
  ST_H0,         /* H at t = 0                                           */
  ST_STATUS,     /* status code                                          */
  ST_T_END,      /* time of the last checkpoint reached                  */
  ST_S_DONE,     /* steps performed                                      */
  ST_NSCAL
};

int64_t ora_state_len(int N, int m_s, int n_l) {
  return ST_NSCAL + 2 * N + (int64_t)(m_s + n_l) * 2 * N + m_s + n_l;
}

typedef struct {
  double *sc, *x, *ws, *wl, *g, *sl;
} ora_view;

static ora_view view(double *st, int N, int m_s, int n_l) {
  ora_view v;
  v.sc = st;
  v.x = st + ST_NSCAL;
  v.ws = v.x + 2 * N;
  v.wl = v.ws + (int64_t)m_s * 2 * N;
  v.g = v.wl + (int64_t)n_l * 2 * N;
  v.sl = v.g + m_s;
  return v;
}

/* Lagrangian-descriptor integrand (the p-norm M-function of Lopesino et al.
 * 2017, cited in the Summary section; the LD-based indicators are in the
 * Functionalities section): sum over all 2N phase-space components of
 * |dx_i/dt|^p, with dq/dt = p and dp/dt = -grad V. */
static double ld_integrand(int kind, int N, const double *pr, const double *x,
                           double ldp) {
  double g[ORA_MAX_DOF], s = 0.0;
  ora_grad(kind, N, pr, x, g);
  for (int i = 0; i < N; ++i) {
    double a = fabs(x[N + i]);
    s += (ldp == 0.5) ? sqrt(a) : pow(a, ldp);
  }
  for (int i = 0; i < N; ++i) {
    double a = fabs(g[i]);
    s += (ldp == 0.5) ? sqrt(a) : pow(a, ldp);
  }
  return s;
}

static int all_finite(int n, const double *a) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

int ora_init(int kind, int N, const double *pr, const double *x0, const double *w0,
             const uint8_t *mask, int64_t n, int m_s, int n_l, uint32_t ind,
             double ldp, double *state) {
  int64_t L = ora_state_len(N, m_s, n_l);
  if (N < 1 || N > ORA_MAX_DOF) return 1;
  for (int64_t o = 0; o < n; ++o) {
    double *st = state + o * L;
    ora_view v = view(st, N, m_s, n_l);
    for (int64_t i = 0; i < L; ++i) st[i] = 0.0;
    for (int i = 0; i < 2 * N; ++i) v.x[i] = x0[o * 2 * N + i];
    v.sc[ST_SALI_MIN] = INFINITY;
    v.sc[ST_SALI_LAST] = NAN;
    v.sc[ST_T_CHAOS] = NAN;
    if (mask && !mask[o]) {
      v.sc[ST_STATUS] = ORA_ST_MASKED;
      continue;
    }
    if (!all_finite(2 * N, v.x)) {
      v.sc[ST_STATUS] = ORA_ST_NONFINITE;
      continue;
    }
    v.sc[ST_STATUS] = ORA_ST_OK;
    v.sc[ST_H0] = ora_hamiltonian(kind, N, pr, v.x);
    /* SALI/GALI set: the given vectors, normalised to unit length. */
    for (int k = 0; k < m_s; ++k) {
      const double *src = w0 + (o * m_s + k) * 2 * N;
      double *dst = v.ws + (int64_t)k * 2 * N;
      double r = sqrt(dot(2 * N, src, src));
      for (int i = 0; i < 2 * N; ++i) dst[i] = src[i] / r;
    }
    /* Lyapunov set: canonical basis. */
    for (int k = 0; k < n_l; ++k)
      for (int i = 0; i < 2 * N; ++i) v.wl[k * 2 * N + i] = (i == k) ? 1.0 : 0.0;
    if (ind & ORA_IND_LD) v.sc[ST_GPREV] = ld_integrand(kind, N, pr, v.x, ldp);
  }
  return 0;
}

/* One checkpoint at step s (time t = s dt). Returns the new status. */
static int checkpoint(int kind, int N, const double *pr, ora_view v, int m_s, int n_l,
                      uint32_t ind, double t, double thr, int early_exit,
                      double escape_r2) {
  if (!all_finite(2 * N, v.x)) return ORA_ST_NONFINITE;
  int escaped = 0;
  if (escape_r2 > 0.0) {
    double r2 = 0.0;
    for (int i = 0; i < N; ++i) r2 += v.x[i] * v.x[i];
    if (r2 > escape_r2) escaped = 1;
  }
  /* Deviation-vector normalisation (Functionalities section): each vector of
   * the SALI/GALI set is rescaled to unit length; ln of its norm is kept. */
  for (int k = 0; k < m_s; ++k) {
    double *w = v.ws + (int64_t)k * 2 * N;
    double r = sqrt(dot(2 * N, w, w));
    v.g[k] += log(r);
    for (int i = 0; i < 2 * N; ++i) w[i] = w[i] / r;
  }
  double sali = NAN;
  if ((ind & ORA_IND_SALI) && m_s >= 2) {
    /* SALI = min(|w1 + w2|, |w1 - w2|) of the two unit vectors. */
    double sp = 0.0, sm = 0.0;
    for (int i = 0; i < 2 * N; ++i) {
      double a = v.ws[i] + v.ws[2 * N + i];
      double b = v.ws[i] - v.ws[2 * N + i];
      sp += a * a;
      sm += b * b;
    }
    sp = sqrt(sp);
    sm = sqrt(sm);
    sali = sp < sm ? sp : sm;
    v.sc[ST_SALI_LAST] = sali;
    if (sali < v.sc[ST_SALI_MIN]) v.sc[ST_SALI_MIN] = sali;
    if (sali < thr && isnan(v.sc[ST_T_CHAOS])) v.sc[ST_T_CHAOS] = t;
  }
  /* Lyapunov set: QR by modified Gram-Schmidt; ln R_jj accumulated. */
  if (n_l > 0) {
    double rd[2 * ORA_MAX_DOF];
    ora_mgs(2 * N, n_l, v.wl, rd);
    for (int j = 0; j < n_l; ++j) v.sl[j] += log(rd[j]);
  }
  if (ind & ORA_IND_ENERGY) {
    double e = fabs(ora_hamiltonian(kind, N, pr, v.x) - v.sc[ST_H0]);
    if (e > v.sc[ST_EERR]) v.sc[ST_EERR] = e;
  }
  if (escaped) return ORA_ST_ESCAPED;
  if (early_exit && (ind & ORA_IND_SALI) && m_s >= 2 && sali < thr) return ORA_ST_EXITED;
  return ORA_ST_OK;
}

int ora_advance(int kind, int N, const double *pr, double *state, int64_t n, int m_s,
                int n_l, uint32_t ind, double dt, int64_t s_begin, int64_t s_end,
                int64_t n_total, int K, double ldp, double thr, int early_exit,
                double escape_r2) {
  int64_t L = ora_state_len(N, m_s, n_l);
  if (K < 1 || s_begin < 0 || s_end > n_total || s_begin > s_end) return 1;
  for (int64_t o = 0; o < n; ++o) {
    double *st = state + o * L;
    ora_view v = view(st, N, m_s, n_l);
    if ((int)v.sc[ST_STATUS] != ORA_ST_OK) continue;
    if ((int64_t)v.sc[ST_S_DONE] != s_begin) return 2;
    for (int64_t s = s_begin + 1; s <= s_end; ++s) {
      /* both vector sets are evolved by the same tangent map */
      ora_step(kind, N, pr, dt, v.x, v.ws, m_s + n_l);
      if (ind & ORA_IND_LD) {
        /* trapezoid rule over the step's endpoints */
        double g = ld_integrand(kind, N, pr, v.x, ldp);
        v.sc[ST_LD] += dt / 2.0 * (v.sc[ST_GPREV] + g);
        v.sc[ST_GPREV] = g;
      }
      v.sc[ST_S_DONE] = (double)s;
      if (s % K == 0 || s == n_total) {
        double t = (double)s * dt;
        int stt = checkpoint(kind, N, pr, v, m_s, n_l, ind, t, thr, early_exit,
                             escape_r2);
        v.sc[ST_T_END] = t;
        if (stt != ORA_ST_OK) {
          v.sc[ST_STATUS] = stt;
          break;
        }
      }
    }
  }
  return 0;
}

int ora_finalize(int N, const double *state, int64_t n, int m_s, int n_l, uint32_t ind,
                 int kmax, double thr, double *x_final, double *t_end,
                 int32_t *status, int8_t *label, double *sali_final, double *sali_min,
                 double *t_chaos, double *gali, double *lyap, double *ld,
                 double *energy_err, double *ln_growth) {
  int64_t L = ora_state_len(N, m_s, n_l);
  for (int64_t o = 0; o < n; ++o) {
    const double *st = state + o * L;
    ora_view v = view((double *)st, N, m_s, n_l);
    int stt = (int)v.sc[ST_STATUS];
    int bad = (stt == ORA_ST_MASKED || stt == ORA_ST_NONFINITE);
    double te = v.sc[ST_T_END];
    if (x_final)
      for (int i = 0; i < 2 * N; ++i) x_final[o * 2 * N + i] = v.x[i];
    if (t_end) t_end[o] = te;
    if (status) status[o] = stt;
    if (label) {
      int8_t lb;
      if (stt == ORA_ST_MASKED) lb = -1;
      else if (stt == ORA_ST_NONFINITE) lb = 3;
      else if (stt == ORA_ST_ESCAPED) lb = 2;
      else lb = (v.sc[ST_SALI_MIN] < thr) ? 1 : 0;
      label[o] = lb;
    }
    if (sali_final) sali_final[o] = bad ? NAN : v.sc[ST_SALI_LAST];
    if (sali_min) sali_min[o] = bad ? NAN : v.sc[ST_SALI_MIN];
    if (t_chaos) t_chaos[o] = bad ? NAN : v.sc[ST_T_CHAOS];
    if (ld) ld[o] = bad ? NAN : v.sc[ST_LD];
    if (energy_err) energy_err[o] = bad ? NAN : v.sc[ST_EERR];
    if (ln_growth)
      for (int k = 0; k < m_s; ++k) ln_growth[o * m_s + k] = bad ? NAN : v.g[k];
    if (lyap)
      for (int j = 0; j < n_l; ++j)
        lyap[o * n_l + j] = (bad || !(te > 0.0)) ? NAN : v.sl[j] / te;
    if (gali && kmax >= 2) {
      if (bad)
        for (int k = 2; k <= kmax; ++k) gali[o * (kmax - 1) + k - 2] = NAN;
      else
        ora_gali(2 * N, kmax, v.ws, kmax, gali + o * (kmax - 1));
    }
  }
  (void)ind;
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Input assembly                                                          */
/* ---------------------------------------------------------------------- */

/* Henon-Heiles section x = 0: on it H = (p_x^2 + p_y^2)/2 + y^2/2 - y^3/3, so
 * at energy E, p_x^2 = 2E - p_y^2 - y^2 + 2y^3/3; the branch p_x >= 0 is
 * taken and points with a negative right-hand side are inaccessible. */
static void hh_point(double E, double y, double py, double *x, uint8_t *m) {
  double r = 2.0 * E - py * py - y * y + 2.0 * y * y * y / 3.0;
  x[0] = 0.0;
  x[1] = y;
  x[3] = py;
  if (r >= 0.0) {
    x[2] = sqrt(r);
    *m = 1;
  } else {
    x[2] = 0.0;
    *m = 0;
  }
}

void ora_hh_grid(double E, double y0, double y1, int ny, double py0, double py1,
                 int npy, double *x0, uint8_t *mask) {
  for (int j = 0; j < npy; ++j) {
    double py = (npy > 1) ? py0 + (py1 - py0) * (double)j / (double)(npy - 1) : py0;
    for (int i = 0; i < ny; ++i) {
      double y = (ny > 1) ? y0 + (y1 - y0) * (double)i / (double)(ny - 1) : y0;
      int64_t o = (int64_t)j * ny + i;
      hh_point(E, y, py, x0 + 4 * o, mask + o);
    }
  }
}

void ora_hh_points(double E, const double *y, const double *py, int64_t n, double *x0,
                   uint8_t *mask) {
  for (int64_t o = 0; o < n; ++o) hh_point(E, y[o], py[o], x0 + 4 * o, mask + o);
}

/* FPU chain with fixed ends, energy in the two lowest normal modes.  Normal
 * modes of the linear chain: Q_k = sqrt(2/(N+1)) sum_i q_i sin(i k pi/(N+1)),
 * frequency omega_k = 2 sin(k pi / (2 (N+1))).  Q_k = a_k cos(phi_k)/omega_k,
 * P_k = a_k sin(phi_k) for k = 1, 2; the resulting (q, p) is scaled by s so
 * that H(s q, s p) = E: with H = s^2 H2 + s^3 H3 + s^4 H4 (the parts of
 * degree 2, 3 and 4), s solves that polynomial; for alpha = 0 in closed form
 * s^2 = (-H2 + sqrt(H2^2 + 4 H4 E)) / (2 H4), evaluated in the equivalent
 * form 2E / (H2 + sqrt(H2^2 + 4 H4 E)), which has no cancellation. */
void ora_fput_ic(int N, const double *pr, const double *u, int64_t n, double *x0) {
  const double PI = 3.14159265358979323846;
  for (int64_t o = 0; o < n; ++o) {
    const double *uu = u + 5 * o;
    double E = 0.1 + 9.9 * uu[0];
    double Qm[2], Pm[2];
    for (int k = 1; k <= 2; ++k) {
      double om = 2.0 * sin((double)k * PI / (2.0 * (double)(N + 1)));
      double a = uu[k], ph = 2.0 * PI * uu[k + 2];
      Qm[k - 1] = a * cos(ph) / om;
      Pm[k - 1] = a * sin(ph);
    }
    double *q = x0 + o * 2 * N, *p = q + N;
    double nrm = sqrt(2.0 / (double)(N + 1));
    for (int i = 1; i <= N; ++i) {
      double s1 = sin((double)i * 1.0 * PI / (double)(N + 1));
      double s2 = sin((double)i * 2.0 * PI / (double)(N + 1));
      q[i - 1] = nrm * (Qm[0] * s1 + Qm[1] * s2);
      p[i - 1] = nrm * (Pm[0] * s1 + Pm[1] * s2);
    }
    /* degree-2, -3 and -4 parts of H at the unscaled point */
    double h2 = 0.0, h3 = 0.0, h4 = 0.0;
    for (int i = 0; i < N; ++i) h2 += p[i] * p[i] / 2.0;
    for (int j = 1; j <= N + 1; ++j) {
      double d = fput_qm(q, N, j) - fput_qm(q, N, j - 1);
      h2 += pr[0] * d * d / 2.0;
      h3 += pr[1] * d * d * d / 3.0;
      h4 += pr[2] * d * d * d * d / 4.0;
    }
    double s;
    if (h3 == 0.0 && h4 > 0.0) {
      s = sqrt(2.0 * E / (h2 + sqrt(h2 * h2 + 4.0 * h4 * E)));
    } else if (h3 == 0.0 && h4 == 0.0) {
      s = sqrt(E / h2);
    } else {
      /* Newton on f(s) = h2 s^2 + h3 s^3 + h4 s^4 - E from the quadratic guess */
      s = sqrt(E / h2);
      for (int it = 0; it < 100; ++it) {
        double f = h2 * s * s + h3 * s * s * s + h4 * s * s * s * s - E;
        double fp = 2.0 * h2 * s + 3.0 * h3 * s * s + 4.0 * h4 * s * s * s;
        double ds = f / fp;
        s = s - ds;
        if (fabs(ds) <= 1e-16 * fabs(s)) break;
      }
    }
    for (int i = 0; i < N; ++i) {
      q[i] = s * q[i];
      p[i] = s * p[i];
    }
  }
}

/* Coupled quartic oscillator at H = 1.  V is homogeneous of degree 4, so
 * V(s u) = s^4 V(u): a point on the ray u with V = f is s = (f/V(u))^(1/4). */
void ora_quartic_ic(int N, const double *pr, const double *draws, int64_t n,
                    double *x0) {
  for (int64_t o = 0; o < n; ++o) {
    const double *dr = draws + o * (2 * N + 1);
    double u[ORA_MAX_DOF], e[ORA_MAX_DOF];
    double nu = sqrt(dot(N, dr, dr)), ne = sqrt(dot(N, dr + N, dr + N));
    for (int i = 0; i < N; ++i) {
      u[i] = dr[i] / nu;
      e[i] = dr[N + i] / ne;
    }
    double f = dr[2 * N];
    double s = pow(f / quartic_V(N, pr, u), 0.25);
    double pm = sqrt(2.0 * (1.0 - f));
    double *q = x0 + o * 2 * N, *p = q + N;
    for (int i = 0; i < N; ++i) {
      q[i] = s * u[i];
      p[i] = pm * e[i];
    }
  }
}
