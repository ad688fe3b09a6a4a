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

/* Dimensionless double pendulum (Examples section: its Hamiltonian in matrix
 * form and Hamilton's equations).  x = (theta_1, theta_2, p_1, p_2),
 * params {alpha, sigma} (length and mass ratios):
 *   H = p^T B^{-1}(c) p / 2 - alpha (1 + sigma) cos theta_1 - cos theta_2,
 *   c = cos(theta_1 - theta_2),
 *   B^{-1}(c) = [[1/alpha^2, -c/alpha], [-c/alpha, 1 + sigma]] / (1 + sigma - c^2).
 * The kinetic part is T = Q / (2 D) with D = 1 + sigma - c^2 and
 * Q = p_1^2/alpha^2 - 2 c p_1 p_2 / alpha + (1 + sigma) p_2^2, so
 *   theta' = dH/dp = B^{-1} p,
 *   p_1' = -dH/dtheta_1 = s dT/dc - alpha (1 + sigma) sin theta_1,
 *   p_2' = -dH/dtheta_2 = -s dT/dc - sin theta_2,
 * with s = sin(theta_1 - theta_2) and dT/dc = (c Q - p_1 p_2 D / alpha) / D^2
 * (the printed equations' (sin/2) p^T C p, C = dB^{-1}/dc).  H is not
 * separable, so only the Runge-Kutta integrators apply.  The variational
 * equations d(dx)/dt = Df(x) dx take the directional derivative Df(x) dx
 * exactly, by evaluating the same formulas on dual numbers a + b e with
 * e^2 = 0 (forward-mode differentiation). */
typedef struct {
  double v, d; /* value and derivative part */
} dual;
static dual dl(double v, double d) {
  dual r;
  r.v = v;
  r.d = d;
  return r;
}
static dual dadd(dual a, dual b) { return dl(a.v + b.v, a.d + b.d); }
static dual dsub(dual a, dual b) { return dl(a.v - b.v, a.d - b.d); }
static dual dmul(dual a, dual b) { return dl(a.v * b.v, a.v * b.d + a.d * b.v); }
static dual ddiv(dual a, dual b) { return dl(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
static dual dscale(double k, dual a) { return dl(k * a.v, k * a.d); }
static dual dsin(dual a) { return dl(sin(a.v), cos(a.v) * a.d); }
static dual dcos(dual a) { return dl(cos(a.v), -sin(a.v) * a.d); }

static void dp_rhs_dual(const double *pr, const dual *x, dual *f) {
  const double al = pr[0], sg = pr[1];
  dual del = dsub(x[0], x[1]);
  dual c = dcos(del), s = dsin(del);
  dual p1 = x[2], p2 = x[3];
  dual D = dsub(dl(1.0 + sg, 0.0), dmul(c, c));
  /* theta' = B^{-1}(c) p */
  dual u1 = ddiv(dsub(dscale(1.0 / (al * al), p1), dscale(1.0 / al, dmul(c, p2))), D);
  dual u2 = ddiv(dadd(dscale(-1.0 / al, dmul(c, p1)), dscale(1.0 + sg, p2)), D);
  dual Q = dadd(dsub(dscale(1.0 / (al * al), dmul(p1, p1)),
                     dscale(2.0 / al, dmul(c, dmul(p1, p2)))),
                dscale(1.0 + sg, dmul(p2, p2)));
  dual dTdc = ddiv(dsub(dmul(c, Q), dscale(1.0 / al, dmul(dmul(p1, p2), D))), dmul(D, D));
  f[0] = u1;
  f[1] = u2;
  f[2] = dsub(dmul(s, dTdc), dscale(al * (1.0 + sg), dsin(x[0])));
  f[3] = dsub(dscale(-1.0, dmul(s, dTdc)), dsin(x[1]));
}

static double dp_H(const double *pr, const double *x) {
  const double al = pr[0], sg = pr[1];
  double c = cos(x[0] - x[1]);
  double D = 1.0 + sg - c * c;
  double p1 = x[2], p2 = x[3];
  double Q = p1 * p1 / (al * al) - 2.0 * c * p1 * p2 / al + (1.0 + sg) * p2 * p2;
  return Q / (2.0 * D) - al * (1.0 + sg) * cos(x[0]) - cos(x[1]);
}

/* f(x) and, if dx is given, Df(x) dx, for the double pendulum. */
void ora_dp_rhs(const double *pr, const double *x, const double *dx, double *f, double *df) {
  dual xd[4], fd[4];
  for (int i = 0; i < 4; ++i) xd[i] = dl(x[i], dx ? dx[i] : 0.0);
  dp_rhs_dual(pr, xd, fd);
  for (int i = 0; i < 4; ++i) {
    f[i] = fd[i].v;
    if (df) df[i] = fd[i].d;
  }
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
  if (kind == ORA_SYS_DOUBLE_PENDULUM) return dp_H(pr, x);
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
/* Integrator: the explicit Runge-Kutta method of order 8 of Dormand and    */
/* Prince (DOP853), with a fixed step                                      */
/* ---------------------------------------------------------------------- */

/* The paper's solvers are built on DOP853 (Functionalities section).  Its
 * coefficients are those published with the method (Prince and Dormand,
 * J. Comput. Appl. Math. 7 (1981) 67; in the 12-stage form of Hairer, Norsett
 * and Wanner, Solving Ordinary Differential Equations I, 2nd ed., Sect.
 * II.10), written to 30 significant digits; the compiler stores the nearest
 * binary64 values.  Only the eighth-order solution is used: no error
 * estimate, no step-size control, no dense output.  Stage i (0-based) is
 * evaluated at t + c_i dt; a[i][j] = 0 where not listed. */
static const double DOP_C[12] = {
    0.0,
    0.526001519587677318785587544488e-01,
    0.789002279381515978178381316732e-01,
    0.118350341907227396726757197510,
    0.281649658092772603273242802490,
    0.333333333333333333333333333333,
    0.25,
    0.307692307692307692307692307692,
    0.651282051282051282051282051282,
    0.6,
    0.857142857142857142857142857142,
    1.0};
static const double DOP_B[12] = {
    5.42937341165687622380535766363e-2, 0.0, 0.0, 0.0, 0.0,
    4.45031289275240888144113950566,
    1.89151789931450038304281599044,
    -5.8012039600105847814672114227,
    3.1116436695781989440891606237e-1,
    -1.52160949662516078556178806805e-1,
    2.01365400804030348374776537501e-1,
    4.47106157277725905176885569043e-2};
static double dop_a(int i, int j) {
  /* rows 2..12 of the published lower-triangular matrix, 1-based */
  switch (i * 100 + j) {
  case 201: return 5.26001519587677318785587544488e-2;
  case 301: return 1.97250569845378994544595329183e-2;
  case 302: return 5.91751709536136983633785987549e-2;
  case 401: return 2.95875854768068491816892993775e-2;
  case 403: return 8.87627564304205475450678981324e-2;
  case 501: return 2.41365134159266685502369798665e-1;
  case 503: return -8.84549479328286085344864962717e-1;
  case 504: return 9.24834003261792003115737966543e-1;
  case 601: return 3.7037037037037037037037037037e-2;
  case 604: return 1.70828608729473871279604482173e-1;
  case 605: return 1.25467687566822425016691814123e-1;
  case 701: return 3.7109375e-2;
  case 704: return 1.70252211019544039314978060272e-1;
  case 705: return 6.02165389804559606850219397283e-2;
  case 706: return -1.7578125e-2;
  case 801: return 3.70920001185047927108779319836e-2;
  case 804: return 1.70383925712239993810214054705e-1;
  case 805: return 1.07262030446373284651809199168e-1;
  case 806: return -1.53194377486244017527936158236e-2;
  case 807: return 8.27378916381402288758473766002e-3;
  case 901: return 6.24110958716075717114429577812e-1;
  case 904: return -3.36089262944694129406857109825;
  case 905: return -8.68219346841726006818189891453e-1;
  case 906: return 2.75920996994467083049415600797e1;
  case 907: return 2.01540675504778934086186788979e1;
  case 908: return -4.34898841810699588477366255144e1;
  case 1001: return 4.77662536438264365890433908527e-1;
  case 1004: return -2.48811461997166764192642586468;
  case 1005: return -5.90290826836842996371446475743e-1;
  case 1006: return 2.12300514481811942347288949897e1;
  case 1007: return 1.52792336328824235832596922938e1;
  case 1008: return -3.32882109689848629194453265587e1;
  case 1009: return -2.03312017085086261358222928593e-2;
  case 1101: return -9.3714243008598732571704021658e-1;
  case 1104: return 5.18637242884406370830023853209;
  case 1105: return 1.09143734899672957818500254654;
  case 1106: return -8.14978701074692612513997267357;
  case 1107: return -1.85200656599969598641566180701e1;
  case 1108: return 2.27394870993505042818970056734e1;
  case 1109: return 2.49360555267965238987089396762;
  case 1110: return -3.0467644718982195003823669022;
  case 1201: return 2.27331014751653820792359768449;
  case 1204: return -1.05344954667372501984066689879e1;
  case 1205: return -2.00087205822486249909675718444;
  case 1206: return -1.79589318631187989172765950534e1;
  case 1207: return 2.79488845294199600508499808837e1;
  case 1208: return -2.85899827713502369474065508674;
  case 1209: return -8.87285693353062954433549289258;
  case 1210: return 1.23605671757943030647266201528e1;
  case 1211: return 6.43392746015763530355970484046e-1;
  }
  return 0.0;
}

void ora_dop853_tableau(double c[12], double a[144], double b[12]) {
  for (int i = 0; i < 12; ++i) {
    c[i] = DOP_C[i];
    b[i] = DOP_B[i];
    for (int j = 0; j < 12; ++j) a[i * 12 + j] = dop_a(i + 1, j + 1);
  }
}

/* Error estimators of DOP853 (same sources): the difference between the
 * eighth-order solution and an embedded fifth-order one, weights er_i, and an
 * embedded third-order solution on stages 1, 9 and 12, weights bhh. */
static const double DOP_ER[12] = {
    0.1312004499419488073250102996e-01, 0.0, 0.0, 0.0, 0.0,
    -0.1225156446376204440720569753e+01,
    -0.4957589496572501915214079952,
    0.1664377182454986536961530415e+01,
    -0.3503288487499736816886487290,
    0.3341791187130174790297318841,
    0.8192320648511571246570742613e-01,
    -0.2235530786388629525884427845e-01};
static const double DOP_BHH[3] = {0.244094488188976377952755905512,
                                  0.733846688281611857341361741547,
                                  0.220588235294117647058823529412e-01};

void ora_dop853_error_weights(double er[12], double bhh[3]) {
  for (int i = 0; i < 12; ++i) er[i] = DOP_ER[i];
  for (int i = 0; i < 3; ++i) bhh[i] = DOP_BHH[i];
}

/* Right-hand side of the extended system y = (x, w_1..w_m, M):
 *   dq/dt = p, dp/dt = -grad V(q)               (Hamilton's equations)
 *   d(dq)/dt = dp, d(dp)/dt = -Hess V(q) dq    (variational equations)
 *   dM/dt = sum over the 2N components of |dx_i/dt|^p  (LD M-function)
 * M is present (the last component) when do_ld is set. */
static void ext_rhs(int kind, int N, const double *pr, int m, int do_ld, double ldp,
                    const double *y, double *f, double *g, double *h) {
  if (kind == ORA_SYS_DOUBLE_PENDULUM) {
    /* general Hamiltonian: f and Df dx by dual numbers */
    ora_dp_rhs(pr, y, NULL, f, NULL);
    for (int v = 0; v < m; ++v) {
      double tmp[4];
      ora_dp_rhs(pr, y, y + 4 + (int64_t)v * 4, tmp, f + 4 + (int64_t)v * 4);
    }
    if (do_ld) {
      double s = 0.0;
      for (int i = 0; i < 4; ++i) {
        double a = fabs(f[i]);
        s += (ldp == 0.5) ? sqrt(a) : pow(a, ldp);
      }
      f[4 + (int64_t)m * 4] = s;
    }
    return;
  }
  const double *q = y, *p = y + N;
  ora_grad(kind, N, pr, q, g);
  ora_hess(kind, N, pr, q, h);
  for (int i = 0; i < N; ++i) {
    f[i] = p[i];
    f[N + i] = -g[i];
  }
  for (int v = 0; v < m; ++v) {
    const double *dq = y + 2 * N + (int64_t)v * 2 * N, *dp = dq + N;
    double *fq = f + 2 * N + (int64_t)v * 2 * N, *fp = fq + N;
    for (int i = 0; i < N; ++i) {
      double s = 0.0;
      for (int j = 0; j < N; ++j) s += h[i * N + j] * dq[j];
      fq[i] = dp[i];
      fp[i] = -s;
    }
  }
  if (do_ld) {
    double s = 0.0;
    for (int i = 0; i < 2 * N; ++i) {
      double a = fabs(f[i]);
      s += (ldp == 0.5) ? sqrt(a) : pow(a, ldp);
    }
    f[2 * N + (int64_t)m * 2 * N] = s;
  }
}

/* One step of size dt: k_i = f(y + dt sum_{j<i} a_ij k_j), i = 1..12, then
 * y <- y + dt sum_i b_i k_i.  ws holds 13 ny + N + N^2 doubles with
 * ny = 2N (1 + m) + (do_ld ? 1 : 0). */
static void dop853_step_ws(int kind, int N, const double *pr, double dt, double *y, int m,
                           int do_ld, double ldp, double *ws) {
  const int64_t ny = (int64_t)2 * N * (1 + m) + (do_ld ? 1 : 0);
  double *k = ws, *Y = ws + 12 * ny, *g = Y + ny, *h = g + N;
  for (int i = 0; i < 12; ++i) {
    for (int64_t c = 0; c < ny; ++c) {
      double s = 0.0;
      for (int j = 0; j < i; ++j) s += dop_a(i + 1, j + 1) * k[j * ny + c];
      Y[c] = y[c] + dt * s;
    }
    ext_rhs(kind, N, pr, m, do_ld, ldp, Y, k + i * ny, g, h);
  }
  for (int64_t c = 0; c < ny; ++c) {
    double s = 0.0;
    for (int i = 0; i < 12; ++i) s += DOP_B[i] * k[i * ny + c];
    y[c] = y[c] + dt * s;
  }
}

/* One attempted step of size h with DOP853's error estimate.  ynew receives
 * y + h sum_i b_i k_i.  The error is measured on the first ne components
 * (the state and the deviation vectors; the LD accumulator is left out: its
 * integrand |dx_i/dt|^p has a square-root cusp at every zero crossing of a
 * component, which no step size resolves):
 *   sk_c = atol + rtol max(|y_c|, |ynew_c|),
 *   e5 = sum_c (sum_i er_i k_i,c / sk_c)^2,
 *   e3 = sum_c ((sum_i b_i k_i,c - bhh1 k_1,c - bhh2 k_9,c - bhh3 k_12,c) / sk_c)^2,
 *   err = |h| e5 / sqrt(ne (e5 + 0.01 e3))   (err = 0 when e5 = e3 = 0).
 * ws as for dop853_step_ws plus ny more doubles. */
static double dop853_attempt(int kind, int N, const double *pr, double h, const double *y,
                             double *ynew, int m, int do_ld, double ldp, double rtol,
                             double atol, double *ws) {
  const int64_t ny = (int64_t)2 * N * (1 + m) + (do_ld ? 1 : 0);
  const int64_t ne = (int64_t)2 * N * (1 + m);
  double *k = ws, *Y = ws + 12 * ny, *g = Y + ny, *hh = g + N;
  for (int i = 0; i < 12; ++i) {
    for (int64_t c = 0; c < ny; ++c) {
      double s = 0.0;
      for (int j = 0; j < i; ++j) s += dop_a(i + 1, j + 1) * k[j * ny + c];
      Y[c] = y[c] + h * s;
    }
    ext_rhs(kind, N, pr, m, do_ld, ldp, Y, k + i * ny, g, hh);
  }
  double e5 = 0.0, e3 = 0.0;
  for (int64_t c = 0; c < ny; ++c) {
    double sb = 0.0, s5 = 0.0;
    for (int i = 0; i < 12; ++i) {
      sb += DOP_B[i] * k[i * ny + c];
      s5 += DOP_ER[i] * k[i * ny + c];
    }
    ynew[c] = y[c] + h * sb;
    if (c < ne) {
      double s3 = sb - DOP_BHH[0] * k[0 * ny + c] - DOP_BHH[1] * k[8 * ny + c] -
                  DOP_BHH[2] * k[11 * ny + c];
      double a = fabs(y[c]), b = fabs(ynew[c]);
      double sk = atol + rtol * (a > b ? a : b);
      e5 += (s5 / sk) * (s5 / sk);
      e3 += (s3 / sk) * (s3 / sk);
    }
  }
  double deno = e5 + 0.01 * e3;
  if (deno <= 0.0) return 0.0;
  return fabs(h) * e5 * sqrt(1.0 / ((double)ne * deno));
}

static double *dop853_workspace(int N, int m) {
  const int64_t ny = (int64_t)2 * N * (1 + m) + 1;
  return (double *)malloc(sizeof(double) * (size_t)(14 * ny + N + (int64_t)N * N));
}

void ora_dop853_step(int kind, int N, const double *pr, double dt, double *x, double *w,
                     int m, int do_ld, double ldp, double *ld) {
  const int64_t ny = (int64_t)2 * N * (1 + m) + (do_ld ? 1 : 0);
  double *ws = dop853_workspace(N, m);
  double *y = (double *)malloc(sizeof(double) * (size_t)ny);
  for (int i = 0; i < 2 * N; ++i) y[i] = x[i];
  for (int64_t c = 0; c < (int64_t)m * 2 * N; ++c) y[2 * N + c] = w[c];
  if (do_ld) y[ny - 1] = *ld;
  dop853_step_ws(kind, N, pr, dt, y, m, do_ld, ldp, ws);
  for (int i = 0; i < 2 * N; ++i) x[i] = y[i];
  for (int64_t c = 0; c < (int64_t)m * 2 * N; ++c) w[c] = y[2 * N + c];
  if (do_ld) *ld = y[ny - 1];
  free(y);
  free(ws);
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
  ST_H,          /* adaptive: the step the controller proposes next      */
  ST_REJ,        /* adaptive: the last attempt was rejected (0 / 1)      */
  ST_NACC,       /* adaptive: accepted steps                             */
  ST_NREJ,       /* adaptive: rejected steps                             */
  ST_ERR_MAX,    /* adaptive: largest error estimate of an accepted step */
  ST_ERR_LAST,   /* adaptive: error estimate of the last accepted step   */
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
  if (kind == ORA_SYS_DOUBLE_PENDULUM) {
    double f[4];
    ora_dp_rhs(pr, x, NULL, f, NULL);
    for (int i = 0; i < 4; ++i) {
      double a = fabs(f[i]);
      s += (ldp == 0.5) ? sqrt(a) : pow(a, ldp);
    }
    return s;
  }
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

int ora_advance_with(int kind, int N, const double *pr, double *state, int64_t n,
                     int m_s, int n_l, uint32_t ind, double dt, int64_t s_begin,
                     int64_t s_end, int64_t n_total, int K, double ldp, double thr,
                     int early_exit, double escape_r2, int integrator) {
  int64_t L = ora_state_len(N, m_s, n_l);
  if (K < 1 || s_begin < 0 || s_end > n_total || s_begin > s_end) return 1;
  if (integrator != ORA_INT_YOSHIDA4 && integrator != ORA_INT_DOP853) return 3;
  if (integrator == ORA_INT_YOSHIDA4 && kind == ORA_SYS_DOUBLE_PENDULUM) return 4;
  const int m = m_s + n_l, do_ld = (ind & ORA_IND_LD) != 0;
  double *ws = NULL, *y = NULL;
  const int64_t ny = (int64_t)2 * N * (1 + m) + (do_ld ? 1 : 0);
  if (integrator == ORA_INT_DOP853) {
    ws = dop853_workspace(N, m);
    y = (double *)malloc(sizeof(double) * (size_t)ny);
  }
  int rc = 0;
  for (int64_t o = 0; o < n && !rc; ++o) {
    double *st = state + o * L;
    ora_view v = view(st, N, m_s, n_l);
    if ((int)v.sc[ST_STATUS] != ORA_ST_OK) continue;
    if ((int64_t)v.sc[ST_S_DONE] != s_begin) {
      rc = 2;
      break;
    }
    for (int64_t s = s_begin + 1; s <= s_end; ++s) {
      if (integrator == ORA_INT_YOSHIDA4) {
        /* both vector sets are evolved by the same tangent map */
        ora_step(kind, N, pr, dt, v.x, v.ws, m);
        if (do_ld) {
          /* trapezoid rule over the step's endpoints */
          double g = ld_integrand(kind, N, pr, v.x, ldp);
          v.sc[ST_LD] += dt / 2.0 * (v.sc[ST_GPREV] + g);
          v.sc[ST_GPREV] = g;
        }
      } else {
        /* the state, both vector sets (contiguous after x) and the LD as
         * one extended system */
        for (int i = 0; i < 2 * N; ++i) y[i] = v.x[i];
        for (int64_t c = 0; c < (int64_t)m * 2 * N; ++c) y[2 * N + c] = v.ws[c];
        if (do_ld) y[ny - 1] = v.sc[ST_LD];
        dop853_step_ws(kind, N, pr, dt, y, m, do_ld, ldp, ws);
        for (int i = 0; i < 2 * N; ++i) v.x[i] = y[i];
        for (int64_t c = 0; c < (int64_t)m * 2 * N; ++c) v.ws[c] = y[2 * N + c];
        if (do_ld) v.sc[ST_LD] = y[ny - 1];
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
  free(ws);
  free(y);
  return rc;
}

int ora_advance(int kind, int N, const double *pr, double *state, int64_t n, int m_s,
                int n_l, uint32_t ind, double dt, int64_t s_begin, int64_t s_end,
                int64_t n_total, int K, double ldp, double thr, int early_exit,
                double escape_r2) {
  return ora_advance_with(kind, N, pr, state, n, m_s, n_l, ind, dt, s_begin, s_end,
                          n_total, K, ldp, thr, early_exit, escape_r2, ORA_INT_YOSHIDA4);
}

/* Adaptive DOP8(5) (the paper's Functionalities section lists the adaptive
 * DOP 8(5) solvers, with the error of each step): the checkpoint schedule is
 * that of the fixed-step driver -- checkpoints at t = s dt for s a multiple
 * of K or the last step -- and between two checkpoints the step size is
 * chosen by the error estimate of dop853_attempt with the controller of
 * Hairer, Norsett and Wanner's DOP853 code (defaults: safety 0.9, step
 * ratio in [1/3.003, 6], exponent 1/8, no step-size memory):
 *   accept iff err <= 1;  q = err^(1/8) (three square roots);
 *   accepted: h <- h / max(1/6, min(1/0.333, q / 0.9)), and not larger than
 *             the accepted step when the attempt before it was rejected;
 *   rejected: h <- h / min(1/0.333, q / 0.9).
 * The first step is dt.  A step that would end within 1.01 h of the next
 * checkpoint is shortened to end on it exactly.  More than 100000 attempts
 * between two checkpoints stop the orbit (ORA_ST_STEPFAIL); a non-finite
 * error or state stops it as ORA_ST_NONFINITE. */
#define ADAPT_SAFE 0.9
#define ADAPT_FACC1 (1.0 / 0.333)
#define ADAPT_FACC2 (1.0 / 6.0)
#define ADAPT_MAX_ATTEMPTS 100000

int ora_advance_adaptive(int kind, int N, const double *pr, double *state, int64_t n,
                         int m_s, int n_l, uint32_t ind, double dt, int64_t s_begin,
                         int64_t s_end, int64_t n_total, int K, double ldp, double thr,
                         int early_exit, double escape_r2, double rtol, double atol) {
  int64_t L = ora_state_len(N, m_s, n_l);
  if (K < 1 || s_begin < 0 || s_end > n_total || s_begin > s_end) return 1;
  if (!(rtol >= 0.0) || !(atol >= 0.0) || !(rtol + atol > 0.0)) return 3;
  const int m = m_s + n_l, do_ld = (ind & ORA_IND_LD) != 0;
  const int64_t ny = (int64_t)2 * N * (1 + m) + (do_ld ? 1 : 0);
  double *ws = dop853_workspace(N, m);
  double *y = (double *)malloc(sizeof(double) * (size_t)ny);
  double *ynew = (double *)malloc(sizeof(double) * (size_t)ny);
  int rc = 0;
  for (int64_t o = 0; o < n && !rc; ++o) {
    double *st = state + o * L;
    ora_view v = view(st, N, m_s, n_l);
    if ((int)v.sc[ST_STATUS] != ORA_ST_OK) continue;
    if ((int64_t)v.sc[ST_S_DONE] != s_begin) {
      rc = 2;
      break;
    }
    if (!(v.sc[ST_H] > 0.0)) v.sc[ST_H] = dt; /* the first step */
    for (int i = 0; i < 2 * N; ++i) y[i] = v.x[i];
    for (int64_t c = 0; c < (int64_t)m * 2 * N; ++c) y[2 * N + c] = v.ws[c];
    if (do_ld) y[ny - 1] = v.sc[ST_LD];
    int64_t s = s_begin;
    while (s < s_end) {
      int64_t sb = (s / K + 1) * K;
      if (sb > n_total) sb = n_total;
      double t = (double)s * dt, tb = (double)sb * dt;
      int stt = ORA_ST_OK, attempts = 0;
      while (t < tb) {
        double h = v.sc[ST_H];
        int last = 0;
        if (t + 1.01 * h >= tb) {
          h = tb - t;
          last = 1;
        }
        double err = dop853_attempt(kind, N, pr, h, y, ynew, m, do_ld, ldp, rtol, atol, ws);
        if (!isfinite(err) || !all_finite((int)ny, ynew)) {
          stt = ORA_ST_NONFINITE;
          break;
        }
        if (++attempts > ADAPT_MAX_ATTEMPTS) {
          stt = ORA_ST_STEPFAIL;
          break;
        }
        double q = sqrt(sqrt(sqrt(err)));
        if (err <= 1.0) {
          double fac = q / ADAPT_SAFE;
          if (fac > ADAPT_FACC1) fac = ADAPT_FACC1;
          if (fac < ADAPT_FACC2) fac = ADAPT_FACC2;
          double hnew = h / fac;
          if (v.sc[ST_REJ] != 0.0 && hnew > h) hnew = h;
          v.sc[ST_REJ] = 0.0;
          v.sc[ST_H] = hnew;
          v.sc[ST_NACC] += 1.0;
          if (err > v.sc[ST_ERR_MAX]) v.sc[ST_ERR_MAX] = err;
          v.sc[ST_ERR_LAST] = err;
          for (int64_t c = 0; c < ny; ++c) y[c] = ynew[c];
          t = last ? tb : t + h;
        } else {
          double fac = q / ADAPT_SAFE;
          if (fac > ADAPT_FACC1) fac = ADAPT_FACC1;
          v.sc[ST_H] = h / fac;
          v.sc[ST_REJ] = 1.0;
          v.sc[ST_NREJ] += 1.0;
        }
      }
      for (int i = 0; i < 2 * N; ++i) v.x[i] = y[i];
      for (int64_t c = 0; c < (int64_t)m * 2 * N; ++c) v.ws[c] = y[2 * N + c];
      if (do_ld) v.sc[ST_LD] = y[ny - 1];
      v.sc[ST_S_DONE] = (double)sb;
      if (stt == ORA_ST_OK) {
        stt = checkpoint(kind, N, pr, v, m_s, n_l, ind, tb, thr, early_exit, escape_r2);
        v.sc[ST_T_END] = tb;
      }
      if (stt != ORA_ST_OK) {
        v.sc[ST_STATUS] = stt;
        break;
      }
      /* the checkpoint renormalised the vectors: continue from them */
      for (int64_t c = 0; c < (int64_t)m * 2 * N; ++c) y[2 * N + c] = v.ws[c];
      s = sb;
    }
  }
  free(ws);
  free(y);
  free(ynew);
  return rc;
}

void ora_step_counts(int N, const double *state, int64_t n, int m_s, int n_l,
                     int64_t *accepted, int64_t *rejected) {
  int64_t L = ora_state_len(N, m_s, n_l);
  for (int64_t o = 0; o < n; ++o) {
    accepted[o] = (int64_t)state[o * L + ST_NACC];
    rejected[o] = (int64_t)state[o * L + ST_NREJ];
  }
}

void ora_step_errors(int N, const double *state, int64_t n, int m_s, int n_l,
                     double *err_max, double *err_last) {
  int64_t L = ora_state_len(N, m_s, n_l);
  for (int64_t o = 0; o < n; ++o) {
    err_max[o] = state[o * L + ST_ERR_MAX];
    err_last[o] = state[o * L + ST_ERR_LAST];
  }
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
    int bad = (stt == ORA_ST_MASKED || stt == ORA_ST_NONFINITE || stt == ORA_ST_STEPFAIL);
    double te = v.sc[ST_T_END];
    if (x_final)
      for (int i = 0; i < 2 * N; ++i) x_final[o * 2 * N + i] = v.x[i];
    if (t_end) t_end[o] = te;
    if (status) status[o] = stt;
    if (label) {
      int8_t lb;
      if (stt == ORA_ST_MASKED) lb = -1;
      else if (stt == ORA_ST_NONFINITE || stt == ORA_ST_STEPFAIL) lb = 3;
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
