/*
 * chx_oracle.h -- the oracle: a plain, slow, scalar FP64 CPU implementation of
 * the ensemble chaos-indicator integrator (arXiv 2507.00622, "Chaoticus").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load or call this library.  It shares
 * no code, header, table or constant with the HIP library under
 * paper_2507_00622_amd/, and it never includes include/chx.h.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (no FMA contraction), so
 * every floating-point operation is one IEEE-754 binary64 operation rounded
 * to nearest, in the order written.
 *
 * What it computes, and where the paper defines it:
 *   - Hamilton's equations of the Henon-Heiles system (Examples section,
 *     the Henon-Heiles Hamiltonian and its equations of motion), of the
 *     Fermi-Pasta-Ulam chain with fixed ends (Examples section, the FPU
 *     Hamiltonian, its equations of motion and the boundary condition
 *     q_0 = q_{N+1} = 0), plus two test systems: a coupled quartic oscillator
 *     and a set of uncoupled harmonic oscillators.
 *   - The deviation vectors, which obey the variational equations (Statement
 *     of need), evolved as the exact tangent map of the discrete step.
 *   - Deviation-vector normalisation, the Lyapunov spectrum by QR, GALI by
 *     the singular values of the unit deviation vectors, SALI, and the
 *     Lagrangian-descriptor M-function (Functionalities section).
 *   - The integrator is the fourth-order symplectic triple-jump composition
 *     of Yoshida (Phys. Lett. A 150 (1990) 262) of kick-drift-kick leapfrog,
 *     or, on request, the eighth-order explicit Runge-Kutta method of Dormand
 *     and Prince (DOP853, the solver the paper's Functionalities section
 *     builds on) with a fixed step, applied to the state, the variational
 *     equations and the LD integrand as one system.
 *
 * All functions are per initial condition, one after another, with no
 * blocking, fusion or reordering beyond the definitions.
 */
#ifndef CHX_ORACLE_H
#define CHX_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* System kinds (the oracle's own numbering). */
#define ORA_SYS_HENON_HEILES 1 /* ndof == 2, no params                         */
#define ORA_SYS_FPUT 2         /* params {k, alpha, beta}; N+1 springs         */
#define ORA_SYS_QUARTIC 3      /* params {eps}; V = sum q^4/4 + eps sum q_i^2 q_j^2 */
#define ORA_SYS_HARMONIC 4     /* params {omega_1..omega_N}; V = sum w^2 q^2/2 */
#define ORA_SYS_DOUBLE_PENDULUM 5 /* ndof == 2, params {alpha, sigma}; not separable:
                                     Runge-Kutta integrators only */

/* Indicator bits (the oracle's own numbering). */
#define ORA_IND_SALI 1
#define ORA_IND_GALI 2
#define ORA_IND_LYAP 4
#define ORA_IND_LD 8
#define ORA_IND_ENERGY 16

/* Integrators. */
#define ORA_INT_YOSHIDA4 0
#define ORA_INT_DOP853 1
#define ORA_INT_DOP853_ADAPTIVE 2 /* driver: ora_advance_adaptive */

/* Orbit status codes. */
#define ORA_ST_OK 0
#define ORA_ST_MASKED 1
#define ORA_ST_ESCAPED 2
#define ORA_ST_NONFINITE 3
#define ORA_ST_EXITED 4
#define ORA_ST_STEPFAIL 5 /* adaptive: too many attempts between checkpoints */

/* Potential, gradient and dense Hessian (row-major ndof x ndof). */
double ora_potential(int kind, int ndof, const double *params, const double *q);
void ora_grad(int kind, int ndof, const double *params, const double *q, double *g);
void ora_hess(int kind, int ndof, const double *params, const double *q, double *h);
/* Double pendulum: f(x) = (dH/dp, -dH/dtheta) and, if dx != NULL, the
 * directional derivative Df(x) dx (x, dx, f, df of length 4). */
void ora_dp_rhs(const double *params, const double *x, const double *dx, double *f,
                double *df);
/* H(q, p) = |p|^2 / 2 + V(q); x = (q_1..q_N, p_1..p_N); the double pendulum's
 * own H. */
double ora_hamiltonian(int kind, int ndof, const double *params, const double *x);

/* The drift and kick coefficients of one Yoshida-4 KDK step. */
void ora_yoshida_coefficients(double c[3], double d[4]);

/* One Yoshida-4 KDK step of size dt applied to the state x[2N] and to m
 * tangent vectors w[m][2N] (each laid out (dq, dp)). */
void ora_step(int kind, int ndof, const double *params, double dt, double *x,
              double *w, int m);

/* The DOP853 coefficients: nodes c[12], row-major lower-triangular a[12][12]
 * (zeros above the diagonal and where the method has none), weights b[12]. */
void ora_dop853_tableau(double c[12], double a[144], double b[12]);
/* Its error estimators: er[12] (eighth minus embedded fifth order) and the
 * embedded third-order weights bhh[3] on stages 1, 9 and 12. */
void ora_dop853_error_weights(double er[12], double bhh[3]);
/* One fixed DOP853 step of size dt of the state x[2N], m tangent vectors
 * w[m][2N] and, if do_ld, the LD M-function *ld (integrand sum |dx_i/dt|^p). */
void ora_dop853_step(int kind, int ndof, const double *params, double dt, double *x,
                     double *w, int m, int do_ld, double ld_p, double *ld);

/* Integration driver with explicit, resumable per-orbit state.
 *
 * state is [n][ora_state_len(ndof, m_s, n_l)] doubles.  ora_init fills it at
 * t = 0, ora_advance performs steps s_begin+1 .. s_end of an n_total-step run
 * (checkpoints where s % K == 0 or s == n_total), ora_finalize writes the
 * outputs.  Splitting a run at any step count gives bit-identical results.
 *
 * w0: [n][m_s][2N] initial SALI/GALI deviation vectors (any non-zero length;
 * normalised at t = 0).  NULL only when m_s == 0.  The Lyapunov set is the
 * canonical basis e_1..e_{n_l}.
 * mask: [n] bytes, 0 = masked (skipped), or NULL (all active).
 */
int64_t ora_state_len(int ndof, int m_s, int n_l);
int ora_init(int kind, int ndof, const double *params, const double *x0,
             const double *w0, const uint8_t *mask, int64_t n, int m_s, int n_l,
             uint32_t indicators, double ld_p, double *state);
int ora_advance(int kind, int ndof, const double *params, double *state, int64_t n,
                int m_s, int n_l, uint32_t indicators, double dt, int64_t s_begin,
                int64_t s_end, int64_t n_total, int K, double ld_p,
                double sali_threshold, int early_exit, double escape_r2);
/* The same with the integrator chosen (ORA_INT_*).  With DOP853 the LD is a
 * component of the integrated system; with Yoshida-4 it is the trapezoid rule
 * over step endpoints. */
int ora_advance_with(int kind, int ndof, const double *params, double *state, int64_t n,
                     int m_s, int n_l, uint32_t indicators, double dt, int64_t s_begin,
                     int64_t s_end, int64_t n_total, int K, double ld_p,
                     double sali_threshold, int early_exit, double escape_r2,
                     int integrator);
/* The same schedule with the adaptive DOP8(5) step-size control between
 * checkpoints (relative and absolute tolerances rtol, atol; first step dt).
 * The error of each attempted step is measured on the state and the
 * deviation vectors. */
int ora_advance_adaptive(int kind, int ndof, const double *params, double *state,
                         int64_t n, int m_s, int n_l, uint32_t indicators, double dt,
                         int64_t s_begin, int64_t s_end, int64_t n_total, int K,
                         double ld_p, double sali_threshold, int early_exit,
                         double escape_r2, double rtol, double atol);
/* Accepted and rejected step counts of the adaptive driver. */
void ora_step_counts(int ndof, const double *state, int64_t n, int m_s, int n_l,
                     int64_t *accepted, int64_t *rejected);
/* The adaptive driver's error estimate (the scaled DOP853 estimate its
 * controller compares with 1) of the accepted steps: the largest and the
 * last, per orbit (0 before the first accepted step). */
void ora_step_errors(int ndof, const double *state, int64_t n, int m_s, int n_l,
                     double *err_max, double *err_last);
/* Outputs (any may be NULL): x_final[n][2N], t_end[n], status[n], label[n],
 * sali_final[n], sali_min[n], t_chaos[n], gali[n][kmax-1], lyap[n][n_l],
 * ld[n], energy_err[n], ln_growth[n][m_s]. */
int ora_finalize(int ndof, const double *state, int64_t n, int m_s, int n_l,
                 uint32_t indicators, int gali_kmax, double sali_threshold,
                 double *x_final, double *t_end, int32_t *status, int8_t *label,
                 double *sali_final, double *sali_min, double *t_chaos,
                 double *gali, double *lyap, double *ld, double *energy_err,
                 double *ln_growth);

/* GALI_k, k = 2..kmax, of the k leading columns of the 2N x m matrix whose
 * columns are the given vectors (normalised first): product of the diagonal
 * of the R factor of a modified Gram-Schmidt QR of a copy. */
void ora_gali(int dim, int m, const double *w, int kmax, double *gali_out);
/* One modified Gram-Schmidt pass in place on m vectors of length dim; writes
 * R_jj to rdiag. */
void ora_mgs(int dim, int m, double *w, double *rdiag);

/* Input assembly ------------------------------------------------------- */
/* Henon-Heiles surface of section x = 0 at energy E: for each (y, p_y)
 * p_x = +sqrt(r), r = 2E - p_y^2 - y^2 + 2 y^3 / 3; mask = (r >= 0).
 * Grid: y_i = y0 + (y1 - y0) i / (ny - 1), py_j likewise, index j*ny + i. */
void ora_hh_grid(double E, double y0, double y1, int ny, double py0, double py1,
                 int npy, double *x0, uint8_t *mask);
void ora_hh_points(double E, const double *y, const double *py, int64_t n,
                   double *x0, uint8_t *mask);
/* FPU chain (fixed ends) with its energy in the two lowest normal modes.
 * u[n][5] uniforms in [0,1): E = 0.1 + 9.9 u0, a_k = u_{k}, phi_k = 2 pi u_{k+2}. */
void ora_fput_ic(int ndof, const double *params, const double *u, int64_t n,
                 double *x0);
/* Coupled quartic oscillator at energy 1: direction d[3] and momentum
 * direction e[3] (Gaussian draws), fraction f in (0,1):
 * q = (f / V(d/|d|))^(1/4) d/|d|, p = sqrt(2 (1 - f)) e/|e|. */
void ora_quartic_ic(int ndof, const double *params, const double *draws, int64_t n,
                    double *x0);

#ifdef __cplusplus
}
#endif
#endif
