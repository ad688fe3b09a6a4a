/*
 * chx.h -- C ABI of libchx: MI355X (gfx950) ensemble integration of
 * Hamiltonian systems with their variational equations, accumulating chaos
 * indicators (arXiv 2507.00622, "Chaoticus").
 *
 * The paper's statement of the problem (Functionalities section): integrate
 * the ODE system derived from a Hamiltonian for many initial conditions and
 * compute indicators that classify each trajectory.  Deviation vectors obey
 * the variational equations (Statement of need), so the library needs the
 * potential, its gradient and its Hessian: they are built in for the
 * systems of the Examples section (Henon-Heiles; the Fermi-Pasta-Ulam chain
 * with fixed ends) and two test systems (coupled quartic oscillator,
 * uncoupled harmonic oscillators).
 *
 * Integrator: fixed-step fourth-order symplectic composition (Yoshida, Phys.
 * Lett. A 150 (1990) 262) of kick-drift-kick leapfrog; deviation vectors are
 * propagated by the exact tangent map of the step.  All arithmetic on the
 * trajectory and the deviation vectors is IEEE binary64.
 *
 * Conventions shared by every entry point
 *   - Phase-space points are x = (q_1..q_N, p_1..p_N), N = ndof; arrays of
 *     points are row-major [n][2N].
 *   - n = 0 is a no-op returning CHX_OK.
 *   - Every argument is validated before any device work; on a non-OK
 *     status nothing is written to any output and chx_last_error() returns a
 *     message (thread-local, valid until the next call on that thread).
 *   - Ownership: the caller allocates every input and output; the library
 *     keeps no caller pointer after returning (an ensemble handle keeps
 *     copies of what it needs).
 *   - Host pointers (flags without CHX_PTR_DEVICE): the call is synchronous.
 *     Device pointers (CHX_PTR_DEVICE): every pointer argument is device
 *     memory, work is ordered on `stream` (a hipStream_t, NULL = the null
 *     stream) and the caller keeps the buffers alive until the stream has
 *     synchronised.  The system's params pointer is always host memory.
 *   - Per-orbit problems (escape, non-finite state) are not call errors:
 *     they are reported in the per-orbit status and label.
 */
#ifndef CHX_H
#define CHX_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CHX_OK = 0,
  CHX_ERR_INVALID_ARG = 1,
  CHX_ERR_UNSUPPORTED = 2,
  CHX_ERR_OUT_OF_MEMORY = 3,
  CHX_ERR_DEVICE = 4,
  CHX_ERR_INTERNAL = 5
} chx_status;

/* Built-in systems.  Kinds 1-4 are separable, H = |p|^2/2 + V(q); kind 5
   is not and takes the DOP853 integrators only. */
enum {
  CHX_SYS_HENON_HEILES = 1, /* Examples section, Henon-Heiles Hamiltonian:
                               V = (x^2+y^2)/2 + x^2 y - y^3/3; ndof = 2, no params */
  CHX_SYS_FPUT = 2,         /* Examples section, FPU Hamiltonian with fixed ends
                               q_0 = q_{N+1} = 0 and N+1 springs:
                               V = sum_j k d^2/2 + alpha d^3/3 + beta d^4/4,
                               d_j = q_j - q_{j-1}; params {k, alpha, beta};
                               ndof 2..16; more than four deviation vectors
                               need ndof 2, 4, 8 or 16 (else
                               CHX_ERR_UNSUPPORTED) */
  CHX_SYS_QUARTIC = 3,      /* V = sum q_i^4/4 + eps sum_{i<j} q_i^2 q_j^2;
                               params {eps}; ndof 1..3 */
  CHX_SYS_HARMONIC = 4,     /* V = sum omega_i^2 q_i^2 / 2; params {omega_i};
                               ndof 1..3 */
  CHX_SYS_DOUBLE_PENDULUM = 5, /* Examples section, dimensionless double pendulum:
                               x = (theta_1, theta_2, p_1, p_2),
                               H = p^T B^{-1}(c) p / 2 - alpha (1+sigma) cos theta_1
                                   - cos theta_2, c = cos(theta_1 - theta_2),
                               B^{-1}(c) = [[1/alpha^2, -c/alpha],
                                            [-c/alpha, 1+sigma]] / (1+sigma-c^2);
                               params {alpha (length ratio) > 0, sigma (mass
                               ratio) > 0}; ndof = 2; integrator CHX_INT_DOP853
                               or CHX_INT_DOP853_ADAPTIVE (else
                               CHX_ERR_UNSUPPORTED); the LD integrand is
                               sum_c |dx_c/dt|^p over the four components */
  CHX_SYS_CUSTOM = 6,       /* a separable system given by the caller (the paper's
                               package integrates any Hamiltonian the user writes):
                               H = |p|^2/2 + V(q), ndof 1..8, up to 16 params
                               (nparams of them, passed as prm).  source holds HIP
                               device code defining
                                 __device__ double chx_potential(const double *q,
                                                                 const double *prm);
                                 __device__ void chx_force(const double *q, double *F,
                                                           const double *prm);
                                     F = grad V (N values)
                                 __device__ void chx_hess(const double *q, double *H,
                                                          const double *prm);
                                     H = Hess V, upper triangle packed row by
                                     row: H[i N - i (i-1)/2 + (j - i)], i <= j.
                               It is compiled for gfx950 with hipRTC together
                               with the library's lane kernels at the first call
                               that needs each kernel variant (about two seconds;
                               cached per process by source, ndof and variant);
                               source that does not compile gives
                               CHX_ERR_INVALID_ARG with the compiler's log.  All
                               integrators; not in the batched form or the gate.
                               One lane holds an orbit with its vectors, so large
                               ndof x vectors run slower (register spills).  The
                               DOP853 kernels keep per-stage values in LDS, at most
                               1024 B per orbit: 8 (12 N + [adaptive] 2 N M) bytes
                               here, 8 (12 [M > 2] 2 N + [adaptive] 2 N M) for
                               CHX_SYS_CUSTOM_GENERAL; more gives
                               CHX_ERR_UNSUPPORTED. */
  CHX_SYS_CUSTOM_GENERAL = 7 /* any Hamiltonian given by the caller, ndof 1..8,
                               up to 16 params.  source defines
                                 template <class T> __device__ void chx_field(
                                     const T *x, T *f, const double *prm);
                                     f = Hamilton's equations J grad H at
                                     x = (q, p), 2N values, written over a
                                     generic number type T (double and the
                                     library's dual numbers, which provide
                                     + - * /, with double operands too, and
                                     sin cos exp log sqrt pow(T, double));
                                 __device__ double chx_hamiltonian(
                                     const double *x, const double *prm);
                               The variational equations take the field's
                               directional derivatives through the dual
                               numbers.  DOP853 and adaptive DOP8(5) only (else
                               CHX_ERR_UNSUPPORTED); compiled and cached as
                               CHX_SYS_CUSTOM. */
};

typedef struct {
  int32_t kind;         /* CHX_SYS_* */
  int32_t ndof;         /* N; phase-space dimension 2N */
  const double *params; /* host memory, nparams values (see above) */
  int32_t nparams;
  const char *source;   /* CHX_SYS_CUSTOM: NUL-terminated device source (host
                           memory, read during the call); ignored otherwise */
} chx_system;

/* Indicator bits (Functionalities section). */
enum {
  CHX_IND_SALI = 1,   /* SALI of two unit deviation vectors */
  CHX_IND_GALI = 2,   /* GALI_k, k = 2..gali_kmax (volume of k unit vectors) */
  CHX_IND_LYAP = 4,   /* Lyapunov spectrum by periodic QR (modified Gram-Schmidt) */
  CHX_IND_LD = 8,     /* Lagrangian-descriptor M-function, forward in time */
  CHX_IND_ENERGY = 16 /* max |H(t) - H(0)| over checkpoints */
};

/* Option flags. */
enum { CHX_PTR_DEVICE = 1 };

/* Integrators (chx_options.integrator). */
enum {
  CHX_INT_YOSHIDA4 = 0, /* fourth-order symplectic triple jump of kick-drift-kick
                           leapfrog (Yoshida 1990); the tangent map is its exact
                           Jacobian; LD by the trapezoid rule over step ends */
  CHX_INT_DOP853 = 1,   /* the eighth-order explicit Runge-Kutta method of
                           Dormand and Prince that the paper's solvers build on
                           (Functionalities section), fixed step, applied to the
                           state, the variational equations and the LD integrand
                           as one system; every system.  FPU chains with more than
                           four deviation vectors keep them in LDS, 1 KB per
                           vector for a block of four orbits (2 KB adaptive):
                           a plan needing more than the device's LDS per block
                           (160 KB on MI355X: every plan up to 4N vectors fits)
                           gets CHX_ERR_UNSUPPORTED */
  CHX_INT_DOP853_ADAPTIVE = 2 /* the adaptive DOP 8(5) solver of the same
                           section: the same system, each orbit with its own step
                           size chosen from DOP853's embedded error estimate
                           (measured on the state and the deviation vectors,
                           tolerances rtol/atol) by the step-size controller of
                           Hairer-Norsett-Wanner's DOP853 (safety 0.9, step ratio
                           in [1/3.003, 6], exponent 1/8).  dt is the first step
                           and the unit of the checkpoint schedule: checkpoints
                           stay at multiples of K dt and at T, which the steps hit
                           exactly.  More than 100000 attempts between two
                           checkpoints stop the orbit (CHX_ORBIT_STEP_FAILED).
                           Systems as for CHX_INT_DOP853. */
};

/* Per-orbit status. */
enum {
  CHX_ORBIT_OK = 0,
  CHX_ORBIT_MASKED = 1,    /* mask[i] == 0: not integrated */
  CHX_ORBIT_ESCAPED = 2,   /* |q|^2 > escape_r2 at a checkpoint: stopped there */
  CHX_ORBIT_NONFINITE = 3, /* non-finite state at t = 0 or at a checkpoint */
  CHX_ORBIT_EXITED = 4,    /* early exit: SALI < threshold at a checkpoint */
  CHX_ORBIT_STEP_FAILED = 5 /* adaptive solver: no acceptable step between two
                              checkpoints (label 3, outputs NaN like non-finite) */
};

typedef struct {
  double dt;              /* step, > 0 */
  double T;               /* final time; T/dt integral to 1e-9 relative */
  uint32_t indicators;    /* CHX_IND_* bits */
  int32_t renorm_every;   /* K: checkpoint every K steps and at the last step
                             (renormalisation, SALI, QR, checks); 0 -> 10 */
  int32_t n_lyap;         /* Lyapunov vectors 1..2N; 0 -> 2N */
  int32_t gali_kmax;      /* 2..2N; 0 -> 2 */
  double ld_p;            /* LD exponent in (0, 1]; 0 -> 0.5.  FPU chains and
                             the batched form: 0.5 only (else
                             CHX_ERR_UNSUPPORTED) */
  double sali_threshold;  /* chaotic iff min SALI < threshold; 0 -> 1e-8 */
  int32_t early_exit;     /* non-zero: stop an orbit at its first checkpoint
                             with SALI < threshold (needs CHX_IND_SALI) */
  int32_t steps_per_launch; /* kernel launch granularity; 0 -> automatic */
  uint64_t seed;          /* deviation vectors when w0 == NULL */
  const double *w0;       /* optional [n][m_s][2N] initial SALI/GALI vectors
                             (normalised at t = 0); m_s = max(2 if SALI,
                             gali_kmax if GALI).  NULL -> Gaussian vectors
                             from SplitMix64(seed) with Box-Muller, element
                             (i, v, c) drawn at counter (i*m_s + v)*2N + c of
                             stream 0 */
  double escape_r2;       /* 0 = off */
  uint32_t flags;         /* CHX_PTR_DEVICE */
  int32_t block_size;     /* threads per block for the lane kernel; 0 -> tuned */
  void *stream;           /* hipStream_t for CHX_PTR_DEVICE calls */
  int32_t integrator;     /* CHX_INT_*; 0 -> Yoshida-4.  The batched form and
                             the convenience calls use Yoshida-4 */
  double rtol, atol;      /* CHX_INT_DOP853_ADAPTIVE tolerances, >= 0, not both
                             0; 0 and 0 -> 1e-10 each.  Ignored otherwise */
} chx_options;

/* Fills *o with dt = T = 0 (must be set) and all defaults above. */
void chx_options_default(chx_options *o);

/* Outputs; any NULL member is skipped.  Layouts are row-major per orbit. */
typedef struct {
  double *x_final;    /* [n][2N] state at t_end */
  double *t_end;      /* [n] time of the last checkpoint reached */
  int32_t *status;    /* [n] CHX_ORBIT_* */
  int8_t *label;      /* [n] -1 masked, 0 regular, 1 chaotic (min SALI <
                         threshold), 2 escaped, 3 non-finite; needs SALI */
  double *sali_final; /* [n] SALI at t_end */
  double *sali_min;   /* [n] min SALI over checkpoints */
  double *t_chaos;    /* [n] first checkpoint time with SALI < threshold, NaN if none */
  double *gali;       /* [n][gali_kmax - 1] GALI_2..GALI_kmax at t_end */
  double *lyap;       /* [n][n_lyap] finite-time exponents at t_end, QR order */
  double *ld;         /* [n] M-function over [0, t_end] */
  double *energy_err; /* [n] max |H - H(0)| */
  double *ln_growth;  /* [n][m_s] sum of ln |w_v| over renormalisations */
  int64_t *steps;     /* [n][2] accepted and rejected steps of the adaptive
                         solver (zeros for the fixed-step integrators) */
  double *step_err;   /* [n][2] the adaptive solver's error estimate of its
                         accepted steps (Functionalities section: the error of
                         each integration step): the largest and the last.
                         The estimate is the scaled DOP853 one the step-size
                         control compares with 1, so both are <= 1; 0 before
                         the first accepted step and for the fixed-step
                         integrators; NaN for masked orbits */
} chx_result;

/* Whole-ensemble integration (Functionalities section: the solvers with
 * deviation-vector normalisation and QR, plus SALI, GALI and LD).
 * x0: [n][2N] initial conditions; mask: [n] (0 = skip) or NULL. */
chx_status chx_integrate_ensemble(const chx_system *sys, const double *x0,
                                  const uint8_t *mask, int64_t n,
                                  const chx_options *opt, chx_result *res);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as chx_integrate_ensemble, with the same arguments, outputs and
 * results, but it calls no hipMalloc, hipFree or other allocating routine.
 * Its working buffers come from a library-owned device array of
 * CHX_NOALLOC_MAX_BYTES that every GPU the library runs on holds until the
 * process ends.  Restrictions: CHX_PTR_DEVICE is required (x0, mask,
 * opt->w0 and every output are device pointers, read and written in place;
 * opt->stream orders the work); built-in systems only (custom systems
 * return CHX_ERR_UNSUPPORTED).  The workspace needed grows with n: about
 * (2N(M + 1) + M + 15) doubles and (M + 1) ints per initial condition,
 * with M = the deviation vectors (plus gali_kmax * 2N doubles when GALI is
 * an output); a call that needs more than CHX_NOALLOC_MAX_BYTES returns
 * CHX_ERR_INVALID_ARG before any device work, its message giving the
 * figure.  Calls that overlap in time on one GPU share its array and race:
 * serialise them.  The call synchronises the stream once (it reads the
 * number of unmasked orbits). */
#define CHX_NOALLOC_MAX_BYTES (64ull << 20)
chx_status chx_integrate_ensemble_noalloc(const chx_system *sys, const double *x0,
                                          const uint8_t *mask, int64_t n,
                                          const chx_options *opt, chx_result *res);

/* Host-pointer convenience calls (synchronous). */
/* SALI (Functionalities section) with two seeded unit vectors, K = 10:
 * min SALI over checkpoints and the label (0 regular, 1 chaotic at 1e-8). */
chx_status chx_sali(const chx_system *sys, const double *x0, int64_t n, double dt,
                    double T, uint64_t seed, double *sali_min_out, int8_t *label_out);
/* GALI_k, k = 2..kmax, of kmax seeded unit vectors renormalised every 10
 * steps (Functionalities section: GALI from the singular values). */
chx_status chx_gali(const chx_system *sys, const double *x0, int64_t n, double dt,
                    double T, int32_t kmax, uint64_t seed,
                    double *gali_out /* [n][kmax-1] */);
/* First n_exp Lyapunov exponents by QR every renorm_every steps
 * (Functionalities section: Lyapunov spectrum via QR factorisation). */
chx_status chx_lyap_spectrum(const chx_system *sys, const double *x0, int64_t n,
                             double dt, double T, int32_t n_exp, int32_t renorm_every,
                             double *lyap_out /* [n][n_exp] */);
/* Lagrangian-descriptor M-function int_0^T sum_i |dx_i/dt|^p dt (Summary and
 * Functionalities sections; trapezoid rule on the step endpoints). */
chx_status chx_ld(const chx_system *sys, const double *x0, int64_t n, double dt,
                  double T, double p, double *ld_out /* [n] */);

/* Chaos indicators from the Lagrangian descriptors of neighbouring orbits
 * (Functionalities section: chaos indicators based on Lagrangian
 * descriptors, and the generation of neighbouring trajectories for them;
 * the paper defers their definitions to the works it cites, and these are
 * the forms used here).  For each initial condition x:
 *   L(x) = M+(x) + M-(x): the M-function of chx_ld over [0, T] plus the
 *     same over [-T, 0] (two_sided; M+ alone otherwise).  M- is computed as
 *     M+ of the momentum-reversed state (q, -p): every built-in Hamiltonian
 *     and every separable user system is even in the momenta, so the
 *     backward orbit is the reflection of that forward orbit and |dx/dt|
 *     has the same components; a general user system
 *     (CHX_SYS_CUSTOM_GENERAL) may not be, and two_sided is refused for it
 *     with CHX_ERR_UNSUPPORTED;
 *   neighbours y_i^(+/-) = x +/- sigma e_c for each coordinate c of the 2N
 *     phase-space coordinates whose bit is set in dirs (n of them);
 *   D = (1/2n) sum_i (|L(x) - L(y_i^+)| + |L(x) - L(y_i^-)|) / L(x)
 *     (difference), R = |1 - (1/2n) sum_i (L(y_i^+) + L(y_i^-)) / L(x)|
 *     (ratio), S = (1/n) sum_i |L(y_i^+) - 2 L(x) + L(y_i^-)| / L(x)
 *     (second derivative).
 * The (1 + 2n) x (2 if two_sided) orbits per initial condition are built on
 * the device and integrated as one ensemble with the LD alone (no
 * variational equations); opt gives dt, T, ld_p, the integrator (and
 * rtol/atol), escape_r2, steps_per_launch, block_size, flags and stream;
 * opt->indicators must be 0 or CHX_IND_LD, opt->w0 NULL, early_exit 0.
 * x0 [n][2N], mask [n] or NULL; all pointers host or device per
 * opt->flags.  Output status[i]: CHX_ORBIT_MASKED for masked initial
 * conditions; otherwise the worst over the member orbits (NONFINITE over
 * STEP_FAILED over ESCAPED over OK), and NaN indicators unless OK.  Device
 * memory of about (1 + 2n)(2)(2N + 30) doubles per initial condition is
 * held during the call.  Any NULL output is skipped. */
typedef struct {
  uint32_t dirs;     /* bit c: neighbours along coordinate c; 0 -> all 2N */
  double sigma;      /* neighbour distance, finite and > 0 */
  int32_t two_sided; /* non-zero: L over [-T, T]; 0: over [0, T] */
} chx_ldn_options;
typedef struct {
  double *ld;       /* [n] L(x) */
  double *D;        /* [n] */
  double *R;        /* [n] */
  double *S;        /* [n] */
  int32_t *status;  /* [n] */
} chx_ldn_result;
chx_status chx_ld_indicators(const chx_system *sys, const double *x0, const uint8_t *mask,
                             int64_t n, const chx_options *opt, const chx_ldn_options *lo,
                             chx_ldn_result *res);

/* Resumable ensemble: checkpoint/resume and chunked launches.  create
 * validates and uploads (no steps); advance integrates up to step s_end,
 * which must be a checkpoint step (a multiple of K, or the last step);
 * results may be read at any checkpoint.  Splitting a run at checkpoints
 * gives results bit-identical to one call. */
typedef struct chx_ensemble chx_ensemble;
chx_status chx_ensemble_create(const chx_system *sys, const double *x0,
                               const uint8_t *mask, int64_t n, const chx_options *opt,
                               chx_ensemble **out);
chx_status chx_ensemble_advance(chx_ensemble *e, int64_t s_end);
chx_status chx_ensemble_results(chx_ensemble *e, chx_result *res);
/* n_total steps, steps done, orbits actually integrated (unmasked). */
chx_status chx_ensemble_info(const chx_ensemble *e, int64_t *n_total, int64_t *s_done,
                             int64_t *n_active);
void chx_ensemble_destroy(chx_ensemble *e);
/* Continue only part of an ensemble: *out is a new ensemble holding the
 * active (unmasked) orbits of e with keep[i] != 0, i < n of e, in increasing
 * i, with their current state, accumulated indicators and step count, so
 * advancing it gives each kept orbit exactly the results it would have had
 * in e.  Its orbits are numbered 0..n2-1 (n2 from chx_ensemble_info);
 * results() arrays have n2 rows.  keep is host or device memory as e's
 * pointers were at creation; e is not changed.  Used to resume a small
 * unresolved part of a large ensemble without idle lanes. */
chx_status chx_ensemble_subset(chx_ensemble *e, const uint8_t *keep, chx_ensemble **out);

/* Batched persistent integration: several systems in one persistent
 * launch, orbits leaving at their first checkpoint with SALI below the
 * threshold when early_exit is set, freed slots refilled at once, repeated
 * launches replayed from a captured hipGraph.  Each item is one system with
 * its own initial conditions, mask, dt and T (T/dt must be a multiple of
 * renorm_every).  Supported items: Henon-Heiles, coupled quartic with
 * ndof 3, FPU with ndof 8 or 16; two deviation vectors per orbit (SALI
 * required; GALI and Lyapunov not available here; LD and energy allowed);
 * opt->w0 must be NULL (item i draws its vectors with seed opt->seed + i);
 * at most 4 items.  opt->block_size and opt->steps_per_launch fix the
 * threads per block and the steps per launch; 0 lets the autotuner choose
 * (it times short probe launches on copies of the ensembles, per system and
 * block size; timings are cached for the process and, if the environment
 * variable CHX_AUTOTUNE_CACHE names a file, in that file).  Results per
 * item as for chx_integrate_ensemble.  stats may be NULL. */
typedef struct {
  chx_system sys;
  const double *x0;     /* [n][2N] */
  const uint8_t *mask;  /* [n] or NULL */
  int64_t n;
  double dt, T;
} chx_batch_item;
typedef struct {
  int32_t threads_per_block, blocks, launches, from_cache;
  int64_t steps_per_launch;
  double integrate_ms;        /* GPU time of the persistent launches */
  int64_t orbit_steps[4];     /* steps integrated per item (sum over orbits) */
  double cost_ps[4];          /* autotuned GPU time per orbit-step, picoseconds */
} chx_batch_stats;
chx_status chx_integrate_batched(const chx_batch_item *items, int32_t n_items,
                                 const chx_options *opt, chx_result *per_item,
                                 chx_batch_stats *stats);

/* Initial-condition assembly. */
/* Henon-Heiles surface of section x = 0 at energy E (Examples section):
 * y_i = y0 + (y1-y0) i/(ny-1), p_y,j likewise, index j*ny + i;
 * p_x = +sqrt(2E - p_y^2 - y^2 + 2y^3/3), mask = 0 where the root's
 * argument is negative (p_x written as 0).  x0_out [ny*npy][4], mask_out. */
chx_status chx_grid_hh_section(double E, double y0, double y1, int32_t ny, double py0,
                               double py1, int32_t npy, double *x0_out,
                               uint8_t *mask_out, uint32_t flags, void *stream);
/* Same for given (y, p_y) lists of length n. */
chx_status chx_hh_section_points(double E, const double *y, const double *py, int64_t n,
                                 double *x0_out, uint8_t *mask_out, uint32_t flags,
                                 void *stream);
/* FPU chain with its energy in the two lowest normal modes of the fixed-end
 * linear chain: u [n][5] uniforms in [0,1): E = 0.1 + 9.9 u0, amplitudes
 * u1, u2, phases 2 pi u3, 2 pi u4; scaled so that H = E. */
chx_status chx_ic_fput_modes(const chx_system *sys, const double *u, int64_t n,
                             double *x0_out, uint32_t flags, void *stream);
/* Coupled quartic oscillator at H = 1 from draws [n][2N+1]: Gaussian
 * position and momentum directions and a potential fraction f in (0,1). */
chx_status chx_ic_quartic(const chx_system *sys, const double *draws, int64_t n,
                          double *x0_out, uint32_t flags, void *stream);

/* Learned gate.  The paper motivates fast chaos indicators as a way to
 * generate large labelled datasets for machine-learning models of dynamics
 * (Introduction and Related research); the gate is such a model, used to
 * label Henon-Heiles orbits from a short integration: a perceptron
 * 6 -> 256 -> 256 -> 2 with erf-GELU activations on the features
 *   f = (y, p_y, p_x, LD(t)/t, G_1(t)/t, G_2(t)/t),
 * (x0 = (x, y, p_x, p_y); LD the M-function; G_v the ln-growth of the two
 * SALI vectors, chx_result.ln_growth) z-scored with the training-set mean
 * and standard deviation.  Products in BF16 with FP32 accumulation (MFMA),
 * FP32 master parameters, softmax cross-entropy, AdamW.  All arithmetic is
 * done by the library's kernels on the current device.
 * Parameters, flat FP32 [CHX_GATE_NPARAM]: W1[16][256] (rows 6..15 zero),
 * b1[256], W2[256][256], b2[256], W3[256][16] (columns 2..15 zero), b3[16]
 * (2..15 zero); logits z = (a2 W3 + b3)[0..1], p(chaotic) = softmax(z)[1]. */
#define CHX_GATE_NFEAT 6
#define CHX_GATE_NPARAM 74256
typedef struct chx_gate chx_gate;
typedef struct {
  int32_t epochs;       /* passes over the training set; 0 -> 1 */
  int32_t batch;        /* rows per step: multiple of 16 in 16..65536; 0 -> 4096 */
  float lr;             /* 0 -> 1e-3 */
  float beta1, beta2;   /* 0 -> 0.9, 0.999 */
  float eps;            /* 0 -> 1e-8 */
  float weight_decay;   /* decoupled (AdamW), >= 0 */
  uint64_t seed;        /* epoch permutations */
} chx_gate_train_cfg;
typedef struct {
  int64_t n_active;     /* unmasked orbits */
  int64_t n_early;      /* stopped before the gate time (label known) */
  int64_t n_accepted;   /* labelled by the gate */
  int64_t n_fallback;   /* integrated on to T */
  double ms_gate;       /* integration to the gate time */
  double ms_infer;      /* features + inference + selection */
  double ms_fallback;   /* subset + integration to T + merge */
} chx_gate_stats;
/* New gate with weights drawn N(0, 2/fan_in) from SplitMix64(seed), zero
 * biases, identity feature scaling. */
chx_status chx_gate_create(uint64_t seed, chx_gate **out);
void chx_gate_destroy(chx_gate *g);
/* Train on features [n][6] (FP32) and labels [n] (1 chaotic, 0 regular;
 * other values contribute nothing but still count in the batch mean).  The
 * first call (or one with reset_stats != 0) sets the z-score statistics
 * from these features.  epoch_loss: host [epochs] mean loss per epoch, or
 * NULL.  Pointers per flags; synchronous. */
chx_status chx_gate_train(chx_gate *g, const float *features, const int8_t *labels, int64_t n,
                          const chx_gate_train_cfg *cfg, int32_t reset_stats,
                          float *epoch_loss, uint32_t flags, void *stream);
/* Mean loss over n <= 65536 rows and its gradient (host [CHX_GATE_NPARAM],
 * zero on padded entries), without updating anything. */
chx_status chx_gate_grad(chx_gate *g, const float *features, const int8_t *labels, int64_t n,
                         float *grad_out, float *loss_out, uint32_t flags, void *stream);
/* p(chaotic) and confidence max(p, 1 - p) per row; either output may be NULL. */
chx_status chx_gate_infer(const chx_gate *g, const float *features, int64_t n,
                          float *p_chaotic, float *confidence, uint32_t flags, void *stream);
/* Read (any output may be NULL) or replace the parameters and the z-score
 * mean / inverse standard deviation [6] (host memory).  Replacing zeroes
 * the padded entries and the optimiser state. */
chx_status chx_gate_get(const chx_gate *g, float *params, float *mean, float *istd);
chx_status chx_gate_set(chx_gate *g, const float *params, const float *mean, const float *istd);
/* Gate features from Henon-Heiles results at time t > 0: x0 [n][4],
 * ld [n], ln_growth [n][2] -> features [n][6]. */
chx_status chx_gate_features(const double *x0, const double *ld, const double *ln_growth,
                             double t, int64_t n, float *features_out, uint32_t flags,
                             void *stream);
/* Label a Henon-Heiles ensemble with the gate: integrate all orbits to
 * t_gate (a checkpoint time before T) with opt's indicators (SALI and LD
 * required, GALI and Lyapunov not allowed), compute the features and the
 * gate's confidence; orbits already stopped keep their label, confident
 * ones (confidence >= conf_min) take the gate's label (p >= 0.5: chaotic),
 * and the rest are resumed from their t_gate state on a compacted ensemble
 * (chx_ensemble_subset) and integrated to T, taking the plain label.
 * label_out [n] as chx_result.label; source_out [n] (or NULL): 0 masked,
 * 1 stopped before t_gate, 2 gate, 3 integrated to T; confidence_out [n]
 * (or NULL; NaN where not evaluated); stats may be NULL. */
chx_status chx_gate_classify(const chx_gate *g, const chx_system *sys, const double *x0,
                             const uint8_t *mask, int64_t n, const chx_options *opt,
                             double t_gate, float conf_min, int8_t *label_out,
                             uint8_t *source_out, float *confidence_out,
                             chx_gate_stats *stats);

/* Releases what the library keeps on the devices between calls: the code
 * objects of user-supplied systems (CHX_SYS_CUSTOM, CHX_SYS_CUSTOM_GENERAL),
 * loaded on each device that ran one.  Each such device is synchronised
 * first; the compiled code stays cached in host memory and is loaded again
 * on its next use, so ensembles and calls made afterwards work as before.
 * Everything else the library allocates lives for one call (or for an
 * ensemble or gate, which its owner destroys), so there is nothing else to
 * release.  Library housekeeping, not an operation of the paper.  No other
 * call of the library may run concurrently.  CHX_ERR_DEVICE if a device
 * call fails (the remaining code objects are still unloaded). */
chx_status chx_shutdown(void);

/* Message for the last non-OK status on this thread ("" if none). */
const char *chx_last_error(void);
/* Library version string. */
const char *chx_version(void);
/* sizeof(chx_system), sizeof(chx_options), sizeof(chx_result),
 * sizeof(chx_batch_item), sizeof(chx_batch_stats), sizeof(chx_gate_train_cfg),
 * sizeof(chx_gate_stats), sizeof(chx_ldn_options), sizeof(chx_ldn_result) for
 * which = 0..8 (0 otherwise): lets a binding check its struct layouts. */
size_t chx_struct_size(int32_t which);

#ifdef __cplusplus
}
#endif
#endif
