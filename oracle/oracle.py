"""ctypes front end of the oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It loads oracle/libchx_oracle.so (built by
oracle/build.py with gcc, no FMA contraction) and exposes the plain FP64
reference: the systems of the paper's Examples section, the Yoshida-4 step
with its tangent map, the fixed-step DOP853 step of the state, the
variational equations and the LD integrand, and the per-orbit chaos-indicator driver (SALI, GALI_k,
Lyapunov spectrum by modified Gram-Schmidt QR, Lagrangian-descriptor
M-function, energy error) with resumable state.
"""
import ctypes as C
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

SYS_HENON_HEILES = 1
SYS_FPUT = 2
SYS_QUARTIC = 3
SYS_HARMONIC = 4
SYS_DOUBLE_PENDULUM = 5

IND_SALI = 1
IND_GALI = 2
IND_LYAP = 4
IND_LD = 8
IND_ENERGY = 16

ST_OK, ST_MASKED, ST_ESCAPED, ST_NONFINITE, ST_EXITED, ST_STEPFAIL = 0, 1, 2, 3, 4, 5

INT_YOSHIDA4 = 0
INT_DOP853 = 1
INT_DOP853_ADAPTIVE = 2

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        d, i, i64, u32 = C.c_double, C.c_int, C.c_int64, C.c_uint32
        P = C.c_void_p
        L.ora_potential.restype = d
        L.ora_potential.argtypes = [i, i, P, P]
        L.ora_hamiltonian.restype = d
        L.ora_hamiltonian.argtypes = [i, i, P, P]
        for f in (L.ora_grad, L.ora_hess):
            f.restype = None
            f.argtypes = [i, i, P, P, P]
        L.ora_yoshida_coefficients.argtypes = [P, P]
        L.ora_step.argtypes = [i, i, P, d, P, P, i]
        L.ora_state_len.restype = i64
        L.ora_state_len.argtypes = [i, i, i]
        L.ora_init.restype = i
        L.ora_init.argtypes = [i, i, P, P, P, P, i64, i, i, u32, d, P]
        L.ora_advance.restype = i
        L.ora_advance.argtypes = [i, i, P, P, i64, i, i, u32, d, i64, i64, i64, i, d, d,
                                  i, d]
        L.ora_advance_with.restype = i
        L.ora_advance_with.argtypes = L.ora_advance.argtypes + [i]
        L.ora_dop853_tableau.argtypes = [P, P, P]
        L.ora_dp_rhs.argtypes = [P, P, P, P, P]
        L.ora_dop853_error_weights.argtypes = [P, P]
        L.ora_advance_adaptive.restype = i
        L.ora_advance_adaptive.argtypes = L.ora_advance.argtypes + [d, d]
        L.ora_step_counts.argtypes = [i, P, i64, i, i, P, P]
        L.ora_step_errors.argtypes = [i, P, i64, i, i, P, P]
        L.ora_dop853_step.argtypes = [i, i, P, d, P, P, i, i, d, P]
        L.ora_finalize.restype = i
        L.ora_finalize.argtypes = [i, P, i64, i, i, u32, i, d] + [P] * 12
        L.ora_gali.argtypes = [i, i, P, i, P]
        L.ora_mgs.argtypes = [i, i, P, P]
        L.ora_hh_grid.argtypes = [d, d, d, i, d, d, i, P, P]
        L.ora_hh_points.argtypes = [d, P, P, i64, P, P]
        L.ora_fput_ic.argtypes = [i, P, P, i64, P]
        L.ora_quartic_ic.argtypes = [i, P, P, i64, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


@dataclass
class System:
    kind: int
    ndof: int
    params: tuple = ()

    def parr(self):
        return np.ascontiguousarray(np.asarray(self.params if self.params else [0.0],
                                               dtype=np.float64))


def henon_heiles():
    return System(SYS_HENON_HEILES, 2, ())


def fput(N, k=1.0, alpha=0.0, beta=1.0):
    return System(SYS_FPUT, N, (k, alpha, beta))


def quartic(N=3, eps=0.1):
    return System(SYS_QUARTIC, N, (eps,))


def harmonic(omegas):
    return System(SYS_HARMONIC, len(omegas), tuple(float(w) for w in omegas))


def double_pendulum(alpha=1.0, sigma=1.0):
    """The dimensionless double pendulum; x = (theta_1, theta_2, p_1, p_2)."""
    return System(SYS_DOUBLE_PENDULUM, 2, (float(alpha), float(sigma)))


def dp_rhs(sys, x, dx=None):
    """f(x) of the double pendulum, and Df(x) dx when dx is given."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    f, df = np.zeros(4), np.zeros(4)
    d = None if dx is None else np.ascontiguousarray(dx, dtype=np.float64)
    lib().ora_dp_rhs(_p(sys.parr()), _p(x), _p(d), _p(f), _p(df) if d is not None else None)
    return f if dx is None else (f, df)


# --- systems ---------------------------------------------------------------

def potential(sys, q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    pr = sys.parr()
    return lib().ora_potential(sys.kind, sys.ndof, _p(pr), _p(q))


def hamiltonian(sys, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    pr = sys.parr()
    return lib().ora_hamiltonian(sys.kind, sys.ndof, _p(pr), _p(x))


def grad(sys, q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    g = np.zeros(sys.ndof)
    pr = sys.parr()
    lib().ora_grad(sys.kind, sys.ndof, _p(pr), _p(q), _p(g))
    return g


def hess(sys, q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    h = np.zeros((sys.ndof, sys.ndof))
    pr = sys.parr()
    lib().ora_hess(sys.kind, sys.ndof, _p(pr), _p(q), _p(h))
    return h


def yoshida_coefficients():
    c = np.zeros(3)
    d = np.zeros(4)
    lib().ora_yoshida_coefficients(_p(c), _p(d))
    return c, d


def step(sys, dt, x, w=None, nsteps=1):
    """Apply nsteps Yoshida-4 KDK steps to a copy of x[2N] (and w[m][2N])."""
    x = np.array(x, dtype=np.float64)
    m = 0 if w is None else len(w)
    w = np.zeros((0, 2 * sys.ndof)) if w is None else np.array(w, dtype=np.float64)
    pr = sys.parr()
    for _ in range(nsteps):
        lib().ora_step(sys.kind, sys.ndof, _p(pr), dt, _p(x), _p(w), m)
    return (x, w) if m else x


def dop853_tableau():
    """Nodes c[12], matrix a[12][12] and weights b[12] of DOP853."""
    c, a, b = np.zeros(12), np.zeros((12, 12)), np.zeros(12)
    lib().ora_dop853_tableau(_p(c), _p(a), _p(b))
    return c, a, b


def dop853_error_weights():
    """er[12] (eighth- minus fifth-order weights) and bhh[3] (third-order
    weights on stages 1, 9, 12) of DOP853's error estimate."""
    er, bhh = np.zeros(12), np.zeros(3)
    lib().ora_dop853_error_weights(_p(er), _p(bhh))
    return er, bhh


def dop853_step(sys, dt, x, w=None, nsteps=1, ld=None, ld_p=0.5):
    """Apply nsteps fixed DOP853 steps to a copy of x[2N] (and w[m][2N]; and
    the LD M-function when ld is a number).  Returns x, (x, w), (x, ld) or
    (x, w, ld) accordingly."""
    x = np.array(x, dtype=np.float64)
    m = 0 if w is None else len(w)
    w = np.zeros((0, 2 * sys.ndof)) if w is None else np.array(w, dtype=np.float64)
    m_ld = np.array([0.0 if ld is None else float(ld)])
    pr = sys.parr()
    for _ in range(nsteps):
        lib().ora_dop853_step(sys.kind, sys.ndof, _p(pr), dt, _p(x), _p(w), m,
                              0 if ld is None else 1, ld_p, _p(m_ld))
    out = (x,) + ((w,) if m else ()) + ((m_ld[0],) if ld is not None else ())
    return out[0] if len(out) == 1 else out


def mgs(w):
    w = np.array(w, dtype=np.float64)
    m, dim = w.shape
    rd = np.zeros(m)
    lib().ora_mgs(dim, m, _p(w), _p(rd))
    return w, rd


def gali(w, kmax):
    w = np.ascontiguousarray(w, dtype=np.float64)
    m, dim = w.shape
    out = np.zeros(kmax - 1)
    lib().ora_gali(dim, m, _p(w), kmax, _p(out))
    return out


# --- driver ----------------------------------------------------------------

def n_steps_for(T, dt):
    """Number of steps n = round(T/dt); T/dt must be integral to 1e-9 relative."""
    r = T / dt
    n = int(round(r))
    if n < 1 or abs(r - n) > 1e-9 * n:
        raise ValueError("T/dt must be a positive integer (to 1e-9 relative)")
    return n


@dataclass
class Run:
    """Everything one integration needs besides the initial conditions."""
    dt: float
    T: float
    indicators: int
    K: int = 10
    n_lyap: int = 0
    gali_kmax: int = 0
    ld_p: float = 0.5
    sali_threshold: float = 1e-8
    early_exit: bool = False
    escape_r2: float = 0.0
    m_s: int = field(default=-1)
    integrator: int = INT_YOSHIDA4
    rtol: float = 1e-10   # adaptive DOP8(5) only
    atol: float = 1e-10

    def __post_init__(self):
        if self.m_s < 0:
            ms = 0
            if self.indicators & IND_SALI:
                ms = 2
            if self.indicators & IND_GALI:
                ms = max(ms, self.gali_kmax)
            self.m_s = ms
        if not (self.indicators & IND_LYAP):
            self.n_lyap = 0


class State:
    """Resumable per-orbit oracle state: [n][len] doubles."""

    def __init__(self, sys, run, x0, w0=None, mask=None):
        self.sys, self.run = sys, run
        x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1, 2 * sys.ndof)
        self.n = len(x0)
        self.len = lib().ora_state_len(sys.ndof, run.m_s, run.n_lyap)
        self.buf = np.zeros((self.n, self.len))
        if run.m_s:
            w0 = np.ascontiguousarray(w0, dtype=np.float64).reshape(
                self.n, run.m_s, 2 * sys.ndof)
        else:
            w0 = None
        mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        pr = sys.parr()
        rc = lib().ora_init(sys.kind, sys.ndof, _p(pr), _p(x0), _p(w0), _p(mask), self.n,
                            run.m_s, run.n_lyap, run.indicators, run.ld_p, _p(self.buf))
        if rc:
            raise ValueError("ora_init failed")
        self.s_done = 0
        self.n_total = n_steps_for(run.T, run.dt)

    def advance(self, s_end, threads=1):
        run, sys = self.run, self.sys
        s_end = min(s_end, self.n_total)
        pr = sys.parr()

        def work(lo, hi):
            sub = self.buf[lo:hi]
            assert sub.flags.c_contiguous
            if run.integrator == INT_DOP853_ADAPTIVE:
                rc = lib().ora_advance_adaptive(
                    sys.kind, sys.ndof, _p(pr), _p(sub), hi - lo, run.m_s, run.n_lyap,
                    run.indicators, run.dt, self.s_done, s_end, self.n_total, run.K, run.ld_p,
                    run.sali_threshold, int(run.early_exit), run.escape_r2, run.rtol, run.atol)
                if rc:
                    raise RuntimeError("ora_advance_adaptive failed (%d)" % rc)
                return
            rc = lib().ora_advance_with(sys.kind, sys.ndof, _p(pr), _p(sub), hi - lo,
                                        run.m_s, run.n_lyap, run.indicators, run.dt,
                                        self.s_done, s_end, self.n_total, run.K, run.ld_p,
                                        run.sali_threshold, int(run.early_exit),
                                        run.escape_r2, run.integrator)
            if rc:
                raise RuntimeError("ora_advance failed (%d)" % rc)

        _parallel(work, self.n, threads)
        self.s_done = s_end

    def step_counts(self):
        """Accepted and rejected steps per orbit (adaptive driver)."""
        acc = np.zeros(self.n, np.int64)
        rej = np.zeros(self.n, np.int64)
        lib().ora_step_counts(self.sys.ndof, _p(self.buf), self.n, self.run.m_s,
                              self.run.n_lyap, _p(acc), _p(rej))
        return acc, rej

    def step_errors(self):
        """Largest and last error estimate of the accepted steps per orbit
        (adaptive driver), as [n][2]."""
        emax = np.zeros(self.n)
        elast = np.zeros(self.n)
        lib().ora_step_errors(self.sys.ndof, _p(self.buf), self.n, self.run.m_s,
                              self.run.n_lyap, _p(emax), _p(elast))
        return np.stack([emax, elast], axis=1)

    def finalize(self):
        run, sys, n, N2 = self.run, self.sys, self.n, 2 * self.sys.ndof
        o = dict(
            x_final=np.zeros((n, N2)), t_end=np.zeros(n),
            status=np.zeros(n, np.int32), label=np.zeros(n, np.int8),
            sali_final=np.zeros(n), sali_min=np.zeros(n), t_chaos=np.zeros(n),
            gali=np.zeros((n, max(run.gali_kmax - 1, 0))),
            lyap=np.zeros((n, run.n_lyap)), ld=np.zeros(n), energy_err=np.zeros(n),
            ln_growth=np.zeros((n, run.m_s)))
        keys = ["x_final", "t_end", "status", "label", "sali_final", "sali_min", "t_chaos",
                "gali", "lyap", "ld", "energy_err", "ln_growth"]
        kmax = run.gali_kmax if run.indicators & IND_GALI else 0
        lib().ora_finalize(sys.ndof, _p(self.buf), n, run.m_s, run.n_lyap, run.indicators,
                           kmax, run.sali_threshold, *[_p(o[k]) for k in keys])
        if not kmax:
            o["gali"] = np.zeros((n, 0))
        return o


def _parallel(fn, n, threads):
    if threads <= 1 or n < 2:
        fn(0, n)
        return
    chunks = np.linspace(0, n, min(threads, n) + 1).astype(int)
    with ThreadPoolExecutor(max_workers=len(chunks) - 1) as ex:
        futs = [ex.submit(fn, int(a), int(b)) for a, b in zip(chunks[:-1], chunks[1:])]
        for f in futs:
            f.result()


def integrate(sys, x0, run, w0=None, mask=None, threads=1):
    st = State(sys, run, x0, w0, mask)
    st.advance(st.n_total, threads=threads)
    out = st.finalize()
    if run.integrator == INT_DOP853_ADAPTIVE:
        out["steps_accepted"], out["steps_rejected"] = st.step_counts()
        out["step_err"] = st.step_errors()
    return out


# --- inputs ----------------------------------------------------------------

def hh_grid(E, ny, npy, y0=-0.4, y1=0.7, py0=-0.45, py1=0.45):
    x0 = np.zeros((ny * npy, 4))
    mask = np.zeros(ny * npy, np.uint8)
    lib().ora_hh_grid(E, y0, y1, ny, py0, py1, npy, _p(x0), _p(mask))
    return x0, mask


def hh_points(E, y, py):
    y = np.ascontiguousarray(y, dtype=np.float64)
    py = np.ascontiguousarray(py, dtype=np.float64)
    n = len(y)
    x0 = np.zeros((n, 4))
    mask = np.zeros(n, np.uint8)
    lib().ora_hh_points(E, _p(y), _p(py), n, _p(x0), _p(mask))
    return x0, mask


def fput_ic(sys, u):
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 5)
    x0 = np.zeros((len(u), 2 * sys.ndof))
    pr = sys.parr()
    lib().ora_fput_ic(sys.ndof, _p(pr), _p(u), len(u), _p(x0))
    return x0


def quartic_ic(sys, draws):
    draws = np.ascontiguousarray(draws, dtype=np.float64).reshape(-1, 2 * sys.ndof + 1)
    x0 = np.zeros((len(draws), 2 * sys.ndof))
    pr = sys.parr()
    lib().ora_quartic_ic(sys.ndof, _p(pr), _p(draws), len(draws), _p(x0))
    return x0



# --- chaos indicators from the LDs of neighbouring orbits ------------------
#
# Functionalities section: chaos indicators based on Lagrangian descriptors,
# with the generation of neighbouring trajectories for them; the paper
# defers their definitions to the works it cites.  Reading taken here:
#   * L(x) = M+(x) + M-(x), the p-norm M-function over [-T, T] (forward and
#     backward parts; forward only when two_sided is False);
#   * the backward part of an orbit of a Hamiltonian even in the momenta is
#     the forward part of its momentum-reversed state: x(-t) = R y(t) with
#     y the orbit of R x, R(q, p) = (q, -p), and |dx/dt| has the same
#     components along both, so M-(x) = M+(R x);
#   * neighbours y_i^(+/-) = x +/- sigma e_{d_i} along the chosen phase-space
#     coordinates d_1..d_n;
#   * D = (1/2n) sum_i (|L(x) - L(y_i^+)| + |L(x) - L(y_i^-)|) / L(x),
#     R = |1 - (1/2n) sum_i (L(y_i^+) + L(y_i^-)) / L(x)|,
#     S = (1/n) sum_i |L(y_i^+) - 2 L(x) + L(y_i^-)| / L(x)
#     (difference, ratio and second derivative of the LDs of neighbouring
#     orbits);
#   * an initial condition whose own orbit or any neighbour's (forward or
#     backward) stops early reports the worst status (non-finite over
#     step failure over escape) and NaN indicators; masked ones status 1.

def ldn_members(x0, dirs, sigma, two_sided=True):
    """The orbits an indicator needs, [n][nb][nm][2N]: b = 0 forward
    states, b = 1 momentum-reversed ones (two_sided); m = 0 the state
    itself, m = 2i+1 and 2i+2 the neighbours +sigma e_{dirs[i]} and
    -sigma e_{dirs[i]}."""
    x0 = np.asarray(x0, dtype=np.float64)
    n, D = x0.shape
    N = D // 2
    nb, nm = (2 if two_sided else 1), 1 + 2 * len(dirs)
    out = np.zeros((n, nb, nm, D))
    for j in range(n):
        for m in range(nm):
            y = x0[j].copy()
            if m > 0:
                c = dirs[(m - 1) // 2]
                y[c] = y[c] + (sigma if m % 2 == 1 else -sigma)
            out[j, 0, m] = y
            if two_sided:
                r = y.copy()
                r[N:] = -r[N:]
                out[j, 1, m] = r
    return out


def ldn_combine(ld, status):
    """Indicators from the members' LDs [n][nb][nm] and statuses."""
    n, nb, nm = ld.shape
    k = (nm - 1) // 2
    L = ld.sum(axis=1)
    res = {"ld": np.full(n, np.nan), "D": np.full(n, np.nan), "R": np.full(n, np.nan),
           "S": np.full(n, np.nan), "status": np.zeros(n, np.int32)}
    rank = {ST_OK: 0, ST_ESCAPED: 1, ST_STEPFAIL: 2, ST_NONFINITE: 3}
    for j in range(n):
        worst = ST_OK
        for s in status[j].ravel():
            if rank[int(s)] > rank[worst]:
                worst = int(s)
        res["status"][j] = worst
        if worst != ST_OK:
            continue
        c = L[j, 0]
        d = r = s2 = 0.0
        for i in range(k):
            lp, lm = L[j, 2 * i + 1], L[j, 2 * i + 2]
            d += abs(c - lp) + abs(c - lm)
            r += lp + lm
            s2 += abs(lp - 2.0 * c + lm)
        res["ld"][j] = c
        res["D"][j] = d / (2 * k) / c
        res["R"][j] = abs(1.0 - r / (2 * k) / c)
        res["S"][j] = s2 / k / c
    return res


def ld_indicators(sys, x0, run, dirs, sigma, two_sided=True, mask=None, threads=1):
    """D, R, S and L of each initial condition (reading above); run gives
    the integrator, dt, T, ld_p and escape radius (its indicators are
    replaced by the LD alone)."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1, 2 * sys.ndof)
    n = len(x0)
    mem = ldn_members(x0, dirs, sigma, two_sided)
    nb, nm = mem.shape[1], mem.shape[2]
    r2 = Run(dt=run.dt, T=run.T, indicators=IND_LD, K=run.K, ld_p=run.ld_p,
             escape_r2=run.escape_r2, integrator=run.integrator, rtol=run.rtol, atol=run.atol)
    out = integrate(sys, mem.reshape(-1, 2 * sys.ndof), r2, threads=threads)
    res = ldn_combine(out["ld"].reshape(n, nb, nm), out["status"].reshape(n, nb, nm))
    if mask is not None:
        off = np.asarray(mask) == 0
        for k in ("ld", "D", "R", "S"):
            res[k][off] = np.nan
        res["status"][off] = ST_MASKED
    return res
