"""Pins of the oracle's fixed-step DOP853 integrator (the eighth-order
Runge-Kutta method of Dormand and Prince that the paper's solvers build on,
Functionalities section) applied to the state, the variational equations and
the LD integrand as one system.

Checked against: Butcher's order conditions for every rooted tree up to
order 8 (a mistyped coefficient fails one of them), the harmonic
oscillator's closed form (eighth-order convergence), an independent solver
(SciPy's adaptive DOP853 at tight tolerance), central finite differences of
the step map (the tangent vectors follow its exact Jacobian), the closed-form
LD M-function of the oscillator over one period, and the trace of the
linearised flow (the sum of the Lyapunov exponents of a Hamiltonian flow is
zero; the method is not symplectic, so only to its truncation error).
"""
from functools import lru_cache
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.integrate import solve_ivp


# --- the tableau -------------------------------------------------------------

@lru_cache(None)
def rooted_trees(n):
    """Rooted trees with n nodes, each a sorted tuple of its subtrees."""
    if n == 1:
        return ((),)
    out = set()

    def forests(rem, acc):
        if rem == 0:
            out.add(tuple(sorted(acc)))
            return
        for k in range(1, rem + 1):
            for t in rooted_trees(k):
                forests(rem - k, acc + [t])

    forests(n - 1, [])
    return tuple(sorted(out))


def order(t):
    return 1 + sum(order(u) for u in t)


def density(t):
    g = order(t)
    for u in t:
        g *= density(u)
    return g


def order_residuals(c, a, b, pmax=8):
    """sum_i b_i Phi_i(t) - 1/gamma(t) for every rooted tree t up to pmax
    nodes, in 60-digit arithmetic on the given binary64 coefficients."""
    mp.mp.dps = 60
    s = len(b)
    A = [[mp.mpf(float(a[i][j])) for j in range(s)] for i in range(s)]
    B = [mp.mpf(float(v)) for v in b]
    memo = {}

    def phi(t):
        if t in memo:
            return memo[t]
        v = [mp.mpf(1)] * s
        for u in t:
            pu = phi(u)
            for i in range(s):
                v[i] *= mp.fsum(A[i][j] * pu[j] for j in range(i))
        memo[t] = v
        return v

    res = []
    for n in range(1, pmax + 1):
        for t in rooted_trees(n):
            lhs = mp.fsum(B[i] * phi(t)[i] for i in range(s))
            res.append((n, float(lhs - mp.mpf(1) / density(t))))
    return res


def test_tree_count():
    # 1, 1, 2, 4, 9, 20, 48, 115 rooted trees of orders 1..8 (OEIS A000081)
    assert [len(rooted_trees(n)) for n in range(1, 9)] == [1, 1, 2, 4, 9, 20, 48, 115]


def test_tableau_is_explicit_and_consistent(O):
    c, a, b = O.dop853_tableau()
    assert np.all(np.triu(a) == 0.0)  # explicit: a_ij = 0 for j >= i
    assert np.max(np.abs(a.sum(axis=1) - c)) < 2e-15  # c_i = sum_j a_ij
    assert c[0] == 0.0 and c[-1] == 1.0
    # the nodes that are rational in the published method
    assert c[5] == pytest.approx(1 / 3, abs=1e-16) and c[6] == 0.25
    assert c[7] == pytest.approx(4 / 13, abs=1e-16) and c[8] == pytest.approx(127 / 195, abs=1e-16)
    assert c[9] == pytest.approx(0.6, abs=1e-16) and c[10] == pytest.approx(6 / 7, abs=1e-16)
    # c_4, c_5 = (6 -/+ sqrt 6)/30 and c_3 = 2 c_4 / 3, c_2 = 2 c_3 / 3
    assert c[3] == pytest.approx((6 - math.sqrt(6)) / 30, abs=1e-16)
    assert c[4] == pytest.approx((6 + math.sqrt(6)) / 30, abs=1e-16)
    assert c[2] == pytest.approx(2 * c[3] / 3, abs=1e-16)
    assert c[1] == pytest.approx(2 * c[2] / 3, abs=1e-16)
    # the eighth-order solution does not use stages 2..5
    assert list(b[1:5]) == [0.0, 0.0, 0.0, 0.0]


def test_all_order_conditions_to_order_8(O):
    c, a, b = O.dop853_tableau()
    res = order_residuals(c, a, b)
    assert len(res) == 200
    worst = max(abs(r) for _, r in res)
    assert worst < 1e-13, worst


def test_order_conditions_catch_a_mistyped_coefficient(O):
    # the check above is sensitive: a change in the 11th digit of one
    # coefficient breaks conditions of order <= 8
    c, a, b = O.dop853_tableau()
    a = a.copy()
    a[8][5] *= 1 + 1e-10
    res = order_residuals(c, a, b)
    assert max(abs(r) for _, r in res) > 1e-10


# --- the integrator ----------------------------------------------------------

def test_eighth_order_convergence_harmonic(O):
    # x'' = -w^2 x: closed form after one period is the initial point
    w = 1.3
    s = O.harmonic([w])
    x0 = np.array([0.7, 0.4])
    T = 2 * math.pi / w
    errs = []
    for n in (12, 24, 48):
        x = O.dop853_step(s, T / n, x0, nsteps=n)
        errs.append(np.max(np.abs(x - x0)))
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(7.8 < p < 8.2 for p in slopes), (errs, slopes)


def hh_rhs(t, y):
    x, yy, px, py = y
    return [px, py, -x - 2 * x * yy, -yy - x * x + yy * yy]


def test_agrees_with_scipy_dop853(O):
    s = O.henon_heiles()
    x0 = np.array([0.0, 0.1, 0.45, 0.05])
    dt, n = 0.01, 5000
    x = O.dop853_step(s, dt, x0, nsteps=n)
    ref = solve_ivp(hh_rhs, (0, dt * n), x0, method="DOP853", rtol=1e-13, atol=1e-13)
    assert np.max(np.abs(x - ref.y[:, -1])) < 1e-10


def test_tangent_vectors_follow_the_step_jacobian(O):
    s = O.henon_heiles()
    x0 = np.array([0.05, -0.2, 0.4, 0.1])
    dt, n, h = 0.05, 8, 1e-6
    _, W = O.dop853_step(s, dt, x0, np.eye(4), nsteps=n)
    J = np.zeros((4, 4))
    for k in range(4):
        e = np.zeros(4)
        e[k] = h
        J[:, k] = (O.dop853_step(s, dt, x0 + e, nsteps=n) - O.dop853_step(s, dt, x0 - e, nsteps=n)) / (2 * h)
    # row v of W is the image of the unit vector e_v
    assert np.max(np.abs(W.T - J)) < 1e-8
    # for a linear system the tangent map is the step map itself
    hs = O.harmonic([0.9, 1.4])
    y0 = np.array([0.3, -0.2, 0.1, 0.5])
    _, W = O.dop853_step(hs, 0.1, y0, np.eye(4), nsteps=5)
    cols = np.array([O.dop853_step(hs, 0.1, e, nsteps=5) for e in np.eye(4)])
    assert np.max(np.abs(W - cols)) < 1e-15


B_QUARTER = 1.198140234735592  # integral of sqrt(sin t) over [0, pi/2]


def test_ld_component_closed_form_oscillator(O):
    # q = A cos t, p = -A sin t: |dq/dt|^(1/2) + |dp/dt|^(1/2) over one period
    # is 8 sqrt(A) B.  The integrand has square-root cusps at the zero
    # crossings, so the error falls like dt^1.5, not dt^8.
    s = O.harmonic([1.0])
    A = 0.64
    exact = 8 * math.sqrt(A) * B_QUARTER
    errs = []
    for n in (500, 2000):
        _, M = O.dop853_step(s, 2 * math.pi / n, [A, 0.0], nsteps=n, ld=0.0)
        errs.append(abs(M - exact))
    assert errs[0] < 2e-3 * exact
    assert errs[1] < errs[0] / 5


def test_driver_matches_the_step_and_resumes_bitwise(O):
    s = O.henon_heiles()
    x0 = np.array([[0.0, 0.1, 0.45, 0.05], [0.0, -0.3, 0.2, 0.1]])
    w0 = np.array([[[1.0, 0.2, -0.1, 0.3], [0.1, 1.0, 0.2, -0.4]]] * 2)
    run = O.Run(dt=0.01, T=3.0, indicators=O.IND_SALI | O.IND_LD | O.IND_LYAP | O.IND_ENERGY,
                K=10, n_lyap=4, integrator=O.INT_DOP853)
    full = O.integrate(s, x0, run, w0=w0)
    # state and LD do not depend on the checkpoints: the same as plain steps
    for i in range(2):
        x, M = O.dop853_step(s, 0.01, x0[i], nsteps=300, ld=0.0)
        assert np.array_equal(full["x_final"][i], x)
        assert full["ld"][i] == M
    st = O.State(s, run, x0, w0=w0)
    st.advance(120)
    st.advance(300)
    part = st.finalize()
    for k in ("x_final", "sali_min", "lyap", "ld", "energy_err"):
        assert np.array_equal(full[k], part[k]), k


def test_lyapunov_sum_and_energy(O):
    s = O.henon_heiles()
    x0 = np.array([[0.0, -0.25, 0.4330127018922193, 0.0]])
    run = O.Run(dt=0.01, T=100.0, indicators=O.IND_LYAP | O.IND_ENERGY, K=10, n_lyap=4,
                integrator=O.INT_DOP853)
    o = O.integrate(s, x0, run)
    # the flow preserves volume, so the exponents sum to zero up to the
    # method's local truncation error
    assert abs(o["lyap"][0].sum()) < 1e-10
    assert o["energy_err"][0] < 1e-12


# --- the adaptive DOP8(5) driver ---------------------------------------------

def plain_residuals(weights, a, pmax):
    """sum_i w_i Phi_i(t) for every rooted tree t up to pmax nodes."""
    mp.mp.dps = 60
    s = len(weights)
    A = [[mp.mpf(float(a[i][j])) for j in range(s)] for i in range(s)]
    W = [mp.mpf(float(v)) for v in weights]
    memo = {}

    def phi(t):
        if t in memo:
            return memo[t]
        v = [mp.mpf(1)] * s
        for u in t:
            pu = phi(u)
            for i in range(s):
                v[i] *= mp.fsum(A[i][j] * pu[j] for j in range(i))
        memo[t] = v
        return v

    out = []
    for n in range(1, pmax + 1):
        for t in rooted_trees(n):
            out.append((n, t, mp.fsum(W[i] * phi(t)[i] for i in range(s))))
    return out


def test_error_estimators_are_embedded_fifth_and_third_order(O):
    c, a, b = O.dop853_tableau()
    er, bhh = O.dop853_error_weights()
    # er = b - bhat5 of a fifth-order solution: it annihilates every tree up
    # to order 5 and not all trees of order 6
    res = plain_residuals(er, a, 6)
    assert max(abs(float(r)) for n, _, r in res if n <= 5) < 1e-13
    assert max(abs(float(r)) for n, _, r in res if n == 6) > 1e-5
    # bhh on stages 1, 9, 12 is a third-order solution: order conditions up
    # to 3 hold, some of order 4 do not
    w3 = np.zeros(12)
    w3[0], w3[8], w3[11] = bhh
    res = plain_residuals(w3, a, 4)
    assert max(abs(float(r) - 1.0 / density(t)) for n, t, r in res if n <= 3) < 1e-14
    assert max(abs(float(r) - 1.0 / density(t)) for n, t, r in res if n == 4) > 1e-3
    # the error weights use the solution's stages only
    assert np.all((er != 0) == (b != 0))


def adaptive_run(O, T, tol, dt=0.1, K=10, ind=None, n_lyap=0):
    return O.Run(dt=dt, T=T, indicators=O.IND_ENERGY if ind is None else ind, K=K,
                 n_lyap=n_lyap, integrator=O.INT_DOP853_ADAPTIVE, rtol=tol, atol=tol)


def test_adaptive_error_follows_the_tolerance(O):
    s = O.henon_heiles()
    x0 = np.array([[0.0, 0.1, 0.45, 0.05], [0.0, -0.25, 0.4330127018922193, 0.0]])
    ref = np.array([solve_ivp(hh_rhs, (0, 100.0), x, method="DOP853", rtol=1e-13,
                              atol=1e-13).y[:, -1] for x in x0])
    errs, steps = [], []
    for tol in (1e-6, 1e-8, 1e-10):
        o = O.integrate(s, x0, adaptive_run(O, 100.0, tol))
        assert np.all(o["status"] == 0) and np.all(o["t_end"] == 100.0)
        errs.append(np.max(np.abs(o["x_final"] - ref)))
        steps.append(o["steps_accepted"].sum())
        assert errs[-1] < 1e3 * tol
    assert errs[0] > errs[1] > errs[2]
    assert steps[0] < steps[1] < steps[2]


def test_adaptive_step_count_scales_like_tol_to_minus_one_eighth(O):
    # one checkpoint interval over the whole run, so the controller alone
    # sets the steps: N(tol) ~ tol^(-1/8)
    s = O.harmonic([1.0])
    x0 = np.array([[1.0, 0.0]])
    n = []
    for tol in (1e-6, 1e-10, 1e-14):
        o = O.integrate(s, x0, adaptive_run(O, 200.0, tol, dt=0.1, K=2000))
        n.append(o["steps_accepted"][0])
        exact = np.array([math.cos(200.0), -math.sin(200.0)])
        assert np.max(np.abs(o["x_final"][0] - exact)) < 1e3 * max(tol, 1e-15)
    r1, r2 = n[1] / n[0], n[2] / n[1]
    assert 2.4 < r1 < 4.0 and 2.4 < r2 < 4.0, n  # (1e4)^(1/8) = 3.16


def test_adaptive_rejections_recover(O):
    # a first step of 4 time units on a unit-frequency oscillator is
    # rejected until the controller has shrunk it; the run is still accurate
    s = O.harmonic([1.0])
    x0 = np.array([[0.3, 0.8]])
    o = O.integrate(s, x0, adaptive_run(O, 40.0, 1e-10, dt=4.0, K=1))
    assert o["steps_rejected"][0] >= 1
    t = 40.0
    exact = np.array([0.3 * math.cos(t) + 0.8 * math.sin(t), -0.3 * math.sin(t) + 0.8 * math.cos(t)])
    assert np.max(np.abs(o["x_final"][0] - exact)) < 1e-7


def test_adaptive_resume_and_checkpoint_times(O):
    s = O.henon_heiles()
    x0 = np.array([[0.0, 0.1, 0.45, 0.05], [0.0, -0.3, 0.2, 0.1]])
    w0 = np.array([[[1.0, 0.2, -0.1, 0.3], [0.1, 1.0, 0.2, -0.4]]] * 2)
    ind = O.IND_SALI | O.IND_LD | O.IND_LYAP | O.IND_ENERGY
    run = adaptive_run(O, 30.0, 1e-9, dt=0.05, K=20, ind=ind, n_lyap=4)
    full = O.integrate(s, x0, run, w0=w0)
    st = O.State(s, run, x0, w0=w0)
    st.advance(200)
    st.advance(600)
    part = st.finalize()
    acc, rej = st.step_counts()
    for k in ("x_final", "sali_min", "lyap", "ld", "energy_err", "t_end"):
        assert np.array_equal(full[k], part[k]), k
    assert np.array_equal(acc, full["steps_accepted"])
    assert np.all(full["t_end"] == 30.0)
    assert np.max(np.abs(full["lyap"].sum(axis=1))) < 1e-8


def test_adaptive_gives_up_on_an_impossible_tolerance(O):
    # tolerance 1e-40 needs steps near 1e-5: more than 100000 attempts in a
    # checkpoint interval of 1 stop the orbit
    s = O.harmonic([1.0])
    o = O.integrate(s, np.array([[1.0, 0.0]]), adaptive_run(O, 1.0, 1e-40, dt=0.1, K=10))
    assert o["status"][0] == O.ST_STEPFAIL and o["label"][0] == 3
    assert np.isnan(o["energy_err"][0])


# --- the adaptive driver's per-step error (Functionalities section: the
# error of each integration step of the adaptive solvers) ---------------------

def hh_ext_rhs(t, y):
    """Henon-Heiles with one deviation vector appended (variational
    equations): d(dq)/dt = dp, d(dp)/dt = -Hess V(q) dq."""
    x, yy, px, py, dx, dy, dpx, dpy = y
    hxx, hxy, hyy = 1 + 2 * yy, 2 * x, 1 - 2 * yy
    return np.array([px, py, -x - 2 * x * yy, -yy - x * x + yy * yy,
                     dpx, dpy, -(hxx * dx + hxy * dy), -(hxy * dx + hyy * dy)])


def scipy_error_norm(fun, y0, h, tol):
    """SciPy's DOP853 error norm of one attempted step of size h from y0
    (its own stage evaluation and estimate, rtol = atol = tol), and the
    relative rounding noise that two implementations may differ by: the
    estimate is h sum_i e_i k_i / sk, a sum of stage derivatives of size
    |k| that cancels to err sk / h, so summing in another order moves it by
    about eps |h| max|k| / (err min sk) relative (times a small count)."""
    from scipy.integrate._ivp import rk
    s = rk.DOP853(fun, 0.0, np.array(y0, float), 1e3, rtol=tol, atol=tol, first_step=h)
    y_new, _ = rk.rk_step(s.fun, 0.0, s.y, s.f, h, s.A, s.B, s.C, s.K)
    scale = tol + np.maximum(np.abs(s.y), np.abs(y_new)) * tol
    err = s._estimate_error_norm(s.K, h, scale)
    noise = 16 * np.finfo(float).eps * abs(h) * np.max(np.abs(s.K)) / (err * np.min(scale))
    return err, noise + 1e-12


@pytest.mark.parametrize("x0,h,tol", [
    ([0.0, 0.1, 0.45, 0.05], 0.2, 1e-10),
    ([0.0, -0.3, 0.2, 0.1], 0.5, 1e-8),
    ([0.0, -0.3, 0.2, 0.1], 0.3, 1e-9),
])
def test_step_error_equals_scipy_dop853_estimate(O, x0, h, tol):
    # one checkpoint interval of one step: the driver's first attempt has
    # size h, is accepted, and its estimate is both the largest and the last
    s = O.henon_heiles()
    o = O.integrate(s, np.array([x0]), adaptive_run(O, h, tol, dt=h, K=1))
    ref, noise = scipy_error_norm(lambda t, y: np.array(hh_rhs(t, y)), x0, h, tol)
    assert o["steps_accepted"][0] == 1 and o["steps_rejected"][0] == 0
    assert o["step_err"][0, 0] == o["step_err"][0, 1]
    assert abs(o["step_err"][0, 1] / ref - 1) < noise, (o["step_err"][0], ref, noise)
    assert noise < 1e-3  # a dropped stage or a wrong weight moves it by O(1)
    # the estimate is measured on the state and the deviation vectors: the
    # Lyapunov set starts as e_1, so SciPy integrates the state with e_1
    run = adaptive_run(O, h, tol, dt=h, K=1, ind=O.IND_LYAP, n_lyap=1)
    st = O.State(s, run, np.array([x0]))
    st.advance(1)
    ref_v, noise_v = scipy_error_norm(hh_ext_rhs, list(x0) + [1.0, 0.0, 0.0, 0.0], h, tol)
    assert abs(st.step_errors()[0, 1] / ref_v - 1) < noise_v, (st.step_errors()[0], ref_v)
    assert abs(ref_v / ref - 1) > 10 * (noise + noise_v)  # the vector counts


def test_step_error_bounds_and_resume(O):
    # every accepted step has an estimate <= 1; the largest bounds the last;
    # the estimates resume bitwise across launches like the rest of the state
    s = O.henon_heiles()
    x0 = np.array([[0.0, 0.1, 0.45, 0.05], [0.0, -0.3, 0.2, 0.1]])
    run = adaptive_run(O, 30.0, 1e-9, dt=0.05, K=20)
    full = O.integrate(s, x0, run)
    e = full["step_err"]
    assert np.all(e[:, 1] <= e[:, 0]) and np.all(e[:, 0] <= 1.0) and np.all(e[:, 1] > 0)
    st = O.State(s, run, x0)
    st.advance(200)
    st.advance(600)
    assert np.array_equal(st.step_errors(), e)
    # a rejected first step is not an accepted step's estimate
    o = O.integrate(O.harmonic([1.0]), np.array([[0.3, 0.8]]),
                    adaptive_run(O, 4.0, 1e-10, dt=4.0, K=1))
    assert o["steps_rejected"][0] >= 1 and o["step_err"][0, 0] <= 1.0
