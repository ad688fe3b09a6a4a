"""Pins of the oracle's Yoshida-4 step and its tangent map.

Checked against: the composition's coefficients computed to 200 bits, the
exact (rational-arithmetic) discrete map of a linear system, the harmonic
oscillator's closed-form solution (fourth-order convergence), an independent
ODE solver (SciPy's DOP853 at tight tolerance), the dt^4 scaling of the
energy error, central finite differences of the step (the tangent map is its
Jacobian), symplecticity and time-reversibility.
"""
from fractions import Fraction as F

import mpmath as mp
import numpy as np
import pytest
from scipy.integrate import solve_ivp

RNG = np.random.default_rng(777)


def true_w():
    mp.mp.prec = 200
    w1 = 1 / (2 - mp.cbrt(2))
    w0 = -mp.cbrt(2) / (2 - mp.cbrt(2))
    return float(w1), float(w0)


def test_coefficients_are_the_triple_jump(O):
    c, d = O.yoshida_coefficients()
    w1, w0 = true_w()
    # drifts w1, w0, w1; kicks the half-sums of neighbouring drifts
    assert list(c) == [w1, w0, w1]
    assert d[0] == w1 / 2 and d[3] == w1 / 2
    assert abs(d[1] - (w1 + w0) / 2) <= 2.3e-16 and d[1] == d[2]
    # consistency: drift and kick weights each sum to one (to rounding)
    assert abs(sum(c) - 1) < 5e-16 and abs(sum(d) - 1) < 5e-16
    # fourth-order condition of the triple jump: 2 w1^3 + w0^3 = 0
    assert abs(2 * w1**3 + w0**3) < 1e-14


def exact_harmonic_map(omega2, dt, n, q0, p0):
    """Exact rational evaluation of n steps of S(w1 h) S(w0 h) S(w1 h), with
    S(h) = K(h/2) D(h) K(h/2) the kick-drift-kick leapfrog of V = omega2 q^2/2."""
    w1, w0 = (F(v) for v in true_w())
    h, o2 = F(dt), F(omega2)
    q, p = F(q0), F(p0)
    for _ in range(n):
        for w in (w1, w0, w1):
            p -= w * h / 2 * o2 * q
            q += w * h * p
            p -= w * h / 2 * o2 * q
    return float(q), float(p)


def test_step_equals_exact_discrete_map(O):
    omega = 1.7
    s = O.harmonic([omega])
    dt, n = 0.05, 120
    x = O.step(s, dt, [0.8, -0.3], nsteps=n)
    q, p = exact_harmonic_map(omega * omega, dt, n, 0.8, -0.3)
    assert abs(x[0] - q) < 1e-13 and abs(x[1] - p) < 1e-13


def test_fourth_order_convergence_harmonic(O):
    s = O.harmonic([1.0])
    T = 10.0
    errs = []
    dts = [0.1, 0.05, 0.025]
    for dt in dts:
        x = O.step(s, dt, [1.0, 0.0], nsteps=int(round(T / dt)))
        errs.append(np.hypot(x[0] - np.cos(T), x[1] + np.sin(T)))
    slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
    assert abs(slope - 4.0) < 0.1, (errs, slope)


def hh_rhs(t, x):
    X, Y, px, py = x
    return [px, py, -X - 2 * X * Y, -Y - X * X + Y * Y]


@pytest.fixture(scope="module")
def hh_ref():
    x0 = np.array([0.0, 0.1, 0.45, 0.05])
    sol = solve_ivp(hh_rhs, (0, 10.0), x0, method="DOP853", rtol=1e-13, atol=1e-13)
    return x0, sol.y[:, -1]


def test_hh_against_dop853_fourth_order(O, hh_ref):
    s = O.henon_heiles()
    x0, xref = hh_ref
    errs = []
    dts = [0.04, 0.02, 0.01]
    for dt in dts:
        x = O.step(s, dt, x0, nsteps=int(round(10.0 / dt)))
        errs.append(np.max(np.abs(x - xref)))
    assert errs[-1] < 1e-8
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(13 < r < 19 for r in ratios), (errs, ratios)


def test_hh_energy_error_scales_as_dt4(O):
    s = O.henon_heiles()
    x0 = np.array([0.0, -0.2, 0.0, 0.1])
    x0[2] = np.sqrt(2 * 0.125 - x0[3] ** 2 - x0[1] ** 2 + 2 * x0[1] ** 3 / 3)
    H0 = O.hamiltonian(s, x0)
    errs = []
    for dt in (0.04, 0.02):
        x = x0.copy()
        e = 0.0
        for _ in range(int(round(40.0 / dt))):
            x = O.step(s, dt, x)
            e = max(e, abs(O.hamiltonian(s, x) - H0))
        errs.append(e)
    assert 14.4 < errs[0] / errs[1] < 17.6, errs


def step_map(O, s, dt, x):
    return O.step(s, dt, x)


@pytest.mark.parametrize("which", ["hh", "fput", "quartic"])
def test_tangent_map_is_fd_jacobian_and_symplectic(O, which):
    if which == "hh":
        s, x = O.henon_heiles(), np.array([0.1, -0.2, 0.3, 0.25])
    elif which == "fput":
        s = O.fput(4, 1.0, 0.3, 1.0)
        x = RNG.uniform(-0.5, 0.5, 8)
    else:
        s = O.quartic(3, 0.1)
        x = RNG.uniform(-0.7, 0.7, 6)
    D = 2 * s.ndof
    dt = 0.05
    _, W = O.step(s, dt, x, np.eye(D))
    M = W.T  # column j = image of e_j
    h = 1e-6
    Mf = np.zeros((D, D))
    for j in range(D):
        e = np.zeros(D)
        e[j] = h
        Mf[:, j] = (O.step(s, dt, x + e) - O.step(s, dt, x - e)) / (2 * h)
    assert np.max(np.abs(M - Mf)) < 1e-8
    J = np.block([[np.zeros((s.ndof, s.ndof)), np.eye(s.ndof)],
                  [-np.eye(s.ndof), np.zeros((s.ndof, s.ndof))]])
    assert np.max(np.abs(M.T @ J @ M - J)) < 1e-13
    _, W100 = O.step(s, dt, x, np.eye(D), nsteps=100)
    M100 = W100.T
    scale = max(1.0, np.max(np.abs(M100)) ** 2)
    assert np.max(np.abs(M100.T @ J @ M100 - J)) < 1e-12 * scale


def test_time_reversibility(O):
    s = O.henon_heiles()
    x0 = np.array([0.0, 0.1, 0.4, -0.1])
    x = O.step(s, 0.01, x0, nsteps=2000)
    xb = O.step(s, -0.01, x, nsteps=2000)
    assert np.max(np.abs(xb - x0)) < 1e-12


def test_tangent_linear_in_vectors(O):
    # the tangent map is linear: propagating a combination equals combining
    s = O.fput(3, 1.0, 0.0, 1.0)
    x = RNG.uniform(-0.5, 0.5, 6)
    a, b = RNG.normal(size=6), RNG.normal(size=6)
    _, W = O.step(s, 0.02, x, np.stack([a, b, 2 * a - 3 * b]), nsteps=50)
    assert np.allclose(W[2], 2 * W[0] - 3 * W[1], rtol=1e-12, atol=1e-12)
