"""Pins of the oracle's double pendulum (Examples section: the Hamiltonian
in matrix form and Hamilton's equations) and of the DOP853 integration of
it with its variational equations.

Checked against: the mechanics of two point masses on rigid rods written in
Cartesian coordinates (energy and angular velocities, nothing of the
printed matrix algebra), the printed equations of motion evaluated with
matrix products (C = -B^{-1} dB/dx B^{-1}), central finite differences of
the Hamiltonian (f = J grad H) and of the field (the tangent map), the
closed-form small-oscillation frequencies, conservation of H, the pairing
of the Lyapunov spectrum, and an independent integrator for the LD.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as O
import seeded_inputs as SI


def cartesian(theta, omega, alpha, sigma):
    """Energy of bob 1 (mass sigma, rod alpha) hanging from the origin and
    bob 2 (mass 1, rod 1) hanging from bob 1, gravity 1, in Cartesian
    coordinates; returns T + V and p = dT/domega (central differences,
    exact for a quadratic form up to rounding)."""
    def kinetic(om):
        t1, t2 = theta
        vx1, vy1 = alpha * math.cos(t1) * om[0], alpha * math.sin(t1) * om[0]
        vx2, vy2 = vx1 + math.cos(t2) * om[1], vy1 + math.sin(t2) * om[1]
        return 0.5 * sigma * (vx1 ** 2 + vy1 ** 2) + 0.5 * (vx2 ** 2 + vy2 ** 2)

    y1 = -alpha * math.cos(theta[0])
    y2 = y1 - math.cos(theta[1])
    V = sigma * y1 + y2
    h = 1e-3
    p = np.zeros(2)
    for i in range(2):
        e = np.zeros(2)
        e[i] = h
        p[i] = (kinetic(omega + e) - kinetic(omega - e)) / (2 * h)
    return kinetic(omega) + V, p


PARAMS = [(1.0, 1.0), (0.7, 2.5), (1.8, 0.4)]


def cases(seed, n=8):
    return SI.dp_states(seed, n, theta_max=math.pi, p_max=2.0)


@pytest.mark.parametrize("alpha,sigma", PARAMS)
def test_energy_and_velocities_match_cartesian_mechanics(alpha, sigma):
    sys = O.double_pendulum(alpha, sigma)
    rng = SI.dp_states(11, 10, theta_max=math.pi, p_max=1.5)
    for row in rng:
        theta, omega = row[:2], row[2:]
        E, p = cartesian(theta, omega, alpha, sigma)
        x = np.array([theta[0], theta[1], p[0], p[1]])
        assert abs(O.hamiltonian(sys, x) - E) <= 1e-9 * (1 + abs(E))
        f = O.dp_rhs(sys, x)
        np.testing.assert_allclose(f[:2], omega, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("alpha,sigma", PARAMS)
def test_field_matches_printed_matrix_equations(alpha, sigma):
    sys = O.double_pendulum(alpha, sigma)

    def binv(c):
        return np.array([[1 / alpha ** 2, -c / alpha], [-c / alpha, 1 + sigma]]) / (
            1 + sigma - c * c)

    for x in cases(3):
        th, p = x[:2], x[2:]
        c, s = math.cos(th[0] - th[1]), math.sin(th[0] - th[1])
        h = 1e-5
        B = lambda z: np.linalg.inv(binv(z))
        dB = (B(c + h) - B(c - h)) / (2 * h)
        C = -binv(c) @ dB @ binv(c)
        thdot = binv(c) @ p
        pdot = (s / 2) * (p @ C @ p) * np.array([1.0, -1.0]) - np.array(
            [alpha * (1 + sigma) * math.sin(th[0]), math.sin(th[1])])
        f = O.dp_rhs(sys, x)
        np.testing.assert_allclose(f[:2], thdot, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(f[2:], pdot, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("alpha,sigma", PARAMS)
def test_field_is_symplectic_gradient_of_h(alpha, sigma):
    sys = O.double_pendulum(alpha, sigma)
    for x in cases(5):
        g = np.zeros(4)
        for i in range(4):
            e = np.zeros(4)
            e[i] = 1e-6
            g[i] = (O.hamiltonian(sys, x + e) - O.hamiltonian(sys, x - e)) / 2e-6
        want = np.concatenate([g[2:], -g[:2]])
        np.testing.assert_allclose(O.dp_rhs(sys, x), want, rtol=1e-7, atol=1e-7)


@pytest.mark.parametrize("alpha,sigma", PARAMS)
def test_tangent_is_jacobian_of_field(alpha, sigma):
    sys = O.double_pendulum(alpha, sigma)
    dirs = SI.dp_states(7, 8, theta_max=1.0, p_max=1.0)
    for x, d in zip(cases(9), dirs):
        _, df = O.dp_rhs(sys, x, d)
        e = 1e-6
        fd = (O.dp_rhs(sys, x + e * d) - O.dp_rhs(sys, x - e * d)) / (2 * e)
        np.testing.assert_allclose(df, fd, rtol=1e-6, atol=1e-7)
        # linear in the direction
        _, df2 = O.dp_rhs(sys, x, -2.5 * d)
        np.testing.assert_allclose(df2, -2.5 * df, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("alpha,sigma", PARAMS)
def test_small_oscillation_frequencies(alpha, sigma):
    # about the stable equilibrium the frequencies solve
    # det(K - w^2 B(1)) = 0, K = diag(alpha (1 + sigma), 1),
    # B(1) = [[alpha^2 (1 + sigma), alpha], [alpha, 1]]:
    # alpha^2 sigma w^4 - alpha (1 + sigma)(1 + alpha) w^2 + alpha (1 + sigma) = 0
    sys = O.double_pendulum(alpha, sigma)
    J = np.zeros((4, 4))
    for k in range(4):
        e = np.zeros(4)
        e[k] = 1.0
        J[:, k] = O.dp_rhs(sys, np.zeros(4), e)[1]
    a, b, c = alpha ** 2 * sigma, -alpha * (1 + sigma) * (1 + alpha), alpha * (1 + sigma)
    disc = math.sqrt(b * b - 4 * a * c)
    w2 = sorted([(-b - disc) / (2 * a), (-b + disc) / (2 * a)])
    ev = np.linalg.eigvals(J)
    np.testing.assert_allclose(np.abs(ev.real), 0, atol=1e-12)
    got = sorted(set(np.round(np.abs(ev.imag) ** 2, 12)))
    np.testing.assert_allclose(got, w2, rtol=1e-10)
    if alpha == 1.0 and sigma == 1.0:
        np.testing.assert_allclose(w2, [2 - math.sqrt(2), 2 + math.sqrt(2)], rtol=1e-14)


def run(integrator, T=50.0, dt=0.01, ind=O.IND_LYAP | O.IND_ENERGY, **kw):
    return O.Run(dt=dt, T=T, indicators=ind, n_lyap=kw.pop("n_lyap", 4),
                 integrator=integrator, **kw)


def test_energy_conserved():
    sys = O.double_pendulum(1.0, 1.0)
    x0 = cases(21, 6)
    out = O.integrate(sys, x0, run(O.INT_DOP853, T=100.0, dt=0.01, ind=O.IND_ENERGY))
    assert (out["status"] == O.ST_OK).all()
    assert out["energy_err"].max() < 1e-10
    out = O.integrate(sys, x0, run(O.INT_DOP853_ADAPTIVE, T=100.0, dt=0.1,
                                   ind=O.IND_ENERGY))
    assert (out["status"] == O.ST_OK).all()
    assert out["energy_err"].max() < 1e-8


def test_lyapunov_spectrum_pairs():
    # Hamiltonian flow: the linearised flow has unit determinant, so the
    # finite-time exponents sum to zero (to the truncation error); they pair
    # as lambda_i = -lambda_{5-i} and the middle pair (along the flow and
    # across the energy surface) vanishes only as T grows (O(1/T) here)
    sys = O.double_pendulum(1.0, 1.0)
    x0 = np.array([[2.0, 2.5, 0.0, 0.0], [0.3, -0.2, 0.0, 0.0]])
    out = O.integrate(sys, x0, run(O.INT_DOP853, T=400.0, dt=0.01))
    ly = out["lyap"]
    assert np.abs(ly.sum(axis=1)).max() < 1e-8
    assert np.abs(ly[:, 0] + ly[:, 3]).max() < 0.02
    assert np.abs(ly[:, 1:3]).max() < 0.05
    assert ly[0, 0] > 0.3          # the high-energy orbit is chaotic
    assert ly[1, 0] < 0.05         # the small oscillation is not


@pytest.mark.parametrize("p,tol", [(0.5, 2e-6), (1.0, 1e-7)])
def test_ld_matches_independent_quadrature(p, tol):
    # |f_c|^p has a cusp where f_c changes sign, so the stage quadrature of
    # the LD converges at a lower order than the state; against SciPy's
    # adaptive DOP853 on the augmented system (rtol 1e-13) the small step
    # agrees to tol and the error shrinks with the step
    sys = O.double_pendulum(0.7, 2.5)
    for x0 in cases(31, 3):
        def rhs(t, y):
            f = O.dp_rhs(sys, y[:4])
            return np.concatenate([f, [np.sum(np.abs(f) ** p)]])

        sol = solve_ivp(rhs, (0.0, 10.0), np.concatenate([x0, [0.0]]), method="DOP853",
                        rtol=1e-13, atol=1e-13)
        ref = sol.y[4, -1]
        errs = []
        for dt in (0.01, 0.00125):
            out = O.integrate(sys, x0[None], run(O.INT_DOP853, T=10.0, dt=dt, ind=O.IND_LD,
                                                 ld_p=p))
            errs.append(abs(out["ld"][0] - ref) / ref)
        assert errs[1] <= tol
        assert errs[1] < errs[0]
        np.testing.assert_allclose(out["x_final"][0], sol.y[:4, -1], rtol=1e-8, atol=1e-9)


def test_equilibria_have_zero_ld_and_stay_put():
    sys = O.double_pendulum(1.0, 1.0)
    x0 = np.array([[0.0, 0.0, 0.0, 0.0], [math.pi, math.pi, 0.0, 0.0],
                   [0.0, math.pi, 0.0, 0.0]])
    out = O.integrate(sys, x0, run(O.INT_DOP853, T=5.0, dt=0.01, ind=O.IND_LD))
    np.testing.assert_allclose(out["x_final"], x0, atol=1e-12)
    assert np.abs(out["ld"]).max() < 1e-5


def test_yoshida_refused():
    sys = O.double_pendulum()
    with pytest.raises(RuntimeError):
        O.integrate(sys, np.zeros((1, 4)), run(O.INT_YOSHIDA4, T=1.0, dt=0.1))


def test_planted_sign_error_is_caught():
    # flipping the sign of the coupling term of p' breaks f = J grad H
    sys = O.double_pendulum(1.0, 1.0)
    x = cases(5, 1)[0]
    f = O.dp_rhs(sys, x)
    bad = f.copy()
    c, s = math.cos(x[0] - x[1]), math.sin(x[0] - x[1])
    bad[2] = 2 * (-math.sin(x[0]) * 2) - f[2]  # reflect about the gravity term
    g = np.zeros(4)
    for i in range(4):
        e = np.zeros(4)
        e[i] = 1e-6
        g[i] = (O.hamiltonian(sys, x + e) - O.hamiltonian(sys, x - e)) / 2e-6
    want = np.concatenate([g[2:], -g[:2]])
    assert np.abs(f - want).max() < 1e-7
    assert np.abs(bad - want).max() > 1e-3
