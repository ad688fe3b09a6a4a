"""Pins of the oracle's LD-based chaos indicators from neighbouring orbits
(Functionalities section; the definitions are a reading of the cited works,
stated in oracle.ld_indicators): the difference D, ratio R and second
derivative S of the two-sided LDs of an orbit and its neighbours.

Checked against: the harmonic oscillator, whose LD over whole periods is
proportional to the square root of the amplitude (so D, R and S have closed
forms in the neighbours' amplitudes, and the quadrature's cusp error, also
proportional to it, cancels from the ratios); a backward integration by
SciPy (the momentum-reversal identity behind the backward part); the
inequalities R <= D and S <= 2 D that the definitions imply; status and
mask handling.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as O
import seeded_inputs as S


def closed(a, sigma, dirs):
    """D, R, S for the oscillator (omega = 1) at (a, 0): L ~ sqrt(amplitude)."""
    c = math.sqrt(a)
    d = r = s = 0.0
    for k in dirs:
        if k == 0:
            lp, lm = math.sqrt(a + sigma), math.sqrt(a - sigma)
        else:
            lp = lm = (a * a + sigma * sigma) ** 0.25
        d += abs(c - lp) + abs(c - lm)
        r += lp + lm
        s += abs(lp - 2 * c + lm)
    n = len(dirs)
    return d / (2 * n) / c, abs(1 - r / (2 * n) / c), s / n / c


@pytest.mark.parametrize("integ", [O.INT_YOSHIDA4, O.INT_DOP853])
def test_oscillator_closed_forms(integ):
    # neighbours along q keep the orbit's phase, so the LD quadrature's cusp
    # error (proportional to sqrt(amplitude) as well) cancels from D, R, S
    s = O.harmonic([1.0])
    T = 2 * math.pi * 4
    run = O.Run(dt=2 * math.pi / 1000, T=T, indicators=O.IND_LD, integrator=integ)
    for a, sg in ((1.0, 0.1), (2.5, 0.05), (0.7, 0.2)):
        res = O.ld_indicators(s, np.array([[a, 0.0]]), run, [0], sg)
        D, R, Sd = closed(a, sg, [0])
        assert res["status"][0] == 0
        np.testing.assert_allclose([res["D"][0], res["R"][0], res["S"][0]], [D, R, Sd],
                                   rtol=2e-7, atol=1e-15)
        # L itself: 2 (forward + backward) x 4 periods x 8 sqrt(a) B
        B = math.gamma(0.75) * math.sqrt(math.pi) / (2 * math.gamma(1.25))
        assert abs(res["ld"][0] / (64 * B * math.sqrt(a)) - 1) < 2e-4


@pytest.mark.parametrize("dirs", [[1], [0, 1]])
def test_oscillator_momentum_neighbours_converge(dirs):
    # neighbours along p shift the phase: their zero crossings fall elsewhere
    # on the step grid, so the cusp errors differ; the indicators converge
    # to the closed forms as the step shrinks (like h^1.5)
    s = O.harmonic([1.0])
    T = 2 * math.pi * 4
    D, R, Sd = closed(1.0, 0.1, dirs)
    err = []
    for nd in (1000, 32000):
        run = O.Run(dt=2 * math.pi / nd, T=T, indicators=O.IND_LD)
        res = O.ld_indicators(s, np.array([[1.0, 0.0]]), run, dirs, 0.1)
        err.append(max(abs(res["D"][0] / D - 1), abs(res["R"][0] / R - 1),
                       abs(res["S"][0] / Sd - 1)))
    assert err[1] < err[0] / 50 and err[1] < 1e-3


def test_backward_part_is_the_reversed_forward_part():
    # M-(x) = int_{-T}^0 sum |dx/dt|^p dt by SciPy backward in time, against
    # the oracle's forward LD of (q, -p)
    hh = O.henon_heiles()
    x0, _ = O.hh_points(0.125, np.array([0.1, -0.2, 0.35]), np.array([0.05, 0.2, -0.1]))
    T = 20.0

    def rhs(t, y):
        g = O.grad(hh, y[:2])
        f = np.array([y[2], y[3], -g[0], -g[1]])
        return np.concatenate([f, [np.sum(np.sqrt(np.abs(f)))]])

    for x in x0:
        sol = solve_ivp(rhs, (0.0, -T), np.concatenate([x, [0.0]]), method="DOP853",
                        rtol=1e-12, atol=1e-12)
        back = -sol.y[4, -1]
        r = x.copy()
        r[2:] = -r[2:]
        out = O.integrate(hh, r[None], O.Run(dt=0.001, T=T, indicators=O.IND_LD,
                                             integrator=O.INT_DOP853))
        assert abs(out["ld"][0] / back - 1) < 2e-6
        # and the orbit itself: reversed final state of the reversed orbit
        xe = out["x_final"][0].copy()
        xe[2:] = -xe[2:]
        np.testing.assert_allclose(xe, sol.y[:4, -1], rtol=1e-8, atol=1e-9)


def test_inequalities_and_forward_only():
    hh = O.henon_heiles()
    y, py = S.section_points(17, 40)
    x0, m = O.hh_points(0.125, y, py)
    x0 = x0[m == 1]
    run = O.Run(dt=0.01, T=60.0, indicators=O.IND_LD)
    res = O.ld_indicators(hh, x0, run, [1, 3], 1e-3, threads=4)
    assert (res["status"] == 0).all()
    assert np.all(res["R"] <= res["D"] + 1e-15)
    assert np.all(res["S"] <= 2 * res["D"] + 1e-15)
    assert np.all(res["D"] > 0) and np.all(res["S"] >= 0)
    fwd = O.ld_indicators(hh, x0, run, [1, 3], 1e-3, two_sided=False, threads=4)
    plain = O.integrate(hh, x0, run, threads=4)
    np.testing.assert_array_equal(fwd["ld"], plain["ld"])
    rev = x0.copy()
    rev[:, 2:] *= -1
    back = O.integrate(hh, rev, run, threads=4)
    np.testing.assert_allclose(res["ld"], plain["ld"] + back["ld"], rtol=1e-15)


def test_members_layout():
    x0 = np.array([[1.0, 2.0, 3.0, 4.0]])
    mem = O.ldn_members(x0, [1, 3], 0.5)
    assert mem.shape == (1, 2, 5, 4)
    np.testing.assert_array_equal(mem[0, 0, 0], [1, 2, 3, 4])
    np.testing.assert_array_equal(mem[0, 0, 1], [1, 2.5, 3, 4])
    np.testing.assert_array_equal(mem[0, 0, 2], [1, 1.5, 3, 4])
    np.testing.assert_array_equal(mem[0, 0, 3], [1, 2, 3, 4.5])
    np.testing.assert_array_equal(mem[0, 0, 4], [1, 2, 3, 3.5])
    np.testing.assert_array_equal(mem[0, 1, 3], [1, 2, -3, -4.5])


def test_status_and_mask():
    hh = O.henon_heiles()
    x0 = np.array([[0.0, 0.1, 0.45, 0.0], [np.nan, 0.1, 0.4, 0.0], [0.0, 0.1, 0.45, 0.0],
                   [0.0, 0.2, 0.3, 0.0]])
    run = O.Run(dt=0.01, T=5.0, indicators=O.IND_LD, escape_r2=0.0)
    res = O.ld_indicators(hh, x0, run, [1], 1e-3, mask=np.array([1, 1, 0, 1]))
    assert list(res["status"]) == [0, 3, 1, 0]
    assert np.isnan(res["D"][1]) and np.isnan(res["S"][2]) and np.isfinite(res["R"][3])
    # an escaping neighbour: a radius that only the +sigma neighbour leaves
    x1 = np.array([[0.0, 0.5, 0.0, 0.0]])
    run = O.Run(dt=0.01, T=0.1, indicators=O.IND_LD, K=1, escape_r2=0.5 ** 2 + 0.04)
    res = O.ld_indicators(hh, x1, run, [1], 0.1)
    assert res["status"][0] == O.ST_ESCAPED and np.isnan(res["D"][0])
