"""Pins of the oracle's chaos indicators and orbit bookkeeping.

Against mathematics rather than the oracle itself: the Lyapunov spectrum of
a symplectic map sums to zero and pairs up; the spectrum at the
Henon-Heiles saddle is (0, 1, 0, -1); linear oscillators have bounded
tangent growth; GALI equals the product of singular values (numpy SVD) and
obeys the power laws of integrable motion (Skokos, Bountis, Antonopoulos,
Physica D 231 (2007) 30); GALI_2 and SALI bound each other; the LD
M-function of a harmonic oscillator has a closed form, and the trapezoid
rule's error at the |.|^(1/2) cusps follows the generalised Euler-Maclaurin
expansion (Navot 1961); the tangent vectors follow the variational equations
integrated independently by SciPy's DOP853.
"""
from fractions import Fraction as F

import mpmath as mp
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import seeded_inputs as S


def hh_ic(E, y, py):
    r = 2 * E - py * py - y * y + 2 * y**3 / 3
    return np.array([0.0, y, np.sqrt(r), py])


# --- Lyapunov spectrum ------------------------------------------------------

@pytest.mark.parametrize("case", ["hh_chaotic", "hh_regular", "fput", "quartic"])
def test_lyapunov_spectrum_sums_to_zero(O, case):
    if case.startswith("hh"):
        s = O.henon_heiles()
        x0 = hh_ic(0.125, -0.25 if case == "hh_chaotic" else 0.1, 0.0)[None]
        dt = 0.01
    elif case == "fput":
        s = O.fput(4, 1.0, 0.0, 1.0)
        x0 = O.fput_ic(s, S.fput_mode_draws(3, 1))
        dt = 0.02
    else:
        s = O.quartic(3, 0.1)
        x0 = O.quartic_ic(s, S.quartic_draws(3, 1))
        dt = 0.01
    r = O.integrate(s, x0, O.Run(dt=dt, T=200.0, indicators=O.IND_LYAP, n_lyap=2 * s.ndof))
    lam = r["lyap"][0]
    assert abs(lam.sum()) < 1e-12, lam
    assert np.all(np.isfinite(lam))


def test_lyapunov_pairs_shrink_like_one_over_T(O):
    s = O.henon_heiles()
    x0 = hh_ic(0.125, -0.25, 0.0)[None]
    pair = []
    for T in (500.0, 2000.0):
        lam = O.integrate(s, x0, O.Run(dt=0.01, T=T, indicators=O.IND_LYAP, n_lyap=4))["lyap"][0]
        pair.append(abs(lam[0] + lam[3]))
        assert lam[0] > 0.03  # this orbit is chaotic
    assert 3.0 < pair[0] / pair[1] < 5.0, pair


def test_lyapunov_spectrum_at_saddle(O):
    # (x, y) = (0, 1) at rest is an exact equilibrium; the linearised flow has
    # Hessian diag(3, -1): the x motion oscillates (exponents 0, 0) and the y
    # motion grows and decays as exp(+-t) (exponents 1, -1).  With the
    # canonical vectors ordered (x, y, p_x, p_y) the MGS order gives
    # (0, 1, 0, -1); finite-time errors decay like 1/T.
    s = O.henon_heiles()
    x0 = np.array([[0.0, 1.0, 0.0, 0.0]])
    errs = []
    for T in (100.0, 400.0):
        r = O.integrate(s, x0, O.Run(dt=0.01, T=T, indicators=O.IND_LYAP, n_lyap=4))
        lam = r["lyap"][0]
        assert np.array_equal(r["x_final"][0], x0[0])
        errs.append(np.max(np.abs(lam - [0, 1, 0, -1])))
    assert errs[1] < 0.01 and errs[1] < errs[0] / 2, errs


def test_lyapunov_bounded_for_linear_oscillators(O):
    # V = sum w_i^2 q_i^2/2: the tangent map is conjugate to a rotation by
    # diag(1, w), so |M^n e| stays within [1/w, w] for w >= 1 and every
    # finite-time exponent is at most ln(w)/T in modulus.
    w = [1.0, np.sqrt(2.0)]
    s = O.harmonic(w)
    T = 300.0
    r = O.integrate(s, np.array([[0.5, 0.3, 0.1, -0.2]]),
                    O.Run(dt=0.01, T=T, indicators=O.IND_LYAP, n_lyap=4))
    assert np.max(np.abs(r["lyap"][0])) <= np.log(np.sqrt(2.0)) / T + 1e-12


# --- GALI and SALI ----------------------------------------------------------

def test_gali_equals_product_of_singular_values(O):
    rng = np.random.default_rng(4)
    for dim, m in [(4, 4), (8, 5), (32, 16)]:
        w = rng.normal(size=(m, dim))
        w[1] = w[0] + 1e-3 * w[1]  # one nearly dependent pair
        g = O.gali(w, m)
        u = w / np.linalg.norm(w, axis=1, keepdims=True)
        for k in range(2, m + 1):
            sv = np.linalg.svd(u[:k].T, compute_uv=False)
            assert abs(g[k - 2] / np.prod(sv) - 1) < 1e-12


def test_mgs_is_a_qr(O):
    rng = np.random.default_rng(5)
    w = rng.normal(size=(6, 6))
    q, rd = O.mgs(w)
    assert np.allclose(q @ q.T, np.eye(6), atol=1e-13)
    R = np.linalg.qr(w.T, mode="r")
    assert np.allclose(rd, np.abs(np.diag(R)), rtol=1e-13)


def test_gali2_and_sali_relations(O):
    # For two unit vectors with angle t: |w1+w2| |w1-w2| / 2 = sin t = GALI_2,
    # and SALI = min(|w1+w2|, |w1-w2|) with |w1+w2|^2 + |w1-w2|^2 = 4, hence
    # SALI/sqrt(2) <= GALI_2 <= SALI <= sqrt(2).
    s = O.henon_heiles()
    x0, mask = O.hh_grid(0.125, 8, 8)
    x0 = x0[mask == 1]
    w0 = S.deviation_vectors(11, len(x0), 2, 4)
    r = O.integrate(s, x0, O.Run(dt=0.01, T=50.0, indicators=O.IND_SALI | O.IND_GALI,
                                 gali_kmax=2), w0=w0)
    g, sl = r["gali"][:, 0], r["sali_final"]
    assert np.all(sl / np.sqrt(2) <= g * (1 + 1e-12))
    assert np.all(g <= sl * (1 + 1e-12))
    assert np.all(sl <= np.sqrt(2) * (1 + 1e-15))
    assert np.all(r["sali_min"] <= sl)


def test_sali_special_cases(O):
    s = O.henon_heiles()
    x0 = hh_ic(0.125, 0.1, 0.05)[None]
    a = np.array([0.3, -0.1, 0.2, 0.5])
    for w in (np.stack([a, a]), np.stack([a, -2 * a])):
        r = O.integrate(s, x0, O.Run(dt=0.01, T=1.0, indicators=O.IND_SALI), w0=w[None])
        assert r["sali_min"][0] == 0.0 and r["t_chaos"][0] == 0.1


@pytest.mark.slow
def test_gali_power_laws_on_integrable_torus(O):
    # Two uncoupled quartic oscillators: integrable with amplitude-dependent
    # frequencies.  On a 2-torus GALI_2 stays bounded while GALI_3 ~ t^-2 and
    # GALI_4 ~ t^-4.
    s = O.quartic(2, 0.0)
    x0 = np.array([[0.5, 0.8, 0.3, -0.2]])
    w0 = S.deviation_vectors(9, 1, 4, 4)
    Ts = [250.0, 2000.0]
    g = [O.integrate(s, x0, O.Run(dt=0.01, T=T, indicators=O.IND_GALI, gali_kmax=4),
                     w0=w0)["gali"][0] for T in Ts]
    slope = np.log(g[1] / g[0]) / np.log(Ts[1] / Ts[0])
    assert abs(slope[0]) < 0.1
    assert -2.3 < slope[1] < -1.7
    assert -4.5 < slope[2] < -3.5


def test_gali2_bounded_on_linear_oscillator(O):
    s = O.harmonic([1.0, np.sqrt(2.0)])
    w0 = S.deviation_vectors(5, 1, 2, 4)
    r = O.integrate(s, np.array([[0.5, 0.3, 0.1, -0.2]]),
                    O.Run(dt=0.01, T=500.0, indicators=O.IND_GALI | O.IND_SALI,
                          gali_kmax=2), w0=w0)
    assert r["gali"][0, 0] > 0.1 and r["sali_min"][0] > 0.1


# --- tangent vectors vs the variational equations ---------------------------

def test_tangent_vectors_follow_variational_equations(O):
    # d/dt (dq, dp) = (dp, -Hess V(q) dq), integrated with the orbit by DOP853.
    def rhs(t, z):
        X, Y, px, py = z[:4]
        H = np.array([[1 + 2 * Y, 2 * X], [2 * X, 1 - 2 * Y]])
        out = [px, py, -X - 2 * X * Y, -Y - X * X + Y * Y]
        for v in range(2):
            dq, dp = z[4 + 4 * v:6 + 4 * v], z[6 + 4 * v:8 + 4 * v]
            out += list(dp) + list(-H @ dq)
        return out

    s = O.henon_heiles()
    x0 = hh_ic(0.125, -0.1, 0.1)
    w0 = S.deviation_vectors(21, 1, 2, 4)[0]
    sol = solve_ivp(rhs, (0, 10.0), np.concatenate([x0, w0.ravel()]), method="DOP853",
                    rtol=1e-13, atol=1e-13)
    err = []
    for dt in (0.02, 0.01):
        _, w = O.step(s, dt, x0, w0, nsteps=int(round(10.0 / dt)))
        err.append(np.max(np.abs(w.ravel() - sol.y[4:, -1])))
    # the discrete tangent map converges to the variational flow at fourth order
    assert err[1] < 3e-7 and 13 < err[0] / err[1] < 19, err


def test_ln_growth_telescopes(O):
    s = O.henon_heiles()
    x0 = hh_ic(0.125, -0.25, 0.0)
    w0 = S.deviation_vectors(2, 1, 2, 4)[0]
    r = O.integrate(s, x0[None], O.Run(dt=0.01, T=30.0, indicators=O.IND_SALI), w0=w0[None])
    _, w = O.step(s, 0.01, x0, w0 / np.linalg.norm(w0, axis=1, keepdims=True), nsteps=3000)
    assert np.allclose(r["ln_growth"][0], np.log(np.linalg.norm(w, axis=1)), rtol=1e-12)


# --- Lagrangian descriptor ---------------------------------------------------

def test_ld_harmonic_closed_form_with_cusp_correction(O):
    # x = A cos(wt), p = -A w sin(wt): |dq/dt|^(1/2) + |dp/dt|^(1/2)
    #   = sqrt(A w)|sin|^(1/2) + sqrt(A w^2)|cos|^(1/2), whose integral over
    # one period P = 2 pi / w is 4 B sqrt(A) (w^(-1/2) + 1), with
    # B = int_0^(pi/2) sin^(1/2) = sqrt(pi) Gamma(3/4) / (2 Gamma(5/4)).
    # Each of the 4 zeros per period lies on a grid point and is a two-sided
    # |t - t0|^(1/2) cusp of local amplitude sqrt(c) (c = A w^2 for the p term,
    # A w^3 for the force term); the trapezoid rule then misses
    # 2 |zeta(-1/2)| sqrt(c) h^(3/2) per cusp, up to O(h^(7/2)).
    B = float(mp.sqrt(mp.pi) * mp.gamma(0.75) / (2 * mp.gamma(1.25)))
    assert abs(B - 1.198140234735592) < 1e-15
    z = abs(float(mp.zeta(-0.5)))
    P, A = 6.28, 0.7
    w = 2 * np.pi / P
    exact = 4 * B * np.sqrt(A) * (1 / np.sqrt(w) + 1)
    s = O.harmonic([w])
    for dt in (0.01, 0.005):
        ld = O.integrate(s, np.array([[A, 0.0]]), O.Run(dt=dt, T=P, indicators=O.IND_LD))["ld"][0]
        cusp = 2 * 2 * z * (np.sqrt(A * w * w) + np.sqrt(A * w**3)) * dt**1.5
        assert abs(ld - (exact - cusp)) < 2e-6, (dt, ld, exact, cusp)
        assert abs(ld - exact) > 1e-5  # the cusp term is really there


def test_ld_zero_at_rest_points(O):
    s = O.henon_heiles()
    for x0 in ([0.0, 0.0, 0.0, 0.0], [0.0, 1.0, 0.0, 0.0]):
        r = O.integrate(s, np.array([x0]), O.Run(dt=0.01, T=5.0, indicators=O.IND_LD))
        assert r["ld"][0] == 0.0


# --- energy error, inputs, resume, status ------------------------------------

def test_energy_error_is_max_over_checkpoints(O):
    s = O.henon_heiles()
    x0 = hh_ic(0.125, 0.2, -0.1)
    r = O.integrate(s, x0[None], O.Run(dt=0.01, T=5.0, indicators=O.IND_ENERGY, K=10))
    H0 = O.hamiltonian(s, x0)
    x, e = x0.copy(), 0.0
    for k in range(50):
        x = O.step(s, 0.01, x, nsteps=10)
        e = max(e, abs(O.hamiltonian(s, x) - H0))
    assert r["energy_err"][0] == e and 0 < e < 1e-9


def test_hh_grid_mask_exact(O):
    # Exact rational sign of r = 2E - py^2 - y^2 + 2y^3/3 at the grid's
    # binary64 points decides accessibility.
    E = 0.125
    n = 32
    x0, mask = O.hh_grid(E, n, n)
    cnt = 0
    for j in range(n):
        py = -0.45 + (0.45 - -0.45) * j / (n - 1)
        for i in range(n):
            y = -0.4 + (0.7 - -0.4) * i / (n - 1)
            r = 2 * F(E) - F(py) ** 2 - F(y) ** 2 + 2 * F(y) ** 3 / 3
            acc = r >= 0
            cnt += acc
            o = j * n + i
            assert mask[o] == acc
            assert x0[o, 0] == 0.0 and x0[o, 1] == y and x0[o, 3] == py
    assert cnt == 796
    s = O.henon_heiles()
    acc = x0[mask == 1]
    assert max(abs(O.hamiltonian(s, x) - E) for x in acc) < 1e-15


@pytest.mark.parametrize("E,expected", [(0.125, 850874), (1 / 6, 992552)])
def test_hh_grid_1024_counts(O, E, expected):
    _, mask = O.hh_grid(E, 1024, 1024)
    y = -0.4 + 1.1 * np.arange(1024) / 1023
    py = -0.45 + 0.9 * np.arange(1024) / 1023
    Y, PY = np.meshgrid(y, py)
    r = 2 * E - PY**2 - Y**2 + 2 * Y**3 / 3
    assert np.min(np.abs(r)) > 1e-9  # no point is within rounding of the boundary
    assert int(mask.sum()) == int((r >= 0).sum()) == expected


def test_fput_initial_conditions(O):
    for N in (4, 8, 16):
        s = O.fput(N)
        u = S.fput_mode_draws(100 + N, 64)
        x0 = O.fput_ic(s, u)
        E = 0.1 + 9.9 * u[:, 0]
        H = np.array([O.hamiltonian(s, x) for x in x0])
        assert np.max(np.abs(H / E - 1)) < 1e-13
        i = np.arange(1, N + 1)
        for k in range(3, N + 1):
            mode = np.sqrt(2 / (N + 1)) * np.sin(i * k * np.pi / (N + 1))
            assert np.max(np.abs(x0[:, :N] @ mode)) < 1e-13
            assert np.max(np.abs(x0[:, N:] @ mode)) < 1e-13


def test_quartic_initial_conditions(O):
    s = O.quartic(3, 0.1)
    x0 = O.quartic_ic(s, S.quartic_draws(8, 200))
    H = np.array([O.hamiltonian(s, x) for x in x0])
    assert np.max(np.abs(H - 1.0)) < 1e-14


def test_resume_is_bitwise(O):
    s = O.henon_heiles()
    x0, mask = O.hh_grid(0.125, 6, 6)
    w0 = S.deviation_vectors(1, len(x0), 2, 4)
    run = O.Run(dt=0.01, T=20.0, indicators=0x1F, n_lyap=4, gali_kmax=2)
    a = O.integrate(s, x0, run, w0=w0, mask=mask)
    st = O.State(s, run, x0, w0, mask)
    for stop in (700, 1300, 2000):
        st.advance(stop)
    b = st.finalize()
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_status_codes(O):
    s = O.henon_heiles()
    x0 = np.array([hh_ic(0.125, 0.1, 0.0), [np.nan, 0, 0, 0], hh_ic(0.2, 0.1, 0.0),
                   hh_ic(0.125, 0.1, 0.0)])
    mask = np.array([1, 1, 1, 0], np.uint8)
    w0 = S.deviation_vectors(3, 4, 2, 4)
    r = O.integrate(s, x0, O.Run(dt=0.01, T=100.0, indicators=O.IND_SALI | O.IND_LD,
                                 escape_r2=4.0), w0=w0, mask=mask)
    assert list(r["status"]) == [O.ST_OK, O.ST_NONFINITE, O.ST_ESCAPED, O.ST_MASKED]
    assert list(r["label"]) == [0, 3, 2, -1]
    assert r["t_end"][0] == 100.0 and 0 < r["t_end"][2] < 100.0
    assert np.isnan(r["ld"][1]) and np.isnan(r["ld"][3])
    assert np.sum(r["x_final"][2, :2] ** 2) > 4.0


def test_early_exit_stops_at_first_low_sali(O):
    s = O.henon_heiles()
    x0 = hh_ic(0.125, -0.25, 0.0)[None]
    w0 = S.deviation_vectors(2, 1, 2, 4)
    run = O.Run(dt=0.01, T=2000.0, indicators=O.IND_SALI | O.IND_LYAP, n_lyap=4)
    full = O.integrate(s, x0, run, w0=w0)
    run.early_exit = True
    ex = O.integrate(s, x0, run, w0=w0)
    assert full["label"][0] == 1 and ex["label"][0] == 1
    assert ex["status"][0] == O.ST_EXITED
    assert ex["t_end"][0] == ex["t_chaos"][0] == full["t_chaos"][0]
    assert ex["t_end"][0] < 2000.0
