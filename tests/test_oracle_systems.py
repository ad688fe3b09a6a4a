"""Pins of the oracle's potentials, forces and Hessians.

Each system is checked against facts that do not come from the oracle's own
formulas: the equations of motion printed in the paper (Examples section),
central finite differences of the potential, the equilibria of the
Henon-Heiles potential and the closed-form normal-mode spectrum of the
harmonic chain with fixed ends.
"""
import numpy as np
import pytest

RNG = np.random.default_rng(12345)


def fd_grad(f, q, h=1e-6):
    g = np.zeros(len(q))
    for i in range(len(q)):
        e = np.zeros(len(q))
        e[i] = h
        g[i] = (f(q + e) - f(q - e)) / (2 * h)
    return g


def systems(O):
    return [O.henon_heiles(), O.fput(5, 1.0, 0.25, 1.0), O.fput(3, 0.7, 0.0, 2.0),
            O.quartic(3, 0.1), O.harmonic([1.0, np.sqrt(2.0), 0.5])]


def test_grad_is_fd_of_potential(O):
    for s in systems(O):
        for _ in range(5):
            q = RNG.uniform(-0.6, 0.6, s.ndof)
            g = O.grad(s, q)
            gf = fd_grad(lambda z: O.potential(s, z), q)
            assert np.allclose(g, gf, rtol=0, atol=2e-9), (s, q, g, gf)


def test_hess_is_fd_of_grad_and_symmetric(O):
    for s in systems(O):
        for _ in range(5):
            q = RNG.uniform(-0.6, 0.6, s.ndof)
            H = O.hess(s, q)
            Hf = np.array([fd_grad(lambda z: O.grad(s, z)[i], q) for i in range(s.ndof)])
            assert np.allclose(H, Hf, rtol=0, atol=2e-9)
            assert np.allclose(H, H.T, rtol=4e-16, atol=0)


def test_hh_printed_equations_of_motion(O):
    # Examples section: dp_x/dt = -x - 2xy, dp_y/dt = -y - x^2 + y^2.
    s = O.henon_heiles()
    for _ in range(20):
        x, y = RNG.uniform(-1, 1, 2)
        assert np.allclose(-O.grad(s, [x, y]), [-x - 2 * x * y, -y - x * x + y * y],
                           rtol=1e-15, atol=1e-15)


def test_hh_printed_hamiltonian(O):
    # Examples section: H = px^2/2 + py^2/2 + (x^2 + y^2)/2 + x^2 y - y^3/3.
    s = O.henon_heiles()
    for _ in range(20):
        x, y, px, py = RNG.uniform(-1, 1, 4)
        ref = px**2 / 2 + py**2 / 2 + (x**2 + y**2) / 2 + x**2 * y - y**3 / 3
        assert abs(O.hamiltonian(s, [x, y, px, py]) - ref) < 1e-15


def test_hh_equilibria(O):
    # The potential has a minimum at the origin and three saddles at energy
    # 1/6: (0, 1) and (+-sqrt(3)/2, -1/2); at (0, 1) the Hessian is diag(3, -1).
    s = O.henon_heiles()
    assert O.potential(s, [0, 0]) == 0.0
    assert np.array_equal(O.hess(s, [0, 0]), np.eye(2))
    for q in ([0.0, 1.0], [np.sqrt(3) / 2, -0.5], [-np.sqrt(3) / 2, -0.5]):
        assert np.max(np.abs(O.grad(s, q))) < 3e-16
        assert abs(O.potential(s, q) - 1 / 6) < 1e-15
        ev = np.linalg.eigvalsh(O.hess(s, q))
        assert np.allclose(ev, [-1.0, 3.0], atol=1e-15)


def test_fput_printed_equations_of_motion(O):
    # Examples section: dp_i/dt = -k[dq_i - dq_{i+1}] - alpha[dq_i^2 - dq_{i+1}^2]
    #                              - beta[dq_i^3 - dq_{i+1}^3],
    # dq_i = q_i - q_{i-1}, q_0 = q_{N+1} = 0.
    for (N, k, a, b) in [(4, 1.0, 0.0, 1.0), (7, 0.8, 0.3, 1.5), (1, 1.0, 0.5, 0.5)]:
        s = O.fput(N, k, a, b)
        for _ in range(5):
            q = RNG.uniform(-1, 1, N)
            qq = np.concatenate([[0.0], q, [0.0]])
            ref = np.zeros(N)
            for i in range(1, N + 1):
                dl = qq[i] - qq[i - 1]
                dr = qq[i + 1] - qq[i]
                ref[i - 1] = -k * (dl - dr) - a * (dl**2 - dr**2) - b * (dl**3 - dr**3)
            assert np.allclose(-O.grad(s, q), ref, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("N", [1, 2, 5, 8, 16])
def test_fput_linear_chain_normal_modes(O, N):
    # With alpha = beta = 0 and spring constant kappa the fixed-end chain
    # (N+1 springs) has normal modes sin(i k pi/(N+1)) with squared
    # frequencies 4 kappa sin^2(k pi/(2(N+1))).
    s = O.fput(N, 1.3, 0.0, 0.0)
    H = O.hess(s, RNG.uniform(-1, 1, N))
    i = np.arange(1, N + 1)
    for kk in range(1, N + 1):
        mode = np.sin(i * kk * np.pi / (N + 1))
        lam = 1.3 * 4 * np.sin(kk * np.pi / (2 * (N + 1))) ** 2
        assert np.allclose(H @ mode, lam * mode, atol=1e-13)


def test_quartic_homogeneity_and_symmetry(O):
    s = O.quartic(3, 0.1)
    for _ in range(10):
        q = RNG.normal(size=3)
        lam = RNG.uniform(0.2, 3)
        assert np.isclose(O.potential(s, lam * q), lam**4 * O.potential(s, q), rtol=1e-14)
        # V = sum q^4/4 + 0.1 sum_{i<j} q_i^2 q_j^2 on a coordinate axis and a diagonal
    assert O.potential(s, [2.0, 0, 0]) == 4.0
    assert np.isclose(O.potential(s, [1.0, 1.0, 1.0]), 0.75 + 0.3, rtol=1e-15)


def test_harmonic_hessian(O):
    s = O.harmonic([1.0, 2.0])
    assert np.array_equal(O.hess(s, [0.3, -0.2]), np.diag([1.0, 4.0]))
