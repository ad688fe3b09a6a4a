"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds random-number generation and nothing of the method's
arithmetic: it never evaluates a Hamiltonian, a force, a step or an
indicator.  Both sides of every parity check take their random inputs from
here, so those inputs are bit-identical.

Generator: SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used counter-based:

    mix64(z):  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
               z = (z ^ (z >> 27)) * 0x94D049BB133111EB
               return z ^ (z >> 31)                      (all mod 2^64)
    key(seed, stream) = mix64(seed ^ mix64(stream + 1))
    out(seed, stream, k) = mix64(key + (k + 1) * 0x9E3779B97F4A7C15)

i.e. the k-th output of a SplitMix64 generator whose state starts at `key`.

    uniform(k)      = (out(k) >> 11) * 2^-53               in [0, 1)
    uniform_open(k) = ((out(k) >> 11) + 0.5) * 2^-53       in (0, 1)
    normal(e)       = sqrt(-2 ln(1 - uniform(2e))) * cos(2 pi uniform(2e + 1))

(the cosine branch of the Box-Muller transform, G. E. P. Box and
M. E. Muller, Ann. Math. Statist. 29 (1958) 610).

Stream ids: 0 = deviation vectors, 1 = initial-condition sampling.
"""
import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

STREAM_DEVIATION = 0
STREAM_IC = 1


def mix64(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        return z ^ (z >> np.uint64(31))


def key(seed, stream):
    return mix64(np.uint64(seed) ^ mix64(np.uint64(stream + 1)))


def raw(seed, stream, k):
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key(seed, stream) + (k + np.uint64(1)) * GOLDEN)


def uniform(seed, stream, k):
    return (raw(seed, stream, k) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def uniform_open(seed, stream, k):
    return ((raw(seed, stream, k) >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def normal(seed, stream, e):
    e = np.asarray(e, dtype=np.uint64)
    u1 = uniform(seed, stream, np.uint64(2) * e)
    u2 = uniform(seed, stream, np.uint64(2) * e + np.uint64(1))
    return np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * np.pi * u2)


def deviation_vectors(seed, n, m, dim, first_ic=0):
    """Raw Gaussian deviation vectors w[i][v][c] = normal((i*m + v)*dim + c).

    The integrator normalises them to unit length at t = 0.  first_ic offsets
    the orbit index, so any slice of an ensemble can be regenerated alone."""
    i = np.arange(first_ic, first_ic + n, dtype=np.uint64)[:, None, None]
    v = np.arange(m, dtype=np.uint64)[None, :, None]
    c = np.arange(dim, dtype=np.uint64)[None, None, :]
    e = (i * np.uint64(m) + v) * np.uint64(dim) + c
    return normal(seed, STREAM_DEVIATION, e)


def section_points(seed, n, y0=-0.4, y1=0.7, py0=-0.45, py1=0.45):
    """n uniform points (y, p_y) in a rectangle of the x = 0 section."""
    k = np.arange(n, dtype=np.uint64)
    uy = uniform(seed, STREAM_IC, np.uint64(2) * k)
    up = uniform(seed, STREAM_IC, np.uint64(2) * k + np.uint64(1))
    return y0 + (y1 - y0) * uy, py0 + (py1 - py0) * up


def fput_mode_draws(seed, n):
    """u[i][j] = uniform(5 i + j): energy, two amplitudes, two phases."""
    k = np.arange(5 * n, dtype=np.uint64)
    return uniform(seed, STREAM_IC, k).reshape(n, 5)


def quartic_draws(seed, n, ndof=3):
    """[i][0:2N] Gaussian directions (position, momentum), [i][2N] a potential
    energy fraction in (0, 1); element e = i*(2N+1) + j."""
    w = 2 * ndof + 1
    e = np.arange(n * w, dtype=np.uint64).reshape(n, w)
    out = normal(seed, STREAM_IC, e)
    out[:, 2 * ndof] = uniform_open(seed, STREAM_IC, np.uint64(2) * e[:, 2 * ndof])
    return out



def dp_states(seed, n, theta_max=np.pi, p_max=0.0):
    """n double-pendulum states (theta_1, theta_2, p_1, p_2): angles uniform
    in [-theta_max, theta_max], momenta uniform in [-p_max, p_max];
    element e = 4 i + j."""
    k = np.arange(4 * n, dtype=np.uint64)
    u = uniform(seed, STREAM_IC, k).reshape(n, 4)
    half = np.array([theta_max, theta_max, p_max, p_max])
    return (2.0 * u - 1.0) * half
