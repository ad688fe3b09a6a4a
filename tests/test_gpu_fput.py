"""GPU parity of the row-per-orbit FPU path against the oracle, through the
C ABI.

Workloads follow the FPU-beta experiments (fixed ends, k = 1, alpha = 0,
beta = 1, energy in the two lowest normal modes, dt = 0.02): the full
Lyapunov spectrum (2N vectors, QR every 10 steps) and GALI_k for k = 2..N
from N seeded vectors, at short T, for every orbit.  Tolerances: state
relative 1e-9, Lyapunov exponents 1e-6 absolute, |log10 GALI| 1e-6 where both
values are >= 1e-8, energy error 1e-12 relative to the energy, LD 1e-9
relative, statuses exactly.
"""
import sys

import numpy as np
import pytest

import seeded_inputs as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2507_00622_amd as P
    from oracle import oracle as O
    return torch, P, O


def run_gpu(env, sys_, x0, mask=None, w0=None, **kw):
    torch, P, _ = env
    dev = torch.device("cuda:0")
    t = lambda a: None if a is None else torch.as_tensor(a, device=dev)
    out = P.integrate_ensemble(sys_, t(x0), mask=t(mask), w0=t(w0), **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def state_err(a, b):
    return np.max(np.abs(a - b), axis=1) / np.maximum(1.0, np.max(np.abs(b), axis=1))


def log_err(a, b, floor):
    ok = (a >= floor) & (b >= floor)
    if not ok.any():
        return 0.0
    return float(np.max(np.abs(np.log10(a[ok]) - np.log10(b[ok]))))


@pytest.mark.parametrize("N", [8, 16])
def test_fput_initial_states(env, N):
    torch, P, O = env
    say(f"case: FPU initial states N={N}")
    u = S.fput_mode_draws(2000 + N, 256)
    xg = P.ic_fput_modes(P.fput(N), u)
    xo = O.fput_ic(O.fput(N), u)
    assert np.max(state_err(xg, xo)) < 1e-13


@pytest.mark.parametrize("N,n,T", [(8, 61, 100.0), (16, 37, 60.0), (4, 45, 100.0),
                                   (2, 30, 100.0)])
def test_fput_lyapunov_gali_parity(env, N, n, T):
    torch, P, O = env
    say(f"case: FPU N={N} n={n} T={T} Lyapunov + GALI")
    so, sg = O.fput(N), P.fput(N)
    x0 = O.fput_ic(so, S.fput_mode_draws(300 + N, n))
    w0 = S.deviation_vectors(400 + N, n, N, 2 * N)
    kw = dict(dt=0.02, T=T, indicators=O.IND_LYAP | O.IND_GALI | O.IND_ENERGY,
              n_lyap=2 * N, gali_kmax=N)
    g = run_gpu(env, sg, x0, None, w0, **kw)
    o = O.integrate(so, x0, O.Run(**kw), w0=w0, threads=8)
    E = np.array([O.hamiltonian(so, x) for x in x0])
    assert np.array_equal(g["status"], o["status"])
    se = state_err(g["x_final"], o["x_final"])
    le = np.max(np.abs(g["lyap"] - o["lyap"]))
    ge = log_err(g["gali"], o["gali"], 1e-8)
    say(f"  state {se.max():.3g} lyap {le:.3g} gali {ge:.3g}")
    assert se.max() < 1e-9
    assert le < 1e-6
    assert ge < 1e-6
    assert np.max(np.abs(g["energy_err"] - o["energy_err"]) / np.maximum(1.0, E)) < 1e-12
    assert np.max(np.abs(g["lyap"].sum(axis=1))) < 1e-9
    assert np.max(np.abs(g["ln_growth"] - o["ln_growth"])) < 1e-6


def test_fput16_four_n_vectors_two_rows(env):
    # N = 16 with more than 48 vectors runs on two rows per orbit (the
    # pivots staged in LDS): the full Lyapunov set and 2N GALI vectors
    torch, P, O = env
    N, n, T = 16, 13, 40.0
    say(f"case: FPU N={N} n={n} T={T} Lyapunov (2N) + GALI_2..2N (2N vectors)")
    so, sg = O.fput(N), P.fput(N)
    x0 = O.fput_ic(so, S.fput_mode_draws(1300, n))
    w0 = S.deviation_vectors(1301, n, 2 * N, 2 * N)
    kw = dict(dt=0.02, T=T, indicators=O.IND_LYAP | O.IND_GALI | O.IND_ENERGY,
              n_lyap=2 * N, gali_kmax=2 * N)
    g = run_gpu(env, sg, x0, None, w0, **kw)
    o = O.integrate(so, x0, O.Run(**kw), w0=w0, threads=8)
    assert np.array_equal(g["status"], o["status"])
    le = np.max(np.abs(g["lyap"] - o["lyap"]))
    ge = log_err(g["gali"], o["gali"], 1e-8)
    say(f"  state {state_err(g['x_final'], o['x_final']).max():.3g} lyap {le:.3g} gali {ge:.3g}")
    assert np.max(state_err(g["x_final"], o["x_final"])) < 1e-9
    assert le < 1e-6 and ge < 1e-6
    assert np.max(np.abs(g["lyap"].sum(axis=1))) < 1e-9


# N = 8 with 17..24 vectors runs two orbits per row: the full Lyapunov set
# with the SALI pair in the third slot (18 vectors, with LD and an early
# exit), a partial Lyapunov set (12: its second slot half full) with 8 GALI
# vectors (20), and the full set with 8 GALI vectors and an escape radius
# that stops 14 of the 45 orbits at different times (rows whose orbits stop
# apart)
@pytest.mark.parametrize("case", ["lyap16_sali", "lyap12_gali8", "lyap16_gali8_escape"])
def test_fput8_two_orbits_per_row(env, case):
    torch, P, O = env
    N, n, T = 8, 45, 60.0
    say(f"case: FPU N=8 two orbits per row, {case}, n={n}, T={T}")
    so, sg = O.fput(N), P.fput(N)
    x0 = O.fput_ic(so, S.fput_mode_draws(1400, n))
    if case == "lyap16_sali":
        kw = dict(dt=0.02, T=T, indicators=O.IND_LYAP | O.IND_SALI | O.IND_LD | O.IND_ENERGY,
                  n_lyap=16)
        w0 = S.deviation_vectors(1401, n, 2, 2 * N)
    elif case == "lyap12_gali8":
        kw = dict(dt=0.02, T=T, indicators=O.IND_LYAP | O.IND_GALI | O.IND_ENERGY,
                  n_lyap=12, gali_kmax=8)
        w0 = S.deviation_vectors(1402, n, 8, 2 * N)
    else:
        kw = dict(dt=0.02, T=T, indicators=O.IND_LYAP | O.IND_GALI | O.IND_ENERGY,
                  n_lyap=16, gali_kmax=8, escape_r2=40.0)
        w0 = S.deviation_vectors(1402, n, 8, 2 * N)
    g = run_gpu(env, sg, x0, None, w0, **kw)
    o = O.integrate(so, x0, O.Run(**kw), w0=w0, threads=8)
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(g["t_end"], o["t_end"])
    se = state_err(g["x_final"], o["x_final"]).max()
    le = np.max(np.abs(g["lyap"] - o["lyap"]))
    say(f"  escaped {int(np.sum(o['status'] == O.ST_ESCAPED))}, state {se:.3g} lyap {le:.3g}")
    assert se < 1e-9 and le < 1e-6
    assert np.max(np.abs(g["ln_growth"] - o["ln_growth"])) < 1e-6
    if case == "lyap16_gali8_escape":
        assert np.sum(o["status"] == O.ST_ESCAPED) == 14
    if case == "lyap16_sali":
        assert np.max(np.abs(g["lyap"].sum(axis=1))) < 1e-9
        assert log_err(g["sali_min"], o["sali_min"], 1e-12) < 1e-6
        assert np.max(np.abs(g["ld"] / o["ld"] - 1)) < 1e-9
        # a threshold inside the SALI minima of these orbits (0.13 .. 1.2 by
        # T = 60), so that some of them stop early
        kw2 = dict(kw, early_exit=True, sali_threshold=0.34)
        g2 = run_gpu(env, sg, x0, None, w0, **kw2)
        o2 = O.integrate(so, x0, O.Run(**kw2), w0=w0, threads=8)
        say("  exited:", int(np.sum(o2["status"] == O.ST_EXITED)))
        assert np.array_equal(g2["status"], o2["status"])
        assert np.array_equal(g2["t_end"], o2["t_end"])
    else:
        assert log_err(g["gali"], o["gali"], 1e-8) < 1e-6


# N = 8 with more than N SALI/GALI vectors stays on one orbit per row (two
# slots of 16): GALI_2..2N with the full spectrum (32 vectors) and with half
# of it (24)
@pytest.mark.parametrize("n_lyap", [16, 8])
def test_fput8_gali_2n_one_orbit_per_row(env, n_lyap):
    torch, P, O = env
    N, n, T = 8, 29, 40.0
    say(f"case: FPU N=8 Lyapunov ({n_lyap}) + GALI_2..2N, n={n}, T={T}")
    so, sg = O.fput(N), P.fput(N)
    x0 = O.fput_ic(so, S.fput_mode_draws(1410, n))
    w0 = S.deviation_vectors(1411, n, 2 * N, 2 * N)
    kw = dict(dt=0.02, T=T, indicators=O.IND_LYAP | O.IND_GALI | O.IND_ENERGY,
              n_lyap=n_lyap, gali_kmax=2 * N)
    g = run_gpu(env, sg, x0, None, w0, **kw)
    o = O.integrate(so, x0, O.Run(**kw), w0=w0, threads=8)
    assert np.array_equal(g["status"], o["status"])
    le = np.max(np.abs(g["lyap"] - o["lyap"]))
    ge = log_err(g["gali"], o["gali"], 1e-8)
    say(f"  state {state_err(g['x_final'], o['x_final']).max():.3g} lyap {le:.3g} gali {ge:.3g}")
    assert np.max(state_err(g["x_final"], o["x_final"])) < 1e-9
    assert le < 1e-6 and ge < 1e-6


@pytest.mark.parametrize("N", [16, 8])
def test_fput_sali_ld_early_exit(env, N):
    torch, P, O = env
    say(f"case: FPU N={N} SALI + LD + early exit")
    so, sg = O.fput(N), P.fput(N)
    n = 50
    x0 = O.fput_ic(so, S.fput_mode_draws(500 + N, n))
    w0 = S.deviation_vectors(600 + N, n, 2, 2 * N)
    kw = dict(dt=0.02, T=100.0, indicators=O.IND_SALI | O.IND_LD | O.IND_ENERGY)
    g = run_gpu(env, sg, x0, None, w0, **kw)
    o = O.integrate(so, x0, O.Run(**kw), w0=w0, threads=8)
    assert np.array_equal(g["status"], o["status"])
    assert log_err(g["sali_min"], o["sali_min"], 1e-12) < 1e-6
    assert log_err(g["sali_final"], o["sali_final"], 1e-12) < 1e-6
    assert np.max(np.abs(g["ld"] / o["ld"] - 1)) < 1e-9
    assert np.max(state_err(g["x_final"], o["x_final"])) < 1e-9
    # early exit with a loose threshold so that some orbits stop
    kw2 = dict(kw, early_exit=True, sali_threshold=1e-2)
    g2 = run_gpu(env, sg, x0, None, w0, **kw2)
    o2 = O.integrate(so, x0, O.Run(dt=0.02, T=100.0, indicators=kw["indicators"],
                                   early_exit=True, sali_threshold=1e-2), w0=w0, threads=8)
    say("  exited:", int(np.sum(o2["status"] == O.ST_EXITED)))
    assert np.array_equal(g2["status"], o2["status"])
    assert np.array_equal(g2["t_end"], o2["t_end"])


def test_fput_masks_ragged_and_resume(env):
    torch, P, O = env
    say("case: FPU masks, ragged rows, resume")
    N = 8
    so, sg = O.fput(N), P.fput(N)
    n = 23
    x0 = O.fput_ic(so, S.fput_mode_draws(700, n))
    x0[5, 3] = np.nan
    mask = np.ones(n, np.uint8)
    mask[[0, 7, 22]] = 0
    w0 = S.deviation_vectors(800, n, N, 2 * N)
    kw = dict(dt=0.02, T=20.0, indicators=O.IND_LYAP | O.IND_GALI | O.IND_ENERGY,
              n_lyap=2 * N, gali_kmax=N)
    g = run_gpu(env, sg, x0, mask, w0, **kw)
    o = O.integrate(so, x0, O.Run(**kw), w0=w0, mask=mask)
    assert np.array_equal(g["status"], o["status"])
    ok = o["status"] == 0
    assert np.max(state_err(g["x_final"][ok], o["x_final"][ok])) < 1e-11
    assert np.max(np.abs(g["lyap"][ok] - o["lyap"][ok])) < 1e-9
    dev = torch.device("cuda:0")
    e = P.Ensemble(sg, torch.as_tensor(x0, device=dev), mask=torch.as_tensor(mask, device=dev),
                   w0=torch.as_tensor(w0, device=dev), steps_per_launch=70, **kw)
    for s in (200, 470, 1000):
        e.advance(s)
    r = {k: v.cpu().numpy() for k, v in e.results().items()}
    e.close()
    for k in g:
        assert np.array_equal(g[k], r[k], equal_nan=True), k


def test_fput_harmonic_chain_exponents_vanish(env):
    # beta = 0: the linear chain is integrable, every exponent -> 0 as
    # O(1/T) (bounded tangent growth), and GALI_k for k <= N stays O(1)
    torch, P, O = env
    say("case: linear chain")
    N = 8
    sg = P.fput(N, 1.0, 0.0, 0.0)
    x0 = O.fput_ic(O.fput(N, 1.0, 0.0, 0.0), S.fput_mode_draws(900, 16))
    w0 = S.deviation_vectors(901, 16, N, 2 * N)
    g = run_gpu(env, sg, x0, None, w0, dt=0.02, T=400.0,
                indicators=O.IND_LYAP | O.IND_GALI, n_lyap=2 * N, gali_kmax=N)
    assert np.max(np.abs(g["lyap"])) < 0.02
    assert np.min(g["gali"][:, N - 2]) > 1e-4


@pytest.mark.parametrize("N", [3, 5, 6, 7, 9, 12, 15])
def test_fput_any_dof_component_rows(env, N):
    # chains whose N is not a power of two run on the component-row kernel
    # (up to four vectors): GALI_4 with SALI, LD and energy, as in the
    # degrees-of-freedom sweep
    torch, P, O = env
    say(f"case: FPU N={N} component rows, SALI + GALI_4 + LD + energy, n=41")
    so, sg = O.fput(N), P.fput(N)
    n = 41
    x0 = O.fput_ic(so, S.fput_mode_draws(700 + N, n))
    w0 = S.deviation_vectors(800 + N, n, 4, 2 * N)
    kw = dict(dt=0.02, T=60.0, indicators=O.IND_SALI | O.IND_GALI | O.IND_LD | O.IND_ENERGY,
              gali_kmax=4)
    g = run_gpu(env, sg, x0, None, w0, **kw)
    o = O.integrate(so, x0, O.Run(**kw), w0=w0, threads=8)
    E = np.array([O.hamiltonian(so, x) for x in x0])
    assert np.array_equal(g["status"], o["status"])
    se = state_err(g["x_final"], o["x_final"])
    ge = log_err(g["gali"], o["gali"], 1e-8)
    say(f"  state {se.max():.3g} gali {ge:.3g}")
    assert se.max() < 1e-9
    assert ge < 1e-6
    assert log_err(g["sali_min"], o["sali_min"], 1e-12) < 1e-6
    assert np.max(np.abs(g["ld"] / o["ld"] - 1)) < 1e-9
    assert np.max(np.abs(g["energy_err"] - o["energy_err"]) / np.maximum(1.0, E)) < 1e-12
    # more than four vectors needs a power of two
    from paper_2507_00622_amd import chx
    with pytest.raises(chx.ChxError) as e:
        run_gpu(env, sg, x0, None, None, dt=0.02, T=1.0, indicators=O.IND_LYAP, n_lyap=2 * N)
    assert e.value.status == chx.ERR_UNSUPPORTED


@pytest.mark.parametrize("N", [4, 7, 16])
def test_fput_without_vectors(env, N):
    # LD and energy alone (no deviation vectors): the state block of an
    # orbit without vectors is followed directly by its accumulators, which
    # a kernel must not treat as vector storage
    torch, P, O = env
    say(f"case: FPU N={N} without vectors, LD + energy")
    so, sg = O.fput(N), P.fput(N)
    n = 37
    x0 = O.fput_ic(so, S.fput_mode_draws(900 + N, n))
    kw = dict(dt=0.02, T=40.0, indicators=O.IND_LD | O.IND_ENERGY)
    g = run_gpu(env, sg, x0, **kw)
    o = O.integrate(so, x0, O.Run(**kw), threads=8)
    E = np.array([O.hamiltonian(so, x) for x in x0])
    assert np.array_equal(g["status"], o["status"])
    assert np.max(state_err(g["x_final"], o["x_final"])) < 1e-9
    assert np.max(np.abs(g["ld"] / o["ld"] - 1)) < 1e-9
    assert np.max(np.abs(g["energy_err"] - o["energy_err"]) / np.maximum(1.0, E)) < 1e-12
