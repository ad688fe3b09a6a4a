"""GPU parity of the FPU component-row DOP853 kernels (fixed step and the
adaptive DOP8(5)) against the oracle's DOP853 drivers, through the C ABI.

FPU-beta chains (k = 1, beta = 1, energy in the two lowest normal modes)
with up to four deviation vectors.  Tolerances as for the other DOP853
tests: state 1e-9 relative, |log10 SALI| and |log10 GALI| 1e-6 above their
floors, exponents 1e-6, LD 1e-9 (fixed step), energy error 1e-12 relative
to the energy; adaptive: step counts equal on at least 99 % of the orbits,
compared where they are, LD 1e-3 (outside the error control).
"""
import sys

import numpy as np
import pytest

import seeded_inputs as S

pytestmark = pytest.mark.gpu
ALL = 1 | 2 | 4 | 8 | 16


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


def oracle_run(O, integ, **kw):
    kw = dict(kw)
    K = kw.pop("renorm_every", 10)
    if integ == "dop853_adaptive":
        tol = kw.pop("rtol")
        kw.pop("atol", None)
        return O.Run(integrator=O.INT_DOP853_ADAPTIVE, rtol=tol, atol=tol, K=K, **kw)
    return O.Run(integrator=O.INT_DOP853, K=K, **kw)


def compare(g, o, sel, E, ld_rel, tag):
    se = state_err(g["x_final"][sel], o["x_final"][sel]).max()
    msg = f"  {tag}: {sel.sum()} orbits, state {se:.2e}"
    assert se < 1e-9
    if "sali_min" in g:
        assert log_err(g["sali_min"][sel], o["sali_min"][sel], 1e-12) < 1e-6
    if "gali" in g:
        ge = log_err(g["gali"][sel], o["gali"][sel], 1e-8)
        msg += f" gali {ge:.2e}"
        assert ge < 1e-6
    if "lyap" in g:
        le = np.max(np.abs(g["lyap"][sel] - o["lyap"][sel]))
        msg += f" lyap {le:.2e}"
        assert le < 1e-6
    if "ld" in g:
        assert np.max(np.abs(g["ld"][sel] / o["ld"][sel] - 1)) < ld_rel
    if "energy_err" in g:
        assert np.max(np.abs(g["energy_err"][sel] - o["energy_err"][sel]) /
                      np.maximum(1.0, E[sel])) < 1e-12
    say(msg)


@pytest.mark.parametrize("N", [2, 5, 8, 16])
def test_fput_dop853_fixed(env, N):
    torch, P, O = env
    say(f"case: FPU N={N} fixed DOP853, SALI + GALI_4 + LD + energy, n=45, T=60")
    so, sg = O.fput(N), P.fput(N)
    n = 45
    x0 = O.fput_ic(so, S.fput_mode_draws(1100 + N, n))
    w0 = S.deviation_vectors(1200 + N, n, 4, 2 * N)
    kw = dict(dt=0.02, T=60.0, indicators=O.IND_SALI | O.IND_GALI | O.IND_LD | O.IND_ENERGY,
              gali_kmax=4)
    g = run_gpu(env, sg, x0, None, w0, integrator="dop853", **kw)
    o = O.integrate(so, x0, oracle_run(O, "dop853", **kw), w0=w0, threads=8)
    E = np.array([O.hamiltonian(so, x) for x in x0])
    assert np.array_equal(g["status"], o["status"])
    compare(g, o, np.ones(n, bool), E, 1e-9, "fixed")


def test_fput_dop853_lyapunov_full_spectrum(env):
    torch, P, O = env
    say("case: FPU N=2 fixed DOP853, full Lyapunov spectrum (4 vectors), T=100")
    so, sg = O.fput(2), P.fput(2)
    x0 = O.fput_ic(so, S.fput_mode_draws(1300, 40))
    kw = dict(dt=0.02, T=100.0, indicators=O.IND_LYAP | O.IND_ENERGY, n_lyap=4)
    g = run_gpu(env, sg, x0, integrator="dop853", **kw)
    o = O.integrate(so, x0, oracle_run(O, "dop853", **kw), threads=8)
    E = np.array([O.hamiltonian(so, x) for x in x0])
    compare(g, o, np.ones(len(x0), bool), E, 1e-9, "lyap")
    assert np.max(np.abs(g["lyap"].sum(axis=1))) < 1e-9


@pytest.mark.parametrize("N", [4, 16])
def test_fput_dop853_adaptive(env, N):
    torch, P, O = env
    say(f"case: FPU N={N} adaptive DOP8(5) 1e-10, SALI + GALI_4 + LD + energy, n=45, T=40")
    so, sg = O.fput(N), P.fput(N)
    n = 45
    x0 = O.fput_ic(so, S.fput_mode_draws(1400 + N, n))
    w0 = S.deviation_vectors(1500 + N, n, 4, 2 * N)
    kw = dict(dt=0.1, T=40.0, indicators=O.IND_SALI | O.IND_GALI | O.IND_LD | O.IND_ENERGY,
              gali_kmax=4, rtol=1e-10, atol=1e-10)
    g = run_gpu(env, sg, x0, None, w0, integrator="dop853_adaptive", **kw)
    o = O.integrate(so, x0, oracle_run(O, "dop853_adaptive", **kw), w0=w0, threads=8)
    E = np.array([O.hamiltonian(so, x) for x in x0])
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(g["t_end"], o["t_end"])
    same = (g["steps"][:, 0] == o["steps_accepted"]) & (g["steps"][:, 1] == o["steps_rejected"])
    say("  same step counts", same.sum(), "of", n, "steps/orbit", g["steps"][:, 0].mean(),
        "rejected", g["steps"][:, 1].sum())
    assert same.sum() >= 0.99 * n
    compare(g, o, same, E, 1e-3, "adaptive")
    # the largest accepted step error (the last one of a step shortened to
    # end on a checkpoint sits near the rounding floor and is not compared)
    se_rel = np.max(np.abs(g["step_err"][same, 0] / o["step_err"][same, 0] - 1))
    say("  largest step_err rel err", se_rel)
    assert se_rel < 3e-4
    e = g["step_err"]
    assert np.all(e[:, 1] <= e[:, 0]) and np.all(e[:, 0] <= 1.0) and np.all(e[:, 1] > 0)


def test_fput_dop853_edges_resume_blocks(env):
    torch, P, O = env
    say("case: FPU N=6 both DOP853 solvers: ragged n=37, masked and non-finite, K=7, "
        "T not a multiple of K dt, resume bit for bit")
    so, sg = O.fput(6), P.fput(6)
    n = 37
    x0 = O.fput_ic(so, S.fput_mode_draws(1600, n))
    x0[4, 2] = np.nan
    mask = (np.arange(n) % 6 != 2).astype(np.uint8)
    mask[4] = 1
    w0 = S.deviation_vectors(1700, n, 2, 12)
    dev = torch.device("cuda:0")
    for integ, extra in (("dop853", {}), ("dop853_adaptive", dict(rtol=1e-9, atol=1e-9))):
        kw = dict(dt=0.02, T=3.06, indicators=ALL, gali_kmax=2, n_lyap=2, renorm_every=7,
                  **extra)
        g = run_gpu(env, sg, x0, mask, w0, integrator=integ, **kw)
        o = O.integrate(so, x0, oracle_run(O, integ, **kw), w0=w0, mask=mask)
        assert g["status"][4] == 3 and o["status"][4] == 3
        assert np.array_equal(g["status"], o["status"])
        act = (mask == 1) & (o["status"] == 0)
        if integ == "dop853_adaptive":
            act &= (g["steps"][:, 0] == o["steps_accepted"]) & (
                g["steps"][:, 1] == o["steps_rejected"])
        assert np.max(state_err(g["x_final"][act], o["x_final"][act])) < 1e-11
        # resume through the ensemble object in pieces: bit-identical
        e = P.Ensemble(sg, torch.as_tensor(x0, device=dev), mask=torch.as_tensor(mask, device=dev),
                       w0=torch.as_tensor(w0, device=dev), steps_per_launch=21,
                       integrator=integ, **kw)
        for st in (70, 140, 153):
            e.advance(st)
        r = {k: v.cpu().numpy() for k, v in e.results().items()}
        e.close()
        for k in g:
            assert np.array_equal(g[k], r[k], equal_nan=True), (integ, k)


# More than four vectors: the component rows keep them in LDS.  The full
# Lyapunov spectrum (2N vectors) under both DOP853 solvers, at N = 8 with
# the SALI/GALI set beside it (3N vectors) and at N = 16 (2N vectors).
@pytest.mark.parametrize("integ", ["dop853", "dop853_adaptive"])
@pytest.mark.parametrize("N,gali", [(8, True), (16, False)])
def test_fput_dop853_full_spectrum_lds(env, N, gali, integ):
    torch, P, O = env
    n, T = 23, 40.0  # ragged: the last block of four orbits has three
    say(f"case: FPU N={N} {integ}, 2N Lyapunov vectors{' + N GALI' if gali else ''}, "
        f"n={n}, T={T}")
    so, sg = O.fput(N), P.fput(N)
    x0 = O.fput_ic(so, S.fput_mode_draws(1600 + N, n))
    ind = O.IND_LYAP | O.IND_ENERGY
    kw = dict(dt=0.02, T=T, n_lyap=2 * N)
    w0 = None
    if gali:
        ind |= O.IND_SALI | O.IND_GALI
        kw["gali_kmax"] = N
        w0 = S.deviation_vectors(1700 + N, n, N, 2 * N)
    kw["indicators"] = ind
    if integ == "dop853_adaptive":
        kw.update(rtol=1e-10, atol=1e-10)
    g = run_gpu(env, sg, x0, None, w0, integrator=integ, **kw)
    o = O.integrate(so, x0, oracle_run(O, integ, **kw), w0=w0, threads=8)
    E = np.array([O.hamiltonian(so, x) for x in x0])
    assert np.array_equal(g["status"], o["status"])
    sel = np.ones(n, bool)
    if integ == "dop853_adaptive":
        sel = (g["steps"][:, 0] == o["steps_accepted"]) & (g["steps"][:, 1] == o["steps_rejected"])
        say("  same step counts", sel.sum(), "of", n, "steps/orbit", g["steps"][:, 0].mean())
        assert sel.sum() >= 0.95 * n
    le = np.max(np.abs(g["lyap"][sel] - o["lyap"][sel]))
    say(f"  lyap {le:.3g}")
    compare(g, o, sel, E, 1e-9, integ)
    assert le < 1e-6
    assert np.max(np.abs(g["energy_err"][sel] - o["energy_err"][sel]) / np.maximum(1.0, E[sel])) < 1e-10


def test_fput_dop853_lds_resume_and_launch_split(env):
    # the LDS kernels write their vectors back at every launch end: split
    # launches give the same bits as one
    torch, P, O = env
    say("case: FPU N=8 DOP853 (LDS vectors): launches of 70 steps against one")
    so, sg = O.fput(8), P.fput(8)
    n = 9
    x0 = O.fput_ic(so, S.fput_mode_draws(1800, n))
    dev = torch.device("cuda:0")
    kw = dict(dt=0.02, T=6.0, indicators=O.IND_LYAP | O.IND_ENERGY, n_lyap=16,
              integrator="dop853")
    one = run_gpu(env, sg, x0, **kw)
    e = P.Ensemble(sg, torch.as_tensor(x0, device=dev), steps_per_launch=70, **kw)
    e.advance()
    r = {k: v.cpu().numpy() for k, v in e.results().items()}
    e.close()
    for k in one:
        assert np.array_equal(one[k], r[k], equal_nan=True), k
