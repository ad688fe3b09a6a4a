"""GPU parity of the double-pendulum DOP853 lane kernels (fixed step and
adaptive DOP8(5)) against the oracle, through the C ABI.

The double pendulum's Hamiltonian is not separable: the kernels evaluate
its field and, through dual numbers, the field's directional derivative;
the oracle does the same arithmetic in its own code.  The two sides round
differently (sin and cos of theta_1 - theta_2 from the angles' on the GPU,
directly in the oracle; fused stage sums on the GPU), so chaotic orbits
are compared where their divergence e^(lambda T) keeps rounding below the
tolerances (T = 10), regular orbits over longer times:
  - state 1e-9 relative; |log10 SALI| and |log10 GALI| 1e-6 where both are
    above their floors; Lyapunov exponents 1e-6 absolute; LD 1e-9 relative
    (fixed step); energy error 1e-12 absolute;
  - status codes, t_end and masks exactly; the adaptive solver's step
    counts equal for at least 99 % of the orbits (a step whose error
    estimate lands within rounding of 1 can be accepted on one side and
    rejected on the other), the rest compared only where they agree.
"""
import math
import sys

import numpy as np
import pytest

import seeded_inputs as S

pytestmark = pytest.mark.gpu

ALL = 1 | 2 | 4 | 8 | 16
PARAMS = [(1.0, 1.0), (0.7, 2.5)]


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


def oracle_run(O, integrator, **kw):
    kw = dict(kw)
    K = kw.pop("renorm_every", 10)
    if integrator == "dop853_adaptive":
        tol = kw.pop("rtol")
        kw.pop("atol", None)
        return O.Run(integrator=O.INT_DOP853_ADAPTIVE, rtol=tol, atol=tol, K=K, **kw)
    return O.Run(integrator=O.INT_DOP853, K=K, **kw)


def state_err(a, b):
    return np.max(np.abs(a - b), axis=1) / np.maximum(1.0, np.max(np.abs(b), axis=1))


def log_err(a, b, floor=1e-12):
    ok = (a >= floor) & (b >= floor)
    if not ok.any():
        return 0.0
    return float(np.max(np.abs(np.log10(a[ok]) - np.log10(b[ok]))))


def dp_x0(seed, n, theta_max=math.pi, p_max=1.0):
    return S.dp_states(seed, n, theta_max, p_max)


def compare(g, o, sel, ld_rel, tag):
    """Compare the outputs both sides produced on the orbits sel."""
    se = state_err(g["x_final"][sel], o["x_final"][sel]).max()
    msg = f"  {tag}: state {se:.2e}"
    assert se < 1e-9
    if "sali_min" in g:
        msg += f" sali {log_err(g['sali_min'][sel], o['sali_min'][sel]):.2e}"
        assert log_err(g["sali_min"][sel], o["sali_min"][sel]) < 1e-6
        assert log_err(g["sali_final"][sel], o["sali_final"][sel]) < 1e-6
    if "gali" in g:
        for k in range(g["gali"].shape[1]):
            assert log_err(g["gali"][sel, k], o["gali"][sel, k], floor=1e-8) < 1e-6, k
    if "lyap" in g:
        lyap = np.max(np.abs(g["lyap"][sel] - o["lyap"][sel]))
        msg += (f" lyap {lyap:.2e} max|sum lyap| "
                f"{np.max(np.abs(g['lyap'][sel].sum(axis=1))):.2e}")
        assert lyap < 1e-6
    if "ld" in g:
        assert np.max(np.abs(g["ld"][sel] / o["ld"][sel] - 1)) < ld_rel
    if "energy_err" in g:
        assert np.max(np.abs(g["energy_err"][sel] - o["energy_err"][sel])) < 1e-12
    say(msg)


@pytest.mark.parametrize("alpha,sigma", PARAMS)
def test_dp_fixed_all_indicators(env, alpha, sigma):
    torch, P, O = env
    say(f"case: DOP853 double pendulum alpha={alpha} sigma={sigma} n=300, all indicators "
        "(GALI_2..4, 4 exponents), T=10")
    x0 = dp_x0(41, 300)
    w0 = S.deviation_vectors(42, len(x0), 4, 4)
    kw = dict(dt=0.01, T=10.0, indicators=ALL, gali_kmax=4, n_lyap=4)
    g = run_gpu(env, P.double_pendulum(alpha, sigma), x0, None, w0, integrator="dop853", **kw)
    o = O.integrate(O.double_pendulum(alpha, sigma), x0, oracle_run(O, "dop853", **kw), w0=w0,
                    threads=8)
    assert np.array_equal(g["status"], o["status"])
    assert (o["status"] == 0).all()
    compare(g, o, np.ones(len(x0), bool), 1e-9, "all orbits")


def test_dp_fixed_regular_T200(env):
    torch, P, O = env
    say("case: DOP853 double pendulum small oscillations n=500, SALI+LD+energy, T=200")
    x0 = dp_x0(43, 500, theta_max=0.3, p_max=0.2)
    w0 = S.deviation_vectors(44, len(x0), 2, 4)
    kw = dict(dt=0.02, T=200.0, indicators=O.IND_SALI | O.IND_LD | O.IND_ENERGY)
    g = run_gpu(env, P.double_pendulum(), x0, None, w0, integrator="dop853", **kw)
    o = O.integrate(O.double_pendulum(), x0, oracle_run(O, "dop853", **kw), w0=w0, threads=8)
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(g["label"], o["label"])
    compare(g, o, np.ones(len(x0), bool), 1e-9, "regular")


@pytest.mark.parametrize("alpha,sigma", PARAMS)
def test_dp_adaptive_all_indicators(env, alpha, sigma):
    torch, P, O = env
    say(f"case: adaptive double pendulum alpha={alpha} sigma={sigma} n=300, all indicators, "
        "T=10, tol 1e-10")
    x0 = dp_x0(45, 300)
    w0 = S.deviation_vectors(46, len(x0), 2, 4)
    kw = dict(dt=0.1, T=10.0, indicators=ALL, gali_kmax=2, n_lyap=4, rtol=1e-10, atol=1e-10)
    g = run_gpu(env, P.double_pendulum(alpha, sigma), x0, None, w0,
                integrator="dop853_adaptive", **kw)
    o = O.integrate(O.double_pendulum(alpha, sigma), x0, oracle_run(O, "dop853_adaptive", **kw),
                    w0=w0, threads=8)
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(g["t_end"], o["t_end"])
    same = (g["steps"][:, 0] == o["steps_accepted"]) & (g["steps"][:, 1] == o["steps_rejected"])
    say("  same step counts", same.sum(), "of", len(same), "steps/orbit",
        g["steps"][:, 0].mean(), "rejected/orbit", g["steps"][:, 1].mean())
    assert same.sum() >= 0.99 * len(same)
    # the LD lies outside the error control (its cusps make it depend on
    # where the stages fall), compared as in the Henon-Heiles adaptive tests
    compare(g, o, same, 1e-3, "same step counts")
    assert g["energy_err"].max() < 1e-8


def test_dp_edges(env):
    torch, P, O = env
    say("case: double pendulum ragged n=333 with masked and non-finite states, K=7, "
        "T=2.53, both integrators; empty ensemble")
    n = 333
    x0 = dp_x0(47, n)
    x0[3] = [np.nan, 0, 0, 0]
    mask = (np.arange(n) % 5 != 1).astype(np.uint8)
    mask[3] = 1
    w0 = S.deviation_vectors(48, n, 2, 4)
    for integ, extra in (("dop853", {}), ("dop853_adaptive", dict(rtol=1e-9, atol=1e-9))):
        kw = dict(dt=0.01, T=2.53, indicators=ALL, gali_kmax=2, n_lyap=4, renorm_every=7,
                  **extra)
        g = run_gpu(env, P.double_pendulum(), x0, mask, w0, integrator=integ, **kw)
        o = O.integrate(O.double_pendulum(), x0, oracle_run(O, integ, **kw), w0=w0, mask=mask)
        act = mask == 1
        assert g["status"][3] == 3 and o["status"][3] == 3
        assert np.array_equal(g["status"], o["status"])
        assert np.array_equal(g["label"] == -1, mask == 0)
        assert np.array_equal(g["t_end"][act], o["t_end"][act])
        ok = act & (o["status"] == 0)
        if integ == "dop853_adaptive":
            ok &= (g["steps"][:, 0] == o["steps_accepted"]) & (
                g["steps"][:, 1] == o["steps_rejected"])
            assert ok.sum() >= 0.99 * (act & (o["status"] == 0)).sum()
            assert np.all(g["steps"][~act] == 0)
        assert np.max(state_err(g["x_final"][ok], o["x_final"][ok])) < 1e-11
    g = run_gpu(env, P.double_pendulum(), np.zeros((0, 4)), None, np.zeros((0, 2, 4)),
                integrator="dop853", dt=0.01, T=1.0, indicators=O.IND_SALI)
    assert g["x_final"].shape == (0, 4)


@pytest.mark.parametrize("integ", ["dop853", "dop853_adaptive"])
def test_dp_resume_bitwise_and_block_sizes(env, integ):
    torch, P, O = env
    say(f"case: double pendulum {integ} resume and block sizes")
    x0 = dp_x0(49, 256)
    w0 = S.deviation_vectors(50, len(x0), 2, 4)
    dev = torch.device("cuda:0")
    extra = dict(rtol=1e-9, atol=1e-9) if integ == "dop853_adaptive" else {}
    kw = dict(dt=0.05, T=30.0, indicators=ALL, gali_kmax=2, n_lyap=4, renorm_every=20,
              integrator=integ, **extra)
    ref = run_gpu(env, P.double_pendulum(), x0, None, w0, **kw)
    e = P.Ensemble(P.double_pendulum(), torch.as_tensor(x0, device=dev),
                   w0=torch.as_tensor(w0, device=dev), steps_per_launch=60, **kw)
    for s in (200, 420, 600):
        e.advance(s)
    r = {k: v.cpu().numpy() for k, v in e.results().items()}
    e.close()
    for k in ref:
        assert np.array_equal(ref[k], r[k], equal_nan=True), k
    for block in (64, 128):
        b = run_gpu(env, P.double_pendulum(), x0, None, w0, block_size=block, **kw)
        for k in ref:
            assert np.array_equal(ref[k], b[k], equal_nan=True), (block, k)


@pytest.mark.parametrize("integ", ["dop853", "dop853_adaptive"])
def test_dp_full_size_sampled(env, integ):
    # the timing workload at its largest size, in the benchmark's launch
    # configuration: 2^19 states from rest on the angle grid, SALI + energy,
    # T = 1e3, fixed dt = 0.02 in launches of 10,000 steps or the adaptive
    # solver at 1e-11; energy held near 1e-9 on every orbit, and sampled
    # regular orbits equal to the oracle's one by one (deviation vectors
    # drawn by the library from seed 7, regenerated here for the oracle)
    torch, P, O = env
    from bench import dp_angle_grid
    x0 = dp_angle_grid(19)
    say(f"case: double pendulum {integ} 2^19 angle grid, SALI+energy, T=1000 (benchmark size)")
    dev = torch.device("cuda:0")
    T = 1000.0
    leg = (dict(dt=0.02, integrator="dop853") if integ == "dop853" else
           dict(dt=0.1, integrator="dop853_adaptive", rtol=1e-11, atol=1e-11))
    n_steps = int(round(T / leg["dt"]))
    spl = min(10000, n_steps)
    e = P.Ensemble(P.double_pendulum(), torch.as_tensor(x0, device=dev), steps_per_launch=spl,
                   T=T, indicators=O.IND_SALI | O.IND_ENERGY, seed=7, **leg)
    s = 0
    while s < n_steps:
        s = min(s + spl, n_steps)
        e.advance(s)
    g = {k: v.cpu().numpy() for k, v in e.results().items()}
    e.close()
    assert (g["status"] == 0).all()
    ee = g["energy_err"]
    say(f"  energy error: median {np.median(ee):.2e} max {ee.max():.2e}; chaotic "
        f"{(g['label'] == 1).mean():.4f}")
    assert np.median(ee) < 1e-9
    assert ee.max() < (5e-8 if integ == "dop853" else 1e-8)
    reg = np.where(g["label"] == 0)[0]
    amp = np.abs(x0[reg, :2]).max(axis=1)
    pick = reg[np.argsort(amp)[np.linspace(0, len(reg) - 1, 6).astype(int)]]
    w0 = np.concatenate([S.deviation_vectors(7, 1, 2, 4, first_ic=int(i)) for i in pick])
    kw = dict(T=T, indicators=O.IND_SALI | O.IND_ENERGY,
              **{k: v for k, v in leg.items() if k != "integrator"})
    o = O.integrate(O.double_pendulum(), x0[pick], oracle_run(O, integ, **kw), w0=w0,
                    threads=6)
    if integ == "dop853_adaptive":
        same = (g["steps"][pick, 0] == o["steps_accepted"]) & (
            g["steps"][pick, 1] == o["steps_rejected"])
        assert same.sum() >= len(pick) - 1
        pick, o = pick[same], {k: v[same] for k, v in o.items()}
    err = state_err(g["x_final"][pick], o["x_final"])
    say("  sampled regular orbits", len(pick), "state error", err.max())
    assert err.max() < 1e-7
    assert np.array_equal(g["label"][pick], o["label"])
    # the energy error is the method's truncation error (same steps on both
    # sides) plus rounding noise
    assert np.all(np.abs(g["energy_err"][pick] - o["energy_err"])
                  <= 0.05 * o["energy_err"] + 1e-12)
