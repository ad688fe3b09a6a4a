"""GPU parity of the lane-per-orbit path (Henon-Heiles, quartic, harmonic)
against the oracle, through the C ABI.

Tolerances (floating point; rounding differs because the HIP path fuses
multiply-adds and merges commuting kicks, the oracle does neither):
  - state, regular orbits (oracle label at T = 1e4), T = 200: relative 1e-9
    (max_c |x_gpu - x_cpu| / max(1, |x_cpu|_inf));
  - every orbit at short T -- about ten Lyapunov times of the fastest orbit
    of the set: T = 100 at E = 0.125, T = 50 at E = 1/6 -- |log10 SALI| 1e-6
    where both values are >= 1e-12, |log10 GALI| 1e-6 where both are >= 1e-8
    (GALI comes from a QR of unit vectors, whose small R_kk carry an absolute
    rounding error near 1e-16 on both sides), Lyapunov exponents
    1e-6 absolute, LD 1e-9 relative, energy error 1e-12 absolute;
  - integers (status, mask, labels of regular orbits) exactly.
"""
import os
import sys

import numpy as np
import pytest

import seeded_inputs as S

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


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


def log_err(a, b, floor=1e-12):
    ok = (a >= floor) & (b >= floor)
    if not ok.any():
        return 0.0
    return float(np.max(np.abs(np.log10(a[ok]) - np.log10(b[ok]))))


def golden_labels():
    lab = {}
    for line in open(os.path.join(HERE, "golden", "hh_e0125_32x32_T1e4.txt")):
        if line.startswith("#"):
            continue
        i, l, _ = line.split()
        lab[int(i)] = int(l)
    return np.array([lab[i] for i in range(len(lab))])


ALL = 1 | 2 | 4 | 8 | 16


def test_hh_sali_ld_state_regular_T200(env):
    torch, P, O = env
    say("case: HH E=0.125 32x32, SALI+LD+energy, T=200")
    x0, mask = O.hh_grid(0.125, 32, 32)
    w0 = S.deviation_vectors(1001, len(x0), 2, 4)
    ind = O.IND_SALI | O.IND_LD | O.IND_ENERGY
    g = run_gpu(env, P.henon_heiles(), x0, mask, w0, dt=0.01, T=200.0, indicators=ind)
    o = O.integrate(O.henon_heiles(), x0, O.Run(dt=0.01, T=200.0, indicators=ind), w0=w0,
                    mask=mask, threads=8)
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(g["label"] == -1, mask == 0)
    lab = golden_labels()
    reg = lab == 0
    assert reg.sum() > 200
    err = state_err(g["x_final"][reg], o["x_final"][reg])
    say("max regular-orbit state error at T=200:", err.max())
    assert err.max() < 1e-9
    act = mask == 1
    assert np.max(np.abs(g["energy_err"][act] - o["energy_err"][act])) < 1e-12
    assert np.max(np.abs(g["ld"][reg] / o["ld"][reg] - 1)) < 1e-9
    # labels at T = 200 of regular orbits cannot flip
    assert np.array_equal(g["label"][reg], o["label"][reg])


def test_hh_all_indicators_T100(env):
    torch, P, O = env
    for E, T in ((0.125, 100.0), (1.0 / 6.0, 50.0)):
        say(f"case: HH E={E:.6f} 24x24, all indicators, T={T}")
        x0, mask = O.hh_grid(E, 24, 24)
        w0 = S.deviation_vectors(7, len(x0), 2, 4)
        kw = dict(dt=0.01, T=T, indicators=ALL, gali_kmax=2, n_lyap=4, escape_r2=4.0)
        g = run_gpu(env, P.henon_heiles(), x0, mask, w0, **kw)
        o = O.integrate(O.henon_heiles(), x0, O.Run(**kw), w0=w0, mask=mask, threads=8)
        act = mask == 1
        assert np.array_equal(g["status"], o["status"])
        ok = act & (o["status"] == 0)
        say("  max lambda_1", np.max(o["lyap"][ok, 0]),
            "sali", log_err(g["sali_min"][ok], o["sali_min"][ok]),
            "gali", log_err(g["gali"][ok, 0], o["gali"][ok, 0], floor=1e-8),
            "lyap", np.max(np.abs(g["lyap"][ok] - o["lyap"][ok])))
        assert log_err(g["sali_min"][ok], o["sali_min"][ok]) < 1e-6
        assert log_err(g["sali_final"][ok], o["sali_final"][ok]) < 1e-6
        assert log_err(g["gali"][ok, 0], o["gali"][ok, 0], floor=1e-8) < 1e-6
        assert np.max(np.abs(g["lyap"][ok] - o["lyap"][ok])) < 1e-6
        assert np.max(np.abs(g["ld"][ok] / o["ld"][ok] - 1)) < 1e-9
        assert np.max(np.abs(g["energy_err"][ok] - o["energy_err"][ok])) < 1e-12
        assert np.max(np.abs(g["ln_growth"][ok] - o["ln_growth"][ok])) < 1e-6
        assert np.max(np.abs(g["lyap"][ok].sum(axis=1))) < 1e-10
        assert np.max(state_err(g["x_final"][ok], o["x_final"][ok])) < 1e-7


@pytest.mark.parametrize("K,T", [(1, 1.0), (7, 3.05), (10, 2.0), (25, 5.0)])
def test_hh_checkpoint_periods_and_ragged_tail(env, K, T):
    torch, P, O = env
    say(f"case: HH K={K} T={T}")
    rng = np.random.default_rng(K)
    n = 333  # not a multiple of the block or the wavefront
    x0, mask = O.hh_points(0.125, rng.uniform(-0.4, 0.7, n), rng.uniform(-0.45, 0.45, n))
    w0 = S.deviation_vectors(3, n, 2, 4)
    kw = dict(dt=0.01, T=T, indicators=ALL, gali_kmax=2, n_lyap=4, renorm_every=K)
    g = run_gpu(env, P.henon_heiles(), x0, mask, w0, **kw)
    o = O.integrate(O.henon_heiles(), x0, O.Run(dt=0.01, T=T, indicators=ALL, gali_kmax=2,
                                                n_lyap=4, K=K), w0=w0, mask=mask)
    act = mask == 1
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(g["t_end"][act], o["t_end"][act])
    assert np.max(np.abs(g["lyap"][act] - o["lyap"][act])) < 1e-9
    assert np.max(state_err(g["x_final"][act], o["x_final"][act])) < 1e-11
    assert np.max(np.abs(g["ld"][act] / o["ld"][act] - 1)) < 1e-11


def test_status_codes_and_early_exit(env):
    torch, P, O = env
    say("case: status codes")

    def hh(E, y, py):
        r = 2 * E - py * py - y * y + 2 * y**3 / 3
        return [0.0, y, np.sqrt(r), py]

    x0 = np.array([hh(0.125, 0.1, 0.0), [np.nan, 0, 0, 0], hh(0.2, 0.1, 0.0),
                   hh(0.125, 0.1, 0.0), hh(0.125, -0.25, 0.0), [np.inf, 1, 0, 0]])
    mask = np.array([1, 1, 1, 0, 1, 1], np.uint8)
    w0 = S.deviation_vectors(2, len(x0), 2, 4)
    kw = dict(dt=0.01, T=2000.0, indicators=O.IND_SALI | O.IND_LD | O.IND_LYAP, n_lyap=4,
              escape_r2=4.0, early_exit=True)
    g = run_gpu(env, P.henon_heiles(), x0, mask, w0, **kw)
    o = O.integrate(O.henon_heiles(), x0, O.Run(**kw), w0=w0, mask=mask)
    say("  status", g["status"], o["status"], "t_end", g["t_end"], o["t_end"])
    assert list(g["status"]) == [0, 3, 2, 1, 4, 3]
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(g["label"], o["label"])
    assert g["t_end"][2] == o["t_end"][2] and g["t_end"][4] == o["t_end"][4]
    assert np.isnan(g["ld"][1]) and np.isnan(g["lyap"][3]).all()


def test_resume_bitwise_and_launch_split_invariance(env):
    torch, P, O = env
    say("case: resume")
    x0, mask = O.hh_grid(0.125, 16, 16)
    w0 = S.deviation_vectors(5, len(x0), 2, 4)
    dev = torch.device("cuda:0")
    kw = dict(dt=0.01, T=50.0, indicators=ALL, gali_kmax=2, n_lyap=4)
    ref = run_gpu(env, P.henon_heiles(), x0, mask, w0, **kw)
    e = P.Ensemble(P.henon_heiles(), torch.as_tensor(x0, device=dev),
                   mask=torch.as_tensor(mask, device=dev), w0=torch.as_tensor(w0, device=dev),
                   steps_per_launch=130, **kw)
    for s in (1000, 2370, 5000):
        e.advance(s)
    r = {k: v.cpu().numpy() for k, v in e.results().items()}
    e.close()
    for k in ref:
        assert np.array_equal(ref[k], r[k], equal_nan=True), k


@pytest.mark.parametrize("block", [64, 128, 256])
def test_block_sizes_agree(env, block):
    torch, P, O = env
    say(f"case: block {block}")
    x0, mask = O.hh_grid(1 / 6, 20, 20)
    w0 = S.deviation_vectors(9, len(x0), 2, 4)
    kw = dict(dt=0.01, T=10.0, indicators=ALL, gali_kmax=2, n_lyap=4)
    a = run_gpu(env, P.henon_heiles(), x0, mask, w0, block_size=block, **kw)
    b = run_gpu(env, P.henon_heiles(), x0, mask, w0, block_size=256, **kw)
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True)


def test_library_generated_deviation_vectors(env):
    torch, P, O = env
    say("case: seeded vectors")
    x0, mask = O.hh_grid(0.125, 12, 12)
    kw = dict(dt=0.01, T=20.0, indicators=O.IND_SALI | O.IND_GALI, gali_kmax=3)
    a = run_gpu(env, P.henon_heiles(), x0, mask, None, seed=77, **kw)
    w0 = S.deviation_vectors(77, len(x0), 3, 4)
    b = run_gpu(env, P.henon_heiles(), x0, mask, w0, **kw)
    act = mask == 1
    assert log_err(a["sali_min"][act], b["sali_min"][act]) < 1e-10
    assert np.max(np.abs(a["ln_growth"][act] - b["ln_growth"][act])) < 1e-10


@pytest.mark.parametrize("N", [1, 2, 3])
def test_quartic_parity(env, N):
    torch, P, O = env
    say(f"case: quartic N={N}")
    so, sg = O.quartic(N, 0.1), P.quartic(N, 0.1)
    draws = S.quartic_draws(31, 200, N)
    x0 = O.quartic_ic(so, draws)
    xg = P.ic_quartic(sg, draws)
    assert np.max(np.abs(xg - x0)) < 1e-14
    w0 = S.deviation_vectors(4, len(x0), 2, 2 * N)
    kw = dict(dt=0.01, T=50.0, indicators=ALL, gali_kmax=2, n_lyap=2 * N)
    g = run_gpu(env, sg, x0, None, w0, **kw)
    o = O.integrate(so, x0, O.Run(**kw), w0=w0)
    assert np.max(state_err(g["x_final"], o["x_final"])) < 1e-9
    assert np.max(np.abs(g["lyap"] - o["lyap"])) < 1e-6
    assert log_err(g["sali_min"], o["sali_min"]) < 1e-6
    assert np.max(np.abs(g["ld"] / o["ld"] - 1)) < 1e-9


def test_harmonic_parity_and_bounds(env):
    torch, P, O = env
    say("case: harmonic")
    w = [1.0, np.sqrt(2.0), 0.5]
    rng = np.random.default_rng(1)
    x0 = rng.uniform(-1, 1, (100, 6))
    w0 = S.deviation_vectors(8, 100, 4, 6)
    kw = dict(dt=0.01, T=100.0, indicators=ALL, gali_kmax=4, n_lyap=6)
    g = run_gpu(env, P.harmonic(w), x0, None, w0, **kw)
    o = O.integrate(O.harmonic(w), x0, O.Run(**kw), w0=w0)
    assert np.max(state_err(g["x_final"], o["x_final"])) < 1e-11
    assert np.max(np.abs(g["lyap"] - o["lyap"])) < 1e-9
    assert np.max(np.abs(g["lyap"])) <= np.log(2.0) / 100.0 + 1e-9
    for k in range(3):
        assert log_err(g["gali"][:, k], o["gali"][:, k]) < 1e-9


def test_general_ld_exponent(env):
    torch, P, O = env
    say("case: ld p=0.3")
    x0, mask = O.hh_grid(0.125, 10, 10)
    kw = dict(dt=0.01, T=20.0, indicators=O.IND_LD, ld_p=0.3)
    g = run_gpu(env, P.henon_heiles(), x0, mask, None, **kw)
    o = O.integrate(O.henon_heiles(), x0, O.Run(**kw), mask=mask)
    act = mask == 1
    assert np.max(np.abs(g["ld"][act] / o["ld"][act] - 1)) < 1e-9


def test_convenience_entry_points(env):
    torch, P, O = env
    say("case: convenience calls")
    x0, mask = O.hh_grid(0.125, 8, 8)
    x0 = x0[mask == 1]
    smin, lab = P.sali(P.henon_heiles(), x0, 0.01, 20.0, 5)
    w0 = S.deviation_vectors(5, len(x0), 2, 4)
    o = O.integrate(O.henon_heiles(), x0, O.Run(dt=0.01, T=20.0, indicators=O.IND_SALI), w0=w0)
    assert log_err(smin, o["sali_min"]) < 1e-9 and np.array_equal(lab, o["label"])
    ly = P.lyap_spectrum(P.henon_heiles(), x0, 0.01, 20.0, 4)
    ol = O.integrate(O.henon_heiles(), x0, O.Run(dt=0.01, T=20.0, indicators=O.IND_LYAP,
                                                  n_lyap=4))
    assert np.max(np.abs(ly - ol["lyap"])) < 1e-9
    ldv = P.ld(P.henon_heiles(), x0, 0.01, 20.0)
    assert np.max(np.abs(ldv / O.integrate(O.henon_heiles(), x0, O.Run(
        dt=0.01, T=20.0, indicators=O.IND_LD))["ld"] - 1)) < 1e-11
    ga = P.gali(P.henon_heiles(), x0, 0.01, 20.0, 4, 5)
    og = O.integrate(O.henon_heiles(), x0, O.Run(dt=0.01, T=20.0, indicators=O.IND_GALI,
                                                  gali_kmax=4),
                     w0=S.deviation_vectors(5, len(x0), 4, 4))
    for k in range(3):
        assert log_err(ga[:, k], og["gali"][:, k], floor=1e-8) < 1e-8


def test_section_grid_kernel(env):
    torch, P, O = env
    for E, cnt in ((0.125, 850874), (1 / 6, 992552)):
        say(f"case: grid E={E}")
        xg, mg = P.grid_hh_section(E, 1024, 1024, device="cuda:0")
        xg, mg = xg.cpu().numpy(), mg.cpu().numpy()
        xo, mo = O.hh_grid(E, 1024, 1024)
        assert np.array_equal(mg, mo) and int(mg.sum()) == cnt
        assert np.array_equal(xg[:, [0, 1, 3]], xo[:, [0, 1, 3]])
        # p_x = sqrt(r): r agrees to rounding, sqrt amplifies that near r = 0
        assert np.max(np.abs(xg[:, 2] ** 2 - xo[:, 2] ** 2)) < 1e-15
    y, py = S.section_points(3, 1000)
    xg, mg = P.hh_section_points(0.125, y, py)
    xo, mo = O.hh_points(0.125, y, py)
    assert np.array_equal(mg, mo) and np.max(np.abs(xg**2 - xo**2)) < 1e-15
