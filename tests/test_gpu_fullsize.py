"""Full-size parity of the benchmark workload in the launch configuration
bench.py times: Henon-Heiles 1024x1024 section grids at E = 0.125 and
E = 1/6 (850,874 + 992,552 orbits) to T = 1e4 with SALI, GALI_2, four
Lyapunov exponents, LD and the energy error in one pass, library-generated
deviation vectors (seed 1002), 25,000 steps per launch.

Checked on every orbit: exact mask counts and properties that hold at any
size (the Lyapunov spectrum sums to zero, SALI/sqrt(2) <= GALI_2 <= SALI,
bounded energy error).  Checked against the oracle, orbit by orbit, on a
strided sample of 1024 orbits: labels (>= 99.9 % agree) and, on orbits
both call regular, the LD (relative 1e-7 at most, 1e-10 in the median),
the energy error (absolute 1e-12) and the final state: relative 1e-5 at
most and 1e-8 in the median.
On a torus, rounding moves the action by a random walk, so the phase
error grows faster than linearly; near-separatrix tori (large d omega/dI)
reach 1e-6 at T = 1e4 while the median orbit stays near 1e-10 (the strict
1e-9 state check is made at T = 200).
"""
import os
import sys

import numpy as np
import pytest

import seeded_inputs as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_benchmark_workload_full_size():
    import torch
    import paper_2507_00622_amd as P
    from oracle import oracle as O

    dev = torch.device("cuda:0")
    say("case: full-size HH 2x1024^2, T=1e4, 25000 steps per launch")
    xs, ms = [], []
    for E in (0.125, 1.0 / 6.0):
        x, m = P.grid_hh_section(E, 1024, 1024, device=dev)
        xs.append(x)
        ms.append(m)
    x0, mask = torch.cat(xs), torch.cat(ms)
    ind = 31
    kw = dict(dt=0.01, T=1e4, indicators=ind, gali_kmax=2, n_lyap=4, renorm_every=10,
              seed=1002, escape_r2=4.0, steps_per_launch=25000)
    with P.Ensemble(P.henon_heiles(), x0, mask=mask, **kw) as e:
        n_total, _, n_active = e.info()
        assert n_active == 850874 + 992552
        for s in range(25000, n_total + 1, 25000):
            e.advance(s)
        g = {k: v.cpu().numpy() for k, v in e.results().items()}
    x0h, maskh = x0.cpu().numpy(), mask.cpu().numpy()
    act = maskh == 1
    ok = act & (g["status"] == 0)
    say("  statuses:", {int(k): int(v) for k, v in zip(*np.unique(g["status"], return_counts=True))})
    # properties on every orbit
    assert np.array_equal(g["status"] == 1, ~act)
    assert np.max(np.abs(g["lyap"][ok].sum(axis=1))) < 1e-9
    # GALI_2 comes from a QR of the two unit vectors: near alignment its R_22
    # carries an absolute rounding error ~1e-16, which SALI (|w1 - w2|) does not
    gal, sal = g["gali"][ok, 0], g["sali_final"][ok]
    assert np.all(sal / np.sqrt(2) <= gal * (1 + 1e-9) + 1e-14)
    assert np.all(gal <= sal * (1 + 1e-9) + 1e-14)
    e125 = ok.copy()
    e125[len(e125) // 2:] = False
    say("  max energy error E=0.125:", np.max(g["energy_err"][e125]))
    assert np.max(g["energy_err"][e125]) < 1e-8
    # strided sample against the oracle
    idx = np.flatnonzero(act)[np.linspace(0, act.sum() - 1, 1024).astype(int)]
    w0 = S.deviation_vectors(1002, len(x0h), 2, 4)[idx]
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    say(f"  oracle on {len(idx)} sampled orbits with {threads} threads")
    o = O.integrate(O.henon_heiles(), x0h[idx], O.Run(dt=0.01, T=1e4, indicators=ind,
                                                       gali_kmax=2, n_lyap=4, escape_r2=4.0),
                    w0=w0, threads=threads)
    lg, lo = g["label"][idx], o["label"]
    agree = np.mean(lg == lo)
    say("  label agreement on the sample:", agree, "mismatches:", int(np.sum(lg != lo)))
    assert agree >= 0.999
    reg = (lg == 0) & (lo == 0)
    assert reg.sum() > 100
    xe = np.max(np.abs(g["x_final"][idx][reg] - o["x_final"][reg]), axis=1)
    xe /= np.maximum(1.0, np.max(np.abs(o["x_final"][reg]), axis=1))
    lde = np.abs(g["ld"][idx][reg] / o["ld"][reg] - 1)
    say("  regular orbits:", int(reg.sum()), "max state err", xe.max(), "max LD rel err",
        lde.max())
    assert xe.max() < 1e-5
    assert np.median(xe) < 1e-8
    assert lde.max() < 1e-7
    assert np.median(lde) < 1e-10
    assert np.max(np.abs(g["energy_err"][idx][reg] - o["energy_err"][reg])) < 1e-12
