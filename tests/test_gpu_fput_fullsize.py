"""Full-size parity of the FPU workload in the launch configuration bench.py
times: 65,536 FPU-beta chains per N (N = 8 and 16), 3N deviation vectors
(2N Lyapunov vectors by Gram-Schmidt every 10 steps + N GALI vectors from
the library's generator, seed 1003), SALI + GALI + Lyapunov + energy,
dt = 0.02, 10,000 steps in one launch (T = 200).

Checked on every orbit: status, the Lyapunov spectrum summing to zero (the
tangent map is symplectic), GALI_k in [0, 1] and non-increasing in k,
energy error below 1e-3 of the energy.  Checked against the oracle, orbit
by orbit, on 16 strided orbits per N: exponents (absolute 1e-6), GALI
(|log10| 1e-6 where both are >= 1e-8), final state (relative 1e-9), energy
error (1e-12 relative to the energy).
"""
import os

import numpy as np
import pytest

import seeded_inputs as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("N", [8, 16])
def test_fput_workload_full_size(N):
    import torch
    import paper_2507_00622_amd as P
    from oracle import oracle as O

    dev = torch.device("cuda:0")
    n = 65536
    say(f"case: full-size FPU N={N}, {n} orbits, 3N vectors, T=200, one launch")
    draws = S.fput_mode_draws(1003 + N, n)
    x0 = P.ic_fput_modes(P.fput(N), torch.as_tensor(draws, device=dev))
    ind = 1 | 2 | 4 | 16
    kw = dict(dt=0.02, T=200.0, indicators=ind, gali_kmax=N, n_lyap=2 * N, renorm_every=10,
              seed=1003, steps_per_launch=10000)
    out = P.integrate_ensemble(P.fput(N), x0, **kw)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    x0h = x0.cpu().numpy()
    assert np.all(g["status"] == 0)
    lsum = np.abs(g["lyap"].sum(axis=1))
    say(f"  max |sum of exponents| {lsum.max():.3g}")
    assert lsum.max() < 1e-9
    gal = g["gali"]
    assert np.all((gal >= 0) & (gal <= 1 + 1e-12))
    assert np.all(gal[:, 1:] <= gal[:, :-1] * (1 + 1e-12) + 1e-300)
    E = np.array([O.hamiltonian(O.fput(N), x) for x in x0h])
    rel = g["energy_err"] / E
    say(f"  max relative energy error {rel.max():.3g} (energies {E.min():.3g}..{E.max():.3g})")
    assert rel.max() < 1e-3
    # strided sample against the oracle
    idx = np.linspace(0, n - 1, 16).astype(int)
    w0 = np.concatenate([S.deviation_vectors(1003, 1, N, 2 * N, first_ic=int(i)) for i in idx])
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    o = O.integrate(O.fput(N), x0h[idx], O.Run(dt=0.02, T=200.0, indicators=ind, gali_kmax=N,
                                               n_lyap=2 * N, K=10), w0=w0, threads=threads)
    # the initial states themselves come from the library's generator; the
    # oracle's generator must give the same states
    xo = O.fput_ic(O.fput(N), draws[idx])
    assert np.max(np.abs(xo - x0h[idx])) < 1e-13
    le = np.max(np.abs(g["lyap"][idx] - o["lyap"]))
    ok = (g["gali"][idx] >= 1e-8) & (o["gali"] >= 1e-8)
    ge = np.max(np.abs(np.log10(g["gali"][idx][ok]) - np.log10(o["gali"][ok])))
    se = np.max(np.abs(g["x_final"][idx] - o["x_final"]), axis=1)
    se /= np.maximum(1.0, np.max(np.abs(o["x_final"]), axis=1))
    Es = np.array([O.hamiltonian(O.fput(N), x) for x in x0h[idx]])
    ee = np.max(np.abs(g["energy_err"][idx] - o["energy_err"]) / np.maximum(1.0, Es))
    say(f"  sample: lyap {le:.3g} gali {ge:.3g} state {se.max():.3g} energy {ee:.3g}")
    assert le < 1e-6
    assert ge < 1e-6
    assert se.max() < 1e-9
    assert ee < 1e-12
