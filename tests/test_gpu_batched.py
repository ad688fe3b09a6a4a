"""The persistent batched form (one launch for Henon-Heiles, quartic and FPU
orbits, early exit, slot refill, autotuned launch, hipGraph replay) against
the plain form, through the C ABI.

The batched kernel runs the same per-orbit code as the plain kernels, so an
orbit's results do not depend on the slot or the launch that integrated it:
the batched outputs must equal the plain outputs bit for bit, whatever the
steps per launch, the block size or the autotuner's choices.  Labels are
also checked against the oracle on a sample.
"""
import os

import numpy as np
import pytest

import seeded_inputs as S

pytestmark = pytest.mark.gpu

IND = 1 | 8 | 16  # SALI, LD, energy


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2507_00622_amd as P
    from oracle import oracle as O
    return torch, P, O


def make_items(P, O, n_hh, n_q, n_f16, n_f8, T_hh, T_f, seed=5):
    y, py = S.section_points(seed, int(n_hh * 1.4) + 16)
    xh, mh = O.hh_points(0.125, y, py)
    xh = xh[mh == 1][:n_hh]
    xq = O.quartic_ic(O.quartic(3, 0.1), S.quartic_draws(seed + 1, n_q))
    items = [dict(sys=P.henon_heiles(), x0=xh, dt=0.01, T=T_hh),
             dict(sys=P.quartic(3, 0.1), x0=xq, dt=0.01, T=T_hh)]
    if n_f16:
        items.append(dict(sys=P.fput(16), x0=O.fput_ic(O.fput(16), S.fput_mode_draws(seed + 2, n_f16)),
                          dt=0.02, T=T_f))
    if n_f8:
        items.append(dict(sys=P.fput(8), x0=O.fput_ic(O.fput(8), S.fput_mode_draws(seed + 3, n_f8)),
                          dt=0.02, T=T_f))
    return items


def plain(P, items, seed, **kw):
    outs = []
    for i, it in enumerate(items):
        outs.append(P.integrate_ensemble(it["sys"], it["x0"], mask=it.get("mask"), dt=it["dt"],
                                         T=it["T"], indicators=IND, seed=seed + i, **kw))
    return outs


def assert_same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("budget,block", [(0, 0), (50, 64), (230, 128), (1000, 256)])
def test_batched_equals_plain(env, budget, block):
    torch, P, O = env
    say(f"case: batched vs plain, steps/launch {budget} block {block}")
    items = make_items(P, O, 700, 300, 90, 45, T_hh=100.0, T_f=60.0)
    # a loose threshold so that early exits occur within this short time
    kw = dict(early_exit=True, sali_threshold=3e-2, escape_r2=4.0)
    outs, stats = P.integrate_batched(items, indicators=IND, seed=77, steps_per_launch=budget,
                                      block_size=block, **kw)
    say("  stats:", {k: stats[k] for k in ("threads_per_block", "blocks", "launches",
                                            "steps_per_launch", "orbit_steps")})
    ref = plain(P, items, 77, **kw)
    for a, b in zip(outs, ref):
        assert_same(a, b)
    exited = sum(int(np.sum(o["status"] == 4)) for o in outs)
    say("  exited orbits:", exited)
    assert exited > 20
    for o, it, nst in zip(outs, items, stats["orbit_steps"]):
        assert nst == int(np.sum(np.round(o["t_end"] / it["dt"])))


def test_batched_device_pointers_and_labels_vs_oracle(env):
    torch, P, O = env
    say("case: batched on device tensors, labels vs oracle")
    items = make_items(P, O, 400, 100, 40, 0, T_hh=200.0, T_f=200.0, seed=11)
    dev = torch.device("cuda:0")
    ditems = [dict(it, x0=torch.as_tensor(it["x0"], device=dev)) for it in items]
    outs, stats = P.integrate_batched(ditems, indicators=IND, seed=3, early_exit=True,
                                      sali_threshold=1e-6)
    torch.cuda.synchronize()
    outs = [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]
    sysmap = [O.henon_heiles(), O.quartic(3, 0.1), O.fput(16)]
    for i, (it, o) in enumerate(zip(items, outs)):
        n = len(it["x0"])
        w0 = S.deviation_vectors(3 + i, n, 2, 2 * sysmap[i].ndof)
        r = O.integrate(sysmap[i], it["x0"], O.Run(dt=it["dt"], T=it["T"], indicators=IND,
                                                   early_exit=True, sali_threshold=1e-6),
                        w0=w0, threads=8)
        agree = np.mean(r["label"] == o["label"])
        say(f"  item {i}: label agreement {agree:.4f}, exited {int(np.sum(o['status'] == 4))}")
        assert agree >= 0.99


def test_autotune_cache_file(env, tmp_path):
    torch, P, O = env
    say("case: autotune cache")
    path = str(tmp_path / "tune.txt")
    os.environ["CHX_AUTOTUNE_CACHE"] = path
    try:
        items = make_items(P, O, 200, 50, 20, 0, T_hh=2.0, T_f=2.0, seed=13)
        # indicators no other test uses, so the first call has to probe
        _, s1 = P.integrate_batched(items, indicators=1, seed=1)
        _, s2 = P.integrate_batched(items, indicators=1, seed=1)
    finally:
        del os.environ["CHX_AUTOTUNE_CACHE"]
    assert s1["from_cache"] == 0 and s2["from_cache"] == 1
    assert s1["threads_per_block"] == s2["threads_per_block"]
    lines = open(path).read().split("\n")
    assert any(l.startswith("gfx950/") and "/ind1 " in l for l in lines)


def test_full_orbit_counts_short_time(env):
    torch, P, O = env
    say("case: batched at full orbit counts (2^20 HH, 2^18 quartic, 2^16 FPU-16), T = 400")
    dev = torch.device("cuda:0")
    y, py = S.section_points(4001, 1400000)
    x, m = P.hh_section_points(0.125, torch.as_tensor(y, device=dev), torch.as_tensor(py, device=dev))
    xh = x[m == 1][: 1 << 20]
    assert xh.shape[0] == 1 << 20
    xq = P.ic_quartic(P.quartic(3, 0.1), torch.as_tensor(S.quartic_draws(4002, 1 << 18), device=dev))
    xf = P.ic_fput_modes(P.fput(16), torch.as_tensor(S.fput_mode_draws(4003, 1 << 16), device=dev))
    items = [dict(sys=P.henon_heiles(), x0=xh, dt=0.01, T=400.0),
             dict(sys=P.quartic(3, 0.1), x0=xq, dt=0.01, T=400.0),
             dict(sys=P.fput(16), x0=xf, dt=0.02, T=400.0)]
    kw = dict(indicators=IND, seed=4000, early_exit=True)
    outs, stats = P.integrate_batched(items, outputs=("status", "label", "sali_min", "t_end"), **kw)
    say("  stats:", stats)
    ref = []
    for i, it in enumerate(items):
        ref.append(P.integrate_ensemble(it["sys"], it["x0"], dt=it["dt"], T=it["T"],
                                        outputs=("status", "label", "sali_min", "t_end"),
                                        indicators=IND, seed=4000 + i, early_exit=True))
    torch.cuda.synchronize()
    for a, b in zip(outs, ref):
        for k in a:
            x, y = a[k], b[k]
            if x.is_floating_point():
                x, y = x.nan_to_num(-7.0), y.nan_to_num(-7.0)
            assert torch.equal(x, y), k
