"""The learned gate and ensemble subsets on the GPU, through the C ABI.

  - chx_ensemble_subset: resuming a subset gives every kept orbit exactly
    (bit for bit) the results of the full run, for every indicator;
  - perceptron forward pass and gradient against the FP64 oracle
    (oracle/mlp.py) on the same BF16-rounded operands: |p| within 2e-3,
    gradient normwise relative 2e-2 per parameter block;
  - one AdamW step against the oracle update applied to the device gradient;
  - the gradient after several AdamW steps against the oracle's at the
    trained parameters (the steps keep the weights' BF16 copies current);
  - training learns a separable rule, and is reproducible bit for bit;
  - chx_gate_classify: with a gate that is never confident every label is
    the plain integrator's (bit for bit); with a mixed gate, resumed orbits
    carry the plain label and gated ones the gate's label.
"""
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
    from oracle import mlp as M
    from oracle import oracle as O
    return torch, P, M, O


def assert_same(a, b, rows=None):
    for k in a:
        x = b[k] if rows is None else b[k][rows]
        assert np.array_equal(a[k], x, equal_nan=True), k


@pytest.mark.parametrize("case", ["hh_all", "quartic_lyap", "fput16_crow", "fput8_row"])
def test_subset_resume_is_bitwise(env, case):
    torch, P, M, O = env
    say(f"case: subset resume {case}")
    if case == "hh_all":
        x0, mask = O.hh_grid(0.125, 24, 24)
        sys_, kw = P.henon_heiles(), dict(indicators=1 | 2 | 4 | 8 | 16, gali_kmax=3, dt=0.01,
                                          T=60.0)
    elif case == "quartic_lyap":
        x0 = O.quartic_ic(O.quartic(3, 0.1), S.quartic_draws(21, 300))
        mask = None
        sys_, kw = P.quartic(3, 0.1), dict(indicators=1 | 4 | 8, dt=0.01, T=60.0)
    elif case == "fput16_crow":
        x0 = O.fput_ic(O.fput(16), S.fput_mode_draws(22, 200))
        mask = None
        sys_, kw = P.fput(16), dict(indicators=1 | 8 | 16, dt=0.02, T=60.0)
    else:
        x0 = O.fput_ic(O.fput(8), S.fput_mode_draws(23, 150))
        mask = None
        sys_, kw = P.fput(8), dict(indicators=1 | 2 | 4 | 16, gali_kmax=4, dt=0.02, T=60.0)
    n = len(x0)
    keep = (np.arange(n) * 7919 % 5 < 2).astype(np.uint8)
    with P.Ensemble(sys_, x0, mask=mask, seed=9, **kw) as e:
        full_total = e.n_total
        mid = (full_total // 2) // 10 * 10
        e.advance(mid)
        sub = e.subset(keep)
        e.advance()
        ref = e.results()
    with sub:
        ns = sub.info()[2]
        sub.advance()
        got = sub.results()
    active = np.ones(n, bool) if mask is None else mask.astype(bool)
    rows = np.flatnonzero((keep == 1) & active)
    assert ns == len(rows) and ns > 0
    say(f"  kept {ns} of {n}")
    assert_same(got, ref, rows)


def random_params(M, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = M.init_params(rng) * scale
    p[M.B1:M.W2] = rng.normal(0, 0.1, M.NH)
    p[M.B2:M.W3] = rng.normal(0, 0.1, M.NH)
    p[M.B3:M.B3 + 2] = rng.normal(0, 0.1, 2)
    return p.astype(np.float32)


def random_features(seed, n):
    rng = np.random.default_rng(seed)
    F = rng.normal(size=(n, 6)) * np.array([0.2, 0.15, 0.3, 0.05, 0.02, 0.02]) \
        + np.array([0.1, 0.0, 0.3, 0.4, 0.01, 0.01])
    return F.astype(np.float32)


def test_forward_matches_oracle(env):
    torch, P, M, O = env
    say("case: gate forward vs oracle")
    g = P.Gate(1)
    p = random_params(M, 2)
    F = random_features(3, 5000)
    mu, istd = M.zscore_stats(F.astype(np.float64))
    g.set(p, mu.astype(np.float32), istd.astype(np.float32))
    pg, cg = g.infer(F)
    _, mu32, is32 = g.get()
    X = M.inputs(F, mu32, is32, rounding=True)
    pr = M.probabilities(M.forward(p.astype(np.float64), X, rounding=True)[4])
    d = np.abs(pg - pr)
    say(f"  max |dp| {d.max():.3e}, median {np.median(d):.3e}")
    assert d.max() <= 2e-3 and np.median(d) <= 1e-5
    assert np.allclose(cg, np.maximum(pg, 1 - pg), rtol=0, atol=0)
    # device tensors give the same bits
    pd, _ = g.infer(torch.as_tensor(F, device="cuda:0"))
    torch.cuda.synchronize()
    assert np.array_equal(pd.cpu().numpy(), pg)
    g.close()


# 4104 rows: a ragged batch (not a multiple of 16; the products' K is not a
# multiple of their 32-deep chunks) split over K; 40 rows: fewer rows than
# one 64-row tile
@pytest.mark.parametrize("n", [4096 + 8, 40])
def test_gradient_matches_oracle(env, n):
    torch, P, M, O = env
    say(f"case: gate gradient vs oracle, {n} rows")
    g = P.Gate(1)
    p = random_params(M, 4, scale=0.7)
    F = random_features(5, n)
    y = (np.random.default_rng(6).random(len(F)) < 0.4).astype(np.int8)
    y[::97] = -1  # ignored rows
    mu, istd = M.zscore_stats(F.astype(np.float64))
    g.set(p, mu.astype(np.float32), istd.astype(np.float32))
    loss, gg = g.grad(F, y)
    _, mu32, is32 = g.get()
    X = M.inputs(F, mu32, is32, rounding=True)
    lr, gr = M.loss_and_grad(p.astype(np.float64), X, y, rounding=True)
    say(f"  loss gpu {loss:.7f} oracle {lr:.7f}")
    assert abs(loss - lr) <= 1e-4 * max(1.0, abs(lr))
    for name, a, b in (("W1", M.W1, M.B1), ("b1", M.B1, M.W2), ("W2", M.W2, M.B2),
                       ("b2", M.B2, M.W3), ("W3", M.W3, M.B3), ("b3", M.B3, M.NPARAM)):
        rel = np.linalg.norm(gg[a:b] - gr[a:b]) / max(np.linalg.norm(gr[a:b]), 1e-30)
        say(f"  {name}: normwise rel {rel:.3e}")
        assert rel <= 2e-2, name
    assert np.all(gg[M.mask() == 0] == 0.0)
    g.close()


def test_adamw_step_matches_oracle(env):
    torch, P, M, O = env
    say("case: one AdamW step vs oracle")
    g = P.Gate(1)
    p = random_params(M, 7, scale=0.5)
    F = random_features(8, 2048)
    y = (np.random.default_rng(9).random(len(F)) < 0.5).astype(np.int8)
    mu, istd = M.zscore_stats(F.astype(np.float64))
    g.set(p, mu.astype(np.float32), istd.astype(np.float32))
    _, gg = g.grad(F, y)
    lr, wd = 1e-3, 0.01
    g.train(F, y, epochs=1, batch=2048, lr=lr, weight_decay=wd)
    p1 = g.get()[0]
    pr, _, _ = M.adamw(p.astype(np.float64), gg.astype(np.float64), np.zeros(M.NPARAM),
                       np.zeros(M.NPARAM), 1, lr=lr, wd=wd, keep=M.mask())
    d = np.abs(p1 - pr)
    # Where |g| is near eps the step g / (|g| + eps) is sensitive to the
    # float32 rounding of g, which differs between the two passes (rows are
    # summed in another order); elsewhere the step is fixed to float32 rounding.
    firm = np.abs(gg) >= 1e-6
    say(f"  max |dp| {d[firm].max():.3e} where |g| >= 1e-6, {d.max():.3e} overall")
    assert d[firm].max() <= 2e-6
    assert d.max() <= 2 * lr * (1.0 + wd * np.abs(p).max())
    assert np.all(p1[M.mask() == 0] == 0.0)
    g.close()


def test_gradient_after_training_steps(env):
    """The training pass reads a transposed BF16 copy of the weights that every
    AdamW step rewrites: a gradient taken after training matches the oracle's
    at the trained parameters."""
    torch, P, M, O = env
    say("case: gate gradient after AdamW steps")
    g = P.Gate(1)
    p = random_params(M, 14, scale=0.7)
    F = random_features(15, 3000)
    y = (np.random.default_rng(16).random(len(F)) < 0.5).astype(np.int8)
    mu, istd = M.zscore_stats(F.astype(np.float64))
    g.set(p, mu.astype(np.float32), istd.astype(np.float32))
    g.train(F, y, epochs=2, batch=512, lr=3e-2, seed=17)  # 12 steps
    p1, mu32, is32 = g.get()
    moved = np.abs(p1 - p).max()
    say(f"  largest parameter change {moved:.3e}")
    assert moved > 1e-2
    n = 1000
    loss, gg = g.grad(F[:n], y[:n])
    X = M.inputs(F[:n], mu32, is32, rounding=True)
    lr, gr = M.loss_and_grad(p1.astype(np.float64), X, y[:n], rounding=True)
    say(f"  loss gpu {loss:.7f} oracle {lr:.7f}")
    assert abs(loss - lr) <= 1e-4 * max(1.0, abs(lr))
    for name, a, b in (("W1", M.W1, M.B1), ("b1", M.B1, M.W2), ("W2", M.W2, M.B2),
                       ("b2", M.B2, M.W3), ("W3", M.W3, M.B3), ("b3", M.B3, M.NPARAM)):
        rel = np.linalg.norm(gg[a:b] - gr[a:b]) / max(np.linalg.norm(gr[a:b]), 1e-30)
        say(f"  {name}: normwise rel {rel:.3e}")
        assert rel <= 2e-2, name
    g.close()


def test_training_is_reproducible(env):
    """Every sum of the training pass runs in a fixed order (split-K parts,
    bias and loss sums), so two runs from the same state agree bit for bit."""
    torch, P, M, O = env
    say("case: training twice from the same state")
    F = random_features(18, 5000)
    y = (np.random.default_rng(19).random(len(F)) < 0.5).astype(np.int8)
    out = []
    for _ in range(2):
        g = P.Gate(20)
        losses = g.train(F, y, epochs=2, batch=1024, lr=1e-2, seed=21)
        out.append((np.asarray(losses), g.get()[0]))
        g.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_training_learns_a_rule(env):
    torch, P, M, O = env
    say("case: training on a separable rule")
    F = random_features(10, 20000)
    Z = (F - F.mean(0)) / F.std(0)
    y = (Z[:, 0] + 0.8 * Z[:, 3] - 0.5 * Z[:, 4] > 0.1).astype(np.int8)
    g = P.Gate(11)
    losses = g.train(F[:16384], y[:16384], epochs=12, batch=512, lr=2e-3, seed=12)
    say("  epoch losses", np.round(losses, 4))
    assert losses[-1] < 0.5 * losses[0]
    pt, _ = g.infer(F[16384:])
    acc = np.mean((pt >= 0.5) == (y[16384:] == 1))
    say(f"  held-out accuracy {acc:.4f}")
    assert acc >= 0.97
    g.close()


def test_features_match_definition(env):
    torch, P, M, O = env
    say("case: gate features")
    rng = np.random.default_rng(13)
    x0 = rng.normal(size=(333, 4))
    ld = rng.random(333) * 50
    lg = rng.normal(size=(333, 2)) * 10
    f = P.gate_features(x0, ld, lg, 200.0)
    assert np.array_equal(f, M.features(x0, ld, lg, 200.0).astype(np.float32))


def plain_labels(P, x0, mask, **kw):
    return P.integrate_ensemble(P.henon_heiles(), x0, mask=mask, outputs=("label", "status"),
                                **kw)


def test_classify_never_confident_equals_plain(env):
    torch, P, M, O = env
    say("case: classify with an unconfident gate")
    x0, mask = O.hh_grid(0.125, 40, 40)
    kw = dict(dt=0.01, T=1000.0, indicators=1 | 8, early_exit=True, sali_threshold=1e-3, seed=31)
    g = P.Gate(1)
    p = random_params(M, 14)
    p[M.W3:] = 0.0  # logits (0, 0): p = 0.5, confidence 0.5
    g.set(p)
    out, st = g.classify(P.henon_heiles(), x0, mask, t_gate=200.0, conf_min=0.98, **kw)
    ref = plain_labels(P, x0, mask, **kw)
    say("  stats", st)
    assert np.array_equal(out["label"], ref["label"])
    src = out["source"]
    assert np.all(src[mask == 0] == 0)
    early = (ref["status"] == 4) & (src == 1)
    assert st["n_early"] == int(np.sum(src == 1)) and st["n_accepted"] == 0
    assert st["n_fallback"] == int(np.sum(src == 3)) > 0
    assert st["n_early"] == int(np.sum(early)) > 0
    g.close()


def test_classify_mixed_gate(env):
    torch, P, M, O = env
    say("case: classify with a mixed gate")
    x0, mask = O.hh_grid(0.125, 40, 40)
    kw = dict(dt=0.01, T=600.0, indicators=1 | 8, seed=33)
    g = P.Gate(1)
    p = random_params(M, 15, scale=1.5)
    g.set(p)
    out, st = g.classify(P.henon_heiles(), x0, mask, t_gate=100.0, conf_min=0.75, **kw)
    say("  stats", st)
    assert st["n_accepted"] > 0 and st["n_fallback"] > 0
    ref = plain_labels(P, x0, mask, **kw)
    src, lab = out["source"], out["label"]
    assert np.array_equal(lab[src == 3], ref["label"][src == 3])
    # gated labels: the gate on features from an ensemble stopped at t_gate
    with P.Ensemble(P.henon_heiles(), x0, mask=mask, **kw) as e:
        e.advance(10000)
        r = e.results(("ld", "ln_growth"))
    f = P.gate_features(x0, r["ld"], r["ln_growth"], 100.0)
    pc, cf = g.infer(f)
    gated = src == 2
    assert np.array_equal(lab[gated], (pc[gated] >= 0.5).astype(np.int8))
    assert np.array_equal(out["confidence"][gated], cf[gated])
    assert np.all(cf[gated] >= 0.75) and np.all(cf[src == 3] < 0.75)
    g.close()


def test_trained_gate_gains_over_plain(env):
    """The workflow end to end at reduced size: labels from the plain
    integrator on 2^18 seeded accessible section points (T = 2000, features
    at t = 200), a gate trained on them by the library's kernels, then a
    fresh 256 x 256 grid classified with the gate and with the plain
    integrator.  The gate must agree with the plain labels on >= 99 % of the
    orbits while integrating to T only the orbits it is unsure of (the
    gain: fewer orbit-steps than the plain run)."""
    torch, P, M, O = env
    say("case: trained gate vs plain (2^18 training orbits, 256^2 test grid, T=2000)")
    dev = torch.device("cuda:0")
    T, dt, tg = 2000.0, 0.01, 200.0
    kw = dict(dt=dt, T=T, indicators=1 | 8, seed=21)
    y, py = S.section_points(2101, 360000)
    x, m = P.hh_section_points(0.125, torch.as_tensor(y, device=dev),
                               torch.as_tensor(py, device=dev))
    xt = x[m == 1][: 1 << 18].contiguous()
    with P.Ensemble(P.henon_heiles(), xt, **kw) as e:
        e.advance(int(round(tg / dt)))
        r = e.results(("ld", "ln_growth"))
        feat = P.gate_features(xt, r["ld"], r["ln_growth"], tg)
        e.advance()
        lab = e.results(("label",))["label"]
    g = P.Gate(22)
    losses = g.train(feat, lab, epochs=6, batch=4096, lr=1e-3, seed=23)
    say("  epoch losses", np.round(losses, 4))
    assert losses[-1] < losses[0]
    xg, mg = P.grid_hh_section(0.125, 256, 256, device=dev)
    out, st = g.classify(P.henon_heiles(), xg, mg, t_gate=tg, conf_min=0.98, **kw)
    ref = P.integrate_ensemble(P.henon_heiles(), xg, mask=mg, outputs=("label",), **kw)
    torch.cuda.synchronize()
    act = (mg == 1).cpu().numpy()
    gl, rl = out["label"].cpu().numpy()[act], ref["label"].cpu().numpy()[act]
    src = out["source"].cpu().numpy()[act]
    agree = np.mean(gl == rl)
    n_total, n_gate = int(round(T / dt)), int(round(tg / dt))
    steps_gate = st["n_active"] * n_gate + st["n_fallback"] * (n_total - n_gate)
    steps_plain = st["n_active"] * n_total
    say(f"  agreement {agree:.4f}, accepted {st['n_accepted']}, fallback {st['n_fallback']}, "
        f"orbit-steps {steps_gate / steps_plain:.3f} of plain")
    assert agree >= 0.99
    assert np.all(gl[src == 3] == rl[src == 3])
    assert steps_gate < 0.6 * steps_plain
    g.close()
