"""Pins of the FP64 gate oracle (oracle/mlp.py) against closed forms, special
cases and finite differences."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def test_gelu_values_and_identity():
    # GELU(u) = u Phi(u): Phi(0) = 1/2, Phi(1) = 0.841344746068542948...
    assert M.gelu(np.array([0.0]))[0] == 0.0
    assert abs(M.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert abs(M.gelu(np.array([-1.0]))[0] + 0.15865525393145707) < 1e-15
    u = np.linspace(-6, 6, 101)
    # Phi(u) + Phi(-u) = 1  =>  GELU(u) - GELU(-u) = u
    assert np.allclose(M.gelu(u) - M.gelu(-u), u, rtol=0, atol=1e-14)
    # large |u|: identity and zero
    assert abs(M.gelu(np.array([40.0]))[0] - 40.0) < 1e-12
    assert abs(M.gelu(np.array([-40.0]))[0]) < 1e-12


def test_gelu_grad_matches_central_differences():
    u = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (M.gelu(u + h) - M.gelu(u - h)) / (2 * h)
    assert np.allclose(M.gelu_grad(u), fd, rtol=0, atol=1e-9)


def test_bf16_rounding_special_values():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9, -2.5, 0.0,
                  3.0e38, 1.0 + 2.0 ** -7])
    r = M.bf16(x)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert r[0] == 1.0 and r[1] == 1.0
    # 1 + 3*2^-8 is halfway between 1+2^-7 and 1+2^-6: ties to even -> 1+2^-6
    assert r[2] == 1.0 + 2.0 ** -6
    assert r[3] == 1.0 and r[4] == -2.5 and r[5] == 0.0
    assert r[7] == 1.0 + 2.0 ** -7
    assert np.isfinite(r[6])
    # every result has at most 8 significant bits
    m, _ = np.frexp(r[np.isfinite(r) & (r != 0)])
    assert np.all((m * 256) == np.round(m * 256))


def test_zero_output_layer_gives_log2_loss_and_half_gradients():
    rng = np.random.default_rng(1)
    p = M.init_params(rng)
    p[M.W3:] = 0.0  # W3 and b3 zero: logits (0, 0)
    X = M.inputs(rng.normal(size=(32, 6)), np.zeros(6), np.ones(6))
    y = rng.integers(0, 2, 32)
    loss, g = M.loss_and_grad(p, X, y)
    assert abs(loss - math.log(2.0)) < 1e-15
    # db3 = mean of (softmax - onehot) = (1/2 - [y==c]) averaged
    assert abs(g[M.B3] - np.mean(0.5 - (y == 0))) < 1e-15
    assert abs(g[M.B3 + 1] - np.mean(0.5 - (y == 1))) < 1e-15
    # nothing flows back through zero W3
    assert np.all(g[M.W1:M.W3] == 0.0)


def test_single_path_network_is_the_scalar_composition():
    # one hidden unit per layer: logit_1 = GELU(GELU(c x)), logit_0 = 0
    p = np.zeros(M.NPARAM)
    c = 0.7
    p[M.W1 + 0 * M.NH + 0] = c
    p[M.W2 + 0 * M.NH + 0] = 1.0
    p[M.W3 + 0 * M.NOUT + 1] = 1.0
    F = np.array([[0.3, 0, 0, 0, 0, 0], [-1.2, 0, 0, 0, 0, 0], [2.0, 0, 0, 0, 0, 0]])
    X = M.inputs(F, np.zeros(6), np.ones(6))
    Z3 = M.forward(p, X)[4]
    for i, x in enumerate(F[:, 0]):
        g1 = 0.5 * c * x * (1 + math.erf(c * x / math.sqrt(2)))
        g2 = 0.5 * g1 * (1 + math.erf(g1 / math.sqrt(2)))
        assert abs(Z3[i, 1] - g2) < 1e-15 and Z3[i, 0] == 0.0
        assert abs(M.probabilities(Z3)[i] - 1 / (1 + math.exp(-g2))) < 1e-15


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    p = M.init_params(rng) * 0.5
    p[M.B1:M.W2] = rng.normal(0, 0.1, M.NH)
    p[M.B2:M.W3] = rng.normal(0, 0.1, M.NH)
    p[M.B3:M.B3 + 2] = rng.normal(0, 0.1, 2)
    F = rng.normal(size=(24, 6))
    X = M.inputs(F, np.zeros(6), np.ones(6))
    y = rng.integers(0, 2, 24)
    y[3] = -1  # ignored row
    loss, g = M.loss_and_grad(p, X, y)
    real = np.flatnonzero(M.mask())
    pick = rng.choice(real, 60, replace=False)
    pick = np.concatenate([pick, [M.W1 + 2 * M.NH + 5, M.B1 + 3, M.B2 + 9, M.B3, M.B3 + 1,
                                  M.W3 + 17 * M.NOUT + 1]])
    h = 1e-6
    for k in pick:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (M.loss_and_grad(pp, X, y)[0] - M.loss_and_grad(pm, X, y)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1e-3, abs(g[k])) + 1e-10, k
    # padded parameters get no gradient
    assert np.all(g[M.mask() == 0] == 0.0)


def test_ignored_labels_count_in_the_mean_only():
    rng = np.random.default_rng(3)
    p = M.init_params(rng)
    X = M.inputs(rng.normal(size=(8, 6)), np.zeros(6), np.ones(6))
    y = np.array([0, 1, 1, 0, 1, 0, 0, 1])
    y2 = np.concatenate([y, [-1, 2]])
    X2 = np.concatenate([X, rng.normal(size=(2, 16))])
    l1, g1 = M.loss_and_grad(p, X, y)
    l2, g2 = M.loss_and_grad(p, X2, y2)
    assert abs(l2 - l1 * 8 / 10) < 1e-14
    assert np.allclose(g2, g1 * 8 / 10, rtol=1e-12, atol=1e-18)


def test_adamw_first_step_is_a_signed_lr_step():
    rng = np.random.default_rng(5)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, wd = 1e-3, 0.01
    p1, m1, v1 = M.adamw(p, g, np.zeros(50), np.zeros(50), 1, lr=lr, wd=wd, eps=0.0)
    # with bias correction m^ = g and v^ = g^2 after one step
    assert np.allclose(p1, p - lr * (np.sign(g) + wd * p), rtol=1e-14, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    keep = np.zeros(50, np.uint8)
    keep[::2] = 1
    p2, _, _ = M.adamw(p, g, np.zeros(50), np.zeros(50), 1, keep=keep)
    assert np.all(p2[1::2] == p[1::2]) and np.all(p2[::2] != p[::2])


def test_adamw_constant_gradient_steady_step():
    # constant gradient: m^ -> g, v^ -> g^2 exactly (bias corrections cancel)
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -0.25])
    m = v = np.zeros(2)
    for t in range(1, 6):
        p_new, m, v = M.adamw(p, g, m, v, t, lr=0.01, eps=0.0)
        assert np.allclose(p - p_new, 0.01 * np.sign(g), rtol=1e-12)
        p = p_new


def test_features_and_zscore():
    x0 = np.array([[0.0, 0.1, 0.3, -0.2], [0.0, -0.25, 0.1, 0.05]])
    f = M.features(x0, np.array([10.0, 20.0]), np.array([[2.0, 4.0], [6.0, 8.0]]), 200.0)
    assert np.array_equal(f[0], [0.1, -0.2, 0.3, 0.05, 0.01, 0.02])
    F = np.random.default_rng(0).normal(3.0, 2.0, (1000, 6))
    mu, istd = M.zscore_stats(F)
    Z = (F - mu) * istd
    assert np.allclose(Z.mean(0), 0, atol=1e-12) and np.allclose(Z.std(0), 1, atol=1e-12)
