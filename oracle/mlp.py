"""FP64 reference of the learned gate (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The paper motivates fast indicators as a source of
large labelled datasets for machine-learning models of dynamics
(Introduction; Related research); the gate is one such model.  Written
from the definitions, in numpy FP64:

  features   f = (y, p_y, p_x, LD(t)/t, G_1(t)/t, G_2(t)/t), x0 = (x, y, p_x, p_y)
  scaling    z = (f - mean) * istd, population statistics of the training set
  network    h1 = GELU(z W1 + b1), h2 = GELU(h1 W2 + b2), logits = h2 W3 + b3
             (6 -> 256 -> 256 -> 2), GELU(u) = u Phi(u) with the erf form of Phi
  loss       mean over the batch of -log softmax(logits)[label]; rows whose
             label is not 0 or 1 contribute zero but count in the mean
  optimiser  AdamW: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
             p -= lr (m/(1-b1^t) / (sqrt(v/(1-b2^t)) + eps) + wd p)

Parameters use the library's flat padded layout (inputs padded to 16,
logits to 16): W1[16][256], b1[256], W2[256][256], b2[256], W3[256][16],
b3[16].  The optional `bf16` switch rounds, like the device products do,
the inputs, the weights, the hidden activations and the back-propagated
logit / pre-activation gradients to bfloat16 (round to nearest even) and
otherwise computes in FP64; it exists so that device results can be
compared on the same rounded operands.
"""
import math

import numpy as np
from scipy.special import erf

NFEAT, NIN, NH, NOUT = 6, 16, 256, 16
W1, B1 = 0, NIN * NH
W2 = B1 + NH
B2 = W2 + NH * NH
W3 = B2 + NH
B3 = W3 + NH * NOUT
NPARAM = B3 + NOUT


def mask():
    """1 for the real parameters, 0 for the padding."""
    m = np.zeros(NPARAM, np.uint8)
    m[W1:B1].reshape(NIN, NH)[:NFEAT] = 1
    m[B1:W2] = 1
    m[W2:B2] = 1
    m[B2:W3] = 1
    m[W3:B3].reshape(NH, NOUT)[:, :2] = 1
    m[B3:B3 + 2] = 1
    return m


def unpack(p):
    p = np.asarray(p, np.float64)
    return (p[W1:B1].reshape(NIN, NH), p[B1:W2], p[W2:B2].reshape(NH, NH), p[B2:W3],
            p[W3:B3].reshape(NH, NOUT), p[B3:B3 + NOUT])


def bf16(x):
    """Round to the nearest bfloat16 value (ties to even), through float32."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isfinite(f), out, f).astype(np.float64)


def gelu(u):
    return 0.5 * u * (1.0 + erf(u / math.sqrt(2.0)))


def gelu_grad(u):
    return 0.5 * (1.0 + erf(u / math.sqrt(2.0))) + u * np.exp(-0.5 * u * u) / math.sqrt(2.0 * math.pi)


def features(x0, ld, ln_growth, t):
    x0 = np.asarray(x0, np.float64)
    lg = np.asarray(ln_growth, np.float64)
    return np.stack([x0[:, 1], x0[:, 3], x0[:, 2], np.asarray(ld) / t, lg[:, 0] / t,
                     lg[:, 1] / t], axis=1)


def zscore_stats(F):
    F = np.asarray(F, np.float64)
    mu = F.mean(axis=0)
    sd = np.sqrt(F.var(axis=0))
    return mu, np.where(sd > 0, 1.0 / np.where(sd > 0, sd, 1.0), 1.0)


def inputs(F, mean, istd, rounding=False):
    """Padded [n][16] network inputs from raw features.  With rounding the
    z-score is taken in float32 (as the device does) and rounded to bf16."""
    F = np.asarray(F)
    n = F.shape[0]
    X = np.zeros((n, NIN))
    if rounding:
        z = (F.astype(np.float32) - np.asarray(mean, np.float32)) * np.asarray(istd, np.float32)
        X[:, :NFEAT] = bf16(z)
    else:
        X[:, :NFEAT] = (np.asarray(F, np.float64) - mean) * istd
    return X


def forward(p, X, rounding=False):
    """Pre-activations and activations of every layer: (Z1, A1, Z2, A2, Z3)."""
    w1, b1, w2, b2, w3, b3 = unpack(p)
    r = bf16 if rounding else (lambda a: a)
    X = r(X)
    Z1 = X @ r(w1) + b1
    A1 = r(gelu(Z1))
    Z2 = A1 @ r(w2) + b2
    A2 = r(gelu(Z2))
    Z3 = A2 @ r(w3) + b3
    return Z1, A1, Z2, A2, Z3


def probabilities(Z3):
    a, b = Z3[:, 0], Z3[:, 1]
    m = np.maximum(a, b)
    ea, eb = np.exp(a - m), np.exp(b - m)
    return eb / (ea + eb)


def loss_and_grad(p, X, labels, rounding=False):
    """Mean cross-entropy over the rows of X and its gradient (flat)."""
    w1, b1, w2, b2, w3, b3 = unpack(p)
    r = bf16 if rounding else (lambda a: a)
    n = X.shape[0]
    labels = np.asarray(labels)
    Z1, A1, Z2, A2, Z3 = forward(p, X, rounding)
    valid = (labels == 0) | (labels == 1)
    y = np.where(labels == 1, 1, 0)
    m = np.maximum(Z3[:, 0], Z3[:, 1])
    lse = m + np.log(np.exp(Z3[:, 0] - m) + np.exp(Z3[:, 1] - m))
    zy = np.where(y == 1, Z3[:, 1], Z3[:, 0])
    loss = np.sum(np.where(valid, lse - zy, 0.0)) / n
    p1 = probabilities(Z3)
    dZ3 = np.zeros_like(Z3)
    dZ3[:, 0] = np.where(valid, (1.0 - p1) - (y == 0), 0.0) / n
    dZ3[:, 1] = np.where(valid, p1 - (y == 1), 0.0) / n
    dZ3r = r(dZ3)
    g = np.zeros(NPARAM)
    g[W3:B3] = (r(A2).T @ dZ3r).ravel()
    g[B3:B3 + NOUT] = dZ3.sum(axis=0)
    dA2 = dZ3r @ r(w3).T
    dZ2 = dA2 * gelu_grad(Z2)
    dZ2r = r(dZ2)
    g[W2:B2] = (A1.T @ dZ2r).ravel()
    g[B2:W3] = dZ2.sum(axis=0)
    dA1 = dZ2r @ r(w2).T
    dZ1 = dA1 * gelu_grad(Z1)
    dZ1r = r(dZ1)
    g[W1:B1] = (r(X).T @ dZ1r).ravel()
    g[B1:W2] = dZ1.sum(axis=0)
    return loss, g


def adamw(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.0, keep=None):
    """One AdamW step (t counts from 1); returns new (p, m, v).  Entries with
    keep == 0 are left unchanged."""
    m2 = beta1 * m + (1.0 - beta1) * g
    v2 = beta2 * v + (1.0 - beta2) * g * g
    mh = m2 / (1.0 - beta1 ** t)
    vh = v2 / (1.0 - beta2 ** t)
    p2 = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    if keep is not None:
        k = np.asarray(keep) != 0
        p2 = np.where(k, p2, p)
        m2 = np.where(k, m2, m)
        v2 = np.where(k, v2, v)
    return p2, m2, v2


def init_params(rng):
    """He-normal weights on the real entries, zero biases and padding."""
    p = np.zeros(NPARAM)
    w1, _, w2, _, w3, _ = (p[W1:B1].reshape(NIN, NH), None, p[W2:B2].reshape(NH, NH), None,
                           p[W3:B3].reshape(NH, NOUT), None)
    w1[:NFEAT] = rng.normal(0, math.sqrt(2.0 / NFEAT), (NFEAT, NH))
    w2[:] = rng.normal(0, math.sqrt(2.0 / NH), (NH, NH))
    w3[:, :2] = rng.normal(0, math.sqrt(2.0 / NH), (NH, 2))
    return p
