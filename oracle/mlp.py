"""FP64 oracle of the learned level-of-detail network (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests use it to check the GPU training and
inference kernels; the renderer never imports it.

The network refines the hierarchy cut of NavGSim Sec. III-B (level-of-
detail selection over the Gaussian tree); the paper gives no learned
component, so its form is the project's: inputs are 8 standardised node
features, layers 8 -> 32 -> 32 -> 1 with ReLU, output a logit of
P(refine).  Loss: mean binary cross-entropy with logits.  Optimiser: Adam.
Weights are held in FP32 and used rounded to BF16 (round to nearest, ties to
even).  Parameter layout: W1[32][8], b1[32], W2[32][32], b2[32], w3[32], b3.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 8, 32
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("w3", (N_H,)), ("b3", ())]
N_PARAMS = sum(int(np.prod(s)) if s else 1 for _, s in SIZES)   # 1377


def unpack(p):
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape)) if shape else 1
        out[name] = np.asarray(p[o:o + k], np.float64).reshape(shape) if shape else float(p[o])
        o += k
    return out


def pack(d):
    return np.concatenate([np.ravel(np.asarray(d[name], np.float64)) for name, _ in SIZES])


def bf16_bits(x):
    """BF16 bit patterns of float32 values, rounded to nearest, ties to even
    (NaN not handled: weights are finite)."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = (b + 0x7FFF + lsb) >> 16
    return r.astype(np.uint16)


def bf16_value(bits):
    return (np.asarray(bits, np.uint32) << 16).view(np.float32).astype(np.float64)


def standardise(F, mean, std):
    return (np.asarray(F, np.float64) - np.asarray(mean, np.float64)) / np.asarray(std, np.float64)


def forward(p, X):
    """Logits z (n,) and the activations (a1, h1, a2, h2) for inputs X (n, 8)."""
    q = unpack(p)
    X = np.asarray(X, np.float64)
    a1 = X @ q["W1"].T + q["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ q["w3"] + q["b3"]
    return z, (a1, h1, a2, h2)


def loss(p, X, y):
    """Mean binary cross-entropy of sigmoid(z) against labels y in {0, 1}:
    mean(log(1 + e^z) - y z), evaluated stably."""
    z, _ = forward(p, X)
    y = np.asarray(y, np.float64)
    return float(np.mean(np.maximum(z, 0) + np.log1p(np.exp(-np.abs(z))) - y * z))


def grad(p, X, y):
    """Gradient of loss(p, X, y) with respect to the packed parameters."""
    q = unpack(p)
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.float64)
    n = X.shape[0]
    z, (a1, h1, a2, h2) = forward(p, X)
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / n
    g = {"w3": h2.T @ dz, "b3": dz.sum()}
    da2 = np.outer(dz, q["w3"]) * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(0)
    da1 = (da2 @ q["W2"]) * (a1 > 0)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(0)
    return pack(g)


def adam(p, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1).  Returns (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
