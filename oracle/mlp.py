"""FP64 oracle of the learned proposal's network -- TEST INFRASTRUCTURE ONLY.

A plain numpy evaluation of the 64 -> 256 -> 256 -> 1 multilayer perceptron
that ranks chirp-mass / sub-band regions, its binary cross-entropy loss, the
gradients by the chain rule, and one Adam update.  Only the tests and the
benchmark's CPU leg may use it.

Readings (the network is not in the paper; its shape is the one the
workload description fixes): ReLU hidden activations, one logit, the mean
binary cross-entropy with logits, Adam with bias correction.  The weights
the GPU multiplies with are the FP32 master weights rounded to bfloat16
(round to nearest even); the oracle receives those rounded values as its
inputs and computes everything else in FP64.

Parameter vector layout (82,689 FP32 values):
    W1 [256][64], b1 [256], W2 [256][256], b2 [256], w3 [256], b3 [1]
with W[out][in] row-major.
"""
from __future__ import annotations

import numpy as np

D_IN, H1, H2 = 64, 256, 256
SHAPES = [("W1", (H1, D_IN)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)),
          ("w3", (H2,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16_round(x):
    """float32 -> nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def weights_as_used(p32):
    """The parameters as the GPU multiplies with them: matrices and the output
    vector rounded to bfloat16, biases kept in FP32."""
    d = unpack(np.asarray(p32, dtype=np.float32).astype(np.float64))
    for name in ("W1", "W2", "w3"):
        d[name] = bf16_round(d[name].astype(np.float32))
    return d


def forward(d, x):
    """Logits and the hidden activations for inputs x [B][64]."""
    x = np.asarray(x, dtype=np.float64)
    a1 = x @ d["W1"].T + d["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ d["W2"].T + d["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ d["w3"] + d["b3"][0]
    return z, (x, a1, h1, a2, h2)


def bce_loss(z, y):
    """Mean binary cross-entropy with logits: mean(softplus(z) - y z)."""
    z = np.asarray(z, dtype=np.float64)
    return float(np.mean(np.logaddexp(0.0, z) - np.asarray(y, dtype=np.float64) * z))


def loss_and_grad(d, x, y):
    """Loss and the gradient (same layout as the parameter vector) by the chain rule."""
    z, (x, a1, h1, a2, h2) = forward(d, x)
    y = np.asarray(y, dtype=np.float64)
    B = len(z)
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / B
    g = {"w3": h2.T @ dz, "b3": np.array([dz.sum()])}
    da2 = np.outer(dz, d["w3"]) * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ d["W2"]) * (a1 > 0)
    g["W1"] = da1.T @ x
    g["b1"] = da1.sum(axis=0)
    return bce_loss(z, y), pack(g)


def adam(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected, step number t >= 1); returns (p, m, v)."""
    p, m, v, g = (np.asarray(a, dtype=np.float64) for a in (p, m, v, g))
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
