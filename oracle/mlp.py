"""Angle-predictor MLP in float64 with bfloat16 storage emulated (oracle).

Test infrastructure only. The paper suggests deriving G-QAOA angles from
statistics of an instance's density of states (Sec. V) and shows that the
optimized single-angle pairs cluster (Sec. III.B, Fig. "clustering"); this
network maps the normalized level histogram plus (n, d, p) to one pair.

Network: x[131] -> Linear(131, 256) -> GELU -> Linear(256, 256) -> GELU
-> Linear(256, 2) -> o; beta = 2 pi sigmoid(o_0), gamma = pi sigmoid(o_1).
Features: w_k = N_k / 2^n for k = 0..127 (zero beyond m), n/24, d/8, log2(p)/6.
GELU is the exact form z * Phi(z), Phi the standard normal CDF.

Storage points rounded to bfloat16 (round to nearest, ties to even), as the
device kernels store them: inputs x, weights W1..W3, post-GELU activations
h1, h2, and the pre-activation gradients dz1, dz2 that feed the backward
products. Everything else (accumulation, biases, z1, z2, outputs, weight
gradients) is kept at full precision here.

Loss: mean over the batch of ((beta - beta*)/(2 pi))^2 + ((gamma - gamma*)/pi)^2.
"""
from __future__ import annotations

import math

import numpy as np

D_IN = 131
D_HID = 256
D_OUT = 2


def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) through float32, as float64."""
    f = np.asarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    cdf = 0.5 * (1.0 + _erf(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def features(hist, n: int, d: float, p: int) -> np.ndarray:
    """Input vector of the network for one instance and round count."""
    hist = np.asarray(hist, dtype=np.float64)
    x = np.zeros(D_IN)
    w = hist / float(1 << n)
    x[:min(128, len(w))] = w[:128]
    x[128] = n / 24.0
    x[129] = d / 8.0
    x[130] = math.log2(p) / 6.0
    return x


def init_params(seed: int):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [(D_IN, D_HID), (D_HID, D_HID), (D_HID, D_OUT)]
    params = {}
    for i, (fi, fo) in enumerate(shapes, start=1):
        bound = 1.0 / math.sqrt(fi)
        params[f"W{i}"] = rng.uniform(-bound, bound, size=(fi, fo))
        params[f"b{i}"] = np.zeros(fo)
    return params


def forward(params, x):
    """Returns (o[B,2], cache)."""
    xb = bf16_round(x)
    W1, W2, W3 = (bf16_round(params[k]) for k in ("W1", "W2", "W3"))
    z1 = xb @ W1 + params["b1"]
    h1 = bf16_round(gelu(z1))
    z2 = h1 @ W2 + params["b2"]
    h2 = bf16_round(gelu(z2))
    o = h2 @ W3 + params["b3"]
    return o, dict(x=xb, z1=z1, h1=h1, z2=z2, h2=h2, W1=W1, W2=W2, W3=W3)


def angles(o):
    """(beta, gamma) from the raw outputs."""
    sig = 1.0 / (1.0 + np.exp(-np.asarray(o)))
    return 2.0 * math.pi * sig[:, 0], math.pi * sig[:, 1]


def loss_and_dout(o, beta_t, gamma_t):
    """Loss and dL/do for the angle MSE defined in the module header."""
    o = np.asarray(o, dtype=np.float64)
    B = o.shape[0]
    sig = 1.0 / (1.0 + np.exp(-o))
    beta = 2.0 * math.pi * sig[:, 0]
    gamma = math.pi * sig[:, 1]
    rb = (beta - beta_t) / (2.0 * math.pi)
    rg = (gamma - gamma_t) / math.pi
    loss = float(np.mean(rb * rb + rg * rg))
    dout = np.empty_like(o)
    # d/do0 of rb^2 = 2 rb * sig' (since d beta/do0 / (2 pi) = sig(1-sig))
    dout[:, 0] = 2.0 * rb * sig[:, 0] * (1.0 - sig[:, 0]) / B
    dout[:, 1] = 2.0 * rg * sig[:, 1] * (1.0 - sig[:, 1]) / B
    return loss, dout


def backward(params, cache, dout):
    """Gradients of the loss with respect to every parameter."""
    h1, h2, x = cache["h1"], cache["h2"], cache["x"]
    g = {}
    g["W3"] = h2.T @ dout
    g["b3"] = dout.sum(axis=0)
    dh2 = dout @ cache["W3"].T
    dz2 = bf16_round(dh2 * gelu_grad(cache["z2"]))
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ cache["W2"].T
    dz1 = bf16_round(dh1 * gelu_grad(cache["z1"]))
    g["W1"] = x.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return g


def backward_exact(params, x, dout):
    """Gradients with no bfloat16 rounding anywhere (for finite differences)."""
    z1 = x @ params["W1"] + params["b1"]
    h1 = gelu(z1)
    z2 = h1 @ params["W2"] + params["b2"]
    h2 = gelu(z2)
    g = {"W3": h2.T @ dout, "b3": dout.sum(axis=0)}
    dz2 = (dout @ params["W3"].T) * gelu_grad(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ params["W2"].T) * gelu_grad(z1)
    g["W1"] = x.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return g


def forward_exact(params, x):
    h1 = gelu(x @ params["W1"] + params["b1"])
    h2 = gelu(h1 @ params["W2"] + params["b2"])
    return h2 @ params["W3"] + params["b3"]


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction, in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = b1 * m + (1.0 - b1) * grads[k]
        v[...] = b2 * v + (1.0 - b2) * grads[k] ** 2
        mhat = m / (1.0 - b1 ** t)
        vhat = v / (1.0 - b2 ** t)
        params[k] = params[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return params
