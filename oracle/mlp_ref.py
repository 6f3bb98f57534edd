"""CPU reference of the pivot network (test infrastructure).

A 16 -> 64 -> 64 -> 1 perceptron, ReLU hidden layers; z = output before the
logistic.  Loss = mean_b (z_b - t_b)^2 / 2.  Written directly from these
definitions in float64 numpy; the backward pass is the chain rule by hand and
is pinned by finite differences in the tests.  bf16=True rounds weights,
inputs and hidden activations to bfloat16 (round to nearest, ties to even)
before each product, as the device kernels do.

Parameter layout (flat float vector): W1[64][16], b1[64], W2[64][64],
b2[64], w3[64], b3.
"""
from __future__ import annotations

import numpy as np

IN, H = 16, 64
SIZES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
P = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + k], np.float64).reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SIZES])


def bf16(a):
    """Round float32 values to the nearest bfloat16 (ties to even)."""
    a32 = np.asarray(a, np.float32)
    b = a32.view(np.uint32).astype(np.uint64)
    finite = (b & 0x7F800000) != 0x7F800000
    r = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    out = np.where(finite, r, b.astype(np.uint32)).view(np.float32)
    return out.astype(np.float64)


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    d = {"W1": rng.normal(0, np.sqrt(2.0 / IN), (H, IN)), "b1": np.zeros(H),
         "W2": rng.normal(0, np.sqrt(2.0 / H), (H, H)), "b2": np.zeros(H),
         "w3": rng.normal(0, np.sqrt(1.0 / H), H), "b3": np.zeros(1)}
    return pack(d)


def forward(p, x, bf=False):
    """x: [B, 16] -> (z [B], cache)."""
    d = unpack(p)
    r = bf16 if bf else (lambda a: np.asarray(a, np.float64))
    W1, b1, W2, b2, w3, b3 = (r(d[k]) for k in ("W1", "b1", "W2", "b2", "w3", "b3"))
    x = r(np.asarray(x, np.float64))
    a1 = x @ W1.T + b1
    h1 = r(np.maximum(a1, 0.0))
    a2 = h1 @ W2.T + b2
    h2 = r(np.maximum(a2, 0.0))
    z = h2 @ w3 + b3[0]
    return z, (x, a1, h1, a2, h2, W2, w3)


def magnitude(p, x):
    """The forward pass on |parameters| and |x| (no activation): for each
    sample, the sum of the absolute values of every product the network
    adds up, propagated through the layers.  Rounding errors of a
    floating-point evaluation of the network scale with it (a dot product of
    k terms errs by at most k * u * the sum of its terms' magnitudes)."""
    d = unpack(np.abs(np.asarray(p, np.float64)))
    xa = np.abs(np.asarray(x, np.float64))
    a1 = xa @ d["W1"].T + d["b1"]
    a2 = a1 @ d["W2"].T + d["b2"]
    return a2 @ d["w3"] + d["b3"][0]


def loss_and_grad(p, x, t, bf=False):
    z, (xx, a1, h1, a2, h2, W2, w3) = forward(p, x, bf)
    B = len(z)
    t = np.asarray(t, np.float64)
    loss = float(np.mean(0.5 * (z - t) ** 2))
    dz = (z - t) / B
    g = {"b3": np.array([dz.sum()]), "w3": h2.T @ dz}
    dh2 = np.outer(dz, w3) * (a2 > 0)
    g["b2"] = dh2.sum(0)
    g["W2"] = dh2.T @ h1
    dh1 = (dh2 @ W2) * (a1 > 0)
    g["b1"] = dh1.sum(0)
    g["W1"] = dh1.T @ xx
    return loss, pack(g)


def quantile(z):
    """Network output as the clamped sample quantile."""
    q = 1.0 / (1.0 + np.exp(-np.asarray(z, np.float64)))
    return np.clip(q, 2.0**-10, 1 - 2.0**-10)
