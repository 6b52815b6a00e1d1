"""FP64 reference of the boundary-closure MLP (test infrastructure only).

Network 36 -> 64 -> 64 -> 3 with exact-erf GELU after the two hidden layers:
    z1 = q(x) q(W1) + b1,  h1 = gelu(z1)
    z2 = q(h1) q(W2) + b2, h2 = gelu(z2)
    y  = q(h2) q(W3) + b3
Loss: mean squared error over the batch and the three outputs.
Backward (the plain chain rule; q on every matrix-product operand, as the GPU
feeds bfloat16 operands to its matrix cores):
    dy  = 2 (y - t) / (3 B)
    dW3 = q(h2)^T q(dy),  db3 = sum dy,  dh2 = q(dy) q(W3)^T,  dz2 = dh2 gelu'(z2)
    dW2 = q(h1)^T q(dz2), db2 = sum dz2, dh1 = q(dz2) q(W2)^T, dz1 = dh1 gelu'(z1)
    dW1 = q(x)^T q(dz1),  db1 = sum dz1
q is round-to-nearest-even to bfloat16 when `bf16=True` and the identity
otherwise (then this is an exact FP64 network, which finite differences pin).
Adam (Kingma & Ba 2015) with bias correction updates FP32 master weights.

The paper contains no network; this is the reference the GPU kernels of the
learned closure are checked against.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SHAPES = [("W1", (36, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 3)), ("b3", (3,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 6723


def bf16(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), from the float32 value."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(flat):
    out, i = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[i:i + n], dtype=np.float64).reshape(shape)
        i += n
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(flat, x, bf16_operands=True):
    q = bf16 if bf16_operands else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(flat)
    z1 = q(x) @ q(p["W1"]) + p["b1"]
    h1 = gelu(z1)
    z2 = q(h1) @ q(p["W2"]) + p["b2"]
    h2 = gelu(z2)
    y = q(h2) @ q(p["W3"]) + p["b3"]
    return y, (z1, h1, z2, h2)


def loss(flat, x, t, bf16_operands=True):
    y, _ = forward(flat, x, bf16_operands)
    return float(np.mean((y - t) ** 2))


def grad(flat, x, t, bf16_operands=True):
    """(loss, flat gradient)."""
    q = bf16 if bf16_operands else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(flat)
    y, (z1, h1, z2, h2) = forward(flat, x, bf16_operands)
    B = x.shape[0]
    dy = 2.0 * (y - t) / (3.0 * B)
    g = {}
    g["W3"] = q(h2).T @ q(dy)
    g["b3"] = dy.sum(0)
    dz2 = (q(dy) @ q(p["W3"]).T) * gelu_grad(z2)
    g["W2"] = q(h1).T @ q(dz2)
    g["b2"] = dz2.sum(0)
    dz1 = (q(dz2) @ q(p["W2"]).T) * gelu_grad(z1)
    g["W1"] = q(x).T @ q(dz1)
    g["b1"] = dz1.sum(0)
    return float(np.mean((y - t) ** 2)), pack(g)


def splitmix64_output(state):
    """SplitMix64 (Steele, Lea & Flood 2014): the output of the generator
    whose state is `state` (uint64 array) before its step, i.e. the state
    advanced by the golden gamma and passed through the two xor-shift-multiply
    rounds and a final xor-shift.  Arithmetic modulo 2^64."""
    with np.errstate(over="ignore"):  # the wrap modulo 2^64 is the definition
        z = np.atleast_1d(np.asarray(state, dtype=np.uint64)) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def input_noise(seed, step, rows, cols=36):
    """Standard normal variates of the training-input noise of train step
    `step` (the definition of lbm_mlp_set_noise): key K = seed * 0x100000001B3
    + step (mod 2^64); feature c of dataset row i takes the SplitMix64 output
    r for the state K ^ (64 i + c), u1 = ((r >> 40) + 1) / (2^24 + 1) in (0, 1),
    u2 = ((r >> 16) mod 2^24) / 2^24 in [0, 1), and the Box-Muller variate
    sqrt(-2 ln u1) cos(2 pi u2) (Box & Muller 1958), here in FP64.  Returns
    [rows][cols]."""
    key = (int(seed) * 0x100000001B3 + int(step)) % (1 << 64)
    i = np.arange(rows, dtype=np.uint64)[:, None]
    c = np.arange(cols, dtype=np.uint64)[None, :]
    r = splitmix64_output(np.uint64(key) ^ (i * np.uint64(64) + c))
    u1 = ((r >> np.uint64(40)).astype(np.float64) + 1.0) / 16777217.0
    u2 = ((r >> np.uint64(16)) & np.uint64(0xFFFFFF)).astype(np.float64) / 16777216.0
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def adam(w, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def init(seed=0):
    """He-style uniform initialisation with a zero last layer (the network
    starts as the plain boundary condition)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SHAPES:
        if name.startswith("W") and name != "W3":
            lim = math.sqrt(6.0 / shape[0])
            p[name] = rng.uniform(-lim, lim, size=shape)
        else:
            p[name] = np.zeros(shape)
    return pack(p)
