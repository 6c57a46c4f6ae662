"""FP64 reference of the candidate-ranking network -- TEST INFRASTRUCTURE ONLY.

The network (not part of the paper's method; it ranks candidate priority
orders before the exact analysis of Sec. IV-F confirms them) is a DeepSets
model over the chains of a set under one order:

    z1_r = W1 x_r + b1,  h1_r = max(z1_r, 0)        for every chain row r
    p    = mean over the rows of the candidate of h1_r
    z2   = W2 p + b2,    h2 = max(z2, 0)
    y    = w3 . h2 + b3                             (predicted max R/D)

with 48 inputs, 256 hidden units and 78,593 parameters.  The fast path keeps
float32 master parameters, multiplies in bfloat16 with float32 accumulation
and rounds at fixed points: the inputs x, the weights W1, W2, w3, the pooled
vector p and the hidden vector h2 enter their products as bfloat16 values.
``forward(..., quant=True)`` applies the same rounding points and does every
sum in float64, so the two differ only by accumulation rounding;
``quant=False`` is the plain float64 model used to check the gradients against
finite differences.  Gradients pass straight through the bfloat16 roundings.

Parameter vector layout (float32 / float64, 78,593 entries):
    W1 [256][48] | b1 [256] | W2 [256][256] | b2 [256] | w3 [256] | b3 [1]
"""
from __future__ import annotations

import numpy as np

from .features import bf16_round

N_IN = 48
N_HID = 256
SIZES = (("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("w3", (N_HID,)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)
assert N_PARAMS == 78593


def unpack(theta) -> dict:
    theta = np.asarray(theta)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], np.float64).reshape(-1) for name, _ in SIZES])


def _q(a, quant):
    """bfloat16 value of a float32 rounding of ``a`` (identity when not quant)."""
    if not quant:
        return np.asarray(a, np.float64)
    return bf16_round(np.asarray(a, np.float64).astype(np.float32))


def forward(theta, x, row_off, quant=True):
    """x: [rows, 48] feature values (bfloat16 values when quant); row_off:
    [n+1] row ranges of the n candidates.  Returns y [n] and the
    intermediates the backward pass needs."""
    P = unpack(np.asarray(theta, np.float64))
    W1, W2, w3 = _q(P["W1"], quant), _q(P["W2"], quant), _q(P["w3"], quant)
    x = np.asarray(x, np.float64)
    n = len(row_off) - 1
    z1 = x @ W1.T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    p = np.zeros((n, N_HID))
    for i in range(n):
        a, b = int(row_off[i]), int(row_off[i + 1])
        p[i] = h1[a:b].sum(axis=0) / (b - a)
    pq = _q(p, quant)
    z2 = pq @ W2.T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    h2q = _q(h2, quant)
    y = h2q @ w3 + P["b3"][0]
    cache = {"x": x, "z1": z1, "p": p, "pq": pq, "z2": z2, "h2q": h2q, "W2": W2, "w3": w3,
             "row_off": np.asarray(row_off)}
    return y, cache


def loss(y, t) -> float:
    """Mean squared error."""
    d = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float(np.mean(d * d))


def backward(theta, cache, y, t) -> np.ndarray:
    """Gradient of the mean squared error wrt the (master) parameters."""
    n = len(y)
    dy = 2.0 * (np.asarray(y, np.float64) - np.asarray(t, np.float64)) / n
    g = {}
    g["b3"] = np.array([dy.sum()])
    g["w3"] = dy @ cache["h2q"]
    dz2 = np.outer(dy, cache["w3"]) * (cache["z2"] > 0)
    g["b2"] = dz2.sum(axis=0)
    g["W2"] = dz2.T @ cache["pq"]
    dp = dz2 @ cache["W2"]
    ro = cache["row_off"]
    dz1 = np.zeros_like(cache["z1"])
    for i in range(n):
        a, b = int(ro[i]), int(ro[i + 1])
        dz1[a:b] = dp[i] / (b - a)
    dz1 *= cache["z1"] > 0
    g["b1"] = dz1.sum(axis=0)
    g["W1"] = dz1.T @ cache["x"]
    return pack(g)


def adam(theta, m, v, grad, lr, b1, b2, eps, step):
    """One Adam step (Kingma & Ba 2015, Algorithm 1) with bias correction;
    ``step`` counts from 1.  Returns the new (theta, m, v)."""
    theta = np.asarray(theta, np.float64)
    g = np.asarray(grad, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
