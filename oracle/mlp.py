"""NumPy FP64 oracle for the learned free-surface classifier -- TEST
INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).

Network: 16 standardised features -> 64 (GELU) -> 64 (GELU) -> 1 logit.
GELU is the tanh form 0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).
Loss: weighted binary cross-entropy on the logit, averaged over the batch:
    loss = (1/B) sum_b w_b [max(s_b, 0) - s_b y_b + log(1 + exp(-|s_b|))].
Optimiser: Adam (bias-corrected first and second moments).

Flat parameter layout (5,313 values), shared by definition (not by code) with
the HIP training and inference kernels:
    W1 [16 x 64] row-major (input-major), b1 [64],
    W2 [64 x 64] row-major,              b2 [64],
    W3 [64],                              b3 [1].
"""
from __future__ import annotations

import numpy as np

NIN, NH = 16, 64
SIZES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
_C = np.sqrt(2.0 / np.pi)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for k, s in SIZES:
        n = int(np.prod(s))
        out[k] = theta[o:o + n].reshape(s)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[k], dtype=np.float64).ravel() for k, _ in SIZES])


def init_params(seed):
    """He-style uniform initialisation from a seeded NumPy generator."""
    rng = np.random.default_rng(seed)
    d = {}
    for k, s in SIZES:
        if k.startswith("W"):
            fan_in = s[0]
            lim = np.sqrt(6.0 / fan_in) * 0.5
            d[k] = rng.uniform(-lim, lim, size=s)
        else:
            d[k] = np.zeros(s)
    return pack(d)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(_C * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    u = _C * (z + 0.044715 * z ** 3)
    th = np.tanh(u)
    return 0.5 * (1.0 + th) + 0.5 * z * (1.0 - th * th) * _C * (1.0 + 3.0 * 0.044715 * z * z)


def standardise(X, mean, std):
    return (np.asarray(X, dtype=np.float64) - np.asarray(mean, dtype=np.float64)) / np.asarray(std, dtype=np.float64)


def forward(theta, X, mean, std):
    """Logits for the rows of X (B x 16)."""
    p = unpack(theta)
    Z = standardise(X, mean, std)
    a1 = gelu(Z @ p["W1"] + p["b1"])
    a2 = gelu(a1 @ p["W2"] + p["b2"])
    return a2 @ p["W3"] + p["b3"][0]


def loss_and_grad(theta, X, y, w, mean, std):
    """Weighted mean BCE-with-logits and its gradient w.r.t. the flat
    parameters (hand-derived backward pass)."""
    p = unpack(theta)
    y = np.asarray(y, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    B = y.shape[0]
    Z = standardise(X, mean, std)
    z1 = Z @ p["W1"] + p["b1"]
    a1 = gelu(z1)
    z2 = a1 @ p["W2"] + p["b2"]
    a2 = gelu(z2)
    s = a2 @ p["W3"] + p["b3"][0]
    l = w * (np.maximum(s, 0.0) - s * y + np.log1p(np.exp(-np.abs(s))))
    loss = l.sum() / B
    sig = 1.0 / (1.0 + np.exp(-s))
    ds = w * (sig - y) / B
    g = {}
    g["W3"] = a2.T @ ds
    g["b3"] = np.array([ds.sum()])
    da2 = np.outer(ds, p["W3"])
    dz2 = da2 * gelu_grad(z2)
    g["W2"] = a1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    da1 = dz2 @ p["W2"].T
    dz1 = da1 * gelu_grad(z1)
    g["W1"] = Z.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def adam_step(theta, m, v, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
