"""Float64 reference of the kernel-selector network. TEST INFRASTRUCTURE ONLY.

The network maps the 6 features of a degree-pair bucket to 3 logits, one per
intersection strategy (merge path, binary search, LDS bitmap):

    h1 = relu(W1 x + b1)      W1: 32 x 6
    h2 = relu(W2 h1 + b2)     W2: 32 x 32
    z  = W3 h2 + b3           W3: 3 x 32

Weights are used after rounding to bfloat16 (round to nearest, ties to even);
biases stay float32. The loss is the weighted softmax cross-entropy
    loss = (1 / B) * sum_s w_s * (logsumexp(z_s) - z_s[y_s]),
and gradients are taken with respect to the float32 master weights through
the rounding (straight-through). Adam (Kingma and Ba, 2015) updates the
master weights.

Parameter vector layout (float32, 1379 entries):
    W1 (192, row-major [out][in]), b1 (32), W2 (1024), b2 (32), W3 (96), b3 (3)

This file shares no code with the GPU kernels; it is the plain definition,
written with numpy matrix products.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 6, 32, 3
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta)
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32 values.

    bfloat16 keeps the top 16 bits of the float32 pattern; rounding adds half
    an ulp of the kept part (0x7FFF) plus the kept part's lowest bit, so exact
    halves go to the even neighbour. NaNs are passed through.
    """
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (r << 16).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(f), f, out)


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initialisation as float32."""
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            parts[name] = rng.normal(0.0, np.sqrt(2.0 / shape[1]), size=shape)
        else:
            parts[name] = np.zeros(shape)
    return pack(parts).astype(np.float32)


def _weights(theta):
    """Float64 copies of the parameters with weights rounded to bfloat16."""
    p = unpack(np.asarray(theta, dtype=np.float32))
    return {k: (bf16_round(v).astype(np.float64) if k.startswith("W") else v.astype(np.float64))
            for k, v in p.items()}


def forward(theta, X):
    """Logits [B, 3] and the activations (h1, h2) in float64."""
    p = _weights(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ p["W1"].T + p["b1"], 0.0)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0.0)
    z = h2 @ p["W3"].T + p["b3"]
    return z, h1, h2


def loss_and_grad(theta, X, y, w=None):
    """(loss, gradient over the 1379 parameters) in float64."""
    p = _weights(theta)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.int64)
    B = X.shape[0]
    w = np.ones(B) if w is None else np.asarray(w, dtype=np.float64)
    z, h1, h2 = forward(theta, X)
    zmax = z.max(axis=1, keepdims=True)
    e = np.exp(z - zmax)
    s = e.sum(axis=1, keepdims=True)
    lse = np.log(s)[:, 0] + zmax[:, 0]
    loss = float(np.sum(w * (lse - z[np.arange(B), y])) / B)
    prob = e / s
    dz = prob.copy()
    dz[np.arange(B), y] -= 1.0
    dz *= (w / B)[:, None]
    g = {"W3": dz.T @ h2, "b3": dz.sum(0)}
    dh2 = (dz @ p["W3"]) * (h2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ p["W2"]) * (h1 > 0)
    g["W1"] = dh1.T @ X
    g["b1"] = dh1.sum(0)
    return loss, pack(g)


def loss_only(theta_rounded_weights_f64, X, y, w=None):
    """Loss with parameters used exactly as given (no rounding), float64.

    Used to check the analytic gradient by central differences.
    """
    p = unpack(np.asarray(theta_rounded_weights_f64, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    B = X.shape[0]
    w = np.ones(B) if w is None else np.asarray(w, dtype=np.float64)
    h1 = np.maximum(X @ p["W1"].T + p["b1"], 0.0)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0.0)
    z = h2 @ p["W3"].T + p["b3"]
    zmax = z.max(axis=1, keepdims=True)
    lse = np.log(np.exp(z - zmax).sum(1)) + zmax[:, 0]
    return float(np.sum(w * (lse - z[np.arange(B), np.asarray(y)])) / B)


def adam_step(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1). Returns (theta, m, v) in float64."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def forward_error_bound(theta, X):
    """Bound on |float32 logits - float64 logits| for the kernel's evaluation order.

    A length-k dot product accumulated in float32 with the bias added last
    errs by at most (k + 1) * u * (sum |w_j x_j| + |b|), u = 2^-24 (standard
    forward error analysis); ReLU is 1-Lipschitz and a later layer multiplies
    an input error by |W|. The inputs X are exact float32 values.
    """
    p = _weights(theta)
    _, h1, h2 = forward(theta, X)
    X = np.abs(np.asarray(X, dtype=np.float64))
    u = 2.0 ** -24
    a1 = X @ np.abs(p["W1"]).T + np.abs(p["b1"])
    e1 = (N_IN + 1) * u * a1
    a2 = np.abs(h1) @ np.abs(p["W2"]).T + np.abs(p["b2"])
    e2 = (N_H + 1) * u * a2 + e1 @ np.abs(p["W2"]).T
    a3 = np.abs(h2) @ np.abs(p["W3"]).T + np.abs(p["b3"])
    e3 = (N_H + 1) * u * a3 + e2 @ np.abs(p["W3"]).T
    return e3
