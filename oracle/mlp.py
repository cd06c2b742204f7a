"""Float64 reference for the planner MLP (40 -> 64 -> 64 -> 2, ReLU).

TEST INFRASTRUCTURE ONLY (see the package docstring). Shares nothing with the
GPU kernels beyond the parameter layout both sides document.

Parameter vector layout (6914 values): W1[40][64], b1[64], W2[64][64], b2[64],
W3[64][2], b3[2], each matrix row-major with the input index first, so that a
layer computes y[o] = b[o] + sum_i x[i] * W[i][o].

Loss: mean squared error over the batch and both outputs,
L = 1/(2B) * sum_b sum_o (y[b,o] - t[b,o])^2.

Adam follows Kingma and Ba (ICLR 2015, Algorithm 1) with bias-corrected first
and second moment estimates.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 40, 64, 2
SHAPES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_H, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 6914


def unpack(theta: np.ndarray) -> dict:
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,), theta.shape
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = theta[o:o + k].reshape(shp)
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def he_uniform(unit_draws: np.ndarray) -> np.ndarray:
    """Parameters from N_PARAMS uniform [0,1) draws: weights U(-a, a) with
    a = sqrt(6 / fan_in), biases zero."""
    u = np.asarray(unit_draws, dtype=np.float64)
    theta = np.zeros(N_PARAMS)
    o = 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        if name.startswith("W"):
            a = np.sqrt(6.0 / shp[0])
            theta[o:o + k] = (2.0 * u[o:o + k] - 1.0) * a
        o += k
    return theta


def forward(theta: np.ndarray, x: np.ndarray):
    """Returns (y, cache). x: [B, 40]."""
    p = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"] + p["b3"]
    return y, (x, z1, h1, z2, h2)


def loss(theta: np.ndarray, x: np.ndarray, t: np.ndarray) -> float:
    y, _ = forward(theta, x)
    return float(np.sum((y - t) ** 2) / (2.0 * x.shape[0]))


def backward(theta: np.ndarray, x: np.ndarray, t: np.ndarray):
    """Returns (loss, grad) with grad in the packed layout."""
    p = unpack(theta)
    y, (x, z1, h1, z2, h2) = forward(theta, x)
    b = x.shape[0]
    dy = (y - np.asarray(t, dtype=np.float64)) / b  # dL/dy
    g = {}
    g["W3"] = h2.T @ dy
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ p["W3"].T
    dz2 = dh2 * (z2 > 0.0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * (z1 > 0.0)
    g["W1"] = x.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    lval = float(np.sum((y - t) ** 2) / (2.0 * b))
    return lval, pack(g)


def adam_step(theta, m, v, grad, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based). Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v
