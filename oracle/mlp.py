"""FP64 reference of the warm-start network (TEST INFRASTRUCTURE).

Not part of the paper: the learned warm start predicts initial spot
intensities z0 and a penalty scale for ADMM-BB from per-spot features.  This
module is the plain float64 statement of the network, its loss, gradient and
Adam step, against which the GPU training kernels are checked.  Pinned by
central finite differences of the loss (tests).

Network, for a batch X (B x F) of the spots of one patient:
  h1 = relu(X W1^T + b1)            W1: H x F
  h2 = relu(h1 W2^T + b2)           W2: H x H
  y  = softplus(h2 w3 + b3)         predicted intensity, >= 0
  lr = mean_b(h2) . wr + br         predicted log of the penalty scale
Loss:  L = mean_b (y_b - t_b)^2 + lam (lr - lr_t)^2
Flat parameter order: W1, b1, W2, b2, w3, b3, wr, br.
"""
from __future__ import annotations

import numpy as np


def shapes(F: int, H: int):
    return [("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,)),
            ("wr", (H,)), ("br", (1,))]


def unflatten(theta: np.ndarray, F: int, H: int) -> dict:
    out, o = {}, 0
    for name, shp in shapes(F, H):
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def flatten(p: dict, F: int, H: int) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in shapes(F, H)])


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def forward(theta, X, F, H):
    p = unflatten(theta, F, H)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ p["w3"] + p["b3"][0]
    y = softplus(z3)
    pooled = h2.mean(axis=0)
    lr = float(pooled @ p["wr"] + p["br"][0])
    return y, lr, dict(z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, pooled=pooled, p=p, X=X)


def loss_and_grad(theta, X, t, lr_t, lam, F, H):
    y, lr, c = forward(theta, X, F, H)
    p = c["p"]
    B = X.shape[0]
    t = np.asarray(t, dtype=np.float64)
    L = float(np.mean((y - t) ** 2) + lam * (lr - lr_t) ** 2)
    dy = 2.0 * (y - t) / B
    dz3 = dy * sigmoid(c["z3"])
    g = {}
    g["w3"] = c["h2"].T @ dz3
    g["b3"] = np.array([dz3.sum()])
    dlr = 2.0 * lam * (lr - lr_t)
    g["wr"] = dlr * c["pooled"]
    g["br"] = np.array([dlr])
    dh2 = np.outer(dz3, p["w3"]) + dlr * p["wr"][None, :] / B
    dz2 = dh2 * (c["z2"] > 0)
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (c["z1"] > 0)
    g["W1"] = dz1.T @ c["X"]
    g["b1"] = dz1.sum(axis=0)
    return L, flatten(g, F, H)


def adam(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
