"""FP64 oracle for the scheduler MLP: Linear(F,H)-ReLU-Linear(H,H)-ReLU-Linear(H,C),
mean-squared-error loss over a mask, and Adam.

TEST INFRASTRUCTURE ONLY.  Plain numpy in float64, written from the
definitions (affine maps, ReLU, chain rule, Adam with bias correction).
Parameter layout: W1 [F,H], b1 [H], W2 [H,H], b2 [H], W3 [H,C], b3 [C];
a layer computes Y = X @ W + b with X row-major [batch, in].
"""
from __future__ import annotations

import numpy as np

PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def forward(params: dict, X: np.ndarray):
    X = np.asarray(X, np.float64)
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], np.float64) for k in PARAM_NAMES)
    Z1 = X @ W1 + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2 + b2
    H2 = np.maximum(Z2, 0.0)
    Y = H2 @ W3 + b3
    return Y, (X, Z1, H1, Z2, H2)


def mse_loss(Y: np.ndarray, T: np.ndarray, mask: np.ndarray):
    """L = sum(mask * (Y - T)^2) / max(1, sum(mask)); returns (L, dL/dY)."""
    Y = np.asarray(Y, np.float64)
    T = np.asarray(T, np.float64)
    Mk = np.asarray(mask, np.float64)
    cnt = max(1.0, float(Mk.sum()))
    D = (Y - T) * Mk
    return float((D * D).sum() / cnt), 2.0 * D / cnt


def backward(params: dict, cache, dY: np.ndarray) -> dict:
    X, Z1, H1, Z2, H2 = cache
    W2 = np.asarray(params["W2"], np.float64)
    W3 = np.asarray(params["W3"], np.float64)
    dY = np.asarray(dY, np.float64)
    g = {}
    g["W3"] = H2.T @ dY
    g["b3"] = dY.sum(axis=0)
    dH2 = dY @ W3.T
    dZ2 = dH2 * (Z2 > 0)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dH1 = dZ2 @ W2.T
    dZ1 = dH1 * (Z1 > 0)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam_step(params: dict, grads: dict, m: dict, v: dict, t: int,
              lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step number t >= 1), in place on float64 copies;
    returns the new (params, m, v)."""
    newp, newm, newv = {}, {}, {}
    for k in PARAM_NAMES:
        gk = np.asarray(grads[k], np.float64)
        mk = beta1 * np.asarray(m[k], np.float64) + (1 - beta1) * gk
        vk = beta2 * np.asarray(v[k], np.float64) + (1 - beta2) * gk * gk
        mhat = mk / (1 - beta1 ** t)
        vhat = vk / (1 - beta2 ** t)
        newp[k] = np.asarray(params[k], np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
        newm[k], newv[k] = mk, vk
    return newp, newm, newv

