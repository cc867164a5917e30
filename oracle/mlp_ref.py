"""Float64 reference of the proposal network -- test infrastructure only.

f(x) = w3 . relu(W2 relu(W1 x + b1) + b2) + b3, sizes 16 -> 64 -> 64 -> 1,
loss L = 0.5 * mean((f(x) - y)^2).  The gradient is the chain rule written
out layer by layer; it is pinned by central finite differences in the tests.
Parameter layout (flat vector): W1[64][16], b1[64], W2[64][64], b2[64],
w3[64], b3.
"""
from __future__ import annotations

import numpy as np

IN, HID = 16, 64
SIZES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("w3", (HID,)), ("b3", (1,))]
NUM_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta: np.ndarray):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def forward(theta: np.ndarray, X: np.ndarray) -> np.ndarray:
    P = unpack(np.asarray(theta, np.float64))
    X = np.asarray(X, np.float64)
    h1 = np.maximum(X @ P["W1"].T + P["b1"], 0.0)
    h2 = np.maximum(h1 @ P["W2"].T + P["b2"], 0.0)
    return h2 @ P["w3"] + P["b3"][0]


def loss(theta: np.ndarray, X: np.ndarray, y: np.ndarray) -> float:
    d = forward(theta, X) - np.asarray(y, np.float64)
    return float(0.5 * np.mean(d * d))


def loss_grad(theta: np.ndarray, X: np.ndarray, y: np.ndarray):
    P = unpack(np.asarray(theta, np.float64))
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.float64)
    n = X.shape[0]
    z1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    f = h2 @ P["w3"] + P["b3"][0]
    d = f - y
    L = float(0.5 * np.mean(d * d))
    g_f = d / n                                  # dL/df
    g = {}
    g["b3"] = np.array([g_f.sum()])
    g["w3"] = h2.T @ g_f
    g_z2 = np.outer(g_f, P["w3"]) * (z2 > 0)
    g["W2"] = g_z2.T @ h1
    g["b2"] = g_z2.sum(axis=0)
    g_z1 = (g_z2 @ P["W2"]) * (z1 > 0)
    g["W1"] = g_z1.T @ X
    g["b1"] = g_z1.sum(axis=0)
    flat = np.concatenate([g[name].ravel() for name, _ in SIZES])
    return L, flat


def finite_difference(theta: np.ndarray, X: np.ndarray, y: np.ndarray, idx, eps: float = 1e-6):
    out = []
    for i in idx:
        tp = np.array(theta, np.float64)
        tm = np.array(theta, np.float64)
        tp[i] += eps
        tm[i] -= eps
        out.append((loss(tp, X, y) - loss(tm, X, y)) / (2 * eps))
    return np.array(out)
