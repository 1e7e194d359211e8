"""FP64 reference of the proposal network.  TEST INFRASTRUCTURE ONLY: the
tests call it to check the GPU kernels; the library never does.

Network (same parameter layout as the library's flat array): x (8) ->
h1 = relu(x W1 + b1) (128) -> h2 = relu(h1 W2 + b2) (128) -> y = h2 W3 + b3.
Loss: mean squared error.  Gradients by the chain rule written out per
layer; Adam with bias correction (beta1 0.9, beta2 0.999, eps 1e-8).
"""
from __future__ import annotations

import numpy as np

IN, H = 8, 128
SIZES = [("W1", (IN, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SIZES])


def forward(flat, X):
    p = unpack(flat)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    out = h2 @ p["W3"] + p["b3"][0]
    return out, (X, z1, h1, z2, h2)


def loss_and_grad(flat, X, Y):
    p = unpack(flat)
    out, (X, z1, h1, z2, h2) = forward(flat, X)
    n = X.shape[0]
    r = out - np.asarray(Y, dtype=np.float64)
    loss = float(np.mean(r * r))
    dout = 2.0 * r / n                        # dL/dout
    g = {"W3": h2.T @ dout, "b3": np.array([dout.sum()])}
    dz2 = np.outer(dout, p["W3"]) * (z2 > 0)  # through relu
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"].T) * (z1 > 0)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def adam(flat, grad, m, v, step: int, lr: float):
    b1, b2, eps = 0.9, 0.999, 1e-8
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v
