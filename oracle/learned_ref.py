"""FP64 reference of the learned index's root network -- test infrastructure only.

The root is a multilayer perceptron 2 -> 64 -> 64 -> 1 with ReLU; its
parameters are one flat vector in this order: W1[64][2], b1[64], W2[64][64],
b2[64], w3[64], b3 (4417 values).  Its loss over rows (x_i, t_i) is the mean
squared error (1/n) sum_i (y(x_i) - t_i)^2.  This module evaluates the loss
and its gradient by the chain rule in float64 with numpy, so the device
training kernels can be checked against it; the central-difference routine
pins the analytic gradient itself.  Nothing here is shared with the library.
"""
from __future__ import annotations

import numpy as np

NH = 64
NPARAM = NH * 2 + NH + NH * NH + NH + NH + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (NPARAM,)
    o = 0
    W1 = p[o:o + 2 * NH].reshape(NH, 2); o += 2 * NH
    b1 = p[o:o + NH]; o += NH
    W2 = p[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = p[o:o + NH]; o += NH
    w3 = p[o:o + NH]; o += NH
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def forward(p, X):
    """Network output y for every row of X (n x 2), and the intermediates."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (X, z1, h1, z2, h2)


def loss(p, X, T):
    y, _ = forward(p, X)
    return float(np.mean((y - np.asarray(T, dtype=np.float64)) ** 2))


def grad(p, X, T):
    """Gradient of the mean squared error with respect to the flat parameters."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    y, (X, z1, h1, z2, h2) = forward(p, X)
    n = X.shape[0]
    dy = 2.0 * (y - np.asarray(T, dtype=np.float64)) / n
    g_w3 = h2.T @ dy
    g_b3 = dy.sum()
    d2 = np.outer(dy, w3) * (z2 > 0)
    g_W2 = d2.T @ h1
    g_b2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (z1 > 0)
    g_W1 = d1.T @ X
    g_b1 = d1.sum(axis=0)
    return np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])


def central_differences(p, X, T, idx, h=1e-6):
    """(loss(p + h e_i) - loss(p - h e_i)) / 2h for each i in idx."""
    p = np.asarray(p, dtype=np.float64)
    out = np.empty(len(idx))
    for j, i in enumerate(idx):
        a = p.copy(); a[i] += h
        b = p.copy(); b[i] -= h
        out[j] = (loss(a, X, T) - loss(b, X, T)) / (2 * h)
    return out
