"""FP64 reference of the learned Verlet-buffer predictor -- TEST INFRASTRUCTURE ONLY.

Not part of the paper: a small multilayer perceptron that maps 8 features
(temperature, mass-weighted displacement width, list lifetime, density,
cut-off, cluster shape one-hot) to a buffer size r_b >= 0.

Network: x (8, normalised to [-1, 1] over the training ranges)
  -> h1 = tanh(W1 x + b1) (64) -> h2 = tanh(W2 h1 + b2) (64)
  -> y = softplus(w3 . h2 + b3).
Loss: mean squared error over the batch.  Optimiser: Adam (Kingma & Ba 2015)
with bias correction, beta1 = 0.9, beta2 = 0.999, eps = 1e-8.
Flat parameter order: W1 (64x8 row-major), b1 (64), W2 (64x64 row-major),
b2 (64), w3 (64), b3 (1): 4801 values.
"""
from __future__ import annotations

import numpy as np

NF, NH = 8, 64
NPARAM = NH * NF + NH + NH * NH + NH + NH + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + NH * NF].reshape(NH, NF); o += NH * NF
    b1 = p[o:o + NH]; o += NH
    W2 = p[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = p[o:o + NH]; o += NH
    w3 = p[o:o + NH]; o += NH
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def normalise(X, lo, hi):
    return 2.0 * (np.asarray(X, np.float64) - lo) / (hi - lo) - 1.0


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def forward(p, Xn):
    W1, b1, W2, b2, w3, b3 = unpack(p)
    h1 = np.tanh(Xn @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    z3 = h2 @ w3 + b3
    return softplus(z3), (Xn, h1, h2, z3)


def loss_and_grad(p, Xn, t):
    """Mean squared error and its gradient with respect to the flat parameters (backpropagation)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    y, (x, h1, h2, z3) = forward(p, Xn)
    B = x.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dz3 = (2.0 / B) * r / (1.0 + np.exp(-z3))          # d loss / d z3, softplus' = sigmoid
    gw3 = h2.T @ dz3
    gb3 = dz3.sum()
    dz2 = np.outer(dz3, w3) * (1.0 - h2 * h2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (1.0 - h1 * h1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    return loss, pack(gW1, gb1, gW2, gb2, gw3, gb3)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
