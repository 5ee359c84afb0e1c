"""FP64 reference of the warm-start network: an MLP with two ReLU hidden layers.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Shapes: X [N, I] -> H1 = relu(X W1^T + b1) [N, H] -> H2 = relu(H1 W2^T + b2)
-> Y = H2 W3^T + b3 [N, O].  Loss = mean over the N*O entries of (Y - T)^2.
Parameters are the list [W1 (H,I), b1, W2 (H,H), b2, W3 (O,H), b3].
Optimiser: Adam (Kingma & Ba 2015) with bias correction.
Matrix products use numpy's matmul as a primitive; everything else is
written out.
"""
from __future__ import annotations

import numpy as np


def forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    Z1 = X @ W1.T + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2.T + b2
    H2 = np.maximum(Z2, 0.0)
    Y = H2 @ W3.T + b3
    return Y, (X, Z1, H1, Z2, H2)


def loss(params, X, T):
    Y, _ = forward(params, X)
    return float(np.mean((Y - T) ** 2))


def grads(params, X, T):
    """Loss and its gradient with respect to every parameter (same order)."""
    W1, b1, W2, b2, W3, b3 = params
    Y, (X, Z1, H1, Z2, H2) = forward(params, X)
    N, O = Y.shape
    L = float(np.mean((Y - T) ** 2))
    dY = 2.0 * (Y - T) / (N * O)
    dW3 = dY.T @ H2
    db3 = dY.sum(axis=0)
    dZ2 = (dY @ W3) * (Z2 > 0.0)
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * (Z1 > 0.0)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(axis=0)
    return L, [dW1, db1, dW2, db2, dW3, db3]


class Adam:
    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, g):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for i, (p, gi) in enumerate(zip(params, g)):
            self.m[i] = self.b1 * self.m[i] + (1.0 - self.b1) * gi
            self.v[i] = self.b2 * self.v[i] + (1.0 - self.b2) * gi * gi
            mhat = self.m[i] / c1
            vhat = self.v[i] / c2
            out.append(p - self.lr * mhat / (np.sqrt(vhat) + self.eps))
        return out


def standardize_stats(X):
    """Per-column mean and population standard deviation (1 where it is 0)."""
    mu = X.mean(axis=0)
    sd = np.sqrt(((X - mu) ** 2).mean(axis=0))
    sd = np.where(sd > 0.0, sd, 1.0)
    return mu, sd
