"""FP64 reference of the learned row-size network.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  This part is not in the
paper: it is the oracle for the project's own learned sizer, written as the
textbook definitions (affine layers, ReLU, logistic output, mean squared error,
the chain rule, and Adam as published by Kingma and Ba, 2015).

Model (1,217 parameters, flat vector order W1, b1, W2, b2, w3, b3):
  x   = (log2(1 + f) - mu) / sd             f = (nnz(A_i), UB_i, maxB_i)
  h1  = relu(W1 x + b1)                     W1: 32 x 3
  h2  = relu(W2 h1 + b2)                    W2: 32 x 32
  z   = w3 . h2 + b3
  rho = 1 / (1 + exp(-z))
  predicted nnz(C_i) = maxB_i + rho * (UB_i - maxB_i)

The paper bounds nnz(C_i) from above by the multiplication count UB_i
(Section IV-B); from below it is at least the longest selected B row, since
those columns all appear in C_i.  The network only places the row inside that
interval.

Loss over samples with UB > maxB (rows with UB == maxB are exact already):
  t = (n - maxB) / (UB - maxB),  L = sum_s w_s (rho_s - t_s)^2 / sum_s w_s.
"""
from __future__ import annotations

import numpy as np

H = 32
NPARAM = H * 3 + H + H * H + H + H + 1   # 1217

_OFF_W1 = 0
_OFF_B1 = _OFF_W1 + H * 3
_OFF_W2 = _OFF_B1 + H
_OFF_B2 = _OFF_W2 + H * H
_OFF_W3 = _OFF_B2 + H
_OFF_B3 = _OFF_W3 + H
assert _OFF_B3 + 1 == NPARAM


def unpack(theta: np.ndarray):
    t = np.asarray(theta, dtype=np.float64)
    return (t[_OFF_W1:_OFF_B1].reshape(H, 3), t[_OFF_B1:_OFF_W2],
            t[_OFF_W2:_OFF_B2].reshape(H, H), t[_OFF_B2:_OFF_W3],
            t[_OFF_W3:_OFF_B3], t[_OFF_B3])


def pack(W1, b1, W2, b2, w3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2),
                           np.ravel(w3), np.atleast_1d(b3)]).astype(np.float64)


def inputs(f1, f2, f3, mu, sd) -> np.ndarray:
    """Network input rows: standardised log2(1 + feature)."""
    F = np.stack([np.asarray(f1), np.asarray(f2), np.asarray(f3)], axis=1).astype(np.float64)
    return (np.log2(1.0 + F) - np.asarray(mu, dtype=np.float64)) / np.asarray(sd, dtype=np.float64)


def targets(n, f2, f3):
    """(t, w): fraction of the interval [maxB, UB] reached, and sample weight."""
    n = np.asarray(n, dtype=np.float64)
    lo = np.asarray(f3, dtype=np.float64)
    hi = np.asarray(f2, dtype=np.float64)
    w = (hi > lo).astype(np.float64)
    t = np.where(hi > lo, (n - lo) / np.where(hi > lo, hi - lo, 1.0), 0.0)
    return t, w


def forward(theta, X):
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    rho = 1.0 / (1.0 + np.exp(-z))
    return rho, (X, a1, h1, a2, h2, z)


def loss(theta, X, t, w) -> float:
    rho, _ = forward(theta, X)
    W = float(np.sum(w))
    return float(np.sum(w * (rho - t) ** 2) / W) if W > 0 else 0.0


def loss_and_grad(theta, X, t, w):
    """Loss and its gradient with respect to the flat parameter vector."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    rho, (X, a1, h1, a2, h2, z) = forward(theta, X)
    Wsum = float(np.sum(w))
    if Wsum == 0:
        return 0.0, np.zeros(NPARAM)
    L = float(np.sum(w * (rho - t) ** 2) / Wsum)
    d_rho = 2.0 * w * (rho - t) / Wsum            # dL/drho
    d_z = d_rho * rho * (1.0 - rho)               # logistic derivative
    g_w3 = h2.T @ d_z
    g_b3 = np.sum(d_z)
    d_h2 = np.outer(d_z, w3)
    d_a2 = d_h2 * (a2 > 0)
    g_W2 = d_a2.T @ h1
    g_b2 = np.sum(d_a2, axis=0)
    d_h1 = d_a2 @ W2
    d_a1 = d_h1 * (a1 > 0)
    g_W1 = d_a1.T @ X
    g_b1 = np.sum(d_a1, axis=0)
    return L, pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)


def adam_step(theta, grad, m, v, step: int, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1); ``step`` counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def predict(theta, mu, sd, f1, f2, f3) -> np.ndarray:
    """Predicted nnz(C_i) as a real number in [maxB_i, UB_i]."""
    rho, _ = forward(theta, inputs(f1, f2, f3, mu, sd))
    f2 = np.asarray(f2, dtype=np.float64)
    f3 = np.asarray(f3, dtype=np.float64)
    return f3 + rho * (f2 - f3)
