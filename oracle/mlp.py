"""FP64 reference of the cost-model MLP (TEST INFRASTRUCTURE ONLY).

Network: x (F features) -> ReLU(W1 x + b1) (H1) -> ReLU(W2 h1 + b2) (H2)
-> y = W3 h2 + b3 (one output).  Loss: mean squared error over the batch,
L = (1/B) sum_b (y_b - t_b)^2.  Optimiser: Adam (Kingma and Ba, 2015):
m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2, w <- w - lr * mhat / (sqrt(vhat) + eps)
with mhat = m / (1 - b1^step), vhat = v / (1 - b2^step).

Weights are row-major: W1 is H1 x F, W2 is H2 x H1, W3 is 1 x H2.
Parity: pinned by central finite differences and by the linear special case
in tests/test_oracle_mlp.py.
"""
from __future__ import annotations

import numpy as np

NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def init(F: int, H1: int = 64, H2: int = 64, seed: int = 0):
    """He-style random initialisation (seeded)."""
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.normal(0, np.sqrt(2.0 / F), size=(H1, F)),
        "b1": np.zeros(H1),
        "W2": rng.normal(0, np.sqrt(2.0 / H1), size=(H2, H1)),
        "b2": np.zeros(H2),
        "W3": rng.normal(0, np.sqrt(1.0 / H2), size=(1, H2)),
        "b3": np.zeros(1),
    }


def forward(p, X):
    """X: B x F.  Returns (y of shape B, cache)."""
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ p["W3"].T + p["b3"])[:, 0]
    return y, (X, z1, h1, z2, h2)


def loss(p, X, t):
    y, _ = forward(p, X)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def backward(p, cache, y, t):
    """Gradients of the mean squared error with respect to every weight."""
    X, z1, h1, z2, h2 = cache
    B = X.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / B          # B
    g = {}
    g["W3"] = dy[None, :] @ h2                                      # 1 x H2
    g["b3"] = np.array([dy.sum()])
    dh2 = dy[:, None] @ p["W3"]                                     # B x H2
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return g


def adam_step(p, g, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; `state` holds m, v and the step count."""
    state["step"] = state.get("step", 0) + 1
    s = state["step"]
    for k in NAMES:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = beta1 * m + (1 - beta1) * g[k]
        v[...] = beta2 * v + (1 - beta2) * g[k] ** 2
        mh = m / (1 - beta1 ** s)
        vh = v / (1 - beta2 ** s)
        p[k] -= lr * mh / (np.sqrt(vh) + eps)
    return p
