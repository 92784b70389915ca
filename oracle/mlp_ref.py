"""Float64 CPU reference of the level-policy network -- TEST INFRASTRUCTURE ONLY.

Only tests may import it.  The network maps 5 level features through two
32-unit ReLU layers to 9 outputs (predicted log2 times: three discover
variants, three summation options of the path-count step, three of the
backward step).  Parameters are packed as W1[32][5], b1[32], W2[32][32],
b2[32], W3[9][32], b3[9].  Loss over samples (x, y, mask):

    L = sum mask * (f(x) - y)^2 / (2 * sum mask)

``loss_grad`` back-propagates by hand (chain rule written out); it is pinned
by central finite differences in tests/test_mlp_ref.py.
"""
from __future__ import annotations

import numpy as np

H, I, O = 32, 5, 9
N_PARAMS = H * I + H + H * H + H + O * H + O


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    o = 0
    W1 = w[o:o + H * I].reshape(H, I); o += H * I
    b1 = w[o:o + H]; o += H
    W2 = w[o:o + H * H].reshape(H, H); o += H * H
    b2 = w[o:o + H]; o += H
    W3 = w[o:o + O * H].reshape(O, H); o += O * H
    b3 = w[o:o + O]; o += O
    assert o == N_PARAMS
    return W1, b1, W2, b2, W3, b3


def forward(w, X):
    W1, b1, W2, b2, W3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3.T + b3
    return y, (X, z1, h1, z2, h2)


def loss(w, X, Y, mask):
    y, _ = forward(w, X)
    m = np.asarray(mask, dtype=np.float64)
    return float(np.sum(m * (y - Y) ** 2) / (2.0 * m.sum()))


def loss_grad(w, X, Y, mask):
    W1, b1, W2, b2, W3, b3 = unpack(w)
    y, (X, z1, h1, z2, h2) = forward(w, X)
    m = np.asarray(mask, dtype=np.float64)
    cnt = m.sum()
    d3 = m * (y - np.asarray(Y, dtype=np.float64)) / cnt          # dL/dy
    gW3 = d3.T @ h2
    gb3 = d3.sum(axis=0)
    d2 = (d3 @ W3) * (z2 > 0)                                    # dL/dz2
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (z1 > 0)                                    # dL/dz1
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return float(np.sum(m * (y - Y) ** 2) / (2.0 * cnt)), g


def init(seed: int = 0):
    """He-style random initialisation (float32 values)."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, np.sqrt(2.0 / I), H * I), np.zeros(H),
             rng.normal(0, np.sqrt(2.0 / H), H * H), np.zeros(H),
             rng.normal(0, np.sqrt(1.0 / H), O * H), np.zeros(O)]
    return np.concatenate(parts).astype(np.float32)
