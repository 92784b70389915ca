"""Pins for the float64 reference of the policy network (CPU only): its
hand-written back-propagation must agree with central finite differences of
the loss, and with an independent autograd (torch float64 on the CPU)."""
from __future__ import annotations

import numpy as np

from oracle import mlp_ref


def _data(n=40, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, (n, mlp_ref.I))
    Y = rng.normal(5, 2, (n, mlp_ref.O))
    M = (rng.uniform(0, 1, (n, mlp_ref.O)) < 0.8).astype(np.uint8)
    M[0] = 1
    return X, Y, M


def test_gradient_matches_central_differences():
    X, Y, M = _data()
    w = mlp_ref.init(1).astype(np.float64)
    w += np.random.default_rng(2).normal(0, 0.05, w.size)  # move off exact zeros of the biases
    L, g = mlp_ref.loss_grad(w, X, Y, M)
    assert abs(L - mlp_ref.loss(w, X, Y, M)) < 1e-12
    rng = np.random.default_rng(4)
    idx = rng.choice(w.size, 120, replace=False)
    h = 1e-6
    for i in idx:
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        fd = (mlp_ref.loss(wp, X, Y, M) - mlp_ref.loss(wm, X, Y, M)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_gradient_matches_torch_autograd():
    import torch
    X, Y, M = _data(60, 9)
    w = mlp_ref.init(5).astype(np.float64)
    L, g = mlp_ref.loss_grad(w, X, Y, M)
    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    o = 0
    def take(k):
        nonlocal o
        t = wt[o:o + k]; o += k
        return t
    W1 = take(32 * 5).reshape(32, 5); b1 = take(32); W2 = take(1024).reshape(32, 32); b2 = take(32)
    W3 = take(9 * 32).reshape(9, 32); b3 = take(9)
    assert o == w.size
    x = torch.tensor(X); y = torch.tensor(Y); m = torch.tensor(M, dtype=torch.float64)
    h1 = torch.relu(x @ W1.T + b1)
    h2 = torch.relu(h1 @ W2.T + b2)
    out = h2 @ W3.T + b3
    lt = (m * (out - y) ** 2).sum() / (2 * m.sum())
    lt.backward()
    assert abs(lt.item() - L) < 1e-12
    np.testing.assert_allclose(wt.grad.numpy(), g, rtol=1e-10, atol=1e-13)


def test_planted_gradient_mistake_is_caught():
    # dropping the ReLU mask of the first layer must be visible to the check
    X, Y, M = _data()
    w = mlp_ref.init(1).astype(np.float64)
    W1, b1, W2, b2, W3, b3 = mlp_ref.unpack(w)
    _, g = mlp_ref.loss_grad(w, X, Y, M)
    y, (Xf, z1, h1, z2, h2) = mlp_ref.forward(w, X)
    d3 = M * (y - Y) / M.sum()
    d2 = (d3 @ W3) * (z2 > 0)
    wrong_gW1 = ((d2 @ W2)).T @ Xf  # mask omitted
    assert not np.allclose(wrong_gW1.ravel(), g[:32 * 5], rtol=1e-6, atol=1e-9)
