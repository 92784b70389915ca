"""GPU tests of the policy network: the HIP loss/gradient/prediction kernels
against the float64 CPU reference (rel 1e-4, abs 1e-6), training, timing
collection, and the learned policy's effect (speed only: BC bits must not
change)."""
from __future__ import annotations

import os
import time

import numpy as np
import pytest

import oracle
from gpu_util import assert_bc_close, say
from oracle import mlp_ref
from paper_2008_05718_amd import binding as b
from paper_2008_05718_amd import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(os.path.dirname(HERE), "paper_2008_05718_amd", "policy_weights.npy")


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, (n, 5)).astype(np.float32)
    Y = (3 + 4 * X[:, [0, 1, 2]] - 2 * X[:, [3, 4, 0]] + rng.normal(0, 0.1, (n, 3))).astype(np.float32)
    M = (rng.uniform(0, 1, (n, 3)) < 0.9).astype(np.uint8)
    M[0] = 1
    return X, Y, M


def test_loss_gradient_matches_cpu_reference():
    say("[mlp grad]")
    X, Y, M = _data(700, 1)
    w = mlp_ref.init(3)
    loss, g = b.bc_mlp_loss_grad(w, X, Y, M)
    L, G = mlp_ref.loss_grad(w.astype(np.float64), X.astype(np.float64), Y.astype(np.float64), M)
    assert abs(loss - L) <= 1e-4 * abs(L) + 1e-6
    np.testing.assert_allclose(g, G, rtol=1e-4, atol=1e-6)


def test_predict_matches_cpu_reference():
    X, Y, M = _data(300, 2)
    w = mlp_ref.init(4)
    got = b.bc_mlp_predict(w, X)
    want, _ = mlp_ref.forward(w.astype(np.float64), X.astype(np.float64))
    np.testing.assert_allclose(got, want, rtol=1e-4, atol=1e-5)


def test_training_reduces_loss():
    X, Y, M = _data(2000, 3)
    w0 = mlp_ref.init(5)
    l0, _ = b.bc_mlp_loss_grad(w0, X, Y, M)
    w, l1 = b.bc_mlp_train(w0, X, Y, M, 600, 3e-3)
    assert np.isfinite(w).all()
    assert l1 < 0.1 * l0, (l0, l1)
    assert abs(l1 - mlp_ref.loss(w.astype(np.float64), X, Y, M)) <= 1e-3 * l1 + 1e-6


def test_invalid_inputs_rejected():
    X, Y, M = _data(10, 4)
    w = mlp_ref.init(0)
    bad = w.copy()
    bad[7] = np.nan
    with pytest.raises(b.BCError):
        b.bc_mlp_train(bad, X, Y, M, 5, 1e-3)
    with pytest.raises(b.BCError):
        b.bc_mlp_loss_grad(w, X, Y, np.zeros_like(M))
    g = W.grid(6)
    with b.Graph(g) as G:
        with pytest.raises(b.BCError):
            G.load_policy(bad)
        with pytest.raises(b.BCError):
            G.load_policy(w[:100])


def test_collect_level_times_keeps_results():
    g = W.rmat(12, 16, seed=31)
    srcs = W.choose_sources(g, 130, seed=2)
    say("[collect] rmat12")
    with b.Graph(g) as G:
        X, Y = G.collect_level_times(srcs)
        assert len(X) >= 3 and np.isfinite(X).all() and np.isfinite(Y).all()
        assert (X >= 0).all() and (X[:, :4] <= 1.0 + 1e-6).all()
        ref, _ = oracle.bc(g, srcs)
        assert_bc_close(G.scores(), ref)  # three variants per level, one result


def test_collect_level_times_deep_grid():
    # a few hundred levels, each run three times with undo steps in between
    g = W.grid(48, 0.10, 0.0, seed=5)
    srcs = W.choose_sources(g, 70, seed=4)
    say("[collect] grid48")
    with b.Graph(g) as G:
        X, Y = G.collect_level_times(srcs)
        assert len(X) > 100 and np.isfinite(Y).all()
        ref, _ = oracle.bc(g, srcs)
        assert_bc_close(G.scores(), ref)


def _weights_or_train(g):
    if os.path.exists(WEIGHTS):
        return np.load(WEIGHTS)
    with b.Graph(g) as G:
        X, Y = G.collect_level_times(W.choose_sources(g, 128, seed=11))
    w, _ = b.bc_mlp_train(mlp_ref.init(0), X, Y, np.ones_like(Y, dtype=np.uint8), 1500, 3e-3)
    return w


def test_learned_policy_same_bits_and_its_gain():
    # held-out graph (not a training graph): R-MAT scale 16, seed 9
    g = W.rmat(16, 16, seed=9)
    srcs = W.choose_sources(g, 512, seed=3)
    w = _weights_or_train(W.rmat(14, 16, seed=130))
    say("[learned policy] rmat16")
    with b.Graph(g) as G:
        G.run(srcs, batch=64, policy=b.BC_POLICY_HEURISTIC)
        h_bits = G.scores().copy()
        G.load_policy(w)
        G.run(srcs, batch=64, policy=b.BC_POLICY_MLP)
        m_bits = G.scores().copy()
        assert np.array_equal(h_bits.view(np.uint64), m_bits.view(np.uint64))
        # best of 7 runs each, the policies taken in turn so that drift of
        # the device clock or of other load hits them alike
        pols = (b.BC_POLICY_HEURISTIC, b.BC_POLICY_MLP, b.BC_POLICY_FORCE_PUSH_TPV, b.BC_POLICY_FORCE_PULL)
        times = {p: 1e30 for p in pols}
        for _ in range(7):
            for pol in pols:
                t = time.perf_counter()
                # the general engine, whose per-level times the network was trained on
                G.run(srcs, batch=64, policy=pol, flags=b.BC_RUN_NO_BLOCKS)
                times[pol] = min(times[pol], time.perf_counter() - t)
        gain = times[b.BC_POLICY_HEURISTIC] / times[b.BC_POLICY_MLP]
        say(f"  heuristic {times[1]*1e3:.2f} ms, mlp {times[2]*1e3:.2f} ms (gain x{gain:.3f}), "
            f"tpv {times[3]*1e3:.2f} ms, pull {times[5]*1e3:.2f} ms")
        # speed is the only thing the network may change: on a graph it was
        # not trained on it must be at least as fast as the rule it replaces,
        # up to 2 % of timing noise
        assert gain >= 0.98
