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
    X = rng.uniform(0, 1, (n, b.BC_MLP_IN)).astype(np.float32)
    Y = (3 + 4 * X[:, [0, 1, 2, 3, 4, 0, 1, 2, 3]] - 2 * X[:, [3, 4, 0, 1, 2, 2, 4, 0, 1]]
         + rng.normal(0, 0.1, (n, b.BC_MLP_OUT))).astype(np.float32)
    M = (rng.uniform(0, 1, (n, b.BC_MLP_OUT)) < 0.9).astype(np.uint8)
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
        assert len(X) >= 9 and np.isfinite(X).all()
        assert (X >= 0).all() and (X[:, :4] <= 1.0 + 1e-6).all()
        _check_samples(Y)
        ref, _ = oracle.bc(g, srcs)
        assert_bc_close(G.scores(), ref)  # three variants / options per step, one result


def _check_samples(Y):
    # every sample times one choice: three finite outputs of one group
    fin = np.isfinite(Y)
    groups = fin.reshape(len(Y), 3, 3)
    assert (fin.sum(axis=1) == 3).all()
    assert (groups.all(axis=2).sum(axis=1) == 1).all()
    per = groups.all(axis=2).sum(axis=0)
    assert (per > 0).all(), per  # discover, path-count and backward samples


def test_collect_level_times_deep_grid():
    # a few hundred levels, each run three times with undo steps in between
    g = W.grid(48, 0.10, 0.0, seed=5)
    srcs = W.choose_sources(g, 70, seed=4)
    say("[collect] grid48")
    with b.Graph(g) as G:
        X, Y = G.collect_level_times(srcs)
        assert len(X) > 300
        _check_samples(Y)
        ref, _ = oracle.bc(g, srcs)
        assert_bc_close(G.scores(), ref)


def _weights_or_train(g):
    if os.path.exists(WEIGHTS):
        return np.load(WEIGHTS)
    with b.Graph(g) as G:
        X, Y = G.collect_level_times(W.choose_sources(g, 128, seed=11))
    M = np.isfinite(Y).astype(np.uint8)
    w, _ = b.bc_mlp_train(mlp_ref.init(0), X, np.nan_to_num(Y), M, 1500, 3e-3)
    return w


def _constant_policy(fwd, sig, bwd):
    # zero layers, output biases only: the network predicts b3 at every level
    w = np.zeros(b.BC_MLP_PARAMS, np.float32)
    b3 = np.ones(b.BC_MLP_OUT, np.float32)
    b3[fwd] = b3[3 + sig] = b3[6 + bwd] = 0.0
    w[-b.BC_MLP_OUT:] = b3
    return w


@pytest.mark.parametrize("flags", [0, b.BC_RUN_NO_BLOCKS])
def test_learned_summation_options_take_effect(flags):
    # the network's path-count / backward choices replace the run's rule:
    # arc counts of those phases follow the option (the (entry, source)
    # summation scans an entry's arcs once per source), scores keep their bits
    g = W.rmat(12, 16, seed=21)
    srcs = W.choose_sources(g, 640, seed=4)
    say(f"[learned summation] rmat12 flags={flags}")
    with b.Graph(g) as G:
        def run(**kw):
            G.run(srcs, batch=64, flags=flags, **kw)
            st = G.stats()
            return G.scores().copy(), st["phase_arcs"][2:4]
        bits_p, arcs_p = run(policy=b.BC_POLICY_HEURISTIC, lanes_per_entry=-1.0)
        bits_i, arcs_i = run(policy=b.BC_POLICY_HEURISTIC, lanes_per_entry=65.0)
        assert np.array_equal(bits_p.view(np.uint64), bits_i.view(np.uint64))
        assert arcs_p != arcs_i
        G.load_policy(_constant_policy(b.BC_VARIANT_PUSH_TPV, b.BC_LB_ITEMS, b.BC_LB_ITEMS))
        bits, arcs = run(policy=b.BC_POLICY_MLP, lanes_per_entry=-1.0)
        assert arcs == arcs_i and np.array_equal(bits.view(np.uint64), bits_p.view(np.uint64))
        G.load_policy(_constant_policy(b.BC_VARIANT_PULL, b.BC_LB_PACKED, b.BC_LB_PACKED))
        bits, arcs = run(policy=b.BC_POLICY_MLP, lanes_per_entry=65.0)
        assert arcs == arcs_p and np.array_equal(bits.view(np.uint64), bits_p.view(np.uint64))
        G.load_policy(_constant_policy(b.BC_VARIANT_PULL, b.BC_LB_ITEMS, b.BC_LB_PACKED))
        bits, arcs = run(policy=b.BC_POLICY_MLP)
        assert arcs[0] == arcs_i[0] and arcs[1] == arcs_p[1]
        assert np.array_equal(bits.view(np.uint64), bits_p.view(np.uint64))


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
