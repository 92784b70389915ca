"""GPU tests of the launch-configuration autotuner: it returns one of its
candidates, leaves the scores reset, and a tuned run gives the same bits as
a default run of the same batch width and replica count (policy,
workgroups, chunk length, WPV threshold and summation never change a sum or
its order) and matches the oracle.  The
tune cache returns a kept result without timing, also to a new handle of the
same graph after a save and load, and BC_TUNE_FRESH tunes again."""
from __future__ import annotations

import time

import numpy as np
import pytest

import oracle
from gpu_util import assert_bc_close, say
from paper_2008_05718_amd import binding as b
from paper_2008_05718_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_candidates_and_same_bits():
    g = W.rmat(14, 16, seed=5)
    srcs = W.choose_sources(g, 384, seed=6)
    say("[autotune] rmat14")
    with b.Graph(g) as G:
        with pytest.raises(b.BCError):
            G.run(srcs, flags=b.BC_RUN_TUNED)
        best = G.autotune(srcs[:128])
        say("  tuned", best)
        assert best["batch"] in (1, 8, 16, 32, 64)
        assert best["policy"] in (b.BC_POLICY_HEURISTIC, b.BC_POLICY_MLP)
        assert best["chunk_steps"] in (8, 16, 32)
        assert best["wpv_degree"] in (12.0, 24.0, 48.0)
        assert best["grid_blocks"] >= 1
        assert best["replicas"] in (4, 8, 16)  # half, default (2^14 vertices: 8) or twice
        assert not G.scores().any()
        # same width and replica count, default policy and launch shape
        G.run(srcs, batch=best["batch"], replicas=best["replicas"])
        ref_bits = G.scores().copy()
        G.run(srcs, flags=b.BC_RUN_TUNED)
        got = G.scores()
        assert np.array_equal(got.view(np.uint64), ref_bits.view(np.uint64))
    ref, _ = oracle.bc(g, srcs)
    assert_bc_close(got, ref)


def test_autotune_rejects_bad_sample():
    g = W.grid(8)
    with b.Graph(g) as G:
        with pytest.raises(b.BCError):
            G.autotune(np.array([], np.int32))
        with pytest.raises(b.BCError):
            G.autotune(np.array([0, 64], np.int32))


def test_tune_cache_hit_save_load_and_fresh(tmp_path):
    g = W.rmat(12, 16, seed=8)
    srcs = W.choose_sources(g, 256, seed=9)
    path = str(tmp_path / "tune.json")
    b.bc_tune_cache_clear()
    say("[autotune] cache, rmat12")
    with b.Graph(g) as G:
        t = time.perf_counter()
        best = G.autotune(srcs[:128])
        t_tune = time.perf_counter() - t
        assert b.bc_tune_cache_size() == 1
        t = time.perf_counter()
        again = G.autotune(srcs[:128])
        t_hit = time.perf_counter() - t
        say(f"  tuned in {t_tune:.2f}s, cached answer in {t_hit:.4f}s: {best}")
        assert again == best and t_hit < t_tune / 5
        b.bc_tune_cache_save(path)
    b.bc_tune_cache_clear()
    b.bc_tune_cache_load(path)
    with b.Graph(g) as H:  # a new handle of the same graph
        t = time.perf_counter()
        assert H.autotune(srcs[:128]) == best
        assert time.perf_counter() - t < t_tune / 5
        H.run(srcs, flags=b.BC_RUN_TUNED)
        got = H.scores().copy()
        H.run(srcs, batch=best["batch"], replicas=best["replicas"])
        assert np.array_equal(got.view(np.uint64), H.scores().view(np.uint64))
        H.autotune(srcs[:64])  # another sample: tuned and kept beside the first
        assert b.bc_tune_cache_size() == 2
        H.autotune(srcs[:64], flags=b.BC_TUNE_FRESH)  # tuned again, replaces its entry
        assert b.bc_tune_cache_size() == 2
    b.bc_tune_cache_clear()


def test_replicas_option_repeats_and_agrees():
    # the number of concurrent state machines of a single graph changes only
    # how batch results are grouped: each count repeats bit for bit, all agree
    # with the oracle
    g = W.rmat(13, 16, seed=31)
    srcs = W.choose_sources(g, 640, seed=7)
    ref, _ = oracle.bc(g, srcs)
    say("[replicas] rmat13")
    with b.Graph(g) as G:
        for r in (1, 2, 5, 16, 2):
            G.run(srcs, batch=64, replicas=r)
            got = G.scores().copy()
            G.run(srcs, batch=64, replicas=r)
            assert np.array_equal(G.scores().view(np.uint64), got.view(np.uint64)), r
            assert_bc_close(got, ref)
