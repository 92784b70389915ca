"""GPU tests of the launch-configuration autotuner: it returns one of its
candidates, leaves the scores reset, and a tuned run gives the same bits as
a default run of the same batch width (policy, workgroups, chunk length and
WPV threshold never change a sum or its order) and matches the oracle."""
from __future__ import annotations

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
        assert best["batch"] in (16, 32, 64)
        assert best["policy"] in (b.BC_POLICY_HEURISTIC, b.BC_POLICY_MLP)
        assert best["chunk_steps"] in (8, 16, 32)
        assert best["wpv_degree"] in (12.0, 24.0, 48.0)
        assert best["grid_blocks"] >= 1
        assert not G.scores().any()
        G.run(srcs, batch=best["batch"])  # same width, default policy and launch shape
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
