"""Deep traversals: thousands of levels, path counts far beyond uint64 and
beyond the FP64 exponent range, under hipGraph capture (the default launch
configuration captures chunks of level steps).

* A chain of diamonds has closed-form path counts 2^j (exact in any binary
  floating-point format), so the per-level power-of-two rescaling of the
  FP64 mode is checked bit for bit, and its dependencies against the closed
  form of Eq. 2 on a chain.
* A chain long enough that one level holds counts 2^2000 apart cannot be
  represented with one power of two per level: the run must report
  BC_ERR_SIGMA_RANGE instead of returning wrong scores.
* The intact 600 x 600 grid from a corner has sigma(i, j) = C(i + j, i), up
  to about 2^1193 at 1199 levels.
* The damaged 1024 x 1024 grid without shortcuts (about 2,000 levels) in the
  benchmark's launch configuration, against the long-double oracle.
"""
from __future__ import annotations

import math
import os
import time

import numpy as np
import pytest

import oracle
from gpu_util import REL, assert_bc_close, check_detail, say
from paper_2008_05718_amd import binding as b
from paper_2008_05718_amd import workloads as W

pytestmark = pytest.mark.gpu
WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2008_05718_amd",
                       "policy_weights.npy")


def diamond_chain(D: int, tail: int = 0, extra_path: int = 0):
    """Source 0, then D diamonds: c_{j-1} - {a_j, b_j} - c_j (c_{-1} = 0),
    with a_j = 3j + 1, b_j = 3j + 2, c_j = 3j + 3; plus a plain path of
    ``tail`` vertices hanging off vertex 0 (ids 3D + 1 ..), plus a separate
    path component of ``extra_path`` vertices (the last ids)."""
    us, vs = [], []
    prev = 0
    for j in range(D):
        a, bb, c = 3 * j + 1, 3 * j + 2, 3 * j + 3
        us += [prev, prev, a, bb]
        vs += [a, bb, c, c]
        prev = c
    prev = 0
    for i in range(tail):
        v = 3 * D + 1 + i
        us.append(prev)
        vs.append(v)
        prev = v
    base = 3 * D + 1 + tail
    for i in range(extra_path - 1):
        us.append(base + i)
        vs.append(base + i + 1)
    n = base + extra_path
    return W.csr_from_edges(n, np.array(us, np.int64), np.array(vs, np.int64), name=f"diamonds{D}_t{tail}")


def _exact_sigma(det):
    """Path counts as Python integers from mantissa * 2^exp (exact: every
    count here is a power of two or has few significant bits)."""
    out = []
    for m, e in zip(det["sigma_mant"], det["sigma_exp"]):
        fm, fe = math.frexp(float(m))
        out.append(int(fm * 2 ** 53) * 2 ** (int(e) + fe - 53) if m != 0 else 0)
    return out


@pytest.mark.parametrize("batch", [1, 64])
def test_diamond_chain_rescaled_counts_exact(batch):
    # 1100 diamonds: counts up to 2^1100 on 2200 levels, beyond the largest
    # double, so the per-level power of two must have been applied; a 2200
    # vertex tail keeps count 1 on the same levels (spread 1100 bits)
    D, tail = 1100, 2200
    g = diamond_chain(D, tail)
    with b.Graph(g) as G:
        det = G.detail([0, 1, 3 * D + tail], dump_index=0, batch=batch)
        st = G.stats()
    say(f"[diamonds K={batch}] mode {det['mode']} levels {det['n_levels']} max_levels {st['max_levels']}")
    assert det["mode"] == 1 and det["n_levels"] == 2 * D + 1
    sig = _exact_sigma(det)
    d = det["d"]
    for j in range(D):
        a, c = 3 * j + 1, 3 * j + 3
        assert d[a] == 2 * j + 1 and d[c] == 2 * j + 2
        assert sig[a] == 2 ** j and sig[a + 1] == 2 ** j and sig[c] == 2 ** (j + 1), j
    # counts up to 2^1100 are beyond the double range: they were stored
    # divided by a power of two (sigma = mantissa * 2^exp, exp > 0)
    assert max(sig) == 2 ** D and max(int(e) for e in det["sigma_exp"]) > 0
    assert all(sig[3 * D + 1 + i] == 1 for i in range(tail))
    # Eq. 2 on the chain: delta(c_j) = 3 (D - 1 - j), delta(a_j) = (1 + delta(c_j)) / 2,
    # tail vertex i: tail - 1 - i
    want = np.zeros(g.n)
    for j in range(D):
        dc = 3.0 * (D - 1 - j)
        want[3 * j + 3] = dc
        want[3 * j + 1] = want[3 * j + 2] = (1.0 + dc) / 2.0
    for i in range(tail):
        want[3 * D + 1 + i] = float(tail - 1 - i)
    assert_bc_close(det["delta"][1:], want[1:], what="delta")
    assert det["delta"][0] == 0
    check_detail(g, det, 0)


def test_diamond_chain_beyond_one_scale_reports_range_error():
    # counts 2^2000 and 1 on one level: no single power of two keeps both in
    # range, so the run fails with BC_ERR_SIGMA_RANGE (and the handle stays
    # usable for a graph region that fits)
    D = 2000
    g = diamond_chain(D, 2 * D, extra_path=9)
    other = g.n - 4  # in the separate path component
    for batch in (1, 64):
        with b.Graph(g) as G:
            with pytest.raises(b.BCError) as ei:
                G.run([0], batch=batch)
            assert ei.value.status == 5, ei.value
            say(f"[diamonds {D} K={batch}] {ei.value}")
            G.run([other], batch=batch)
            got = G.scores()
        ref, _ = oracle.bc(g, [other])
        assert_bc_close(got, ref)


@pytest.mark.parametrize("batch", [1, 64])
def test_intact_grid_corner_binomial_counts(batch):
    L = 600
    g = W.grid(L)
    srcs = np.array([0, L - 1, (L // 2) * L + L // 2, L * L - 1], np.int32)
    with b.Graph(g) as G:
        det = G.detail(srcs, dump_index=0, batch=batch)
        say(f"[grid{L} K={batch}] levels {det['n_levels']}, max exponent {int(det['sigma_exp'].max())}")
        assert det["n_levels"] == 2 * L - 1
        # corner source: d(i, j) = i + j, sigma(i, j) = C(i + j, i); check a
        # diagonal of vertices against exact binomials (relative 2^-50)
        for i in range(0, L, 37):
            for j in (0, i, L - 1):
                v = i * L + j
                assert det["d"][v] == i + j
                want = math.comb(i + j, i)
                e = int(det["sigma_exp"][v])
                # compare in scaled form to stay inside the double range
                wf = want / (2 ** e) if want.bit_length() - e < 1000 else float("inf")
                assert abs(float(det["sigma_mant"][v]) - wf) <= 2.0 ** -50 * abs(wf), (i, j)
        check_detail(g, det, 0)
        det2 = G.detail(srcs, dump_index=2, batch=batch)
        check_detail(g, det2, int(srcs[2]))
        got = G.scores()
    ref, modes = oracle.bc(g, srcs)
    assert modes.all()
    assert_bc_close(got, ref)


def test_grid1024_noshortcut_deep_levels():
    # The damaged grid without shortcuts: about 2,000 levels per source, every
    # source in the scaled FP64 mode, chunks of level steps captured as
    # hipGraphs (the default launch configuration), learned policy.
    t = time.time()
    g, srcs = W.workload("grid1024_noshortcut")
    say(f"[grid1024_noshortcut] n={g.n} m={g.m} sources={len(srcs)} ({time.time() - t:.1f}s)")
    with b.Graph(g) as G:
        if os.path.exists(WEIGHTS):
            G.load_policy(np.load(WEIGHTS))
        t = time.time()
        G.run(srcs, batch=64)
        bits = G.scores().copy()
        st = G.stats()
        say(f"  run {time.time() - t:.2f}s: max levels {st['max_levels']}, f64 sources {st['f64_sources']}, "
            f"launches {st['launches']}")
        assert st["max_levels"] >= 1500
        assert st["f64_sources"] == len(srcs)
        want = float(oracle.path_excess(g, srcs).sum())
        assert abs(float(bits.sum()) - want) <= REL * want
        for k in (0, 131, 255):
            det = G.detail(srcs, dump_index=k, batch=64)
            say(f"  detail #{k}: {det['n_levels']} levels, max exponent {int(det['sigma_exp'].max())}")
            check_detail(g, det, int(srcs[k]))
            assert np.array_equal(G.scores().view(np.uint64), bits.view(np.uint64))
        G.run(srcs[:8], batch=64)
        got = G.scores()
    ref, _ = oracle.bc_sliced(g, srcs[:8], threads=8)
    assert_bc_close(got, ref)
