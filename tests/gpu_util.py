"""Helpers for the GPU parity tests (comparison against the CPU oracle)."""
from __future__ import annotations

import sys

import numpy as np

import oracle
from paper_2008_05718_amd import binding as b

REL = 1e-10  # FP64 tolerance on BC and delta, relative per vertex


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def assert_bc_close(got, ref, rel=REL, what="bc"):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape
    zero = ref == 0
    assert np.all(got[zero] == 0), f"{what}: nonzero where the oracle is exactly zero"
    nz = ~zero
    if nz.any():
        err = np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])
        i = int(np.argmax(err))
        assert err[i] <= rel, f"{what}: rel err {err[i]:.3e} at {np.nonzero(nz)[0][i]}"


def check_detail(g, det, s, rel=REL):
    """d bit-exact; uint64 sigma bit-exact; FP64 sigma and delta within rel."""
    o = oracle.source(g, int(s))
    assert det["mode"] == o.mode, ("mode", det["mode"], o.mode)
    # weighted graphs: int64 distances
    np.testing.assert_array_equal(det["d64"] if o.d.dtype == np.int64 else det["d"], o.d)
    reached = o.d >= 0
    if o.mode == 0:
        np.testing.assert_array_equal(det["sigma_u64"], o.sigma_u64)
    else:
        mant = det["sigma_mant"][reached].astype(np.longdouble)
        ex = det["sigma_exp"][reached].astype(np.int64)
        got = np.ldexp(mant, ex)
        want = o.sigma_ld[reached]
        err = np.abs(got - want) / want
        assert float(err.max()) <= rel, ("sigma f64", float(err.max()))
    inner = o.d >= 1  # reached, not the source (weights are >= 1)
    assert_bc_close(det["delta"][inner], o.delta[inner], rel, what="delta")
    assert np.all(det["delta"][~inner] == 0)


def run_bc(g, sources=None, **opts):
    with b.Graph(g) as G:
        G.run(sources, **opts)
        return G.scores(), G.stats()
