"""The autotuner's tune cache as a file (bc_tune_cache_save / _load /
_clear / _size): the JSON format round-trips, entries with the same key
replace each other, malformed files are refused with BC_ERR_INVALID_ARG
and add nothing.  None of these calls touches the GPU."""
from __future__ import annotations

import json

import pytest

from paper_2008_05718_amd import binding as b

ENTRY = {"device": "gfx950:256", "graph": "00000000000000ab", "sample": "0123456789abcdef",
         "base": "fedcba9876543210", "batch": 32, "policy": 1, "grid_blocks": 192, "chunk_steps": 8,
         "wpv_degree": 12.0, "lanes_per_entry": -1.0, "policy_margin": 0.25, "replicas": 8, "flags": 0}


def _write(path, obj):
    with open(path, "w") as f:
        f.write(obj if isinstance(obj, str) else json.dumps(obj))


@pytest.fixture(autouse=True)
def _empty_cache():
    b.bc_tune_cache_clear()
    yield
    b.bc_tune_cache_clear()


def test_round_trip_and_replacement(tmp_path):
    e2 = dict(ENTRY, graph="00000000000000ac", batch=64, policy=2, lanes_per_entry=4.0, extra={"ignored": [1, 2]})
    src = tmp_path / "in.json"
    _write(src, {"format": "bc-autotune-cache", "version": 1, "comment": "x", "entries": [ENTRY, e2]})
    b.bc_tune_cache_load(str(src))
    assert b.bc_tune_cache_size() == 2
    b.bc_tune_cache_load(str(src))  # same keys: replaced, not added
    assert b.bc_tune_cache_size() == 2
    out = tmp_path / "out.json"
    b.bc_tune_cache_save(str(out))
    got = json.load(open(out))
    assert got["format"] == "bc-autotune-cache" and got["version"] == 1
    want = [ENTRY, {k: v for k, v in e2.items() if k != "extra"}]
    assert got["entries"] == want
    # a changed value under an existing key replaces it
    _write(src, {"entries": [dict(ENTRY, batch=8)]})
    b.bc_tune_cache_load(str(src))
    b.bc_tune_cache_save(str(out))
    got = json.load(open(out))["entries"]
    assert len(got) == 2 and got[0]["batch"] == 8
    b.bc_tune_cache_clear()
    assert b.bc_tune_cache_size() == 0
    b.bc_tune_cache_save(str(out))
    assert json.load(open(out))["entries"] == []


@pytest.mark.parametrize("text", [
    "",
    "[]",
    "{}",
    '{"entries": 3}',
    '{"entries": [',
    '{"entries": [{"device": "gfx950:256"}]}',
    '{"entries": [' + json.dumps(dict(ENTRY, graph="not-hex")) + "]}",
    '{"entries": [' + json.dumps(dict(ENTRY, batch="64")) + "]}",
    '{"entries": [' + json.dumps(ENTRY) + ", 5]}",
    '{"entries": [' + json.dumps(ENTRY) + "]",
])
def test_malformed_files_are_refused(tmp_path, text):
    p = tmp_path / "bad.json"
    _write(p, text)
    with pytest.raises(b.BCError) as e:
        b.bc_tune_cache_load(str(p))
    assert e.value.status == 1
    assert b.bc_tune_cache_size() == 0


def test_missing_file_and_null_path(tmp_path):
    with pytest.raises(b.BCError) as e:
        b.bc_tune_cache_load(str(tmp_path / "nope.json"))
    assert e.value.status == 1
    with pytest.raises(b.BCError) as e:
        b.bc_tune_cache_save(str(tmp_path / "no_dir" / "x.json"))
    assert e.value.status == 1
    L = b.lib()
    assert L.bc_tune_cache_load(None) == 1
    assert L.bc_tune_cache_save(None) == 1
