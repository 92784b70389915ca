"""Host-side logic of bench.py (no GPU): the kernel-source hash that decides
whether committed counter summaries still describe the built kernel, and the
reading of those summaries."""
from __future__ import annotations

import os
import shutil

import bench


def _copy_sources(tmp_path):
    for rel in bench.KERNEL_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, rel), dst)


def _hash_at(root):
    old = bench.ROOT
    try:
        bench.ROOT = str(root)
        return bench.kernel_sources_sha256()
    finally:
        bench.ROOT = old


def test_hash_ignores_comments_but_not_code(tmp_path):
    _copy_sources(tmp_path)
    h0 = _hash_at(tmp_path)
    hip = tmp_path / "paper_2008_05718_amd/csrc/bc_batched.hip"
    text = hip.read_text()
    hip.write_text("// a new comment line\n" + text.replace("\n", "\n  ", 3) + "\n/* trailing\n block */\n")
    assert _hash_at(tmp_path) == h0
    hip.write_text(text.replace("constexpr int kUnroll = BC_UNROLL;", "constexpr int kUnroll = BC_UNROLL + 0;"))
    assert _hash_at(tmp_path) != h0


def test_summaries_are_read_only_for_their_sources():
    # a summary's traffic is used while its recorded hash is the current one
    # and ignored (null in the bench line) once the kernel sources change
    import re
    cur = bench.kernel_sources_sha256()
    tags = {"batch_step_u64": "batch_step<0>", "batch_step_f64": "batch_step<1>"}
    found = 0
    for name in os.listdir(os.path.join(bench.ROOT, "profiles")):
        m = re.match(r"(batch_step_[uf]64)_(\w+)\.md$", name)
        if not m:
            continue
        found += 1
        text = open(os.path.join(bench.ROOT, "profiles", name)).read()
        rec = re.search(r"- kernel_sources_sha256: (\w+)", text).group(1)
        t = bench.measured_traffic(tags[m.group(1)], m.group(2))
        assert (t is not None and t > 0) if rec == cur else t is None, name
    assert found >= 1
    assert bench.measured_traffic("batch_step<0>", "no_such_workload") is None
