"""Build libbc.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2008_05718_amd.build

Every translation unit is compiled for gfx950 only, with packed-FP32
instruction selection disabled, then linked into one shared library next to
this file.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libbc.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["bc_api.hip", "bc_plain.hip", "bc_batched.hip", "bc_mlp.hip", "bc_weighted.hip", "bc_wbatch.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(HERE, "..", "include")]


def _compile(src: str, build_dir: str, extra: list) -> str:
    obj = os.path.join(build_dir, src.replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        # surface warnings other than the host pass's unknown-feature note
        lines = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    return obj


def build(out: str = OUT, defines: dict | None = None) -> str:
    """Compile and link libbc.so (out); defines override tuning constants
    (e.g. {"BC_GROUP": 8}) for experiments."""
    extra = [f"-D{k}={v}" for k, v in (defines or {}).items()]
    build_dir = BUILD if not defines else os.path.join(BUILD, "_".join(f"{k}{v}" for k, v in defines.items()))
    os.makedirs(build_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda f: _compile(f, build_dir, extra), SOURCES))
    tmp = out + f".tmp{os.getpid()}"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
