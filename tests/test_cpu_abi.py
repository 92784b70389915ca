"""Host-only checks: libbc.so loads and exports every function include/bc.h
declares; option/struct layouts agree with the header; the generators give
the documented shapes.  No GPU compute is called."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2008_05718_amd import binding as b
from paper_2008_05718_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bc.h")


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bc_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = b.lib()
    declared = _declared_functions()
    assert set(declared) >= {"bc_graph_create", "bc_run", "bc_scores", "bc_destroy"}
    for name in declared:
        assert hasattr(L, name), f"libbc.so does not export {name}"
    assert sorted(b.EXPORTS) == declared


def test_exports_are_plain_c_symbols():
    out = subprocess.run(["nm", "-D", "--defined-only", b.LIB_PATH], capture_output=True, text=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if " T " in l}
    for name in _declared_functions():
        assert name in syms


def test_status_strings_and_options_defaults():
    L = b.lib()
    for code, name in b.STATUS.items():
        assert L.bc_status_string(code).decode() == name
    o = b.make_options()
    assert (o.flags, o.batch, o.policy, o.grid_blocks, o.chunk_steps, o.sigma_limit) == (0, 0, 0, 0, 0, 0)


def _c_sizeof(struct_src: str, name: str) -> int:
    prog = f'#include "{HEADER}"\n#include <stdio.h>\nint main(void){{printf("%zu\\n", sizeof({name}));return 0;}}\n'
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "s.c")
        exe = os.path.join(td, "s")
        open(c, "w").write(prog)
        subprocess.check_call(["gcc", c, "-o", exe])
        return int(subprocess.check_output([exe]).decode())


@pytest.mark.parametrize("cname,pyt", [("bc_run_options", b.RunOptions), ("bc_detail", b.Detail),
                                       ("bc_stats", b.Stats), ("bc_level_stats", b.LevelStats)])
def test_struct_layouts_match_header(cname, pyt):
    assert _c_sizeof("", cname) == ctypes.sizeof(pyt)


@pytest.mark.parametrize("cname,pyt", [("bc_run_options", b.RunOptions), ("bc_detail", b.Detail),
                                       ("bc_stats", b.Stats), ("bc_level_stats", b.LevelStats)])
def test_struct_field_offsets_match_header(cname, pyt):
    # every field of the binding sits where the C compiler puts the field of
    # the same name (sizes alone would not catch two fields swapped)
    import tempfile
    names = [f[0] for f in pyt._fields_]
    body = "".join(f'printf("%zu\\n", offsetof({cname}, {n}));' for n in names)
    prog = f'#include "{HEADER}"\n#include <stddef.h>\n#include <stdio.h>\nint main(void){{{body}return 0;}}\n'
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "o.c")
        exe = os.path.join(td, "o")
        open(c, "w").write(prog)
        subprocess.check_call(["gcc", c, "-o", exe])
        got = [int(x) for x in subprocess.check_output([exe]).decode().split()]
    assert got == [getattr(pyt, n).offset for n in names]


def test_mlp_param_count_matches_header():
    txt = open(HEADER).read()
    m = re.search(r"#define BC_MLP_PARAMS \((.*?)\)\n", txt)
    assert eval(m.group(1)) == b.BC_MLP_PARAMS == 1545
    for name in ("BC_MLP_IN", "BC_MLP_OUT", "BC_LB_PACKED", "BC_LB_RULE", "BC_LB_ITEMS"):
        v = re.search(rf"#define {name} +(\d+)", txt)
        assert v and int(v.group(1)) == getattr(b, name), name
    assert b.BC_MLP_PARAMS == 32 * b.BC_MLP_IN + 32 + 32 * 32 + 32 + b.BC_MLP_OUT * 32 + b.BC_MLP_OUT


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(b, "_lib", None)
    monkeypatch.setattr(b, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(b.LibraryMissing):
        b.lib()


def test_generators_shapes():
    g = W.erdos_renyi(2000, 8.0, seed=1)
    assert g.n == 2000 and 7600 < g.m < 8400
    rp, ci = g.row_ptr, g.col_idx
    assert rp[0] == 0 and rp[-1] == g.nnz
    for v in range(0, g.n, 97):
        nb = ci[rp[v]:rp[v + 1]]
        assert (np.diff(nb) > 0).all() and v not in nb
    r = W.rmat(12, 16, seed=2)
    assert r.n == 4096 and r.nnz % 2 == 0
    deg = r.degrees()
    assert deg.max() > 20 * deg[deg > 0].mean()  # skewed
    gr = W.grid(20, 0.1, 0.01, seed=3)
    assert gr.n <= 400 and gr.degrees().max() <= 4 + 4
    ba = W.barabasi_albert(500, 4, seed=1)
    assert ba.m == 6 + (500 - 4) * 4
    u = W.union([W.grid(3), W.grid(4)])
    assert u.n == 25 and list(u.vtx_offsets) == [0, 9, 25]


def test_grid_full_size_recipe_counts():
    # the 1024^2 damaged grid: 10 % of 2,095,104 edges deleted, LCC, +0.1 % shortcuts
    g = W.grid(1024, 0.10, 0.001, seed=3)
    assert 1_040_000 < g.n < 1_048_576
    lcc_m = g.m - round(0.001 * (g.m / 1.001))
    assert abs(g.m - lcc_m) > 1000


def test_null_handles_and_pointers_are_argument_errors():
    # every entry point rejects a NULL handle or a NULL required pointer with
    # BC_ERR_INVALID_ARG before touching the device (no GPU needed)
    L = b.lib()
    INV = 1
    P = ctypes.c_void_p
    out = P()
    rp = np.array([0, 1, 2], np.int32)
    ci = np.array([1, 0], np.int32)
    prp, pci = rp.ctypes.data_as(P), ci.ctypes.data_as(P)
    o = b.make_options()
    st = b.Stats()
    det = b.Detail()
    lv = b.LevelStats()
    nl = ctypes.c_int64()
    cnt = ctypes.c_int64()
    src = np.array([0], np.int32)
    ps = src.ctypes.data_as(P)
    f = np.zeros(4096, np.float32)
    pf = f.ctypes.data_as(P)
    mask = np.ones(4096, np.uint8)
    calls = {
        "create out NULL": lambda: L.bc_graph_create(2, 2, prp, pci, 0, None),
        "create row_ptr NULL": lambda: L.bc_graph_create(2, 2, None, pci, 0, ctypes.byref(out)),
        "create col NULL": lambda: L.bc_graph_create(2, 2, prp, None, 0, ctypes.byref(out)),
        "create n < 0": lambda: L.bc_graph_create(-1, 2, prp, pci, 0, ctypes.byref(out)),
        "create nnz < 0": lambda: L.bc_graph_create(2, -2, prp, pci, 0, ctypes.byref(out)),
        "multi offsets NULL": lambda: L.bc_graph_create_multi(1, None, 2, 2, prp, pci, 0, ctypes.byref(out)),
        "info": lambda: L.bc_graph_info(None, None, None, None, None),
        "limit": lambda: L.bc_set_device_limit(None, 0),
        "run": lambda: L.bc_run(None, ps, 1, ctypes.byref(o), None),
        "run all": lambda: L.bc_run(None, None, 0, None, None),
        "detail": lambda: L.bc_run_detail(None, ps, 1, ctypes.byref(o), 0, ctypes.byref(det), None),
        "detail out NULL": lambda: L.bc_run_detail(None, ps, 1, ctypes.byref(o), 0, None, None),
        "scores": lambda: L.bc_scores(None, pf, 10, 0, None),
        "stats": lambda: L.bc_run_stats(None, ctypes.byref(st)),
        "level stats": lambda: L.bc_run_level_stats(None, ctypes.byref(lv), 1, ctypes.byref(nl)),
        "autotune": lambda: L.bc_autotune(None, ps, 1, None, ctypes.byref(o), None),
        "load policy": lambda: L.bc_load_policy(None, pf, b.BC_MLP_PARAMS),
        "collect": lambda: L.bc_collect_level_times(None, ps, 1, None, pf, pf, 10, ctypes.byref(cnt), None),
        "mlp grad NULL X": lambda: L.bc_mlp_loss_grad(pf, None, pf, mask.ctypes.data_as(P), 1, None, pf, None),
        "mlp train NULL w": lambda: L.bc_mlp_train(None, pf, pf, mask.ctypes.data_as(P), 1, 1, ctypes.c_float(0.01),
                                                   None, None),
        "mlp predict NULL Y": lambda: L.bc_mlp_predict(pf, pf, 1, None, None),
    }
    for name, call in calls.items():
        assert call() == INV, name
        assert L.bc_last_error().decode(), name
    assert out.value is None  # never set on failure
    L.bc_destroy(None)  # NULL-safe
