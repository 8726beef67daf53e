"""The C ABI: every declared function is exported, and the ctypes mirrors of
the structs match the C layout (CPU only: no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "macproj.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mg_setup", "mac_project", "mg_vcycle", "project_batch", "serve_submit",
                 "serve_create", "serve_poll", "serve_wait", "serve_destroy", "mg_destroy",
                 "mg_strerror", "mg_last_error", "mg_workspace_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1910_12979_amd import macproj
    if not os.path.exists(macproj.LIB_PATH):
        from paper_1910_12979_amd import build
        build.build()
    lib = macproj.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.mg_strerror(-3) == b"incompatible right-hand side"


def test_struct_layouts_match_ctypes(tmp_path):
    from paper_1910_12979_amd import macproj as M
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "macproj.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(mg_params), sizeof(mg_stats),"
        " sizeof(mg_problem), offsetof(mg_params, rtol), offsetof(mg_stats, resid_hist),"
        " offsetof(mg_problem, phi), offsetof(mg_problem, kind), offsetof(mg_problem, box));return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(M.Params), ctypes.sizeof(M.Stats), ctypes.sizeof(M.Problem),
            M.Params.rtol.offset, M.Stats.resid_hist.offset, M.Problem.phi.offset, M.Problem.kind.offset,
            M.Problem.box.offset]
    assert got == want


def test_host_side_validation_without_gpu():
    """Parameter checks that never touch the device."""
    from paper_1910_12979_amd import macproj as M
    p = M.make_params((256, 256, 256), 1 / 256)
    assert M.mg_num_levels_for(p) == 7
    assert M.mg_workspace_bytes(p) > 5 * 8 * 256 ** 3
    bad = M.make_params((37, 37, 37), 1 / 37)
    assert M.mg_num_levels_for(bad) == 0 and M.mg_workspace_bytes(bad) == 0
    mixed = M.make_params((64, 64, 64), 1 / 64, precision="mixed")
    plain = M.make_params((64, 64, 64), 1 / 64)
    assert M.mg_workspace_bytes(mixed) > M.mg_workspace_bytes(plain)


def test_setters_reject_a_null_handle_without_gpu():
    from paper_1910_12979_amd import macproj as M
    lib = M.lib()
    box = (ctypes.c_int32 * 3)(16, 16, 16)
    assert lib.mg_set_boxes(None, box) == -1
    assert lib.mg_set_graphs(None, 1) == -1
    assert lib.mg_set_bottom(None, 1) == -1


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; --gpus N > 1 exits with a message
    before anything touches a device."""
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
