"""The C-ABI library loads and exports every entry point that include/blr.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2112_02695_amd", "libblr.so")


def _declared():
    src = open(os.path.join(ROOT, "include", "blr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(blr_[a-z_]+)\s*\(", src)))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("blr_collision_pairs", "blr_dlr_step", "blr_steady_solve", "blr_create",
              "blr_destroy", "blr_last_error", "blr_workspace_bytes", "blr_state_from_full"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libblr.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_2112_02695_amd as blr
    with pytest.raises(ImportError):
        blr._LIB = None
        blr.load_library(str(tmp_path / "nope.so"))
    blr._LIB = None


STRUCTS = [("VGrid", "blr_vgrid"), ("Problem", "blr_problem"), ("State", "blr_state"),
           ("StepParams", "blr_step_params"), ("StepInfo", "blr_step_info"),
           ("SolveParams", "blr_solve_params"), ("SolveInfo", "blr_solve_info"),
           ("ServerParams", "blr_server_params"), ("Request", "blr_request"),
           ("Completion", "blr_completion")]


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (a C program built against include/blr.h prints them)."""
    import shutil
    import subprocess
    import paper_2112_02695_amd as blr
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "blr.h"', "int main(void) {"]
    for py, c in STRUCTS:
        lines.append(f'  printf("{py} size %zu\\n", sizeof({c}));')
        for f in getattr(blr, py)._fields_:
            lines.append(f'  printf("{py}.{f[0]} %zu\\n", offsetof({c}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    for py, c in STRUCTS:
        cls = getattr(blr, py)
        assert int(got[f"{py} size"]) == ctypes.sizeof(cls), py
        for f in cls._fields_:
            assert int(got[f"{py}.{f[0]}"]) == getattr(cls, f[0]).offset, f"{py}.{f[0]}"
