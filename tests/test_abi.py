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
