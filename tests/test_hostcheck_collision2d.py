"""Bounds check on the CPU of the generic collision pipeline at 2D 48 and 64
points per axis, the grids switched off on the GPU after a memory fault whose
cause was not found.

tests/hostcheck/collision2d_bounds.cpp runs every thread of every launch of
that pipeline (basis spectra, filtered or shifted fields, sigma reduce, pair
transforms, final, moment projection) through the kernels' own per-thread
bodies, on buffers of exactly the requested sizes, under AddressSanitizer.
The library's table builder is compiled into it with the 2D size restriction
lifted (a copy made here; the library itself keeps refusing these grids).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_02695_amd", "csrc")
RESTRICTION = 'require(vg.n == 16 || vg.n == 32, "2D vgrid.n must be 16 or 32"'
LIFTED = 'require(vg.n == 16 || vg.n == 32 || vg.n == 48 || vg.n == 64, "2D vgrid.n"'


def test_generic_pipeline_2d_48_64_stays_in_bounds(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    src = open(os.path.join(CSRC, "tables.cpp")).read()
    assert RESTRICTION in src, "the 2D size restriction moved; update this test"
    tables = tmp_path / "tables_all2d.cpp"
    tables.write_text(src.replace(RESTRICTION, LIFTED).replace(
        '#include "internal.hpp"', '#include "%s"' % os.path.join(CSRC, "internal.hpp")))
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    # AddressSanitizer on the host pass only (no GPU code is built or run)
    asan = ["-Xarch_host", "-fsanitize=address", "-fno-omit-frame-pointer"]
    hc_o, tb_o, exe = tmp_path / "hc.o", tmp_path / "tables.o", tmp_path / "hc"
    subprocess.run(["hipcc", "-x", "hip", "--cuda-host-only", "-std=c++17", "-O1", "-g", *asan,
                    *inc, "-c", os.path.join(ROOT, "tests", "hostcheck", "collision2d_bounds.cpp"),
                    "-o", str(hc_o)], check=True, capture_output=True)
    subprocess.run(["hipcc", "-std=c++17", "-O1", "-g", *asan, *inc, "-c", str(tables), "-o",
                    str(tb_o)], check=True, capture_output=True)
    subprocess.run(["hipcc", *asan, str(hc_o), str(tb_o), "-o", str(exe)], check=True,
                   capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out
    assert out.count("  ok:") == 16 and "all cases done" in out, out[-4000:]
