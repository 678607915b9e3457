"""The rendezvous of the server's shared collision launches (csrc/rendezvous.hpp),
stressed on the CPU with many threads under ThreadSanitizer
(tests/hostcheck/rendezvous_check.cpp): every item runs exactly once, rounds
hold at most one item per participant and, with a fixed set, one of each,
errors reach every item of a round, and stopping releases the waiters."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_02695_amd", "csrc")


def test_rendezvous_rounds_under_thread_sanitizer(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "rv"
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=thread", "-I" + CSRC,
                    os.path.join(ROOT, "tests", "hostcheck", "rendezvous_check.cpp"), "-o",
                    str(exe)], check=True, capture_output=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "ThreadSanitizer" not in out, out[-4000:]
    assert out.strip().endswith("ok"), out[-2000:]
