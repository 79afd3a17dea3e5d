"""The serving engine's host bookkeeping (device-arena allocator, request
footprint) built with the host C++ compiler and checked on the CPU against
a brute-force model (tests/srv_sched_check.cpp)."""
import os
import shutil
import subprocess

import pytest

from _util import ROOT


def test_arena_allocator_and_footprint(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    exe = tmp_path / "srv_sched_check"
    src = os.path.join(ROOT, "tests", "srv_sched_check.cpp")
    inc = os.path.join(ROOT, "paper_2410_04001_amd", "csrc")
    subprocess.run([cxx, "-O1", "-std=c++17", "-I", inc, src, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout + out.stderr
