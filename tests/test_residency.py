"""Host logic of the persistent-grid admission (csrc/residency.hpp), built with g++ and run on the
CPU: a grid's CU-slot charge per XCD, tickets, and concurrent holders that never exceed the pool."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_residency_admission(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "residency_check"
    src = os.path.join(HERE, "native", "residency_check.cpp")
    inc = os.path.join(ROOT, "paper_2507_02809_amd", "csrc")
    subprocess.run([gxx, "-std=c++17", "-O1", "-pthread", "-I", inc, src, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "residency ok" in r.stdout
