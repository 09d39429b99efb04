"""The stream tile choice's host logic on the CPU (tile_spec.h, no HIP):
tile-cache lines, the FJOFC_TILE override (plain and scoped entries, strict
parsing) and the choice of a cache row by architecture, nearest d and
smallest covering n-bucket.  Built with g++ from tests/cpu/tile_spec_test.cpp."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tile_spec_logic(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "tile_spec_test"
    src = os.path.join(ROOT, "tests", "cpu", "tile_spec_test.cpp")
    inc = f"-I{os.path.join(ROOT, 'paper_1502_03391_amd', 'csrc')}"
    subprocess.run([gxx, "-O1", "-std=c++17", "-Wall", inc, src, "-o", str(exe)], check=True,
                   capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
