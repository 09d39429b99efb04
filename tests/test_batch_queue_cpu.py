"""The persistent batch's queue logic on the CPU: a host-only simulation
(tests/cpu/batch_queue_sim.cpp, built with hipcc, run without a GPU) drives
the dependency rule the kernel uses (batch_dep in fjofc_internal.h) with
random problem sets, worker counts, transform counts and task durations,
and checks that the queue never deadlocks and that no task starts before
the tasks it depends on in Algorithm 2's order."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_batch_queue_simulation(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = tmp_path / "batch_queue_sim"
    src = os.path.join(ROOT, "tests", "cpu", "batch_queue_sim.cpp")
    inc = [f"-I{os.path.join(ROOT, 'include')}",
           f"-I{os.path.join(ROOT, 'paper_1502_03391_amd', 'csrc')}"]
    subprocess.run([HIPCC, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", *inc,
                    src, "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
