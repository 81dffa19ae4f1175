"""Host-side invariants of the planner's tables that the GPU kernels rely on (gridding lane
nodes and LDS addressing, FFT factorisation, the z band of the mid-range transforms):
tests/planner_checks.cpp compiled with the host compiler against the library's planner
source and run on the CPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROCM_INCLUDE = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INCLUDE),
                    reason="needs g++ and the ROCm headers")
def test_planner_invariants(tmp_path):
    exe = tmp_path / "planner_checks"
    cmd = ["g++", "-O2", "-std=c++17", f"-I{ROCM_INCLUDE}", "-D__HIP_PLATFORM_AMD__",
           os.path.join(HERE, "planner_checks.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:]
    assert r.stdout.strip().endswith("bad 0")
