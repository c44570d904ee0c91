"""Host check of the sweep-block packer (no GPU): tests/host/sweep_pack_check.cpp
is built with g++ against the library's MDF factorization and packer sources
and replays the packed ILU(0) sweeps the way the patch kernel consumes them,
against a direct level-ordered triangular solve, in float and double, on
interior, face, edge, corner and degenerate box shapes in 2D and 3D.  The
MDF result itself is pinned against the oracle in test_abi.py."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1908_07071_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


def test_sweep_blocks_replay_to_triangular_solves(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(ROCM_INC):
        pytest.skip("g++ or the ROCm headers are not available")
    exe = str(tmp_path / "sweep_pack_check")
    cmd = [gxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, "-I" + CSRC,
           os.path.join(ROOT, "tests", "host", "sweep_pack_check.cpp"),
           os.path.join(CSRC, "sweep_pack.cpp"), os.path.join(CSRC, "mdf.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(run.stdout)
    assert run.returncode == 0, run.stdout[-3000:]
    assert "all ok" in run.stdout
