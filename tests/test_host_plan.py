"""Host check of the planning helpers (no GPU): tests/host/plan_check.cpp is
built with g++ against csrc/host_plan.cpp and checks the box colours (boxes
of one colour never overlap, each box takes the smallest colour its earlier
neighbours leave, vertex boxes one element either way on a structured
block need 2^d colours) and the batched solve's grouping (every part in
exactly one group; shared groups only with more parts than streams, of
small multi-right-hand-side parts of one dimension and precision, within
the job and block limits; groups spread over the streams)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1908_07071_amd", "csrc")


def test_box_colours_and_batch_groups(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    exe = str(tmp_path / "plan_check")
    cmd = [gxx, "-O2", "-std=c++17", "-I" + CSRC, os.path.join(ROOT, "tests", "host", "plan_check.cpp"),
           os.path.join(CSRC, "host_plan.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0 and run.stdout.strip().endswith("OK"), run.stdout + run.stderr
