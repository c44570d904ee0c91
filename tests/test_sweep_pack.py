"""Host check of the sweep-block packer (no GPU): tests/host/sweep_pack_check.cpp
is built with g++ against the library's MDF factorization and packer sources
and replays the packed ILU(0) sweeps the way the patch kernel consumes them,
against a direct level-ordered triangular solve, in float and double.  Cases:
random diagonally dominant stencils on interior, face, edge, corner and
degenerate box shapes in 2D and 3D, and the LOR patch stencils of a
perturbed 2^3 mesh at p = 6 (every patch type, levels 0 to 2) and a 2D mesh
at p = 8, taken from the oracle's hierarchy.  The MDF result itself is pinned
against the oracle in test_abi.py."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import lor as OL, mesh as M, schwarz as S
from paper_1908_07071_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1908_07071_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


def _lor_patch_cases():
    """(dim, shape, stencil rows) of LOR patches from the oracle's hierarchy."""
    out = []
    for dim, n, p, verts in ((3, 2, 6, [(1, 1, 1), (0, 1, 1), (0, 0, 1), (0, 0, 0)]), (2, 3, 8, [(1, 2), (0, 1)])):
        mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n, 0.1, seed=4))
        H = OL.LORHierarchy(mesh, p)
        for v in verts:
            for k in range(min(3, H.nlevels - 1)):
                rng = S.patch_ranges(mesh, H.sizes[k], v)
                shape = [hi - lo + 1 for lo, hi in rng]
                if min(shape) <= 0:
                    continue
                idx = np.indices(shape).reshape(dim, -1, order="F")
                flat = M.lex_index([idx[i] + rng[i][0] for i in range(dim)], H.shapes[k])
                out.append((dim, shape, H.stencils[k][flat]))
    return out


def test_sweep_blocks_replay_to_triangular_solves(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(ROCM_INC):
        pytest.skip("g++ or the ROCm headers are not available")
    exe = str(tmp_path / "sweep_pack_check")
    cmd = [gxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, "-I" + CSRC,
           os.path.join(ROOT, "tests", "host", "sweep_pack_check.cpp"),
           os.path.join(CSRC, "sweep_pack.cpp"), os.path.join(CSRC, "mdf.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    cases = _lor_patch_cases()
    path = tmp_path / "lor_patches.txt"
    with open(path, "w") as f:
        f.write(f"{len(cases)}\n")
        for dim, shape, rows in cases:
            m = list(shape) + [1] * (3 - len(shape))
            f.write(f"{dim} {m[0]} {m[1]} {m[2]}\n")
            np.savetxt(f, rows, fmt="%.17g")
    run = subprocess.run([exe, str(path)], capture_output=True, text=True, timeout=300)
    print(run.stdout)
    assert run.returncode == 0, run.stdout[-3000:]
    assert "all ok" in run.stdout
    assert run.stdout.count("file ") == 2 * len(cases) and len(cases) >= 12
