"""Build the HIP library ``liblor.so`` for gfx950 with hipcc (in-tree).

Run ``python -m paper_1908_07071_amd.build`` (or call :func:`build`).  Every
call recompiles all sources.  The files that must reproduce float64 results
bit for bit (the LOR stencil assembly and the MDF ordering) are compiled
without floating-point contraction.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "liblor.so")
OBJDIR = os.path.join(HERE, "_build")

SOURCES = [
    ("basis.cpp", []),
    ("mdf.cpp", ["-ffp-contract=off"]),
    ("sweep_pack.cpp", []),
    ("lor_api.cpp", []),
    ("k_setup.hip", ["-ffp-contract=off"]),
    ("k_operator.hip", []),
    ("k_schwarz.hip", []),
    ("k_krylov.hip", []),
    ("k_dg.hip", []),
    ("coarse_inverse.cpp", []),
    ("k_dgemm.hip", []),
    ("k_nn.hip", []),
    ("k_nnconv.hip", []),
    ("nn_api.cpp", []),
    ("noalloc.hip", []),
    ("box_patch.cpp", ["-ffp-contract=off"]),
    ("host_plan.cpp", []),
    ("k_single.hip", []),
]

ARCH = "gfx950"
COMMON = [
    "-O3", "-fPIC", "-std=c++17", f"-I{INCLUDE}", "-Wall", "-Wno-unused-function",
    "-Wno-unused-variable", "-Wno-unused-but-set-variable",
]
# device code: no packed FP32 instructions
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, extra: list) -> str:
    hipcc = _hipcc()
    obj = os.path.join(OBJDIR, src + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [hipcc, "-x", "hip", *COMMON, *HIP_FLAGS, *extra, "-c", path, "-o", obj]
    else:
        cmd = [hipcc, "-x", "c++", *COMMON, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *extra,
               "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(*s), SOURCES))
    tmp = LIB + ".tmp"
    # every GPU kernel is built from the sources above; only the HIP runtime is linked
    cmd = [_hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
