"""Writes oracle_bands.json: iteration bands and attainable residuals that
the GPU tests compare against, computed by the CPU oracle alone.

Each entry is keyed by the case id the tests use.  A band is
``krylov.iteration_band`` of the oracle's own preconditioned CG: the lowest
and highest count over the unperturbed run and runs whose preconditioner
output carries relative perturbations of the given size (the parity
tolerance of the float64 preconditioner, 1e-12).  These solves take minutes
in the oracle, too long for a GPU test, so they are stored.

Run from the repository root:  python tests/golden/make_oracle_bands.py
"""
from __future__ import annotations

import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import gll, highorder as HO, krylov, mesh as M, schwarz as S  # noqa: E402
from paper_1908_07071_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_bands.json")

# 3D CG cases at the degrees the small-case GPU tests do not otherwise reach
# (dim, n, p, perturb, seed); right-hand side gaussian_rhs(N, 21), rtol 1e-10
CG_CASES = [
    (3, (2, 2, 2), 5, 0.1, 8),
    (3, (2, 1, 2), 7, 0.1, 9),
    (3, (1, 2, 2), 8, 0.1, 10),
]


def cg_id(c):
    return f"cg-d{c[0]}-n{'x'.join(map(str, c[1]))}-p{c[2]}"


def cg_band(c):
    dim, n, p, pert, seed = c
    V = inputs.structured_vertices(dim, list(n), pert, seed=seed)
    mesh = M.make_mesh(dim, list(n), V)
    K = HO.cg_stiffness(mesh, p)
    B = S.SchwarzLOR(mesh, p)
    b = inputs.gaussian_rhs(K.shape[0], 21)
    lo, hi = krylov.iteration_band(K, b, B.apply, tol=1e-10)
    return cg_id(c), {"lo": int(lo), "hi": int(hi), "rtol": 1e-10, "rhs": "gaussian_rhs(N, 21)"}


def cfg0_band(_):
    """2D unit square, 8x8 uniform quads, p = 3, f = 2 pi^2 sin(pi x) sin(pi y)
    at the GLL nodes, b = M_p f, PCG to 1e-10."""
    dim, n, p = 2, [8, 8], 3
    V = inputs.structured_vertices(dim, n)
    mesh = M.make_mesh(dim, n, V)
    x, _ = gll.gll(p)
    coords = M.global_node_coords(mesh, x, p)
    b = HO.cg_rhs(mesh, p, inputs.manufactured_f(coords))
    K = HO.cg_stiffness(mesh, p)
    B = S.SchwarzLOR(mesh, p)
    lo, hi = krylov.iteration_band(K, b, B.apply, tol=1e-10)
    return "cg-square-8x8-p3-manufactured", {"lo": int(lo), "hi": int(hi), "rtol": 1e-10,
                                             "N": int(K.shape[0])}


def main():
    jobs = [(cg_band, c) for c in CG_CASES] + [(cfg0_band, None)]
    out = {}
    with ProcessPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for key, val in ex.map(_run, jobs):
            out[key] = val
            print(key, val, flush=True)
    with open(OUT, "w") as f:
        json.dump(dict(sorted(out.items())), f, indent=1)
        f.write("\n")


def _run(job):
    fn, arg = job
    return fn(arg)


if __name__ == "__main__":
    main()
