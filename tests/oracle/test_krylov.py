"""Pins of the preconditioned / flexible CG oracle."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import gll, highorder as HO, krylov, mesh as M, schwarz as S
from paper_1908_07071_amd import inputs


@pytest.mark.parametrize("dim,n,p", [(2, 4, 3), (3, 2, 2)])
def test_pcg_matches_direct_solve(dim, n, p):
    mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n, 0.1, seed=9))
    K = HO.cg_stiffness(mesh, p)
    b = inputs.gaussian_rhs(K.shape[0], 3)
    B = S.SchwarzLOR(mesh, p)
    x, it, hist = krylov.pcg(K, b, B.apply, tol=1e-10)
    xd = spla.spsolve(K.tocsc(), b)
    assert hist[-1] <= 1e-10
    assert np.linalg.norm(b - K @ x) <= 1.01e-10 * np.linalg.norm(b)
    assert np.abs(x - xd).max() <= 1e-8 * np.abs(xd).max()
    # flexible CG with a fixed symmetric preconditioner gives the same iterates
    xf, itf, histf = krylov.pcg(K, b, B.apply, tol=1e-10, flexible=True)
    assert abs(itf - it) <= 1
    assert np.abs(xf - x).max() <= 1e-8 * np.abs(x).max()


def test_cartesian_iteration_shape():
    """Shape of Table cart-iters-patch: bounded counts with mild growth in n.
    (Coarse solver and stopping norm differ from the paper: shape only.)"""
    its = []
    for n in (2, 4, 8):
        mesh = M.make_mesh(2, n, inputs.structured_vertices(2, n))
        x, _ = gll.gll(2)
        K = HO.cg_stiffness(mesh, 2)
        b = HO.cg_rhs(mesh, 2, inputs.manufactured_f(M.global_node_coords(mesh, x, 2)))
        _, it, _ = krylov.pcg(K, b, S.SchwarzLOR(mesh, 2).apply, tol=1e-8)
        its.append(it)
    assert its == sorted(its) and its[-1] <= 20, its


def test_identity_preconditioner_is_cg():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 30))
    A = A @ A.T + 30 * np.eye(30)
    b = rng.standard_normal(30)
    x, it, _ = krylov.pcg(A, b, lambda r: r, tol=1e-12)
    assert np.allclose(A @ x, b, rtol=0, atol=1e-10)
    assert it <= 30


def test_iteration_band():
    """The band holds the unperturbed count, collapses to it without
    perturbation, and widens on a problem whose residual history has a plateau
    at the tolerance (3D IP-DG, p = 2, where a 1e-13 relative change of the
    preconditioner moves the count by two)."""
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 30))
    A = A @ A.T + 30 * np.eye(30)
    b = rng.standard_normal(30)
    _, it, _ = krylov.pcg(A, b, lambda r: r, tol=1e-12)
    assert krylov.iteration_band(A, b, lambda r: r, tol=1e-12, rel=0.0) == (it, it)
    lo, hi = krylov.iteration_band(A, b, lambda r: r, tol=1e-12)
    assert lo <= it <= hi
    mesh = M.make_mesh(3, [2, 2, 1], inputs.structured_vertices(3, [2, 2, 1], 0.1, seed=44))
    D = HO.dg_operator(mesh, 2, "ip", 13.5)
    bd = inputs.gaussian_rhs(D.shape[0], 77)
    B = S.SchwarzDG(mesh, 2, D)
    _, itd, _ = krylov.pcg(D, bd, B.apply, tol=1e-10)
    lo, hi = krylov.iteration_band(D, bd, B.apply, tol=1e-10)
    assert lo <= itd <= hi and hi - lo >= 1, (lo, itd, hi)
