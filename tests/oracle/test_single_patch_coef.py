"""Pins of the single-patch preconditioner B(1) (Section 4.1) and of the
variable coefficient b of -div(b grad u) = f (Section 4.2) in the high-order
operator and in the LOR hierarchy."""
import numpy as np
import pytest

from oracle import gll, highorder as HO, krylov, lor, mdf, mesh as M, schwarz as S
from paper_1908_07071_amd import inputs


def _elem_coef(mesh, p, name, seed=0):
    X = HO.dg_node_coords(mesh, p)          # element-major GLL nodes
    nq = (p + 1) ** mesh.dim
    elem = np.repeat(np.arange(mesh.nel), nq)
    return inputs.coefficient(name, X, elem=elem, seed=seed).reshape(mesh.nel, nq)


@pytest.mark.parametrize("dim,n,p", [(2, [3, 2], 4), (3, [2, 2, 1], 3)])
def test_single_patch_exact_smoothers_invert_Kh(dim, n, p):
    """With exact solves in place of the IC(0) smoothers the first smoothing
    step already solves, so the whole-domain V-cycle is K_h^-1."""
    mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n, 0.1, seed=1))
    B = S.SchwarzLOR(mesh, p, exact_local=True, patch_mode="single")
    Kh = B.Kh.toarray()
    Z = B.as_matrix()
    assert np.abs(Z - np.linalg.inv(Kh)).max() <= 1e-11 * np.abs(Z).max()


@pytest.mark.parametrize("dim,n,p", [(2, [3, 3], 4), (3, [2, 2, 2], 2), (2, [2, 2], 6)])
def test_single_patch_error_propagation(dim, n, p):
    """The whole-domain V-cycle equals the recursive two-grid error
    propagation of its levels (one IC(0) step before and after the coarse
    correction, exact on T_p)."""
    from tests.oracle.test_pins_worked import _vcycle_matrix
    mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n, 0.1, seed=2))
    B = S.SchwarzLOR(mesh, p, patch_mode="single")
    P = B.patches[0]
    Vt = _vcycle_matrix(P, 0)
    Z = B.as_matrix()
    assert np.abs(Z - Vt).max() <= 1e-11 * np.abs(Vt).max()
    assert np.abs(Z - Z.T).max() <= 1e-11 * np.abs(Z).max()
    assert np.linalg.eigvalsh(0.5 * (Z + Z.T)).min() > 0


def test_single_patch_condition_flat_in_h_and_p():
    """kappa(B(1) K_p) bounded in h and p (Table cart-iters: counts level off);
    B(1) as a dense matrix from its error propagation (pinned equal to the
    V-cycle above)."""
    from tests.oracle.test_pins_worked import _vcycle_matrix
    kap = {}
    for n in (4, 8):
        for p in (3, 5):
            mesh = M.make_mesh(2, [n, n], inputs.structured_vertices(2, n))
            K = HO.cg_stiffness(mesh, p).toarray()
            B = _vcycle_matrix(S.SchwarzLOR(mesh, p, patch_mode="single").patches[0], 0)
            ev = np.linalg.eigvals(B @ K).real
            kap[n, p] = ev.max() / ev.min()
    assert kap[8, 5] / kap[4, 5] <= 1.25 and kap[8, 3] / kap[4, 3] <= 1.25, kap
    assert kap[8, 5] / kap[8, 3] <= 1.6, kap


def test_coefficient_constant_scales_everything():
    mesh = M.make_mesh(3, [2, 2, 2], inputs.structured_vertices(3, 2, 0.1, seed=3))
    p = 3
    c = np.full((mesh.nel, (p + 1) ** 3), 2.5)
    K1, Kc = HO.cg_stiffness(mesh, p), HO.cg_stiffness(mesh, p, coef=c)
    assert abs(Kc - 2.5 * K1).max() <= 1e-13 * abs(Kc).max()
    H1, Hc = lor.LORHierarchy(mesh, p), lor.LORHierarchy(mesh, p, coef=c)
    for a, b in zip(H1.stencils, Hc.stencils):
        assert np.abs(b - 2.5 * a).max() <= 1e-14 * np.abs(b).max()


def test_cell_coefficient_is_corner_mean():
    """For b linear in x the mean over a cell's corners is b at the mean of
    its corner coordinates (affine mesh: the cell centre)."""
    dim, n, p = 2, [3, 2], 4
    mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n))
    X = HO.dg_node_coords(mesh, p)
    b = (1.0 + 3.0 * X[:, 0] - 2.0 * X[:, 1]).reshape(mesh.nel, -1)
    H = lor.LORHierarchy(mesh, p)
    for k in range(H.nlevels):
        cc = lor.level_cell_coef(mesh, p, k, b)
        corners = lor.subelement_corners(H.coords[k], H.shapes[k])   # (2^d, d, cells)
        centre = corners.mean(axis=0)
        assert np.allclose(cc, 1.0 + 3.0 * centre[0] - 2.0 * centre[1], rtol=0, atol=1e-13)


@pytest.mark.parametrize("p", [2, 3])
def test_variable_coefficient_manufactured_rate(p):
    """-div(b2 grad u) = f with u = sin(pi x) sin(pi y): L2 error O(h^(p+1))."""
    def f_exact(x):
        xp, yp = 2 * x[:, 0] - 1, 2 * x[:, 1] - 1
        b = 100 * xp ** 2 + yp ** 2 + 1
        bx, by = 400 * xp, 4 * yp
        s, c = np.sin(np.pi * x), np.cos(np.pi * x)
        ux, uy = np.pi * c[:, 0] * s[:, 1], np.pi * s[:, 0] * c[:, 1]
        return -(bx * ux + by * uy) + b * 2 * np.pi ** 2 * s[:, 0] * s[:, 1]

    errs = []
    for n in (2, 4, 8):
        mesh = M.make_mesh(2, [n, n], inputs.structured_vertices(2, n))
        coef = _elem_coef(mesh, p, "b2")
        K = HO.cg_stiffness(mesh, p, coef=coef)
        xg, _ = gll.gll(p)
        coords = M.global_node_coords(mesh, xg, p)
        bvec = HO.cg_rhs(mesh, p, f_exact(coords))
        u = np.linalg.solve(K.toarray(), bvec)
        num = M.interior_numbering(M.grid_shape(mesh, p))
        ug = np.zeros(len(num))
        ug[num >= 0] = u
        errs.append(HO.l2_error_cg(mesh, p, ug, inputs.manufactured_u))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] >= p + 1 - 0.3, (errs, rates)


@pytest.mark.parametrize("name", ["b1", "b2", "b3", "b4"])
def test_coefficients_single_and_vertex_patches_converge(name):
    """Section 4.2: bounded counts for every coefficient with both B(1) and
    B(V) (the paper's meshes are not available; 2D 4 x 4, p = 4)."""
    mesh = M.make_mesh(2, [4, 4], inputs.structured_vertices(2, 4, 0.1, seed=5))
    p = 4
    coef = _elem_coef(mesh, p, name, seed=7)
    K = HO.cg_stiffness(mesh, p, coef=coef)
    b = inputs.gaussian_rhs(K.shape[0], 8)
    for mode in ("single", "vertex"):
        B = S.SchwarzLOR(mesh, p, coef=coef, patch_mode=mode)
        x, it, _ = krylov.pcg(K, b, B.apply, tol=1e-8)
        assert np.linalg.norm(b - K @ x) <= 1.05e-8 * np.linalg.norm(b)
        assert it <= 80, (name, mode, it)
