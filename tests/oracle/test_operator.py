"""Pins of the assembled high-order CG operator K_p and right-hand side
(eq. fem / eq. system) against closed forms, invariants and convergence."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import gll, highorder as HO, mesh as M
from paper_1908_07071_amd import inputs


def _box_mesh(dim, lengths):
    """One element [0,a]x[0,b](x[0,c]) as a mesh."""
    V = inputs.structured_vertices(dim, 1)
    V = V * np.array(lengths)[None, :]
    return M.make_mesh(dim, 1, V)


@pytest.mark.parametrize("dim,p,lengths", [(2, 3, (1.0, 0.5)), (3, 2, (0.5, 1.5, 2.0)), (3, 4, (1.0, 0.7, 0.3))])
def test_kronecker_closed_form(dim, p, lengths):
    """Section 3.1: on an affine box, K_p = sum_j (x) (K1D in slot j, M1D elsewhere)."""
    mesh = _box_mesh(dim, lengths)
    K = HO.cg_stiffness(mesh, p, dirichlet=False).toarray()
    x, w = gll.gll(p)
    D = gll.lagrange_derivative_matrix(x)
    K1 = [D.T @ np.diag(w) @ D / L for L in lengths]
    M1 = [np.diag(w) * L for L in lengths]
    ref = 0
    for j in range(dim):
        mats = [K1[i] if i == j else M1[i] for i in range(dim)]
        T = mats[-1]
        for A in reversed(mats[:-1]):
            T = np.kron(T, A)  # x fastest: kron(z, y, x)
        ref = ref + T
    assert np.abs(K - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("dim,n,p", [(2, 3, 3), (3, 2, 2), (3, 2, 3)])
def test_symmetry_nullspace_spd(dim, n, p):
    mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n, 0.1, seed=7))
    Kn = HO.cg_stiffness(mesh, p, dirichlet=False)
    A = Kn.toarray()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    # pure Neumann: constants are annihilated
    assert np.abs(Kn @ np.ones(A.shape[0])).max() <= 1e-13 * np.abs(A).max()
    Kd = HO.cg_stiffness(mesh, p).toarray()
    assert np.linalg.eigvalsh(Kd).min() > 0


@pytest.mark.parametrize("dim,n,p", [(2, 3, 2), (3, 2, 2), (3, 2, 4)])
def test_volume_exact(dim, n, p):
    """sum_q w_q |J_q| is the exact volume (det J of a Q1 map is integrated
    exactly by GLL with p >= 2); interior perturbation keeps the unit volume."""
    mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n, 0.1, seed=11))
    vol = 0.0
    for e in mesh.elements():
        _, dets, _, wq = HO.element_geometry(mesh, p, e)
        vol += np.sum(wq * dets)
    assert abs(vol - 1.0) < 1e-14


def _mms_error(dim, n, p, pert):
    mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n, pert, seed=2))
    x, _ = gll.gll(p)
    coords = M.global_node_coords(mesh, x, p)
    K = HO.cg_stiffness(mesh, p)
    b = HO.cg_rhs(mesh, p, inputs.manufactured_f(coords))
    u = spla.spsolve(K.tocsc(), b)
    num = M.interior_numbering(M.grid_shape(mesh, p))
    ug = np.zeros(len(num))
    ug[num >= 0] = u
    return HO.l2_error_cg(mesh, p, ug, inputs.manufactured_u)


@pytest.mark.parametrize("dim,p,ns,pert", [(2, 2, (2, 4, 8), 0.1), (2, 3, (2, 4, 8), 0.1), (3, 2, (2, 4), 0.0)])
def test_manufactured_convergence(dim, p, ns, pert):
    """L2 error of the discrete solution decays like h^{p+1}."""
    errs = [_mms_error(dim, n, p, pert) for n in ns]
    rates = [np.log2(errs[i] / errs[i + 1]) * np.log(2) / np.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)]
    assert rates[-1] >= p + 1 - 0.3, (errs, rates)


def test_apply_rows_matches_assembled():
    mesh = M.make_mesh(3, 2, inputs.structured_vertices(3, 2, 0.1, seed=4))
    p = 3
    K = HO.cg_stiffness(mesh, p)
    x = inputs.uniform_vector(K.shape[0], 5)
    rows = np.array([0, 17, K.shape[0] // 2, K.shape[0] - 1])
    assert np.allclose(HO.cg_apply_rows(mesh, p, x, rows), (K @ x)[rows], rtol=1e-13, atol=1e-13)


def test_rhs_collocated_mass():
    """b = M_p f: for f = 1 the entries sum to the measure of the support of
    the interior basis functions; on an affine box they are w_i |J| summed."""
    mesh = M.make_mesh(2, 2, inputs.structured_vertices(2, 2))
    p = 2
    shape = M.grid_shape(mesh, p)
    b = HO.cg_rhs(mesh, p, np.ones(int(np.prod(shape))), dirichlet=False)
    assert abs(b.sum() - 1.0) < 1e-15
    _, w = gll.gll(p)
    # centre node of the 5x5 grid: shared by 4 elements, each w_0 * w_0 * h^2 (h = 1/2)
    centre = 2 + 5 * 2
    assert abs(b[centre] - 4 * w[0] * w[0] * 0.25) < 1e-16
