"""Pins of the curved (isoparametric) element geometry: every element is the
image of [0,1]^d under the interpolant of its own GLL node coordinates
(Section 2 allows any suitable map; Section 4.2 uses curved meshes)."""
import numpy as np
import pytest

from oracle import gll, highorder as HO, lor, mesh as M, schwarz as S, krylov
from paper_1908_07071_amd import inputs


def _curved(dim, n, p, amp=0.15, perturb=0.0, seed=None):
    return M.make_mesh(dim, [n] * dim, inputs.curved_vertices(dim, n, amp, perturb, seed),
                       nodes=inputs.curved_nodes(dim, n, p, amp, perturb, seed), nodes_p=p)


@pytest.mark.parametrize("dim,n,p", [(2, 3, 3), (3, 2, 2)])
def test_straight_nodes_reproduce_the_trilinear_map(dim, n, p):
    """Nodes placed by the elements' Q1 maps (no bending): the nodal
    geometry gives the same operator as the vertex map."""
    Vs = inputs.structured_vertices(dim, n, 0.1, seed=3)
    straight = M.make_mesh(dim, [n] * dim, Vs)
    nodal = _curved(dim, n, p, amp=0.0, perturb=0.1, seed=3)
    assert np.abs(nodal.vertices - Vs).max() == 0.0
    K0, K1 = HO.cg_stiffness(straight, p), HO.cg_stiffness(nodal, p)
    assert abs(K0 - K1).max() <= 1e-12 * abs(K0).max()


@pytest.mark.parametrize("p", [2, 3, 5])
def test_curved_volume_and_neumann_kernel(p):
    """2D: |J| of the degree-p interpolant has degree 2p - 1 per direction,
    which GLL quadrature integrates exactly, and the bent block is still the
    unit square: sum w |J| = 1.  Constants lie in the Neumann kernel."""
    mesh = _curved(2, 3, p)
    vol = 0.0
    for e in mesh.elements():
        _, dets, _, wq = HO.element_geometry(mesh, p, e)
        assert dets.min() > 0
        vol += float(np.sum(wq * dets))
    assert abs(vol - 1.0) <= 1e-13
    Kn = HO.cg_stiffness(mesh, p, dirichlet=False)
    assert np.abs(Kn @ np.ones(Kn.shape[0])).max() <= 1e-12 * abs(Kn).max()
    Kd = HO.cg_stiffness(mesh, p).toarray()
    assert np.abs(Kd - Kd.T).max() <= 1e-13 * np.abs(Kd).max()
    assert np.linalg.eigvalsh(Kd).min() > 0


@pytest.mark.parametrize("p", [2, 3])
def test_curved_manufactured_rate(p):
    """-Laplace u = f on the unit square with bent elements, u = sin(pi x)
    sin(pi y): L2 error O(h^(p+1))."""
    errs = []
    for n in (2, 4, 8):
        mesh = _curved(2, n, p)
        K = HO.cg_stiffness(mesh, p)
        coords = M.global_node_coords(mesh, gll.gll(p)[0], p)
        b = HO.cg_rhs(mesh, p, inputs.manufactured_f(coords))
        u = np.linalg.solve(K.toarray(), b)
        num = M.interior_numbering(M.grid_shape(mesh, p))
        ug = np.zeros(len(num))
        ug[num >= 0] = u
        errs.append(HO.l2_error_cg(mesh, p, ug, inputs.manufactured_u))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] >= p + 1 - 0.3, (errs, rates)


def test_curved_preconditioner_converges():
    """The LOR hierarchy of a curved mesh uses its GLL nodes as the
    sub-element corners; B stays spectrally equivalent (the count is close
    to the straight mesh's)."""
    p = 4
    its = []
    for amp in (0.0, 0.15):
        mesh = _curved(2, 4, p, amp=amp)
        K = HO.cg_stiffness(mesh, p)
        b = inputs.gaussian_rhs(K.shape[0], 3)
        _, it, _ = krylov.pcg(K, b, S.SchwarzLOR(mesh, p).apply, tol=1e-8)
        its.append(it)
    assert its[1] <= 1.3 * its[0] + 2, its
