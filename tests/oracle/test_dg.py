"""Pins of the IP / BR2 DG operators (eq. ip, eq. br2) and the DG Schwarz
preconditioner (eq. dg-as)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import gll, highorder as HO, mesh as M, schwarz as S
from paper_1908_07071_amd import inputs


def _mesh(dim, n, pert=0.1, seed=6):
    return M.make_mesh(dim, n, inputs.structured_vertices(dim, n, pert, seed=seed))


@pytest.mark.parametrize("method", ["ip", "br2"])
@pytest.mark.parametrize("dim,n,p", [(2, 3, 3), (3, 2, 2)])
def test_conforming_restriction_is_cg(method, dim, n, p):
    """For H^1_0-conforming functions every face term vanishes: E^T A E = K_p."""
    mesh = _mesh(dim, n)
    A = HO.dg_operator(mesh, p, method, eta=10.0)
    E = HO.cg_to_dg(mesh, p)
    K = HO.cg_stiffness(mesh, p)
    d = (E.T @ A @ E - K).toarray()
    assert np.abs(d).max() <= 1e-12 * abs(K).max()
    Ad = A.toarray()
    assert np.abs(Ad - Ad.T).max() <= 1e-12 * np.abs(Ad).max()


@pytest.mark.parametrize("method", ["ip", "br2"])
def test_neumann_constants_in_kernel(method):
    mesh = _mesh(3, 2)
    A = HO.dg_operator(mesh, 2, method, eta=5.0, boundary=False)
    assert np.abs(A @ np.ones(A.shape[0])).max() <= 1e-12 * abs(A).max()


def test_br2_nodewise_penalty_equals_lifting():
    """The BR2 term eta sum_e (r_e([u]), r_e([v])) with liftings solved from the
    collocated mass equals the node-wise IP form of the stabilisation."""
    mesh = _mesh(2, 2)
    p, eta = 3, 7.0
    S_nodewise = (HO.dg_operator(mesh, p, "br2", eta) - HO.dg_operator(mesh, p, "br2", 0.0)).toarray()
    S_lift = HO.br2_lifting_matrix(mesh, p, eta).toarray()
    assert np.abs(S_nodewise - S_lift).max() <= 1e-13 * np.abs(S_lift).max()


def test_br2_cartesian_closed_form():
    """Uniform Cartesian mesh: sigma = eta p(p+1)/(2h) on interior faces and
    eta p(p+1)/h on boundary faces (w_0 = 1/(p(p+1)) on [0,1])."""
    n, p, eta = 3, 4, 2.0
    mesh = M.make_mesh(2, n, inputs.structured_vertices(2, n))
    h = 1.0 / n
    fl, nrm, om, volw_m, _ = HO._face_geometry(mesh, p, 0, (0, 0), 1)
    _, _, _, volw_p, _ = HO._face_geometry(mesh, p, 0, (1, 0), 0)
    assert np.allclose(HO.br2_sigma(eta, om, [volw_m, volw_p]), eta * p * (p + 1) / (2 * h), rtol=1e-13)
    fl, nrm, om, volw, _ = HO._face_geometry(mesh, p, 0, (0, 0), 0)
    assert np.allclose(HO.br2_sigma(eta, om, [volw]), eta * p * (p + 1) / h, rtol=1e-13)
    assert np.allclose(nrm, [[-1.0, 0.0]] * len(fl))


@pytest.mark.parametrize("method", ["ip", "br2"])
def test_spd_for_config_penalties(method):
    """eta in {1.5(p+1)^2, x10, x100, x1e4} gives SPD operators."""
    mesh = _mesh(2, 2)
    p = 3
    for eta in (1.5 * (p + 1) ** 2 * f for f in (1, 10, 100, 1e4)):
        A = HO.dg_operator(mesh, p, method, eta).toarray()
        assert np.linalg.eigvalsh(A).min() > 0


def _dg_l2_error(mesh, p, u, uex):
    dim = mesh.dim
    x, _ = gll.gll(p)
    nq = p + 3
    g, wg = np.polynomial.legendre.leggauss(nq)
    g, wg = (g + 1) / 2, wg / 2
    B = gll.lagrange_eval_matrix(x, g)
    Bt = B
    for _ in range(dim - 1):
        Bt = np.kron(B, Bt)
    qloc = np.indices([nq] * dim).reshape(dim, -1, order="F").T
    nloc = (p + 1) ** dim
    err = 0.0
    for k, e in enumerate(mesh.elements()):
        corners = mesh.element_corners(e)
        uh = Bt @ u[k * nloc:(k + 1) * nloc]
        pts = [g[qloc[:, i]] for i in range(dim)]
        X = np.stack(M.map_point(corners[:, :, None] * np.ones(len(qloc)), pts), axis=1)
        dets = np.array([np.linalg.det(M.map_jacobian(corners, [g[q[i]] for i in range(dim)])) for q in qloc])
        err += np.sum(np.prod(wg[qloc], axis=1) * dets * (uh - uex(X)) ** 2)
    return np.sqrt(err)


@pytest.mark.parametrize("method,p", [("ip", 2), ("br2", 3)])
def test_dg_manufactured_convergence(method, p):
    errs = []
    for n in (2, 4, 8):
        mesh = _mesh(2, n, seed=13)
        A = HO.dg_operator(mesh, p, method, eta=1.5 * (p + 1) ** 2)
        b = HO.dg_rhs(mesh, p, inputs.manufactured_f(HO.dg_node_coords(mesh, p)))
        u = spla.spsolve(A.tocsc(), b)
        errs.append(_dg_l2_error(mesh, p, u, inputs.manufactured_u))
    rate = np.log2(errs[-2] / errs[-1])
    assert rate >= p + 1 - 0.3, errs


@pytest.mark.slow
@pytest.mark.parametrize("method", ["ip", "br2"])
def test_dg_preconditioner_penalty_robust(method):
    """Thm/Cor of Section 3.5: kappa(B_DG A) bounded independently of eta."""
    mesh = _mesh(2, 3)
    p = 3
    ks = []
    for f in (1, 10, 100, 1e4):
        A = HO.dg_operator(mesh, p, method, 1.5 * (p + 1) ** 2 * f)
        P = S.SchwarzDG(mesh, p, A)
        N = A.shape[0]
        Bm = np.column_stack([P.apply(np.eye(N)[:, i]) for i in range(N)])
        ev = np.sort(np.real(sla.eigvals(Bm @ A.toarray())))
        assert ev[0] > 0
        ks.append(ev[-1] / ev[0])
    assert max(ks) / min(ks) <= 1.6, ks


@pytest.mark.parametrize("dim,n,p,method", [(3, (2, 2, 1), 2, "ip"), (3, (2, 1, 2), 3, "br2"), (2, (3, 2), 4, "ip"),
                                            (2, (2, 3), 3, "br2")])
def test_dg_apply_rows_matches_assembled(dim, n, p, method):
    """The row-by-row DG apply (used at full size on sampled rows) equals the
    assembled operator on every row, with boundary faces."""
    V = inputs.structured_vertices(dim, list(n), 0.1, seed=3)
    mesh = M.make_mesh(dim, list(n), V)
    eta = 1.5 * (p + 1) ** 2
    A = HO.dg_operator(mesh, p, method, eta)
    x = inputs.uniform_vector(A.shape[0], 4)
    rows = np.arange(A.shape[0])
    y = HO.dg_apply_rows(mesh, p, method, eta, x, rows)
    ref = A @ x
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
