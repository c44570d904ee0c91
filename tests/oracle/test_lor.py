"""Pins of the low-order refined operator and its element-structured
hierarchy (Sections 3.1 and 3.3)."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import gll, highorder as HO, lor, mesh as M
from paper_1908_07071_amd import inputs


def test_coarsening_rule():
    """Delete every other interior point, left to right, until none remain."""
    assert lor.kept_points(6) == [[0, 1, 2, 3, 4, 5, 6], [0, 2, 4, 6], [0, 4, 6], [0, 6]]
    assert lor.kept_points(3) == [[0, 1, 2, 3], [0, 2, 3], [0, 3]]
    assert lor.kept_points(2) == [[0, 1, 2], [0, 2]]
    assert lor.kept_points(8) == [list(range(9)), [0, 2, 4, 6, 8], [0, 4, 8], [0, 8]]
    for p in range(1, 21):
        kp = lor.kept_points(p)
        assert kp[-1] == [0, p]
        assert len(kp) == 1 + math.ceil(math.log2(p))  # O(log p) levels


def _p1_1d(nodes):
    n = len(nodes)
    K = np.zeros((n, n))
    Mm = np.zeros((n, n))
    for i in range(n - 1):
        h = nodes[i + 1] - nodes[i]
        K[i:i + 2, i:i + 2] += np.array([[1, -1], [-1, 1]]) / h
        Mm[i:i + 2, i:i + 2] += np.array([[2, 1], [1, 2]]) * h / 6
    return K, Mm


@pytest.mark.parametrize("dim,n,p", [(2, 2, 3), (2, 3, 4), (3, 2, 3)])
def test_kronecker_lor_closed_form(dim, n, p):
    """Section 3.1: on a Cartesian mesh K_h = sum_j (x) (K1D_h in slot j, M1D_h
    elsewhere) with the exact P1 matrices on the GLL sub-intervals; this holds
    on every level of the hierarchy."""
    mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n))
    H = lor.LORHierarchy(mesh, p)
    for k in range(H.nlevels):
        A = H.matrix(k).toarray()
        # 1D node positions of the level grid (uniform mesh: coordinate of x-axis)
        shape = H.shapes[k]
        coords1d = H.coords[k][:shape[0], 0]
        K1, M1 = _p1_1d(coords1d)
        I = slice(1, shape[0] - 1)
        K1, M1 = K1[I, I], M1[I, I]
        ref = 0
        for j in range(dim):
            mats = [K1 if i == j else M1 for i in range(dim)]
            T = mats[-1]
            for B in reversed(mats[:-1]):
                T = np.kron(T, B)
            ref = ref + T
        assert np.abs(A - ref).max() <= 1e-12 * np.abs(ref).max(), k


@pytest.mark.parametrize("dim,n,p", [(2, 3, 4), (3, 2, 3)])
def test_lor_constants_and_symmetry(dim, n, p):
    mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n, 0.1, seed=8))
    H = lor.LORHierarchy(mesh, p)
    for k in range(H.nlevels):
        st = H.stencils[k]
        shape = H.shapes[k]
        num = M.interior_numbering(shape)
        # rows of interior points sum to zero (K_h 1 = 0 before boundary conditions)
        rowsum = st[num >= 0].sum(axis=1)
        assert np.abs(rowsum).max() <= 1e-13 * np.abs(st).max()
        A = H.matrix(k).toarray()
        assert np.array_equal(A, A.T)  # bit-exact symmetry of the pinned assembly


@pytest.mark.parametrize("dim,n,p", [(2, 2, 4), (3, 2, 4)])
def test_rediscretized_equals_galerkin_on_affine(dim, n, p):
    """Nested spaces and exact 2-point Gauss integration on affine cells:
    the rediscretized coarser level equals P^T A P."""
    V = inputs.structured_vertices(dim, n) * np.array([1.0, 0.6, 0.8][:dim])
    mesh = M.make_mesh(dim, n, V)
    H = lor.LORHierarchy(mesh, p)
    for k in range(H.nlevels - 1):
        Af = H.matrix(k).toarray()
        Ac = H.matrix(k + 1).toarray()
        P = lor.kron_x_fastest([lor.interp_1d(mesh, p, k, i) for i in range(dim)])
        fnum = M.interior_numbering(H.shapes[k])
        cnum = M.interior_numbering(H.shapes[k + 1])
        P = P[np.flatnonzero(fnum >= 0)][:, np.flatnonzero(cnum >= 0)]
        assert np.abs(P.T @ Af @ P - Ac).max() <= 1e-12 * np.abs(Ac).max()


def test_interpolation_reproduces_linears():
    mesh = M.make_mesh(2, 3, inputs.structured_vertices(2, 3))
    p = 6
    x, _ = gll.gll(p)
    for k in range(len(lor.kept_points(p)) - 1):
        P = lor.interp_1d(mesh, p, k, 0)
        fpos = lor.level_fine_index(mesh, p, k, 0)
        cpos = lor.level_fine_index(mesh, p, k + 1, 0)
        # reference coordinate of a grid point = element index + GLL coordinate
        def ref(fi):
            e = np.minimum(fi // p, mesh.n[0] - 1)
            return e + x[fi - e * p]
        for f in (np.ones_like, lambda t: t):
            assert np.allclose(P @ f(ref(cpos).astype(float)), f(ref(fpos).astype(float)), atol=1e-14)


def test_spectral_equivalence_bounded_in_p():
    """Prop. fem-sem: c K_h <= K_p <= C K_h with constants independent of p."""
    mesh = M.make_mesh(2, 2, inputs.structured_vertices(2, 2, 0.1, seed=3))
    lam = []
    for p in (2, 4, 6, 8):
        Kp = HO.cg_stiffness(mesh, p).toarray()
        Kh = lor.LORHierarchy(mesh, p).matrix(0).toarray()
        ev = sla.eigvalsh(Kp, Kh)
        lam.append((ev[0], ev[-1]))
    lo = min(l for l, _ in lam)
    hi = max(h for _, h in lam)
    assert lo > 0.8 and hi < 7.0, lam
    # growth from p = 6 to p = 8 is small (pre-asymptotic regime ends)
    assert lam[-1][1] / lam[-2][1] < 1.15, lam
