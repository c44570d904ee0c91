"""Pins of the reverse Cuthill-McKee ordering of the patch smoothers and of
the counting-weighted (partition of unity) Schwarz sum (Sections 3.4, 4.1)."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

from oracle import highorder as HO, krylov, lor, mdf, mesh as M, schwarz as S
from paper_1908_07071_amd import inputs


def _box_adjacency(shape):
    g = mdf.PatchGraph(shape, np.ones((int(np.prod(shape)), 3 ** len(shape))))
    rows, cols = [], []
    for i in range(g.n):
        for sl in range(3 ** g.dim):
            j = g.nb[i, sl]
            if j >= 0 and j != i:
                rows.append(i)
                cols.append(j)
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(g.n, g.n))


@pytest.mark.parametrize("shape", [(3, 3), (5, 4), (7, 7), (1, 6), (5, 7, 3), (11, 11, 11),
                                   (6, 1, 1), (11, 5, 11), (3, 3, 3)])
def test_rcm_equals_scipy(shape):
    """The oracle's RCM is the same permutation as SciPy's implementation on
    the box graph (minimum-degree start, neighbours by increasing degree,
    reversed), hence the same bandwidth."""
    A = _box_adjacency(shape)
    ref = reverse_cuthill_mckee(A, symmetric_mode=True)
    got = mdf.rcm_order(shape)
    assert np.array_equal(got, ref)
    inv = np.empty_like(got)
    inv[got] = np.arange(len(got))
    Ac = A.tocoo()
    bw = np.abs(inv[Ac.row] - inv[Ac.col]).max() if Ac.nnz else 0
    # a breadth-first order has bandwidth below the largest level set plus its
    # neighbours; on a box from a corner that is at most the number of points
    # within Chebyshev distance one of a face of the box
    assert bw < 3 * int(np.prod(shape)) // max(shape) + 3


def test_factor_in_order_is_ilu0():
    mesh = M.make_mesh(3, [2, 2, 2], inputs.structured_vertices(3, 2, 0.1, seed=3))
    H = lor.LORHierarchy(mesh, 3)
    for ordering in ("rcm", "natural"):
        for v in S.vertices(mesh):
            P = S.Patch(H, v, ordering=ordering)
            for k in range(H.nlevels - 1):
                lv = P.levels[k]
                if lv["graph"] is None:
                    continue
                g = lv["graph"]
                F = mdf.factor_product(g, lv["order"], lv["L"], lv["D"])
                A = g.dense()
                assert np.abs((F - A)[A != 0]).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("dim,n,p", [(2, [3, 2], 4), (3, [2, 2, 2], 3)])
def test_pou_counts_closed_form_and_partition(dim, n, p):
    """c(i) counted over the patches equals prod_d c_d(g_d) with c_d = 1 on a
    vertex line (g_d a multiple of p) and 2 between vertices, and the
    weighted restrictions sum to the identity: sum_j P_j^T Theta_j P_j = I."""
    mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n, 0.1, seed=2))
    B = S.SchwarzLOR(mesh, p, weights="pou")
    shape = M.grid_shape(mesh, p)
    num = M.interior_numbering(shape)
    g = np.array(np.unravel_index(np.flatnonzero(num >= 0), shape, order="F"))
    closed = np.prod(np.where(g % p == 0, 1.0, 2.0), axis=0)
    assert np.array_equal(B.count, closed)
    acc = np.zeros(B.Kh.shape[0])
    for P in B.patches:
        lv = P.levels[0]
        if lv["graph"] is not None:
            u = B.fnum[lv["flat"]]
            acc[u] += 1.0 / B.count[u]
    assert np.allclose(acc, 1.0, rtol=0, atol=1e-15)


def test_rcm_and_pou_iterations():
    """Section 3.4 finds MDF- and RCM-ordered ILU smoothing comparable in
    iterations; the partition-of-unity weighting converges with flexible CG."""
    dim, n, p = 2, [4, 4], 4
    mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n, 0.1, seed=1))
    K = HO.cg_stiffness(mesh, p)
    b = inputs.gaussian_rhs(K.shape[0], 5)
    its = {}
    for ordering in ("mdf", "rcm"):
        B = S.SchwarzLOR(mesh, p, ordering=ordering)
        x, its[ordering], _ = krylov.pcg(K, b, B.apply, tol=1e-8)
        assert np.linalg.norm(b - K @ x) <= 1.05e-8 * np.linalg.norm(b)
    assert abs(its["rcm"] - its["mdf"]) <= max(2, 0.1 * its["mdf"]), its
    Bp = S.SchwarzLOR(mesh, p, weights="pou")
    x, itp, _ = krylov.pcg(K, b, Bp.apply, tol=1e-8, flexible=True)
    assert np.linalg.norm(b - K @ x) <= 1.05e-8 * np.linalg.norm(b)
    assert itp <= 2 * its["mdf"], (itp, its)
    # the weighted preconditioner is not symmetric
    Zp = Bp.as_matrix()
    assert np.abs(Zp - Zp.T).max() > 1e-6 * np.abs(Zp).max()
