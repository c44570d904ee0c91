"""Pins of the MDF ordering and the ILU(0)/IC(0) factor it produces (Section 3.4)."""
import numpy as np
import pytest

from oracle import lor, mdf, mesh as M, schwarz as S
from paper_1908_07071_amd import inputs


def _patch_graphs(dim, n, p, pert, seed=1, level=0):
    mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n, pert, seed=seed))
    H = lor.LORHierarchy(mesh, p)
    out = []
    for v in S.vertices(mesh):
        rng = S.patch_ranges(mesh, H.sizes[level], v)
        shape = [hi - lo + 1 for lo, hi in rng]
        if min(shape) <= 0:
            continue
        idx = np.indices(shape).reshape(dim, -1, order="F")
        flat = M.lex_index([idx[i] + rng[i][0] for i in range(dim)], H.shapes[level])
        out.append(mdf.PatchGraph(shape, H.stencils[level][flat]))
    return out


@pytest.mark.parametrize("dim,n,p,pert", [(2, 2, 4, 0.0), (2, 3, 3, 0.1), (3, 2, 2, 0.1), (3, 2, 3, 0.0)])
def test_heap_equals_brute_force(dim, n, p, pert):
    """The O(n log n) heap selection equals the O(n^2) greedy definition."""
    for g in _patch_graphs(dim, n, p, pert):
        o1, L1, D1 = mdf.mdf_factor(g)
        o2, L2, D2 = mdf.mdf_factor(g, brute_force=True)
        assert np.array_equal(o1, o2)
        assert np.array_equal(L1, L2) and np.array_equal(D1, D2)
        assert sorted(o1.tolist()) == list(range(g.n))


@pytest.mark.parametrize("dim,n,p,pert", [(2, 3, 4, 0.1), (3, 2, 3, 0.1)])
def test_ilu0_defining_identity(dim, n, p, pert):
    """ILU(0): (L D L^T)_ij = A_ij on the sparsity pattern of A."""
    for g in _patch_graphs(dim, n, p, pert):
        order, L, D = mdf.mdf_factor(g)
        A = g.dense()
        F = mdf.factor_product(g, order, L, D)
        mask = A != 0
        assert np.abs((F - A)[mask]).max() <= 1e-12 * np.abs(A).max()
        y = mdf.ic0_solve(g, order, L, D, np.arange(g.n, dtype=float))
        assert np.allclose(F @ y, np.arange(g.n), rtol=1e-10, atol=1e-10)


def test_no_fill_pattern_is_exact():
    """A 1D chain (tridiagonal) or a fully coupled 2x2 box has no discarded
    fill: the factor is exact and MDF keeps index order on the ties."""
    rng = np.random.default_rng(0)
    for shape in ([7, 1], [1, 6], [2, 2], [2, 2, 2]):
        dim = len(shape)
        n = int(np.prod(shape))
        # random SPD matrix with the stencil pattern: diagonally dominant
        g0 = mdf.PatchGraph(shape, np.zeros((n, 3 ** dim)))
        rows = np.zeros((n, 3 ** dim))
        for i in range(n):
            for sl in range(3 ** dim):
                j = g0.nb[i, sl]
                if j >= 0 and j > i:
                    v = -rng.uniform(0.1, 1.0)
                    rows[i, sl] = v
                    rows[j, g0.slot_of([-t for t in g0.slots[sl]])] = v
        for i in range(n):
            rows[i, g0.center] = -rows[i].sum() + 1.0
        g = mdf.PatchGraph(shape, rows)
        order, L, D = mdf.mdf_factor(g)
        assert np.allclose(mdf.factor_product(g, order, L, D), g.dense(), rtol=1e-13, atol=1e-13)
        assert list(order) == list(range(n))


def test_corners_first_on_3x3():
    """On a 3x3 box with the 9-point pattern a corner's three neighbours are
    mutually coupled, so its discarded fill is zero; every edge midpoint and
    the centre have uncoupled neighbour pairs.  MDF therefore starts with the
    four corners in index order."""
    for g in _patch_graphs(2, 2, 4, 0.0, level=1):
        if g.shape == (3, 3):
            order, _, _ = mdf.mdf_factor(g)
            assert list(order[:4]) == [0, 2, 6, 8]
            break
    else:
        pytest.fail("no 3x3 patch")


def test_pivot_failure_is_reported():
    shape = [2, 1]
    rows = np.zeros((2, 9))
    rows[:, 4] = [-1.0, 2.0]
    with pytest.raises(mdf.PivotError):
        mdf.mdf_factor(mdf.PatchGraph(shape, rows))


def test_dependency_depth_consistent():
    for g in _patch_graphs(2, 3, 4, 0.1):
        order, _, _ = mdf.mdf_factor(g)
        d = mdf.dependency_depth(g, order)
        assert 1 <= d <= g.n
        # natural order on an m x m 9-point box: point (i, j) waits for
        # (i+1, j-1), so the depth is 2(m_y - 1) + m_x
        dn = mdf.dependency_depth(g, np.arange(g.n))
        mx, my = g.shape
        assert dn == 2 * (my - 1) + mx
