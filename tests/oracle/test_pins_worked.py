"""Worked-example pins of three oracle parts whose structural pins alone
would let a plausible mistake through:

* the MDF discarded-fill value (Section 3.4; reading C16): hand-computed
  values on a 3 x 3 anisotropic box, before and after the first
  elimination (so that the metric must use the ILU(0)-updated matrix and the
  squared products), and the full order against an exact-rational brute
  force of the same reading;
* the interior-penalty coefficient sigma = eta p^2 / h_e of eq. ip with
  h_e = |K| / |e| (reading C6): on a uniform Cartesian block the penalty part
  of the operator has a closed form (interior and boundary faces);
* the patch V-cycle of Section 3.3 (reading C14): exact on patches that are
  a single grid line (tridiagonal, so IC(0) has no discarded fill), and equal
  on every patch to the textbook two-grid error propagation
  I - V A = (I - M^-T A)(I - P V_c P^T A)(I - M^-1 A), applied recursively.
"""
from fractions import Fraction as Fr
from itertools import product

import numpy as np
import pytest

from oracle import gll, highorder as HO, lor, mdf, mesh as M, schwarz as S
from paper_1908_07071_amd import inputs

# --------------------------------------------------------------------------
# MDF on a 3 x 3 box with the 9-point stencil: centre 16, horizontal -1,
# vertical -4, diagonal -1/2 (node i = x + 3 y).

_W = {(0, 0): 16.0, (1, 0): -1.0, (-1, 0): -1.0, (0, 1): -4.0, (0, -1): -4.0}


def _box_rows():
    rows = np.zeros((9, 9))
    for i in range(9):
        for sl in range(9):
            o = (sl % 3 - 1, sl // 3 - 1)
            rows[i, sl] = _W.get(o, -0.5)
    return rows


def test_mdf_discarded_fill_worked_example():
    g = mdf.PatchGraph([3, 3], _box_rows())
    a = g.rows.copy()
    elim = np.zeros(9, dtype=bool)
    # before any elimination, by hand (uncoupled neighbour pairs of each node):
    # corners: every pair of their 3 neighbours is coupled -> 0
    # node 1: (0,2) 1/16, (0,5) and (3,2) 1/32, (3,5) 1/64, squared -> 25/4096
    # node 3: (0,6) 1, (0,7) and (1,6) 1/8, (1,7) 1/64, squared -> 4225/4096
    # node 4: 16 uncoupled pairs: opposite (1/4)^2 x2, 16^2, 1; rows and
    #         columns of corners (1/4)^2 x4; corner-horizontal (1/2)^2 x4;
    #         corner-vertical 2^2 x4 -> 274.375 / 16^2 = 4390/4096
    want0 = [0, Fr(25, 4096), 0, Fr(4225, 4096), Fr(4390, 4096), Fr(4225, 4096), 0, Fr(25, 4096), 0]
    got0 = [mdf._disc(g, a, elim, m) for m in range(9)]
    for m in range(9):
        assert got0[m] == pytest.approx(float(want0[m]), rel=1e-15, abs=0), m
    # eliminate node 0 (pivot 16): rows 1, 3, 4 are updated on the pattern
    #   a11 = 16 - 1/16 = 255/16, a33 = 16 - 16/16 = 15, a44 = 16 - 1/64
    #   a13 = -1/2 - 4/16 = -3/4, a14 = -4 - 1/32, a34 = -1 - 2/16 = -9/8
    L = np.zeros((9, 9))
    D = np.zeros(9)
    mdf._eliminate(g, a, elim, 0, L, D)
    assert D[0] == 16.0
    assert a[1, 4] == 255 / 16 and a[3, 4] == 15.0 and a[4, 4] == 16 - 1 / 64
    # node 1 now: remaining neighbours 2 (-1), 3 (-3/4), 4, 5 (-1/2);
    # uncoupled pairs (2,3) and (3,5): ((3/4)(16/255))^2 + ((3/8)(16/255))^2
    want1 = (Fr(3, 4) * Fr(16, 255)) ** 2 + (Fr(3, 8) * Fr(16, 255)) ** 2
    assert want1 == Fr(4, 1445)
    # node 3 now: neighbours 1 (-3/4), 4 (-9/8), 6 (-4), 7 (-1/2), pivot 15;
    # uncoupled (1,6) and (1,7): (3/15)^2 + (3/120)^2
    want3 = Fr(3, 15) ** 2 + Fr(3, 120) ** 2
    # node 4 now: pivot 1023/64, neighbours 1 (-129/32), 2 (-1/2), 3 (-9/8),
    # 5 (-1), 6 (-1/2), 7 (-4), 8 (-1/2); its 11 uncoupled pairs:
    prods = [Fr(129, 32) * 4, Fr(129, 64), Fr(129, 64), Fr(9, 16), Fr(1, 4), Fr(2), Fr(1, 4),
             Fr(9, 8), Fr(9, 16), Fr(1, 2), Fr(1, 4)]
    want4 = sum(q * q for q in prods) / Fr(1023, 64) ** 2
    for m, w in ((1, want1), (3, want3), (4, want4)):
        assert mdf._disc(g, a, elim, m) == pytest.approx(float(w), rel=1e-14), m
    # the same metric on the original (not updated) matrix would differ
    assert abs(float(want1) - float(Fr(5, 4096))) > 1e-4
    order, _, _ = mdf.mdf_factor(g)
    assert order.tolist()[:4] == [0, 2, 6, 8]   # corners first, ties to the smallest index
    assert order.tolist() == _exact_mdf_order(_box_rows(), (3, 3))


def _exact_mdf_order(rows, shape):
    """The MDF reading in exact rational arithmetic on a dense matrix:
    pattern = points whose offsets differ by at most one per direction;
    disc(m) = sum over pairs j < l of not-yet-eliminated neighbours of m that
    are not coupled of (a_mj a_ml / a_mm)^2; pick the smallest, ties to the
    smallest index; eliminating i updates a_jl -= a_ji a_il / a_ii on the
    pattern only."""
    nx, ny = shape
    n = nx * ny
    xy = [(i % nx, i // nx) for i in range(n)]
    coupled = [[abs(xy[i][0] - xy[j][0]) <= 1 and abs(xy[i][1] - xy[j][1]) <= 1 for j in range(n)]
               for i in range(n)]
    a = [[Fr(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            if coupled[i][j]:
                dx, dy = xy[j][0] - xy[i][0], xy[j][1] - xy[i][1]
                a[i][j] = Fr(rows[i][(dx + 1) + 3 * (dy + 1)])
    alive = set(range(n))
    order = []
    while alive:
        def disc(m):
            nb = sorted(j for j in alive if j != m and coupled[m][j])
            return sum(((a[m][j] * a[m][l] / a[m][m]) ** 2
                        for x, j in enumerate(nb) for l in nb[x + 1:] if not coupled[j][l]), Fr(0))
        best = min(sorted(alive), key=disc)
        order.append(best)
        alive.remove(best)
        nb = [j for j in alive if coupled[best][j]]
        for j in nb:
            for l in nb:
                if coupled[j][l]:
                    a[j][l] -= a[j][best] * a[best][l] / a[best][best]
    return order


# --------------------------------------------------------------------------
# IP penalty on a uniform Cartesian block

def _dg_index(n, p, dim, e, loc):
    ef = sum(e[t] * n ** t for t in range(dim))
    lf = sum(loc[t] * (p + 1) ** t for t in range(dim))
    return ef * (p + 1) ** dim + lf


@pytest.mark.parametrize("dim,n,p", [(2, 2, 2), (2, 3, 3), (3, 2, 2)])
def test_ip_penalty_closed_form(dim, n, p):
    """A_IP(eta) - A_IP(0) = eta sum_faces sigma_1 omega_q [u][v] with
    sigma_1 = p^2 / h_e, h_e = |K|/|e| = h = 1/n, and the face quadrature
    weight omega_q = h^(d-1) prod of the GLL weights of the face node's
    tangential indices: per face node c = p^2 n^(2-d) prod w.  Interior faces
    couple the two sides (+c on both diagonals, -c between them), boundary
    faces add c to the one side."""
    mesh = M.make_mesh(dim, [n] * dim, inputs.structured_vertices(dim, n))
    eta = 3.0
    Sg = (HO.dg_operator(mesh, p, "ip", eta) - HO.dg_operator(mesh, p, "ip", 0.0)).toarray()
    _, w = gll.gll(p)
    Sw = np.zeros_like(Sg)
    for e in product(range(n), repeat=dim):
        for s in range(dim):                # face normal direction
            for side in (0, 1):             # low / high face of element e
                nb = list(e)
                nb[s] += 1 if side else -1
                for tq in product(range(p + 1), repeat=dim - 1):
                    loc = list(tq[:s]) + [p if side else 0] + list(tq[s:])
                    c = eta * p ** 2 * float(n) ** (2 - dim) * np.prod([w[q] for q in tq])
                    i = _dg_index(n, p, dim, e, loc)
                    Sw[i, i] += c
                    if 0 <= nb[s] < n:      # interior face: the neighbour's mirror node
                        lo = list(loc)
                        lo[s] = 0 if side else p
                        Sw[i, _dg_index(n, p, dim, nb, lo)] -= c
    assert np.abs(Sg - Sw).max() <= 1e-12 * np.abs(Sw).max()


# --------------------------------------------------------------------------
# patch V-cycle

@pytest.mark.parametrize("dim,n,p", [(2, (1, 3), 2), (3, (1, 1, 3), 2), (2, (3, 1), 2)])
def test_vcycle_exact_on_line_patches(dim, n, p):
    """With one element across the block in all directions but one and p = 2,
    every level-0 patch is a single grid line (s - 1 = 1 point across), the
    patch matrix is tridiagonal, IC(0) is its exact factorization, and the
    V-cycle returns A_patch^-1 b (the coarser patch levels are empty)."""
    mesh = M.make_mesh(dim, list(n), inputs.structured_vertices(dim, list(n), 0.1, seed=4))
    H = lor.LORHierarchy(mesh, p)
    rng = np.random.default_rng(2)
    seen = 0
    for v in S.vertices(mesh):
        P = S.Patch(H, v)
        lv = P.levels[0]
        if lv["graph"] is None:
            continue
        assert sorted(lv["shape"])[:-1] == [1] * (dim - 1)
        A = lv["A"]
        assert np.count_nonzero(np.triu(A, 2)) == 0
        b = rng.standard_normal(A.shape[0])
        x = P.solve(b)
        assert np.abs(x - np.linalg.solve(A, b)).max() <= 1e-13 * np.abs(x).max()
        seen += 1
    assert seen > 0


def _vcycle_matrix(P, k):
    """Dense V_k from the error propagation of one pre-smoothing step,
    the coarse correction with V_{k+1}, and one post-smoothing step."""
    lv = P.levels[k]
    A = lv["A"]
    if "Ainv" in lv:
        return np.linalg.inv(A)
    n = A.shape[0]
    I = np.eye(n)
    Minv = np.linalg.inv(mdf.factor_product(lv["graph"], lv["order"], lv["L"], lv["D"]))
    Es = I - Minv @ A
    if lv.get("P") is not None:
        Pk = lv["P"]
        Ec = I - Pk @ _vcycle_matrix(P, k + 1) @ Pk.T @ A
        E = Es @ Ec @ Es
    else:
        E = Es @ Es
    return (I - E) @ np.linalg.inv(A)


@pytest.mark.parametrize("dim,n,p", [(2, (3, 3), 4), (3, (2, 2, 2), 3), (2, (2, 3), 6)])
def test_vcycle_equals_two_grid_error_propagation(dim, n, p):
    mesh = M.make_mesh(dim, list(n), inputs.structured_vertices(dim, list(n), 0.1, seed=5))
    H = lor.LORHierarchy(mesh, p)
    for v in S.vertices(mesh):
        P = S.Patch(H, v)
        if P.levels[0]["graph"] is None:
            continue
        nloc = P.levels[0]["A"].shape[0]
        Vo = np.column_stack([P.solve(np.eye(nloc)[:, i]) for i in range(nloc)])
        Vt = _vcycle_matrix(P, 0)
        assert np.abs(Vo - Vt).max() <= 1e-11 * np.abs(Vt).max(), v
