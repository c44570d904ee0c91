"""Low-order refined (LOR) operator on the Gauss-Lobatto sub-mesh and its hierarchy.

Section 3.1: every element of T_p is cut into the sub-elements spanned by
adjacent GLL points, giving the refined mesh T_h; K_h is the multilinear (Q1)
finite element stiffness on T_h.  Section 3.3: the element-structured
multigrid hierarchy deletes every other interior 1D GLL point per element,
left to right, until none is left (the last level is T_p itself).

Readings (the paper is silent):
* each sub-element is the image of a reference sub-box under its element's
  map, which is again a Q1 map with the sub-box's 8 (4) corner images as
  vertices; its stiffness uses 2^d Gauss-Legendre points;
* coarser levels are rediscretized the same way on the coarser sub-grid;
* transfers are tensor products of 1D linear interpolation in reference
  coordinates, restriction is the transpose.

The sub-element stiffness and the stencil assembly follow a fixed float64
operation order (spelled out in :func:`q1_stiffness` and
:func:`level_stencils`), so that an independent implementation using the
same order obtains identical bits -- the MDF ordering is decided by
comparisons of these values.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import gll as _gll
from . import mesh as _mesh


# ---------------------------------------------------------------------------
# hierarchy (Section 3.3)
# ---------------------------------------------------------------------------

def kept_points(p: int) -> list:
    """Per-level kept 1D GLL indices, level 0 = all p+1 points.

    From [0, i_1, ..., i_m, p] delete i_1, i_3, i_5, ... (every other interior
    point, from the left) until no interior point remains.
    """
    levels = [list(range(p + 1))]
    while len(levels[-1]) > 2:
        cur = levels[-1]
        interior = cur[1:-1]
        keep = [interior[k] for k in range(len(interior)) if k % 2 == 1]
        levels.append([0] + keep + [p])
    return levels


def level_sizes(p: int) -> list:
    """Sub-intervals per element and direction at each level."""
    return [len(k) - 1 for k in kept_points(p)]


def level_fine_index(mesh, p: int, k: int, axis: int) -> np.ndarray:
    """For each level-k 1D grid index G, the level-0 (GLL grid) index."""
    X = kept_points(p)[k]
    s = len(X) - 1
    G = np.arange(mesh.n[axis] * s + 1)
    e = np.minimum(G // s, mesh.n[axis] - 1)
    m = G - e * s
    return e * p + np.array(X)[m]


def level_coords(mesh, p: int, k: int, fine_coords: np.ndarray) -> np.ndarray:
    """Coordinates of the level-k grid points, taken from the GLL grid nodes."""
    dim = mesh.dim
    fshape = _mesh.grid_shape(mesh, p)
    s = level_sizes(p)[k]
    shape = _mesh.grid_shape(mesh, s)
    idx = np.indices(shape).reshape(dim, -1, order="F")
    fidx = [level_fine_index(mesh, p, k, i)[idx[i]] for i in range(dim)]
    return fine_coords[_mesh.lex_index(fidx, fshape)]


# ---------------------------------------------------------------------------
# Q1 sub-element stiffness, pinned operation order
# ---------------------------------------------------------------------------

def gauss2():
    """Two-point Gauss-Legendre abscissae on [0,1]: 1/2 -+ (1/2)/sqrt(3)."""
    gm = 0.5 / math.sqrt(3.0)
    return (0.5 - gm, 0.5 + gm)


def q1_stiffness(corners: np.ndarray) -> np.ndarray:
    """Q1 stiffness of many sub-elements at once.

    ``corners`` is (2^d, d, m): corner c (bits c_x, c_y, c_z) of each of m
    sub-elements.  Returns (2^d, 2^d, m).  Operation order, per Gauss point
    q = q_x + 2 q_y + 4 q_z in ascending order (weight w = 2^-d):

      l(0,t) = 1 - t, l(1,t) = t
      g_c[s] = +-(product of l(c_t, xi_t) over t != s in ascending t)
               (minus when c_s = 0)
      J[r][s] = sum over c ascending of corners[c][r] * g_c[s]  (from 0.0)
      A = adjugate(J) (explicit 2x2 / 3x3 formulas below),
      det = J00*A00 + J01*A10 (+ J02*A20)
      coef = w / det
      u_c[r] = (A[0][r]*g_c[0] + A[1][r]*g_c[1]) (+ A[2][r]*g_c[2])
      K[a][b] += coef * ((u_a[0]*u_b[0] + u_a[1]*u_b[1]) (+ u_a[2]*u_b[2]))
    """
    nc, dim, m = corners.shape
    g = gauss2()
    K = np.zeros((nc, nc, m))
    w = 0.125 if dim == 3 else 0.25
    for q in range(nc):
        xi = [g[(q >> i) & 1] for i in range(dim)]
        lv = [[1.0 - xi[i], xi[i]] for i in range(dim)]
        grads = []
        for c in range(nc):
            bits = [(c >> i) & 1 for i in range(dim)]
            gc = []
            for s in range(dim):
                others = [t for t in range(dim) if t != s]
                val = lv[others[0]][bits[others[0]]]
                for t in others[1:]:
                    val = val * lv[t][bits[t]]
                gc.append(val if bits[s] else -val)
            grads.append(gc)
        J = [[None] * dim for _ in range(dim)]
        for r in range(dim):
            for s in range(dim):
                acc = 0.0
                for c in range(nc):
                    acc = acc + corners[c, r] * grads[c][s]
                J[r][s] = acc
        if dim == 3:
            A = [[J[1][1] * J[2][2] - J[1][2] * J[2][1],
                  J[0][2] * J[2][1] - J[0][1] * J[2][2],
                  J[0][1] * J[1][2] - J[0][2] * J[1][1]],
                 [J[1][2] * J[2][0] - J[1][0] * J[2][2],
                  J[0][0] * J[2][2] - J[0][2] * J[2][0],
                  J[0][2] * J[1][0] - J[0][0] * J[1][2]],
                 [J[1][0] * J[2][1] - J[1][1] * J[2][0],
                  J[0][1] * J[2][0] - J[0][0] * J[2][1],
                  J[0][0] * J[1][1] - J[0][1] * J[1][0]]]
            det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0]
        else:
            A = [[J[1][1], -J[0][1]], [-J[1][0], J[0][0]]]
            det = J[0][0] * J[1][1] - J[0][1] * J[1][0]
        coef = w / det
        us = []
        for c in range(nc):
            u = []
            for r in range(dim):
                acc = A[0][r] * grads[c][0] + A[1][r] * grads[c][1]
                if dim == 3:
                    acc = acc + A[2][r] * grads[c][2]
                u.append(acc)
            us.append(u)
        for a in range(nc):
            for b in range(nc):
                dot = us[a][0] * us[b][0] + us[a][1] * us[b][1]
                if dim == 3:
                    dot = dot + us[a][2] * us[b][2]
                K[a, b] = K[a, b] + coef * dot
    return K


def subelement_corners(coords: np.ndarray, shape) -> np.ndarray:
    """(2^d, d, m) corner coordinates of every cell of a grid of points."""
    dim = len(shape)
    cshape = [s - 1 for s in shape]
    cidx = np.indices(cshape).reshape(dim, -1, order="F")
    out = np.zeros((2 ** dim, dim, cidx.shape[1]))
    for c in range(2 ** dim):
        pidx = [cidx[i] + ((c >> i) & 1) for i in range(dim)]
        out[c] = coords[_mesh.lex_index(pidx, shape)].T
    return out


def stencil_slots(dim: int):
    """Stencil offsets o in {-1,0,1}^d, slot = sum_i (o_i+1) 3^i, ascending."""
    return [tuple(((sl // 3 ** i) % 3) - 1 for i in range(dim)) for sl in range(3 ** dim)]


def level_cell_coef(mesh, p: int, k: int, coef: np.ndarray) -> np.ndarray:
    """Coefficient of every cell of the level-k grid (reading: a LOR
    sub-element takes the mean of b at its 2^d corners, which are GLL nodes
    of the element containing it): corners c = c_x + 2 c_y + 4 c_z summed
    in ascending order from 0.0, then multiplied by 2^-d.  coef is
    (n_el, (p+1)^d) as in highorder.cg_stiffness."""
    dim = mesh.dim
    X = kept_points(p)[k]
    s = len(X) - 1
    cshape = [mesh.n[i] * s for i in range(dim)]
    cidx = np.indices(cshape).reshape(dim, -1, order="F")
    e = [cidx[i] // s for i in range(dim)]
    m = [cidx[i] - e[i] * s for i in range(dim)]
    eflat = _mesh.lex_index(e, list(mesh.n))
    acc = np.zeros(cidx.shape[1])
    for c in range(2 ** dim):
        loc = [np.array(X)[m[i] + ((c >> i) & 1)] for i in range(dim)]
        lflat = _mesh.lex_index(loc, [p + 1] * dim)
        acc = acc + coef[eflat, lflat]
    return acc * (0.125 if dim == 3 else 0.25)


def level_stencils(coords: np.ndarray, shape, cell_coef=None) -> np.ndarray:
    """Assembled Q1 stiffness of a grid as (num_points, 3^d) stencil values.

    Entry (g, slot o) = sum over the cells S adjacent to g, in the order
    s = s_x + 2 s_y + 4 s_z of S = g - 1 + s, of K_S[corner of g][corner of
    g+o] whenever g+o is also a corner of S; accumulated from 0.0.  With a
    coefficient each K_S entry is first multiplied by the cell's b_S.
    Entries reaching outside the grid are zero.
    """
    dim = len(shape)
    K = q1_stiffness(subelement_corners(coords, shape))
    if cell_coef is not None:
        K = K * cell_coef[None, None, :]
    cshape = [s - 1 for s in shape]
    npts = int(np.prod(shape))
    gidx = np.indices(shape).reshape(dim, -1, order="F")
    slots = stencil_slots(dim)
    out = np.zeros((npts, len(slots)))
    for sl, o in enumerate(slots):
        acc = np.zeros(npts)
        for sc in range(2 ** dim):
            S = [gidx[i] - 1 + ((sc >> i) & 1) for i in range(dim)]
            ok = np.ones(npts, dtype=bool)
            ca = np.zeros(npts, dtype=np.int64)
            cb = np.zeros(npts, dtype=np.int64)
            for i in range(dim):
                ok &= (S[i] >= 0) & (S[i] < cshape[i])
                la = gidx[i] - S[i]          # corner bit of g in S
                lb = gidx[i] + o[i] - S[i]   # corner bit of g+o in S
                ok &= (lb >= 0) & (lb <= 1)
                ca += la << i
                cb += lb << i
            cell = _mesh.lex_index([np.clip(S[i], 0, cshape[i] - 1) for i in range(dim)], cshape)
            vals = K[np.clip(ca, 0, 2 ** dim - 1), np.clip(cb, 0, 2 ** dim - 1), cell]
            acc = np.where(ok, acc + vals, acc)
        out[:, sl] = acc
    return out


def stencil_matrix(stencils: np.ndarray, shape, rows_mask=None) -> sp.csr_matrix:
    """Sparse matrix of a stencil field restricted to the interior points."""
    dim = len(shape)
    num = _mesh.interior_numbering(shape)
    npts = int(np.prod(shape))
    gidx = np.indices(shape).reshape(dim, -1, order="F")
    rows, cols, vals = [], [], []
    for sl, o in enumerate(stencil_slots(dim)):
        nb = [gidx[i] + o[i] for i in range(dim)]
        ok = num >= 0
        for i in range(dim):
            ok &= (nb[i] >= 0) & (nb[i] < shape[i])
        nbflat = _mesh.lex_index([np.clip(nb[i], 0, shape[i] - 1) for i in range(dim)], shape)
        ok &= num[nbflat] >= 0
        rows.append(num[ok])
        cols.append(num[nbflat[ok]])
        vals.append(stencils[ok, sl])
    n = int((num >= 0).sum())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()


class LORHierarchy:
    """Global LOR level grids, coordinates and stencils for a mesh and degree p."""

    def __init__(self, mesh, p: int, fine_coords=None, coef=None):
        """fine_coords: the GLL node coordinates of mesh (computed when None);
        given for a submesh, they keep the nodes on its boundary bitwise equal
        to the enclosing mesh's, which evaluates interface nodes with the
        lower-indexed element's map.  coef: b at the elements' GLL nodes
        (n_el, (p+1)^d), None for b = 1."""
        self.mesh, self.p = mesh, p
        self.ref_nodes, _ = _gll.gll(p)
        self.fine_coords = (_mesh.global_node_coords(mesh, self.ref_nodes, p) if fine_coords is None
                            else np.asarray(fine_coords, dtype=np.float64))
        self.kept = kept_points(p)
        self.sizes = [len(k) - 1 for k in self.kept]
        self.nlevels = len(self.kept)
        self.shapes = [_mesh.grid_shape(mesh, s) for s in self.sizes]
        self.coords = [level_coords(mesh, p, k, self.fine_coords) for k in range(self.nlevels)]
        self.coef = coef
        self.stencils = [level_stencils(self.coords[k], self.shapes[k],
                                        None if coef is None else level_cell_coef(mesh, p, k, coef))
                         for k in range(self.nlevels)]

    def matrix(self, k: int) -> sp.csr_matrix:
        return stencil_matrix(self.stencils[k], self.shapes[k])


# ---------------------------------------------------------------------------
# transfers (1D linear interpolation in reference coordinates)
# ---------------------------------------------------------------------------

def interp_1d(mesh, p: int, k: int, axis: int) -> np.ndarray:
    """Dense (n s_k + 1) x (n s_{k+1} + 1) interpolation from level k+1 to k."""
    x, _ = _gll.gll(p)
    Xf, Xc = kept_points(p)[k], kept_points(p)[k + 1]
    sf, sc = len(Xf) - 1, len(Xc) - 1
    n = mesh.n[axis]
    P = np.zeros((n * sf + 1, n * sc + 1))
    for G in range(n * sf + 1):
        e = min(G // sf, n - 1)
        a = Xf[G - e * sf]
        if a in Xc:
            P[G, e * sc + Xc.index(a)] = 1.0
            continue
        hi = min(j for j in range(len(Xc)) if Xc[j] > a)
        lo = hi - 1
        xl, xh = x[Xc[lo]], x[Xc[hi]]
        P[G, e * sc + lo] = (xh - x[a]) / (xh - xl)
        P[G, e * sc + hi] = (x[a] - xl) / (xh - xl)
    return P


def kron_x_fastest(mats):
    """Kronecker product acting on x-fastest flattened tensors: kron(z, y, x)."""
    M = mats[-1]
    for A in reversed(mats[:-1]):
        M = np.kron(M, A)
    return M


def coarse_interp_1d(mesh, p: int, axis: int) -> np.ndarray:
    """(n p + 1) x (n + 1) interpolation from element vertices to the GLL grid."""
    x, _ = _gll.gll(p)
    n = mesh.n[axis]
    P = np.zeros((n * p + 1, n + 1))
    for g in range(n * p + 1):
        e = min(g // p, n - 1)
        a = g - e * p
        P[g, e] += 1.0 - x[a]
        P[g, e + 1] += x[a]
    return P
