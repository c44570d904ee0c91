"""Structured tensor-product meshes and their trilinear element maps.

Section 2: every element of the mesh T_p is the image of the unit cube
[0,1]^d under a map; on a structured block the map of element e is the
(bi/tri)linear interpolation of its 2^d vertices.  Numbering conventions
(the paper is silent on them):

* vertices, elements, element-local nodes and global nodes are lexicographic
  with x fastest;
* element corner c has bits (c_x, c_y[, c_z]), c = c_x + 2 c_y + 4 c_z;
* the global Gauss-Lobatto node grid has n_i p + 1 points per direction; a
  global node with 1D index g is evaluated with the map of element
  min(g // p, n_i - 1), at local index g - p*e.

The coordinates of global nodes are computed with a fixed sequence of float64
operations (documented in :func:`map_point`), so that an independent
implementation that follows the same order reproduces them exactly.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    dim: int
    n: tuple  # elements per direction
    vertices: np.ndarray  # (prod(n+1), dim)
    # curved (isoparametric) geometry: the coordinates of every global GLL
    # node for degree nodes_p, x fastest; element e is then the image of
    # [0,1]^d under the degree-nodes_p interpolant of its own nodes
    nodes: np.ndarray | None = None
    nodes_p: int | None = None

    @property
    def nel(self) -> int:
        return int(np.prod(self.n))

    def vertex_index(self, v):
        """Flat vertex index of integer vertex coordinates v (x fastest)."""
        idx, stride = 0, 1
        for i in range(self.dim):
            idx += v[i] * stride
            stride *= self.n[i] + 1
        return idx

    def element_corners(self, e_multi) -> np.ndarray:
        """(2^d, dim) corner coordinates of element with multi-index e."""
        out = []
        for c in range(2 ** self.dim):
            v = [e_multi[i] + ((c >> i) & 1) for i in range(self.dim)]
            out.append(self.vertices[self.vertex_index(v)])
        return np.array(out)

    def elements(self):
        """Element multi-indices in lexicographic order (x fastest)."""
        shape = list(self.n)
        for flat in range(self.nel):
            e, r = [], flat
            for i in range(self.dim):
                e.append(r % shape[i])
                r //= shape[i]
            yield tuple(e)


def make_mesh(dim: int, n, vertices: np.ndarray, nodes=None, nodes_p=None) -> Mesh:
    n = tuple([int(n)] * dim) if np.isscalar(n) else tuple(int(v) for v in n)
    vertices = np.asarray(vertices, dtype=np.float64)
    if vertices.shape != (int(np.prod([v + 1 for v in n])), dim):
        raise ValueError("vertex array has the wrong shape")
    if nodes is not None:
        nodes = np.asarray(nodes, dtype=np.float64)
        if nodes.shape != (int(np.prod([v * nodes_p + 1 for v in n])), dim):
            raise ValueError("node array has the wrong shape")
    return Mesh(dim, n, vertices, nodes, nodes_p)


def shape_q1(dim: int, xi) -> list:
    """Q1 shape functions phi_c(xi) in the pinned evaluation order.

    l(0, t) = 1 - t, l(1, t) = t;  phi_c = (l(c_x, xi_0) * l(c_y, xi_1)) * l(c_z, xi_2).
    Works elementwise on arrays of points.
    """
    one_m = [1.0 - xi[i] for i in range(dim)]
    phis = []
    for c in range(2 ** dim):
        f = xi[0] if (c & 1) else one_m[0]
        for i in range(1, dim):
            f = f * (xi[i] if ((c >> i) & 1) else one_m[i])
        phis.append(f)
    return phis


def map_point(corners: np.ndarray, xi) -> list:
    """Physical coordinates of reference point(s) xi under the Q1 map.

    X_r = sum over corners c = 0, 1, ... of corners[c, r] * phi_c(xi),
    accumulated left to right starting from 0.0.  ``corners`` may be
    (2^d, dim) or (2^d, dim, m) for m maps evaluated at once.
    """
    dim = corners.shape[1]
    phis = shape_q1(dim, xi)
    out = []
    for r in range(dim):
        acc = 0.0
        for c in range(2 ** dim):
            acc = acc + corners[c, r] * phis[c]
        out.append(acc)
    return out


def map_jacobian(corners: np.ndarray, xi) -> np.ndarray:
    """J[r, s] = dX_r / dxi_s of the Q1 map at reference point xi."""
    dim = corners.shape[1]
    J = np.zeros((dim, dim))
    for c in range(2 ** dim):
        bits = [(c >> i) & 1 for i in range(dim)]
        for s in range(dim):
            g = 1.0
            for i in range(dim):
                if i == s:
                    g *= 1.0 if bits[i] else -1.0
                else:
                    g *= xi[i] if bits[i] else 1.0 - xi[i]
            J[:, s] += corners[c] * g
    return J


def global_node_coords(mesh: Mesh, ref_nodes: np.ndarray, p: int) -> np.ndarray:
    """Coordinates of all (n_i p + 1)^d global Gauss-Lobatto nodes.

    Returns (num_nodes, dim), lexicographic with x fastest.  A node on an
    element interface is evaluated with the map of the lower-indexed
    neighbour (the element min(g // p, n - 1) in each direction).
    """
    dim = mesh.dim
    if mesh.nodes is not None:
        if p != mesh.nodes_p:
            raise ValueError("a curved mesh carries its nodes for one degree")
        return mesh.nodes.copy()
    ng = [mesh.n[i] * p + 1 for i in range(dim)]
    gidx = np.indices(ng).reshape(dim, -1, order="F")  # (dim, num), x fastest
    elem = [np.minimum(gidx[i] // p, mesh.n[i] - 1) for i in range(dim)]
    loc = [gidx[i] - p * elem[i] for i in range(dim)]
    num = gidx.shape[1]
    # corners of each node's element, shape (2^d, dim, num)
    corners = np.zeros((2 ** dim, dim, num))
    for c in range(2 ** dim):
        vflat = np.zeros(num, dtype=np.int64)
        stride = 1
        for i in range(dim):
            vflat += (elem[i] + ((c >> i) & 1)) * stride
            stride *= mesh.n[i] + 1
        corners[c] = mesh.vertices[vflat].T
    xi = [ref_nodes[loc[i]] for i in range(dim)]
    X = map_point(corners, xi)
    return np.stack(X, axis=1)


def grid_shape(mesh: Mesh, s: int):
    """Points per direction of the global grid with s sub-intervals per element."""
    return [mesh.n[i] * s + 1 for i in range(mesh.dim)]


def lex_index(idx, shape) -> np.ndarray:
    """Flat lexicographic index (x fastest) of multi-index arrays idx[i]."""
    out = np.zeros_like(np.asarray(idx[0]), dtype=np.int64)
    stride = 1
    for i in range(len(shape)):
        out = out + np.asarray(idx[i], dtype=np.int64) * stride
        stride *= shape[i]
    return out


def interior_numbering(shape) -> np.ndarray:
    """Map flat grid index -> unknown index (-1 on the boundary).

    Unknowns are the grid points not on the boundary of the block, numbered
    lexicographically with x fastest (the conforming "L-vector").
    """
    dim = len(shape)
    idx = np.indices(shape).reshape(dim, -1, order="F")
    inside = np.ones(idx.shape[1], dtype=bool)
    for i in range(dim):
        inside &= (idx[i] > 0) & (idx[i] < shape[i] - 1)
    num = -np.ones(idx.shape[1], dtype=np.int64)
    num[inside] = np.arange(int(inside.sum()))
    return num
