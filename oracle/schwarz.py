"""Vertex-patch additive Schwarz preconditioner with LOR patch V-cycles.

eq. as: B = sum_{j=0}^J R_j Q_j.  j = 0 is the coarse space V_0 (Q1 on the
original mesh T_p); j >= 1 are the vertex patches (eq. patch) carrying the
LOR space with homogeneous Dirichlet conditions on the patch boundary, each
solved approximately by one element-structured V-cycle (Section 3.3) with
MDF-ordered ILU(0) smoothing (Section 3.4).  eq. dg-as extends it to DG.

Readings (the paper is silent or uses a component that is not available):
* one patch per mesh vertex, boundary vertices included; the patch unknowns
  at level k are the level-k grid points strictly inside the union of the
  elements around the vertex and not on the domain boundary;
* patch matrices are principal sub-matrices of the global level matrices;
* V-cycle: one IC(0) pre-smoothing step from zero, residual, restriction,
  recursion, prolongation, one IC(0) post-smoothing step; the coarsest patch
  level (at most one unknown) is solved exactly;
* the coarse operator is the Galerkin product A_0 = P_0^T K_h P_0 with P_0
  the Q1 interpolation of the element vertices, and it is solved exactly
  (the paper uses one AMG V-cycle here);
* the patch corrections are summed without weights (eq. as);
* DG (eq. dg-as): V_p taken as the Dirichlet-conforming space injected by
  copying node values (E), R_B is point Jacobi with diag(A_DG) on the nodes
  with some local index in {0, p}.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import gll as _gll
from . import lor as _lor
from . import mdf as _mdf
from . import mesh as _mesh
from . import highorder as _ho


def patch_ranges(mesh, s: int, v):
    """Per-direction inclusive [lo, hi] level-grid ranges of the patch of vertex v."""
    out = []
    for i in range(mesh.dim):
        n = mesh.n[i]
        lo = (v[i] - 1) * s + 1 if v[i] > 0 else 1
        hi = (v[i] + 1) * s - 1 if v[i] < n else n * s - 1
        out.append((lo, hi))
    return out


def vertices(mesh):
    """Vertex multi-indices in lexicographic order (x fastest)."""
    shape = [m + 1 for m in mesh.n]
    for flat in range(int(np.prod(shape))):
        v, r = [], flat
        for i in range(mesh.dim):
            v.append(r % shape[i])
            r //= shape[i]
        yield tuple(v)


def domain_ranges(mesh, s: int):
    """Per-direction inclusive level-grid ranges of all interior points."""
    return [(1, mesh.n[i] * s - 1) for i in range(mesh.dim)]


def box_ranges(s: int, box):
    """Level-grid ranges of the points strictly inside an element box
    [(a_d, b_d)] (elements a_d .. b_d - 1 in direction d)."""
    return [(a * s + 1, b * s - 1) for a, b in box]


def vertex_box(mesh, v):
    """The elements around vertex v: its patch (eq. patch) as an element box."""
    return [(max(v[i] - 1, 0), min(v[i] + 1, mesh.n[i])) for i in range(mesh.dim)]


def isotropic_boxes(mesh):
    """Vertex patches enlarged for isotropic overlap (Section 4.5: patches
    holding anisotropic elements are extended so that the overlap stays
    isotropic).  Reading: delta = the longest mesh edge at vertex v; in each
    direction and sense the box grows from v, one element at a time, until
    the vertex reached lies at least 0.9 delta away from v (so that edges
    equal up to rounding or a small perturbation count as reached) or the
    boundary is reached.  Distances compare squared Euclidean lengths,
    summed over the coordinates in order, against 0.81 delta^2."""
    X = mesh.vertices
    out = []
    for v in vertices(mesh):
        xv = X[mesh.vertex_index(v)]

        def d2(w):
            diff = X[mesh.vertex_index(w)] - xv
            acc = 0.0
            for t in range(mesh.dim):
                acc = acc + diff[t] * diff[t]
            return acc

        delta2 = 0.0
        for i in range(mesh.dim):
            for sgn in (-1, 1):
                w = list(v)
                w[i] += sgn
                if 0 <= w[i] <= mesh.n[i]:
                    delta2 = max(delta2, d2(w))
        box = []
        for i in range(mesh.dim):
            ext = []
            for sgn in (-1, 1):
                k = 0
                while True:
                    k += 1
                    w = list(v)
                    w[i] += sgn * k
                    if w[i] <= 0 or w[i] >= mesh.n[i] or d2(w) >= 0.81 * delta2:
                        break
                ext.append(k)
            box.append((max(v[i] - ext[0], 0), min(v[i] + ext[1], mesh.n[i])))
        out.append(box)
    return out


def slab_boxes(mesh, nslabs: int, axis: int = 0, overlap: int = 1):
    """B(n) of Section 4.5: n subdomains, here slabs of nearly equal element
    counts along one axis (bounds i n // nslabs), each widened by `overlap`
    elements on its inner sides; the other directions span the domain."""
    n = mesh.n[axis]
    out = []
    for i in range(nslabs):
        a, b = i * n // nslabs, (i + 1) * n // nslabs
        box = [(0, mesh.n[t]) for t in range(mesh.dim)]
        box[axis] = (max(a - overlap, 0), min(b + overlap, n))
        out.append(box)
    return out


class Patch:
    """All levels of one vertex patch: graphs, MDF factors, transfers.

    v = None gives the single patch of the whole domain (Section 4.1,
    "single patch"): every interior point of every level grid, the V-cycle
    running down to the original mesh T_p, whose level is solved exactly."""

    def __init__(self, H: _lor.LORHierarchy, v, exact_local: bool = False, ordering: str = "mdf",
                 box=None):
        mesh = H.mesh
        dim = mesh.dim
        self.v = v
        self.levels = []
        for k in range(H.nlevels):
            if box is not None:
                rng = box_ranges(H.sizes[k], box)
            elif v is not None:
                rng = patch_ranges(mesh, H.sizes[k], v)
            else:
                rng = domain_ranges(mesh, H.sizes[k])
            shape = [hi - lo + 1 for lo, hi in rng]
            if min(shape) <= 0:
                shape = [0] * dim
            idx = np.indices(shape).reshape(dim, -1, order="F") if min(shape) > 0 else np.zeros((dim, 0), int)
            gl = [idx[i] + rng[i][0] for i in range(dim)]
            flat = _mesh.lex_index(gl, H.shapes[k]) if idx.shape[1] else np.zeros(0, np.int64)
            g = _mdf.PatchGraph(shape, H.stencils[k][flat]) if idx.shape[1] else None
            self.levels.append(dict(range=rng, shape=shape, flat=flat, graph=g))
        self.exact_local = exact_local
        nl = H.nlevels
        for k in range(nl):
            lv = self.levels[k]
            g = lv["graph"]
            if g is None:
                continue
            lv["A"] = g.dense()
            if k == nl - 1 or exact_local:
                lv["Ainv"] = np.linalg.inv(lv["A"])
            elif ordering == "mdf":
                lv["order"], lv["L"], lv["D"] = _mdf.mdf_factor(g)
            elif ordering == "rcm":
                lv["order"], lv["L"], lv["D"] = _mdf.factor_in_order(g, _mdf.rcm_order(lv["shape"]))
            elif ordering == "natural":
                lv["order"], lv["L"], lv["D"] = _mdf.factor_in_order(g, np.arange(g.n))
            else:
                raise ValueError(f"unknown ordering {ordering!r}")
        for k in range(nl - 1):
            f, c = self.levels[k], self.levels[k + 1]
            if f["graph"] is None or c["graph"] is None:
                f["P"] = None
                continue
            mats = []
            for i in range(dim):
                P1 = _lor.interp_1d(mesh, H.p, k, i)
                (flo, fhi), (clo, chi) = f["range"][i], c["range"][i]
                mats.append(P1[flo:fhi + 1, clo:chi + 1])
            f["P"] = _lor.kron_x_fastest(mats)

    def smooth(self, k, r):
        lv = self.levels[k]
        return _mdf.ic0_solve(lv["graph"], lv["order"], lv["L"], lv["D"], r)

    def vcycle(self, k, b):
        lv = self.levels[k]
        if lv["graph"] is None:
            return np.zeros(0)
        if "Ainv" in lv:
            return lv["Ainv"] @ b
        A = lv["A"]
        x = self.smooth(k, b)
        if lv.get("P") is not None:
            r = b - A @ x
            xc = self.vcycle(k + 1, lv["P"].T @ r)
            x = x + lv["P"] @ xc
        r = b - A @ x
        return x + self.smooth(k, r)

    def solve(self, r_patch):
        return self.vcycle(0, r_patch)


def local_patch(mesh, p: int, v, fine_coords=None):
    """The patch of vertex v built on the submesh of the (up to 2^d) elements
    around v, with the enclosing mesh's node coordinates.  Rows of the level
    matrices at patch unknowns involve only sub-elements of those elements,
    so the patch (matrices, MDF orders, factors, transfers, V-cycle) equals
    the one built on the whole mesh (pinned), at the cost of 2^d elements.
    Returns (patch, global L-vector index of each level-0 patch unknown in
    the patch's order)."""
    dim = mesh.dim
    if fine_coords is None:
        ref, _ = _gll.gll(p)
        fine_coords = _mesh.global_node_coords(mesh, ref, p)
    elo = [max(v[i] - 1, 0) for i in range(dim)]
    ne = [min(v[i], mesh.n[i] - 1) - elo[i] + 1 for i in range(dim)]
    vidx = np.indices([ne[i] + 1 for i in range(dim)]).reshape(dim, -1, order="F")
    vflat = _mesh.lex_index([vidx[i] + elo[i] for i in range(dim)], [m + 1 for m in mesh.n])
    sub = _mesh.make_mesh(dim, ne, mesh.vertices[vflat])
    gshape = _mesh.grid_shape(mesh, p)
    sshape = _mesh.grid_shape(sub, p)
    gidx = np.indices(sshape).reshape(dim, -1, order="F")
    gflat = _mesh.lex_index([gidx[i] + elo[i] * p for i in range(dim)], gshape)
    H = _lor.LORHierarchy(sub, p, fine_coords=fine_coords[gflat])
    P = Patch(H, tuple(v[i] - elo[i] for i in range(dim)))
    lv = P.levels[0]
    loc = np.unravel_index(lv["flat"], sshape, order="F") if len(lv["flat"]) else [np.zeros(0, int)] * dim
    glob = _mesh.lex_index([np.asarray(loc[i]) + elo[i] * p for i in range(dim)], gshape)
    num = _mesh.interior_numbering(gshape)
    return P, num[glob]


class CoarseSpace:
    """V_0: Q1 on T_p, P_0 = vertex interpolation, A_0 = P_0^T K_h P_0, exact solve."""

    def __init__(self, H: _lor.LORHierarchy, Kh: sp.csr_matrix):
        mesh = H.mesh
        dim = mesh.dim
        mats = [_lor.coarse_interp_1d(mesh, H.p, i) for i in range(dim)]
        P = _lor.kron_x_fastest(mats)
        fnum = _mesh.interior_numbering(H.shapes[0])
        cnum = _mesh.interior_numbering([m + 1 for m in mesh.n])
        P = P[np.flatnonzero(fnum >= 0)][:, np.flatnonzero(cnum >= 0)]
        self.P = sp.csr_matrix(P)
        self.A0 = (self.P.T @ Kh @ self.P).toarray()
        self.n = self.A0.shape[0]
        self.chol = sla.cho_factor(self.A0) if self.n else None

    def apply(self, r):
        if self.n == 0:
            return np.zeros_like(r)
        return self.P @ sla.cho_solve(self.chol, self.P.T @ r)


class SchwarzLOR:
    """z = B r for the conforming problem on the Dirichlet unknowns.

    patch_mode="vertex": one patch per mesh vertex plus the coarse space
    (eq. as); "single": B(1), the V-cycle over the whole domain (Section 4.1);
    "slabs": B(n), nslabs overlapping slabs (Section 4.5); "vertex_iso": the
    vertex patches enlarged for isotropic overlap, plus the coarse space
    (Section 4.5).
    coef: the coefficient b at the elements' GLL nodes (Section 4.2).
    weights="sum": eq. as, the patch corrections added unweighted.
    weights="pou": each patch correction multiplied by Theta_j = diag(1/c(i)),
    c(i) the number of patches whose level-0 unknowns include i (the
    counting-matrix weighting Section 4.1 names as a refinement; a partition
    of unity, sum_j P_j^T Theta_j P_j = I; B is then not symmetric and needs
    flexible CG).  ordering: "mdf" (Section 3.4), "rcm" or "natural" for the
    IC(0) smoother of every patch level."""

    def __init__(self, mesh, p: int, exact_local: bool = False, coarse: bool = True,
                 ordering: str = "mdf", weights: str = "sum", coef=None, patch_mode: str = "vertex",
                 nslabs: int = 2):
        self.H = _lor.LORHierarchy(mesh, p, coef=coef)
        self.Kh = self.H.matrix(0)
        self.fnum = _mesh.interior_numbering(self.H.shapes[0])
        if patch_mode == "single":
            # B(1): one V-cycle over the whole domain; its coarsest level is
            # T_p itself, solved exactly, so no separate coarse space
            self.coarse = None
            self.patches = [Patch(self.H, None, exact_local, ordering)]
        elif patch_mode == "slabs":
            # B(n): n overlapping subdomains, each V-cycle down to its own
            # part of T_p, solved exactly there; no separate coarse space
            self.coarse = None
            self.patches = [Patch(self.H, None, exact_local, ordering, box=b)
                            for b in slab_boxes(mesh, nslabs)]
        elif patch_mode == "vertex_iso":
            self.coarse = CoarseSpace(self.H, self.Kh) if coarse else None
            self.patches = [Patch(self.H, v, exact_local, ordering, box=b)
                            for v, b in zip(vertices(mesh), isotropic_boxes(mesh))]
        elif patch_mode == "vertex":
            self.coarse = CoarseSpace(self.H, self.Kh) if coarse else None
            self.patches = [Patch(self.H, v, exact_local, ordering) for v in vertices(mesh)]
        else:
            raise ValueError(f"unknown patch mode {patch_mode!r}")
        if weights not in ("sum", "pou"):
            raise ValueError(f"unknown weights {weights!r}")
        self.weights = weights
        self.count = np.zeros(self.Kh.shape[0])
        for P in self.patches:
            lv = P.levels[0]
            if lv["graph"] is not None:
                self.count[self.fnum[lv["flat"]]] += 1.0

    def apply(self, r: np.ndarray, with_coarse: bool = True, with_patches: bool = True) -> np.ndarray:
        z = np.zeros_like(r)
        if with_coarse and self.coarse is not None:
            z += self.coarse.apply(r)
        if with_patches:
            for P in self.patches:
                lv = P.levels[0]
                if lv["graph"] is None:
                    continue
                u = self.fnum[lv["flat"]]
                c = P.solve(r[u])
                z[u] += c / self.count[u] if self.weights == "pou" else c
        return z

    def as_matrix(self, **kw) -> np.ndarray:
        n = self.Kh.shape[0]
        return np.column_stack([self.apply(np.eye(n)[:, i], **kw) for i in range(n)])


class SchwarzDG:
    """z = B_DG r = Pi_B^T D_B^-1 Pi_B r + E B E^T r  (eq. dg-as)."""

    def __init__(self, mesh, p: int, A_dg: sp.csr_matrix, **kw):
        self.B = SchwarzLOR(mesh, p, **kw)
        self.E = _ho.cg_to_dg(mesh, p)
        self.mask = _ho.dg_boundary_mask(mesh, p)
        self.diag = A_dg.diagonal()

    def apply(self, r: np.ndarray) -> np.ndarray:
        z = np.where(self.mask, r / self.diag, 0.0)
        return z + self.E @ self.B.apply(self.E.T @ r)
