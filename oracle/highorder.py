"""High-order CG stiffness, right-hand side and the IP / BR2 DG operators.

Everything here is the plain definition, assembled from dense element
matrices built with explicit tensor-product basis derivatives -- no sum
factorization (eq. fem / eq. system for CG, eq. ip / eq. br2 for DG).

Readings where the paper is silent:
* nodal Lagrange basis at the p+1 GLL points of [0,1] and collocated GLL
  quadrature in the volume ((p+1)^d points) and on faces ((p+1)^(d-1) points);
* right-hand side b = M_p f with the collocated (diagonal) mass matrix;
* CG: homogeneous Dirichlet conditions by eliminating boundary nodes;
* DG: boundary faces impose u = 0 weakly with [u] = u n and {grad u} = grad u;
* IP penalty sigma = eta p^2 / h_e, h_e = min over the adjacent elements K of
  |K| / |e| (GLL quadrature), constant on each face;
* BR2 lifting with the collocated element mass matrix, so that the lifting of
  a face lives only on that face's nodes and the BR2 term is an IP term with a
  node-wise penalty (see :func:`br2_sigma`).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import gll as _gll
from . import mesh as _mesh


def _tensor_ref_grad(p: int, dim: int):
    """Reference derivative tables Gs[s][q, i] = d phi_i / d xi_s at node q."""
    x, _ = _gll.gll(p)
    D = _gll.lagrange_derivative_matrix(x)
    I = np.eye(p + 1)
    mats = []
    for s in range(dim):
        # flat local index is x fastest, i.e. kron(..., z, y, x) with x last
        factors = [D if t == s else I for t in range(dim)]
        M = factors[dim - 1]
        for t in range(dim - 2, -1, -1):
            M = np.kron(M, factors[t])
        mats.append(M)
    return mats


def _local_multi(p: int, dim: int) -> np.ndarray:
    """(nloc, dim) local node multi-indices, x fastest."""
    return np.indices([p + 1] * dim).reshape(dim, -1, order="F").T


def element_geometry(mesh, p: int, e):
    """Jacobian, determinant and inverse at the (p+1)^d GLL nodes of element e.

    Straight-sided elements: the Q1 map of the element's vertices.  Curved
    (isoparametric) elements: J[q][r][s] = sum_j X_j[r] d phi_j/d xi_s (x_q)
    from the element's own GLL node coordinates X_j."""
    x, w = _gll.gll(p)
    dim = mesh.dim
    loc = _local_multi(p, dim)
    if mesh.nodes is not None:
        if p != mesh.nodes_p:
            raise ValueError("a curved mesh carries its nodes for one degree")
        Xe = mesh.nodes[element_global_nodes(mesh, p, e)]
        Gs = _tensor_ref_grad(p, dim)
        Js = np.stack([np.stack([Gs[s_] @ Xe[:, r] for s_ in range(dim)], axis=1) for r in range(dim)], axis=1)
        dets = np.linalg.det(Js)
        Jinv = np.linalg.inv(Js)
        wq = np.prod(w[loc], axis=1)
        return Js, dets, Jinv, wq
    corners = mesh.element_corners(e)
    Js = np.array([_mesh.map_jacobian(corners, [x[q[i]] for i in range(dim)]) for q in loc])
    dets = np.linalg.det(Js)
    Jinv = np.linalg.inv(Js)
    wq = np.prod(w[loc], axis=1)
    return Js, dets, Jinv, wq


def element_stiffness(mesh, p: int, e, coef=None) -> np.ndarray:
    """A_e[i, j] = sum_q w_q |J_q| b_q grad(phi_i)(x_q) . grad(phi_j)(x_q)."""
    dim = mesh.dim
    Gs = _tensor_ref_grad(p, dim)
    _, dets, Jinv, wq = element_geometry(mesh, p, e)
    wd = wq * dets
    if coef is not None:
        wd = wd * coef
    A = np.zeros((len(wq), len(wq)))
    for r in range(dim):
        # physical derivative d/dx_r = sum_s (J^-1)[s, r] d/dxi_s
        Gr = sum(Jinv[:, s, r][:, None] * Gs[s] for s in range(dim))
        A += Gr.T @ (wd[:, None] * Gr)
    return A


def physical_grad_rows(mesh, p: int, e):
    """(dim, nq, nloc) physical gradients of all basis functions at all nodes."""
    dim = mesh.dim
    Gs = _tensor_ref_grad(p, dim)
    _, _, Jinv, _ = element_geometry(mesh, p, e)
    return np.stack([sum(Jinv[:, s, r][:, None] * Gs[s] for s in range(dim)) for r in range(dim)])


def element_global_nodes(mesh, p: int, e) -> np.ndarray:
    """Flat global GLL-grid index of each local node of element e."""
    dim = mesh.dim
    loc = _local_multi(p, dim)
    shape = _mesh.grid_shape(mesh, p)
    idx = [e[i] * p + loc[:, i] for i in range(dim)]
    return _mesh.lex_index(idx, shape)


def cg_stiffness(mesh, p: int, dirichlet: bool = True, coef=None) -> sp.csr_matrix:
    """Assembled K_p over the unknowns (all grid nodes if not dirichlet).

    coef: the coefficient b of -div(b grad u) = f (Section 4.2) at every
    element's GLL nodes, (n_el, (p+1)^d) with elements and local nodes
    lexicographic (x fastest); None for b = 1.  With collocated quadrature b
    enters as a factor of each node's weight."""
    shape = _mesh.grid_shape(mesh, p)
    num = _mesh.interior_numbering(shape) if dirichlet else np.arange(int(np.prod(shape)))
    rows, cols, vals = [], [], []
    for e in mesh.elements():
        A = element_stiffness(mesh, p, e, None if coef is None else coef[_elem_flat(mesh, e)])
        g = num[element_global_nodes(mesh, p, e)]
        keep = g >= 0
        gi, gj = np.meshgrid(g[keep], g[keep], indexing="ij")
        rows.append(gi.ravel())
        cols.append(gj.ravel())
        vals.append(A[np.ix_(keep, keep)].ravel())
    n = int((num >= 0).sum())
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return K.tocsr()


def cg_rhs(mesh, p: int, f_nodes: np.ndarray, dirichlet: bool = True) -> np.ndarray:
    """b = M_p f with the collocated mass: b_i = sum_{e containing i} w_i |J_i| f(x_i).

    ``f_nodes`` holds f at every point of the global GLL grid (x fastest).
    """
    shape = _mesh.grid_shape(mesh, p)
    num = _mesh.interior_numbering(shape) if dirichlet else np.arange(int(np.prod(shape)))
    b = np.zeros(int((num >= 0).sum()))
    for e in mesh.elements():
        _, dets, _, wq = element_geometry(mesh, p, e)
        gl = element_global_nodes(mesh, p, e)
        g = num[gl]
        keep = g >= 0
        np.add.at(b, g[keep], (wq * dets * f_nodes[gl])[keep])
    return b


def cg_apply_rows(mesh, p: int, x: np.ndarray, rows: np.ndarray, coef=None) -> np.ndarray:
    """(K_p x)[rows] for selected unknowns, assembling only the elements touching them."""
    dim = mesh.dim
    shape = _mesh.grid_shape(mesh, p)
    num = _mesh.interior_numbering(shape)
    inv = np.flatnonzero(num >= 0)  # unknown -> flat grid index
    out = np.zeros(len(rows))
    for k, r in enumerate(rows):
        g = np.unravel_index(inv[r], shape, order="F")
        elems = set()
        for c in range(2 ** dim):
            e = []
            for i in range(dim):
                ei = g[i] // p - ((c >> i) & 1) if g[i] % p == 0 else g[i] // p
                e.append(ei)
            if all(0 <= e[i] < mesh.n[i] for i in range(dim)):
                elems.add(tuple(e))
        acc = 0.0
        for e in sorted(elems):
            A = element_stiffness(mesh, p, e, None if coef is None else coef[_elem_flat(mesh, e)])
            gl = element_global_nodes(mesh, p, e)
            li = int(np.flatnonzero(gl == inv[r])[0])
            u = num[gl]
            xe = np.where(u >= 0, x[np.maximum(u, 0)], 0.0)
            acc += A[li] @ xe
        out[k] = acc
    return out


# ----------------------------------------------------------------------------
# Discontinuous Galerkin (eq. ip, eq. br2)
# ----------------------------------------------------------------------------

def dg_node_coords(mesh, p: int) -> np.ndarray:
    """Coordinates of the E-vector nodes (element-major, local x fastest)."""
    x, _ = _gll.gll(p)
    dim = mesh.dim
    loc = _local_multi(p, dim)
    out = []
    for e in mesh.elements():
        corners = mesh.element_corners(e)
        xi = [x[loc[:, i]] for i in range(dim)]
        out.append(np.stack(_mesh.map_point(corners[:, :, None] * np.ones(len(loc)), xi), axis=1))
    return np.concatenate(out)


def faces(mesh):
    """All faces: (s, f_multi, e_minus or None, e_plus or None).

    Faces normal to direction s = 0, 1, 2 in turn; within one direction,
    lexicographic in the face multi-index f (f_s in 0..n_s, x fastest).
    """
    dim = mesh.dim
    out = []
    for s in range(dim):
        shape = [mesh.n[i] + (1 if i == s else 0) for i in range(dim)]
        for flat in range(int(np.prod(shape))):
            f, r = [], flat
            for i in range(dim):
                f.append(r % shape[i])
                r //= shape[i]
            em = list(f)
            em[s] -= 1
            ep = list(f)
            minus = tuple(em) if f[s] > 0 else None
            plus = tuple(ep) if f[s] < mesh.n[s] else None
            out.append((s, tuple(f), minus, plus))
    return out


def _face_local(p: int, dim: int, s: int, side: int) -> np.ndarray:
    """Local node indices of an element's face normal to s (side 0: xi_s=0, 1: xi_s=1)."""
    loc = _local_multi(p, dim)
    return np.flatnonzero(loc[:, s] == (p if side else 0))


def _elem_flat(mesh, e) -> int:
    idx, stride = 0, 1
    for i in range(mesh.dim):
        idx += e[i] * stride
        stride *= mesh.n[i]
    return idx


def _face_geometry(mesh, p, s, e, side):
    """Outward unit normal, surface weights and volume weights on one face of e."""
    x, w = _gll.gll(p)
    dim = mesh.dim
    Js, dets, Jinv, wq = element_geometry(mesh, p, e)
    fl = _face_local(p, dim, s, side)
    loc = _local_multi(p, dim)
    # n dS = det(J) J^-T e_s dS_ref ; sign flips on the xi_s = 0 side
    a = dets[fl][:, None] * Jinv[fl][:, s, :]
    if side == 0:
        a = -a
    area = np.linalg.norm(a, axis=1)
    normal = a / area[:, None]
    wf = np.ones(len(fl))
    for t in range(dim):
        if t != s:
            wf = wf * w[loc[fl, t]]
    omega = wf * area
    vol_w = wq[fl] * dets[fl]
    return fl, normal, omega, vol_w, float(np.sum(wq * dets))


def br2_sigma(eta, omega, volw_list):
    """Node-wise BR2 penalty from the collocated lifting (reading of eq. br2).

    With the diagonal GLL mass, r_e([u]) on element K is
    -c * omega_i [u]_i n / (w_i^K |J_i^K|) at the face nodes i (c = 1/2 on
    interior faces, 1 on boundary faces) and zero elsewhere, so
    eta * sum_K (r_e([u]), r_e([v]))_K = sum_i omega_i sigma_i [u]_i [v]_i with
    sigma_i = eta * c^2 * sum_K omega_i / (w_i^K |J_i^K|).
    """
    c = 0.5 if len(volw_list) == 2 else 1.0
    return eta * c * c * sum(omega / vw for vw in volw_list)


def dg_operator(mesh, p: int, method: str, eta: float, boundary: bool = True) -> sp.csr_matrix:
    """Assembled A_IP or A_BR2 on the E-vector (element-major)."""
    if method not in ("ip", "br2"):
        raise ValueError(method)
    dim = mesh.dim
    nloc = (p + 1) ** dim
    N = mesh.nel * nloc
    rows, cols, vals = [], [], []

    def add_block(ri, ci, B):
        gi, gj = np.meshgrid(ri, ci, indexing="ij")
        rows.append(gi.ravel())
        cols.append(gj.ravel())
        vals.append(B.ravel())

    for e in mesh.elements():
        base = _elem_flat(mesh, e) * nloc
        add_block(base + np.arange(nloc), base + np.arange(nloc), element_stiffness(mesh, p, e))

    for s, f, em, ep in faces(mesh):
        if em is None or ep is None:
            if not boundary:
                continue
            e, side = (ep, 0) if em is None else (em, 1)
            fl, nrm, omega, volw, volK = _face_geometry(mesh, p, s, e, side)
            G = physical_grad_rows(mesh, p, e)
            base = _elem_flat(mesh, e) * nloc
            if method == "ip":
                he = volK / omega.sum()
                sig = np.full(len(fl), eta * p * p / he)
            else:
                sig = br2_sigma(eta, omega, [volw])
            for q in range(len(fl)):
                jv = np.zeros(nloc)
                jv[fl[q]] = 1.0
                fv = sum(nrm[q, r] * G[r, fl[q]] for r in range(dim))
                B = omega[q] * (-np.outer(jv, fv) - np.outer(fv, jv) + sig[q] * np.outer(jv, jv))
                add_block(base + np.arange(nloc), base + np.arange(nloc), B)
            continue
        flm, nrm, omega, volwm, volm = _face_geometry(mesh, p, s, em, 1)
        flp, _, _, volwp, volp = _face_geometry(mesh, p, s, ep, 0)
        Gm = physical_grad_rows(mesh, p, em)
        Gp = physical_grad_rows(mesh, p, ep)
        bm = _elem_flat(mesh, em) * nloc
        bp = _elem_flat(mesh, ep) * nloc
        if method == "ip":
            he = min(volm, volp) / omega.sum()
            sig = np.full(len(flm), eta * p * p / he)
        else:
            sig = br2_sigma(eta, omega, [volwm, volwp])
        idx = np.concatenate([bm + np.arange(nloc), bp + np.arange(nloc)])
        for q in range(len(flm)):
            jv = np.zeros(2 * nloc)
            jv[flm[q]] = 1.0
            jv[nloc + flp[q]] = -1.0
            fv = np.concatenate([
                0.5 * sum(nrm[q, r] * Gm[r, flm[q]] for r in range(dim)),
                0.5 * sum(nrm[q, r] * Gp[r, flp[q]] for r in range(dim)),
            ])
            B = omega[q] * (-np.outer(jv, fv) - np.outer(fv, jv) + sig[q] * np.outer(jv, jv))
            add_block(idx, idx, B)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return A.tocsr()


_physical_grad_rows = physical_grad_rows
_face_geometry_ = _face_geometry


def dg_apply_rows(mesh, p: int, method: str, eta: float, x: np.ndarray, rows) -> np.ndarray:
    """(A_IP or A_BR2 x)[rows] for selected E-vector rows, from the same face
    terms as dg_operator written row by row: for a face node q with jump
    vector j_q and average normal-flux vector f_q (both over the two
    elements' nodes), row r receives
    omega_q (-j_q[r] (f_q . x) - f_q[r] (j_q . x) + sigma_q j_q[r] (j_q . x)),
    plus the element row (A_K x_K)[r].  Only the elements of the sampled
    rows and their face neighbours are visited."""
    if method not in ("ip", "br2"):
        raise ValueError(method)
    dim = mesh.dim
    nloc = (p + 1) ** dim
    elems = list(mesh.elements())
    out = np.zeros(len(rows))
    cache = {}

    def memo(key, f):  # rows of one element share its matrices and faces
        if key not in cache:
            cache[key] = f()
        return cache[key]

    def physical_grad_rows(mesh_, p_, e_):
        return memo(("G", e_), lambda: _physical_grad_rows(mesh_, p_, e_))

    def _face_geometry(mesh_, p_, s_, e_, side_):
        return memo(("F", s_, e_, side_), lambda: _face_geometry_(mesh_, p_, s_, e_, side_))

    for k, r in enumerate(rows):
        e = elems[int(r) // nloc]
        i = int(r) % nloc
        xe = x[_elem_flat(mesh, e) * nloc + np.arange(nloc)]
        acc = memo(("A", e), lambda: element_stiffness(mesh, p, e))[i] @ xe
        Ge = physical_grad_rows(mesh, p, e)
        for s in range(dim):
            for side in (0, 1):
                nb = list(e)
                nb[s] += 1 if side else -1
                if 0 <= nb[s] < mesh.n[s]:
                    nb = tuple(nb)
                    em, ep = (e, nb) if side else (nb, e)
                    flm, nrm, omega, volwm, volm = _face_geometry(mesh, p, s, em, 1)
                    flp, _, _, volwp, volp = _face_geometry(mesh, p, s, ep, 0)
                    Gm = physical_grad_rows(mesh, p, em)
                    Gp = Ge if ep == e else physical_grad_rows(mesh, p, ep)
                    if em == e:
                        Gm = Ge
                    xm = x[_elem_flat(mesh, em) * nloc + np.arange(nloc)]
                    xp = x[_elem_flat(mesh, ep) * nloc + np.arange(nloc)]
                    if method == "ip":
                        he = min(volm, volp) / omega.sum()
                        sig = np.full(len(flm), eta * p * p / he)
                    else:
                        sig = br2_sigma(eta, omega, [volwm, volwp])
                    for q in range(len(flm)):
                        jx = xm[flm[q]] - xp[flp[q]]
                        fx = 0.5 * (sum(nrm[q, t] * Gm[t, flm[q]] for t in range(dim)) @ xm
                                    + sum(nrm[q, t] * Gp[t, flp[q]] for t in range(dim)) @ xp)
                        if e == em:
                            jr = 1.0 if i == flm[q] else 0.0
                            fr = 0.5 * sum(nrm[q, t] * Gm[t, flm[q], i] for t in range(dim))
                        else:
                            jr = -1.0 if i == flp[q] else 0.0
                            fr = 0.5 * sum(nrm[q, t] * Gp[t, flp[q], i] for t in range(dim))
                        acc += omega[q] * (-jr * fx - fr * jx + sig[q] * jr * jx)
                else:
                    # boundary face of e (side 0: xi_s = 0, side 1: xi_s = 1)
                    fl, nrm, omega, volw, volK = _face_geometry(mesh, p, s, e, side)
                    if method == "ip":
                        he = volK / omega.sum()
                        sig = np.full(len(fl), eta * p * p / he)
                    else:
                        sig = br2_sigma(eta, omega, [volw])
                    for q in range(len(fl)):
                        jx = xe[fl[q]]
                        fx = sum(nrm[q, t] * Ge[t, fl[q]] for t in range(dim)) @ xe
                        jr = 1.0 if i == fl[q] else 0.0
                        fr = sum(nrm[q, t] * Ge[t, fl[q], i] for t in range(dim))
                        acc += omega[q] * (-jr * fx - fr * jx + sig[q] * jr * jx)
        out[k] = acc
    return out


def br2_lifting_matrix(mesh, p: int, eta: float) -> sp.csr_matrix:
    """The BR2 stabilisation eta sum_e (r_e([u]), r_e([v])) built from explicit liftings.

    For every face e and adjacent element K the vector lifting r_e([u])|_K is
    obtained by solving M_K r = -(face integral of [u] . {tau}) with the
    collocated element mass M_K, component by component; the stabilisation
    matrix is then eta * sum R^T M_K R.  Used to check :func:`br2_sigma`.
    """
    dim = mesh.dim
    nloc = (p + 1) ** dim
    N = mesh.nel * nloc
    S = np.zeros((N, N))
    for s, f, em, ep in faces(mesh):
        adj = [(k, side) for k, side in ((em, 1), (ep, 0)) if k is not None]
        c = 0.5 if len(adj) == 2 else 1.0
        # jump operator on the face: [u]_q n_q (vector), from the minus side's normal
        ref_e, ref_side = adj[0]
        fl0, nrm, omega, _, _ = _face_geometry(mesh, p, s, ref_e, ref_side)
        nq = len(fl0)
        Jmp = np.zeros((nq, N))
        for k, side in adj:
            fl, _, _, _, _ = _face_geometry(mesh, p, s, k, side)
            sign = 1.0 if (k, side) == adj[0] else -1.0
            Jmp[np.arange(nq), _elem_flat(mesh, k) * nloc + fl] = sign
        for k, side in adj:
            fl, _, _, volw, _ = _face_geometry(mesh, p, s, k, side)
            _, dets, _, wq = element_geometry(mesh, p, k)
            Mk = wq * dets  # diagonal collocated mass
            for r in range(dim):
                # component r of the lifting on K, as a map from the E-vector
                R = np.zeros((nloc, N))
                R[fl, :] = -(c * omega * nrm[:, r])[:, None] * Jmp / Mk[fl][:, None]
                S += eta * R.T @ (Mk[:, None] * R)
    return sp.csr_matrix(S)


def dg_rhs(mesh, p: int, f_dg_nodes: np.ndarray) -> np.ndarray:
    """b = M f on the E-vector with the collocated element mass."""
    nloc = (p + 1) ** mesh.dim
    b = np.zeros(mesh.nel * nloc)
    for e in mesh.elements():
        _, dets, _, wq = element_geometry(mesh, p, e)
        base = _elem_flat(mesh, e) * nloc
        b[base:base + nloc] = wq * dets * f_dg_nodes[base:base + nloc]
    return b


def cg_to_dg(mesh, p: int) -> sp.csr_matrix:
    """E: conforming unknowns (Dirichlet-eliminated) -> E-vector, by copying node values."""
    nloc = (p + 1) ** mesh.dim
    shape = _mesh.grid_shape(mesh, p)
    num = _mesh.interior_numbering(shape)
    rows, cols = [], []
    for e in mesh.elements():
        base = _elem_flat(mesh, e) * nloc
        g = num[element_global_nodes(mesh, p, e)]
        keep = np.flatnonzero(g >= 0)
        rows.append(base + keep)
        cols.append(g[keep])
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    return sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(mesh.nel * nloc, int((num >= 0).sum())))


def dg_boundary_mask(mesh, p: int) -> np.ndarray:
    """True on E-vector nodes with some local index in {0, p} (the space V_B)."""
    loc = _local_multi(p, mesh.dim)
    m = np.any((loc == 0) | (loc == p), axis=1)
    return np.tile(m, mesh.nel)


def _interp_derivative(nodes: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """(len(pts), len(nodes)) derivatives of the Lagrange basis of `nodes` at
    `pts` (the product rule on l_j(t) = prod_{m != j} (t - x_m)/(x_j - x_m))."""
    n = len(nodes)
    out = np.zeros((len(pts), n))
    for j in range(n):
        den = np.prod([nodes[j] - nodes[m] for m in range(n) if m != j])
        for k in range(n):
            if k == j:
                continue
            term = np.ones(len(pts))
            for m in range(n):
                if m != j and m != k:
                    term = term * (pts - nodes[m])
            out[:, j] += term
        out[:, j] /= den
    return out


def l2_error_cg(mesh, p: int, u_grid: np.ndarray, u_exact, nq: int | None = None) -> float:
    """||u_h - u||_{L2} with u_h given at every GLL grid node (x fastest).

    Uses nq-point Gauss-Legendre quadrature per direction (default p + 3) on
    each element; u_h is evaluated by Lagrange interpolation of its nodal
    values, points are mapped with the element's Q1 map (or, on a curved mesh,
    the interpolant of its GLL node coordinates).
    """
    dim = mesh.dim
    nq = nq or p + 3
    x, _ = _gll.gll(p)
    g, wg = np.polynomial.legendre.leggauss(nq)
    g, wg = (g + 1) / 2, wg / 2
    B = _gll.lagrange_eval_matrix(x, g)  # (nq, p+1)
    qloc = np.indices([nq] * dim).reshape(dim, -1, order="F").T
    err2 = 0.0
    Bt = B
    for _ in range(dim - 1):
        Bt = np.kron(B, Bt)
    if mesh.nodes is not None:
        # derivative tables of the nodal interpolant at the Gauss points
        Dq = _interp_derivative(x, g)
        Bd = []
        for s_ in range(dim):
            f = [Dq if t == s_ else B for t in range(dim)]
            M = f[dim - 1]
            for t in range(dim - 2, -1, -1):
                M = np.kron(M, f[t])
            Bd.append(M)
    for e in mesh.elements():
        ue = u_grid[element_global_nodes(mesh, p, e)]
        uh = Bt @ ue
        if mesh.nodes is not None:
            Xe = mesh.nodes[element_global_nodes(mesh, p, e)]
            X = Bt @ Xe
            J = np.stack([np.stack([Bd[s_] @ Xe[:, r] for s_ in range(dim)], axis=1) for r in range(dim)], axis=1)
            dets = np.linalg.det(J)
        else:
            corners = mesh.element_corners(e)
            pts = [g[qloc[:, i]] for i in range(dim)]
            X = np.stack(_mesh.map_point(corners[:, :, None] * np.ones(len(qloc)), pts), axis=1)
            dets = np.array([np.linalg.det(_mesh.map_jacobian(corners, [g[q[i]] for i in range(dim)]))
                             for q in qloc])
        w = np.prod(wg[qloc], axis=1)
        err2 += float(np.sum(w * dets * (uh - u_exact(X)) ** 2))
    return np.sqrt(err2)
