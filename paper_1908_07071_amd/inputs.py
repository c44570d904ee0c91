"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method itself: it only produces the
problem data that the paper's experiments are shaped like (Section 4):
structured quad/hex meshes of the unit square/cube with optionally perturbed
interior vertices, the manufactured solution u = prod_i sin(pi x_i) with its
forcing f = -Laplace(u), and Gaussian right-hand sides.

It imports nothing from the rest of the package, so the CPU oracle and the GPU
path can both be fed from it without depending on each other.
"""
from __future__ import annotations

import numpy as np


def structured_vertices(dim: int, n, perturb: float = 0.0, seed=None) -> np.ndarray:
    """Vertex coordinates of an n^dim block of quads/hexes on [0,1]^dim.

    Returns an array of shape (prod(n_i+1), dim), float64, vertices ordered
    lexicographically with x fastest.  When ``perturb`` > 0, every vertex not
    on the boundary is moved by h_i * U(-perturb, perturb) in each coordinate
    i, drawn from ``numpy.random.default_rng(seed)`` in vertex order, one
    coordinate after the other (h_i = 1/n_i).  ``perturb`` = 0.1 is the
    "interior vertices randomly perturbed by at most 10% of h" recipe.
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    n = [int(n)] * dim if np.isscalar(n) else [int(v) for v in n]
    if len(n) != dim or min(n) < 1:
        raise ValueError("bad element counts")
    axes = [np.linspace(0.0, 1.0, ni + 1) for ni in n]
    grids = np.meshgrid(*axes, indexing="ij")
    # lexicographic with x fastest: flatten in Fortran order over (x, y, z)
    xyz = np.stack([g.reshape(-1, order="F") for g in grids], axis=1).copy()
    if perturb > 0.0:
        rng = np.random.default_rng(seed)
        shape = [ni + 1 for ni in n]
        idx = np.indices(shape).reshape(dim, -1, order="F").T
        interior = np.all((idx > 0) & (idx < np.array(n)), axis=1)
        h = 1.0 / np.array(n, dtype=np.float64)
        disp = rng.uniform(-perturb, perturb, size=(int(interior.sum()), dim))
        xyz[interior] += disp * h
    return xyz


def manufactured_u(x: np.ndarray) -> np.ndarray:
    """u(x) = prod_i sin(pi x_i), which vanishes on the boundary of [0,1]^d."""
    return np.prod(np.sin(np.pi * x), axis=1)


def manufactured_f(x: np.ndarray) -> np.ndarray:
    """f = -Laplace(u) = d * pi^2 * prod_i sin(pi x_i)."""
    d = x.shape[1]
    return d * np.pi ** 2 * np.prod(np.sin(np.pi * x), axis=1)


def gaussian_rhs(n: int, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) right-hand side of length n (float64)."""
    return np.random.default_rng(seed).standard_normal(n)


def uniform_vector(n: int, seed: int) -> np.ndarray:
    """i.i.d. U(-1,1) vector of length n (float64), used as operator input."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def batch_problems(nprob: int = 64, seed: int = 7, nmin: int = 4, nmax: int = 24,
                   pmin: int = 2, pmax: int = 8):
    """Sizes of a batch of independent 3D problems: n ~ U{nmin..nmax} elements
    per direction and p ~ U{pmin..pmax}, drawn with a seeded generator.
    Problem i uses mesh seed 100 + i and right-hand-side seeds 1000 i + k."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=nprob)
    ps = rng.integers(pmin, pmax + 1, size=nprob)
    return [(int(n), int(p), 100 + i) for i, (n, p) in enumerate(zip(ns, ps))]


def nn_initial_params(channels: int = 32, seed: int = 11, cin: int = 2, layers: int = 3):
    """Initial weights of the patch network as one flat float64 vector (layer
    by layer: W [27 cin, cout] row-major, then the bias [cout]); W uniform in
    +-sqrt(6 / fan_in) (He / Kaiming uniform), biases zero."""
    rng = np.random.default_rng(seed)
    out, c = [], cin
    for li in range(layers):
        co = 1 if li == layers - 1 else channels
        bound = np.sqrt(6.0 / (27 * c))
        out.append(rng.uniform(-bound, bound, size=27 * c * co))
        out.append(np.zeros(co))
        c = co
    return np.concatenate(out)


def coefficient(name: str, x: np.ndarray, elem=None, seed: int = 0) -> np.ndarray:
    """Variable coefficients b of -div(b grad u) = f shaped like the paper's
    examples (Section 4.2, defined there on [-1,1]^2), evaluated at points x
    of [0,1]^d through x' = 2x - 1 (extended to 3D with the same pattern):
      b1 = 1e4 prod_i (1 - x'_i^2)        sharp gradients near the boundary
      b2 = 100 x'_0^2 + sum_{i>0} x'_i^2 + 1   anisotropic
      b3 = (1 + |x'|^2)^4
      b4 = 10 or 1 per element, drawn at random (elem: the element index of
           each point; numpy default_rng(seed), one draw per element)
    Returns b at every row of x."""
    xp = 2.0 * np.asarray(x, dtype=np.float64) - 1.0
    if name == "b1":
        return 1e4 * np.prod(1.0 - xp ** 2, axis=1)
    if name == "b2":
        return 100.0 * xp[:, 0] ** 2 + np.sum(xp[:, 1:] ** 2, axis=1) + 1.0
    if name == "b3":
        return (1.0 + np.sum(xp ** 2, axis=1)) ** 4
    if name == "b4":
        if elem is None:
            raise ValueError("b4 needs the element index of every point")
        elem = np.asarray(elem)
        vals = np.where(np.random.default_rng(seed).random(int(elem.max()) + 1) < 0.5, 10.0, 1.0)
        return vals[elem]
    raise ValueError(f"unknown coefficient {name!r}")


def strip_vertices(n: int, aspect: float, strip_rows: int = 2, dim: int = 2) -> np.ndarray:
    """An n^dim block of [0,1]^dim with a strip of thin elements (Section 4.5
    shape): element width 1/n in x (and z); in y, `strip_rows` rows in the
    middle have height (1/n)/aspect -- elements of aspect ratio `aspect` --
    and the other rows share the rest of the height equally.  Vertices as in
    structured_vertices (x fastest)."""
    if not (1 <= strip_rows < n):
        raise ValueError("need 1 <= strip_rows < n")
    hs = (1.0 / n) / aspect
    ho = (1.0 - strip_rows * hs) / (n - strip_rows)
    first = (n - strip_rows) // 2
    heights = [hs if first <= j < first + strip_rows else ho for j in range(n)]
    y = np.concatenate([[0.0], np.cumsum(heights)])
    y[-1] = 1.0
    axes = [np.linspace(0.0, 1.0, n + 1) for _ in range(dim)]
    axes[1] = y
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.reshape(-1, order="F") for g in grids], axis=1).copy()


def curved_nodes(dim: int, n, p: int, amp: float = 0.15, perturb: float = 0.0, seed=None) -> np.ndarray:
    """GLL-grid node coordinates of a block of [0,1]^dim with curved elements:
    the straight block (optionally with perturbed vertices, as in
    structured_vertices) at the 1D GLL points of [0,1] given by `gll_x`
    below, then moved by the smooth map x_i -> x_i + amp * 16 * prod_j
    x_j (1 - x_j) (zero on the boundary, so the domain stays the unit cube
    while element faces inside bend).  Nodes lexicographic with x fastest,
    n_i p + 1 per direction.  The interior vertices of the block are the
    images of the straight vertices, so structured_vertices(...) with the
    same map applied gives the matching vertex array (curved_vertices)."""
    n = [int(n)] * dim if np.isscalar(n) else [int(v) for v in n]
    x = gll_x(p)
    V = structured_vertices(dim, n, perturb, seed)
    # straight nodes: each element's Q1 interpolation of its vertices
    ng = [n[i] * p + 1 for i in range(dim)]
    g = np.indices(ng).reshape(dim, -1, order="F")
    e = [np.minimum(g[i] // p, n[i] - 1) for i in range(dim)]
    t = [x[g[i] - p * e[i]] for i in range(dim)]
    out = np.zeros((g.shape[1], dim))
    for c in range(2 ** dim):
        vidx = np.zeros(g.shape[1], dtype=np.int64)
        stride = 1
        wgt = np.ones(g.shape[1])
        for i in range(dim):
            b = (c >> i) & 1
            vidx += (e[i] + b) * stride
            stride *= n[i] + 1
            wgt = wgt * (t[i] if b else 1.0 - t[i])
        out += wgt[:, None] * V[vidx]
    return _bend(out, amp)


def curved_vertices(dim: int, n, amp: float = 0.15, perturb: float = 0.0, seed=None) -> np.ndarray:
    """The vertices of the block of curved_nodes (the same bending map)."""
    return _bend(structured_vertices(dim, n, perturb, seed), amp)


def _bend(X: np.ndarray, amp: float) -> np.ndarray:
    bump = 16.0 * np.prod(X * (1.0 - X), axis=1)
    return X + amp * bump[:, None]


def gll_x(p: int) -> np.ndarray:
    """The p + 1 Gauss-Lobatto points of [0,1] in float64 (roots of the
    derivative of the Legendre polynomial, from numpy), for placing curved
    mesh nodes; the library and the oracle use their own correctly rounded
    points for the discretization itself."""
    if p == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(p + 1)
    c[p] = 1.0
    r = np.polynomial.legendre.Legendre(c).deriv().roots()
    return np.concatenate([[0.0], (np.sort(r.real) + 1.0) / 2.0, [1.0]])
