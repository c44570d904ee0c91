"""Minimum-discarded-fill (MDF) ordering and the ILU(0) factor it produces.

Section 3.4: the ILU(0) smoother is applied in MDF order (D'Azevedo, Forsyth
and Tang; Persson and Peraire), computed with a min-heap in
O(n log n).  The paper gives no formulas; the reading used here:

* the matrix is symmetric with the structural pattern of the Q1 stencil
  (two points are coupled iff their grid offsets differ by at most one in
  every direction);
* elimination works on the ILU(0)-updated matrix a~: eliminating node i
  applies a~_jl -= a~_ji a~_il / a~_ii to every pair (j, l) of not yet
  eliminated neighbours of i that lies in the pattern (j = l included) and
  discards the rest;
* the discarded fill of a candidate m is
  disc(m) = sum over neighbour pairs j < l of m (not eliminated, not coupled)
            of ((a~_mj * a~_ml) / a~_mm)^2,
  with j ascending, then l ascending, summed left to right from 0.0;
* the next node is the one with the smallest disc, exact ties going to the
  smallest patch-local index; after an elimination only the neighbours of the
  eliminated node change and are re-evaluated;
* the factor is unit lower L and diagonal D with l_ji = a~_ji / a~_ii taken
  when i is eliminated and D_i = a~_ii (this is ILU(0) in that order, which
  for a symmetric matrix is the symmetric IC(0) = L D L^T).

A non-positive or non-finite pivot is an error (no shifting).
"""
from __future__ import annotations

import heapq

import numpy as np


class PivotError(ArithmeticError):
    pass


def _slots(dim):
    return [tuple(((sl // 3 ** i) % 3) - 1 for i in range(dim)) for sl in range(3 ** dim)]


class PatchGraph:
    """A box of grid points with 3^d-slot symmetric rows (patch-local, x fastest)."""

    def __init__(self, shape, rows: np.ndarray):
        self.shape = tuple(int(s) for s in shape)
        self.dim = len(self.shape)
        self.n = int(np.prod(self.shape))
        self.slots = _slots(self.dim)
        self.center = (3 ** self.dim) // 2
        self.rows = np.array(rows, dtype=np.float64).reshape(self.n, 3 ** self.dim)
        # neighbour table: nb[i, slot] = patch-local index or -1
        self.nb = -np.ones((self.n, 3 ** self.dim), dtype=np.int64)
        for i in range(self.n):
            c = self._coords(i)
            for sl, o in enumerate(self.slots):
                q = [c[t] + o[t] for t in range(self.dim)]
                if all(0 <= q[t] < self.shape[t] for t in range(self.dim)):
                    self.nb[i, sl] = self._index(q)
        # drop couplings to points outside the box
        self.rows[self.nb < 0] = 0.0

    def _coords(self, i):
        out = []
        for t in range(self.dim):
            out.append(i % self.shape[t])
            i //= self.shape[t]
        return out

    def _index(self, q):
        idx, stride = 0, 1
        for t in range(self.dim):
            idx += q[t] * stride
            stride *= self.shape[t]
        return idx

    def slot_of(self, o):
        return sum((o[t] + 1) * 3 ** t for t in range(self.dim))

    def dense(self) -> np.ndarray:
        A = np.zeros((self.n, self.n))
        for i in range(self.n):
            for sl in range(3 ** self.dim):
                j = self.nb[i, sl]
                if j >= 0:
                    A[i, j] = self.rows[i, sl]
        return A


def _coupled(oj, ol):
    return all(abs(a - b) <= 1 for a, b in zip(oj, ol))


def _disc(g: PatchGraph, a: np.ndarray, elim: np.ndarray, m: int) -> float:
    nbr = [(sl, g.nb[m, sl]) for sl in range(3 ** g.dim)
           if sl != g.center and g.nb[m, sl] >= 0 and not elim[g.nb[m, sl]]]
    acc = 0.0
    amm = a[m, g.center]
    for x in range(len(nbr)):
        sj, _ = nbr[x]
        for y in range(x + 1, len(nbr)):
            sl, _ = nbr[y]
            if _coupled(g.slots[sj], g.slots[sl]):
                continue
            f = (a[m, sj] * a[m, sl]) / amm
            acc = acc + f * f
    return float(acc)


def _eliminate(g: PatchGraph, a, elim, i, L, D):
    piv = a[i, g.center]
    if not (np.isfinite(piv) and piv > 0.0):
        raise PivotError(f"IC(0) pivot {piv!r} at patch-local row {i}")
    D[i] = piv
    nbr = [sl for sl in range(3 ** g.dim)
           if sl != g.center and g.nb[i, sl] >= 0 and not elim[g.nb[i, sl]]]
    for sj in nbr:
        j = g.nb[i, sj]
        oj = g.slots[sj]
        lji = a[i, sj] / piv
        L[i, sj] = lji                                   # later neighbour j of i
        L[j, g.slot_of([-t for t in oj])] = lji          # earlier neighbour i of j
        for sl in nbr:
            ol = g.slots[sl]
            if not _coupled(oj, ol):
                continue
            t = (a[i, sj] * a[i, sl]) / piv
            rel = g.slot_of([ol[k] - oj[k] for k in range(g.dim)])
            a[j, rel] = a[j, rel] - t
    elim[i] = True
    return nbr


def mdf_factor(g: PatchGraph, brute_force: bool = False):
    """MDF elimination order and its IC(0) factor.

    Returns (order, L, D): order[t] = patch-local node eliminated at step t;
    L is (n, 3^d) with, in row i, l_im at earlier neighbours m and l_mi at
    later neighbours m (the two halves a forward and a backward sweep need);
    D is the pivot of each row.
    """
    n = g.n
    a = g.rows.copy()
    elim = np.zeros(n, dtype=bool)
    L = np.zeros((n, 3 ** g.dim))
    D = np.zeros(n)
    disc = np.array([_disc(g, a, elim, m) for m in range(n)])
    order = []
    if brute_force:
        for _ in range(n):
            best = None
            for m in range(n):
                if not elim[m] and (best is None or disc[m] < disc[best]):
                    best = m
            order.append(best)
            for sl in _eliminate(g, a, elim, best, L, D):
                j = g.nb[best, sl]
                disc[j] = _disc(g, a, elim, j)
        return np.array(order), L, D
    version = np.zeros(n, dtype=np.int64)
    heap = [(disc[m], m, 0) for m in range(n)]
    heapq.heapify(heap)
    while len(order) < n:
        dm, m, ver = heapq.heappop(heap)
        if elim[m] or ver != version[m]:
            continue
        order.append(m)
        for sl in _eliminate(g, a, elim, m, L, D):
            j = g.nb[m, sl]
            disc[j] = _disc(g, a, elim, j)
            version[j] += 1
            heapq.heappush(heap, (disc[j], j, int(version[j])))
    return np.array(order), L, D


def factor_in_order(g: PatchGraph, order):
    """IC(0) factor (L, D as in :func:`mdf_factor`) for a given elimination
    order: the same elimination steps, the order fixed in advance."""
    a = g.rows.copy()
    elim = np.zeros(g.n, dtype=bool)
    L = np.zeros((g.n, 3 ** g.dim))
    D = np.zeros(g.n)
    for i in order:
        _eliminate(g, a, elim, int(i), L, D)
    return np.asarray(order, dtype=np.int64), L, D


def rcm_order(shape) -> np.ndarray:
    """Reverse Cuthill-McKee order of a box of grid points (Section 3.4 names
    RCM beside MDF; Cuthill and McKee 1969, reversed as George proposed).

    The graph is the structural pattern of the patch matrices: two points are
    adjacent iff their offsets differ by at most one per direction (the
    values play no part, so every box of one shape gets one order).  Reading
    of the unspecified choices: the start is a node of minimum degree, the
    smallest index among them; the breadth-first search visits the not yet
    numbered neighbours of each node in increasing degree, ties to the
    smallest index; the Cuthill-McKee sequence is then reversed."""
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    n = int(np.prod(shape))
    strides = [int(np.prod(shape[:t])) for t in range(dim)]
    coords = [[(i // strides[t]) % shape[t] for t in range(dim)] for i in range(n)]
    offs = [o for o in _slots(dim) if any(o)]
    nbrs = []
    for c in coords:
        row = []
        for o in offs:
            q = [c[t] + o[t] for t in range(dim)]
            if all(0 <= q[t] < shape[t] for t in range(dim)):
                row.append(sum(q[t] * strides[t] for t in range(dim)))
        nbrs.append(sorted(row))
    deg = [len(r) for r in nbrs]
    numbered = [False] * n
    cm = []
    while len(cm) < n:
        start = min((i for i in range(n) if not numbered[i]), key=lambda i: (deg[i], i))
        numbered[start] = True
        queue = [start]
        head = 0
        while head < len(queue):
            u = queue[head]
            head += 1
            cm.append(u)
            nxt = sorted((v for v in nbrs[u] if not numbered[v]), key=lambda v: (deg[v], v))
            for v in nxt:
                numbered[v] = True
                queue.append(v)
    return np.array(cm[::-1], dtype=np.int64)


def ic0_solve(g: PatchGraph, order, L, D, r: np.ndarray) -> np.ndarray:
    """y = (L D L^T)^{-1} r with the factor of :func:`mdf_factor`."""
    n = g.n
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    w = np.array(r, dtype=np.float64).copy()
    for i in order:                      # forward: L w = r
        acc = w[i]
        for sl in range(3 ** g.dim):
            m = g.nb[i, sl]
            if sl != g.center and m >= 0 and pos[m] < pos[i]:
                acc -= L[i, sl] * w[m]
        w[i] = acc
    y = w / D
    for i in order[::-1]:                # backward: L^T y = D^-1 w
        acc = y[i]
        for sl in range(3 ** g.dim):
            m = g.nb[i, sl]
            if sl != g.center and m >= 0 and pos[m] > pos[i]:
                acc -= L[i, sl] * y[m]
        y[i] = acc
    return y


def factor_product(g: PatchGraph, order, L, D) -> np.ndarray:
    """Dense L D L^T in the original (patch-local) numbering."""
    n = g.n
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    Lm = np.eye(n)
    for i in range(n):
        for sl in range(3 ** g.dim):
            m = g.nb[i, sl]
            if sl != g.center and m >= 0 and pos[m] < pos[i]:
                Lm[i, m] = L[i, sl]
    return Lm @ np.diag(D) @ Lm.T


def dependency_depth(g: PatchGraph, order) -> int:
    """Length of the longest chain of the forward sweep (levels of the DAG)."""
    n = g.n
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    lev = np.zeros(n, dtype=np.int64)
    for i in order:
        best = 0
        for sl in range(3 ** g.dim):
            m = g.nb[i, sl]
            if sl != g.center and m >= 0 and pos[m] < pos[i]:
                best = max(best, lev[m] + 1)
        lev[i] = best
    return int(lev.max()) + 1 if n else 0
