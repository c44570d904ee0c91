"""Gauss-Lobatto (GLL) points, weights and the Lagrange derivative matrix.

Section 3.1 (FEM-SEM equivalence): the high-order basis is nodal at the p+1
Gauss-Lobatto points of [0,1], integrated with the same points (G-NI), and the
low-order refined mesh is built on these points.

The nodes and weights are returned *correctly rounded* to float64: they are
computed with Newton's method in 60-digit decimal arithmetic and rounded once.
Any independent implementation that also rounds the exact values therefore
reproduces them bit for bit.
"""
from __future__ import annotations

import math
from decimal import Decimal, getcontext
from functools import lru_cache

import numpy as np

_DIGITS = 60


def _legendre(p: int, x: Decimal):
    """(P_{p-1}(x), P_p(x)) by the three-term recurrence."""
    p0, p1 = Decimal(1), x
    for k in range(2, p + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    return p0, p1


def _legendre_and_derivs(p: int, x: Decimal):
    """P_p(x), P_p'(x), P_p''(x) for |x| < 1."""
    p0, p1 = _legendre(p, x)
    # (1 - x^2) P' = p (P_{p-1} - x P_p);  differentiate once more for P''.
    one_m_x2 = 1 - x * x
    dp = p * (p0 - x * p1) / one_m_x2
    d2p = (2 * x * dp - p * (p + 1) * p1) / one_m_x2
    return p1, dp, d2p


@lru_cache(maxsize=None)
def gll(p: int):
    """GLL nodes x_0 < ... < x_p on [0,1] and weights w_i (sum w_i = 1).

    Interior nodes are the roots of P_p' on (-1,1), mapped by x -> (x+1)/2; the
    weights are 2 / (p(p+1) P_p(x)^2) on [-1,1], halved on [0,1].
    """
    if p < 1:
        raise ValueError("p >= 1 required")
    getcontext().prec = _DIGITS
    xs = [Decimal(-1)]
    for j in range(1, p):
        # Chebyshev-Gauss-Lobatto initial guess, then Newton on P_p'.
        x = Decimal(repr(-math.cos(math.pi * j / p)))
        for _ in range(200):
            _, dp, d2p = _legendre_and_derivs(p, x)
            step = dp / d2p
            x -= step
            if abs(step) < Decimal(10) ** (-_DIGITS + 5):
                break
        xs.append(x)
    xs.append(Decimal(1))
    nodes, weights = [], []
    for x in xs:
        _, pp = _legendre(p, x)
        w = Decimal(2) / (p * (p + 1) * pp * pp)
        nodes.append(float((x + 1) / 2))
        weights.append(float(w / 2))
    return np.array(nodes), np.array(weights)


def lagrange_derivative_matrix(nodes: np.ndarray) -> np.ndarray:
    """D[i, j] = l_j'(x_i) for the Lagrange basis on ``nodes``.

    Written straight from the product rule on
    l_j(x) = prod_{k != j} (x - x_k) / (x_j - x_k).
    """
    n = len(nodes)
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            s = 0.0
            for m in range(n):
                if m == j:
                    continue
                t = 1.0 / (nodes[j] - nodes[m])
                for k in range(n):
                    if k in (j, m):
                        continue
                    t *= (nodes[i] - nodes[k]) / (nodes[j] - nodes[k])
                s += t
            D[i, j] = s
    return D


def lagrange_eval_matrix(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """B[q, j] = l_j(x_q): values of the Lagrange basis at points ``x``."""
    B = np.ones((len(x), len(nodes)))
    for j in range(len(nodes)):
        for k in range(len(nodes)):
            if k != j:
                B[:, j] *= (x - nodes[k]) / (nodes[j] - nodes[k])
    return B
