"""Preconditioned and flexible conjugate gradients.

The paper reports CG iterations to a 10^8 reduction of the residual
(Section 4); the norm and the start are not stated.  Reading: x_0 = 0, stop
when ||r_k||_2 <= tol ||b||_2 with the recursively updated residual.
FCG(1) uses beta = z_{k+1} . (r_{k+1} - r_k) / rho_k, which equals the PCG
beta for a fixed symmetric preconditioner in exact arithmetic and stays
robust when the preconditioner is not (reduced precision, learned parts).
"""
from __future__ import annotations

import numpy as np


def pcg(A, b, prec, tol=1e-8, maxit=1000, flexible=False, x0=None):
    """Returns (x, iterations, history of ||r||/||b||)."""
    apply = A if callable(A) else (lambda v: A @ v)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply(x) if x0 is not None else b.copy()
    bnorm = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bnorm if bnorm else 0.0]
    if bnorm == 0.0:
        return x, 0, hist
    z = prec(r)
    p = z.copy()
    rho = r @ z
    it = 0
    while it < maxit and hist[-1] > tol:
        q = apply(p)
        pq = p @ q
        if not pq > 0:
            raise ArithmeticError("p^T A p <= 0")
        alpha = rho / pq
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        it += 1
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= tol:
            break
        z = prec(r)
        rho_new = r @ z
        if not rho_new > 0:
            raise ArithmeticError("r^T z <= 0")
        beta = (z @ (r - r_old)) / rho if flexible else rho_new / rho
        p = z + beta * p
        rho = rho_new
    return x, it, hist


def iteration_band(A, b, prec, tol=1e-8, maxit=1000, rel=1e-12, seeds=(1, 2), flexible=False):
    """(lowest, highest) iteration count of pcg when the preconditioner's
    output carries relative perturbations of size rel (the unperturbed run
    and one run per seed).  Near a plateau of the residual history the count
    moves with rounding; a second implementation whose preconditioner agrees
    with this one to rel should fall inside the band, give or take one."""
    its = [pcg(A, b, prec, tol=tol, maxit=maxit, flexible=flexible)[1]]
    for s in seeds:
        rng = np.random.default_rng(s)
        def noisy(r, rng=rng):
            z = prec(r)
            return z * (1.0 + rel * rng.standard_normal(z.shape))
        its.append(pcg(A, b, noisy, tol=tol, maxit=maxit, flexible=flexible)[1])
    return min(its), max(its)
