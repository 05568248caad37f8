"""Conjugate gradient solvers (Sec. 3.2: Alg. 1 uses CG with tolerance
tol_lin; Alg. 2 and Alg. 3 use (preconditioned) CG).

Reading (A23): the stopping test is on the unpreconditioned residual,
||r_k||_2 <= tol ||b||_2, evaluated as r.r <= tol^2 b.b right after the
residual update; the initial guess is zero.  The inner product is the
Euclidean sum over all voxels and components.
"""
from __future__ import annotations

import numpy as np


class Breakdown(RuntimeError):
    """p^T A p <= 0 inside CG (operator not positive definite)."""


def dot(a, b):
    return float(np.sum(a * b))


def cg(apply_A, b, tol, maxit, fixed_iters=None):
    """Hestenes-Stiefel CG for A x = b, x0 = 0.

    ``fixed_iters``: run exactly that many iterations (tol ignored); used to
    force matching iteration counts in parity runs.
    Returns (x, iterations, final relative residual).
    """
    x = np.zeros_like(b)
    r = b.copy()
    rr0 = dot(b, b)
    if rr0 == 0.0:
        return x, 0, 0.0
    p = r.copy()
    rr = rr0
    limit = maxit if fixed_iters is None else fixed_iters
    it = 0
    for it in range(1, limit + 1):
        Ap = apply_A(p)
        pAp = dot(p, Ap)
        if not pAp > 0.0:
            raise Breakdown("p.Ap <= 0")
        alpha = rr / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = dot(r, r)
        if fixed_iters is None and rr_new <= tol * tol * rr0:
            rr = rr_new
            break
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
    return x, it, float(np.sqrt(rr / rr0))


def pcg(apply_A, apply_M, b, tol, maxit, fixed_iters=None):
    """Preconditioned CG for A x = b with preconditioner M ~ A^-1, x0 = 0.
    Returns (x, iterations, final relative residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    rr0 = dot(b, b)
    if rr0 == 0.0:
        return x, 0, 0.0
    z = apply_M(r)
    p = z.copy()
    rz = dot(r, z)
    rr = rr0
    limit = maxit if fixed_iters is None else fixed_iters
    it = 0
    for it in range(1, limit + 1):
        Ap = apply_A(p)
        pAp = dot(p, Ap)
        if not pAp > 0.0:
            raise Breakdown("p.Ap <= 0")
        alpha = rz / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        rr = dot(r, r)
        if fixed_iters is None and rr <= tol * tol * rr0:
            break
        z = apply_M(r)
        rz_new = dot(r, z)
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
    return x, it, float(np.sqrt(rr / rr0))
