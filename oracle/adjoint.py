"""Adjoint sensitivity of the homogenised stress (derived from eq. (30)).

Loss L = <P_11> (voxel mean) at a converged state, G*P(F; theta) = 0.
For a parameter field theta, the response dF is compatible, zero-mean and
solves G*(K : dF) = -G*(dP/dtheta dtheta).  With the adjoint field lambda
(compatible, zero-mean)
    G*(K : lambda) = -G*(K : E11),   E11 = e1 (x) e1 (uniform),
the major symmetry of K and the symmetry of the projector give
    dL/dtheta(x) = (1/N) (E11 + lambda(x)) : dP/dtheta(x).
For theta = log E, dP/dtheta = P; for theta = Omega see
``constitutive.stress_param_derivatives``.

Reading A26: the finite-difference reference perturbs one voxel and solves
the *difference* problem from the converged base state, so the base
residual cancels exactly.
"""
from __future__ import annotations

import numpy as np

from .constitutive import apply_tangent, law_of, stress, stress_param_derivatives, tangent
from .krylov import cg
from .mechanics import norm, operator
from .spectral import project


def adjoint_gradient(F, c, d, mat, tol_lin=1e-10, maxit=20000):
    """Returns (dL/dlogE, dL/dOmega, adjoint CG iterations), fields of the
    grid's shape."""
    spacing = mat["spacing"]
    shape = F.shape[2:]
    K = tangent(F, c, d, mat["E"], mat["nu"], mat["Omega"], law_of(mat))
    E11 = np.zeros((3, 3) + tuple(shape))
    E11[0, 0] = 1.0
    rhs = -project(apply_tangent(K, E11), spacing)
    lam, it, _ = cg(lambda X: operator(K, X, spacing), rhs, tol_lin, maxit)
    P, dP_dOm = stress_param_derivatives(F, c, d, mat["E"], mat["nu"], mat["Omega"], law_of(mat))
    W = E11 + lam
    N = float(np.prod(shape))
    gE = np.einsum("ij...,ij...->...", W, P) / N
    gO = np.einsum("ij...,ij...->...", W, dP_dOm) / N
    return gE, gO, it


def _difference_solve(F0, c, d, mat_pert, P0, tol=1e-11, max_newton=30, tol_lin=1e-12):
    """Newton on dF for G*[P(F0 + dF; theta') - P0] = 0; returns dF."""
    spacing = mat_pert["spacing"]
    dF = np.zeros_like(F0)
    ref = None
    for _ in range(max_newton):
        P = stress(F0 + dF, c, d, mat_pert["E"], mat_pert["nu"], mat_pert["Omega"], law_of(mat_pert))
        b = -project(project(P - P0, spacing), spacing)
        nb = norm(b)
        if ref is None:
            ref = max(nb, 1e-300)
        if nb <= tol * ref:
            break
        K = tangent(F0 + dF, c, d, mat_pert["E"], mat_pert["nu"], mat_pert["Omega"], law_of(mat_pert))
        x, _, _ = cg(lambda X: operator(K, X, spacing), b, tol_lin, 20000)
        dF = dF + x
    return dF


def fd_gradient(F0, c, d, mat, voxel, param, eta):
    """Central finite difference of L = <P_11> with respect to log E
    (``param='logE'``) or Omega (``param='Omega'``) at one voxel (flat
    index), by two difference solves."""
    P0 = stress(F0, c, d, mat["E"], mat["nu"], mat["Omega"], law_of(mat))
    out = []
    for sgn in (+1.0, -1.0):
        m = dict(mat)
        if param == "logE":
            E = mat["E"].copy().ravel()
            E[voxel] *= np.exp(sgn * eta)
            m["E"] = E.reshape(mat["E"].shape)
        else:
            Om = mat["Omega"].copy().ravel()
            Om[voxel] += sgn * eta
            m["Omega"] = Om.reshape(mat["Omega"].shape)
        dF = _difference_solve(F0, c, d, m, P0)
        P = stress(F0 + dF, c, d, m["E"], m["nu"], m["Omega"], law_of(m))
        out.append(float(np.mean(P[0, 0] - P0[0, 0])))
    return (out[0] - out[1]) / (2.0 * eta)
