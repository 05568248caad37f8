"""Exact solution for a periodic two-phase laminate (used as a pin of the
mechanics of Sec. 3.2).

Layers normal to e_n, phase A for index < k along axis n (fraction
phi = k / N_n), phase B elsewhere, homogeneous fields c, d per phase.  The
piecewise-constant field
    F_A = Fbar + (1 - phi) a (x) e_n,   F_B = Fbar - phi a (x) e_n
is compatible (its spectrum lies on the q_n axis, where the rotated vector
r is parallel to e_n) and has mean Fbar; it is in equilibrium iff the
traction is continuous, P_A e_n = P_B e_n, three equations for a in R^3
solved here by Newton with the analytic tangent.
"""
from __future__ import annotations

import numpy as np

from .constitutive import law_of, stress, tangent


def _pt(F, c, d, E, nu, Om, law="neo_hookean"):
    Fp = F.reshape(3, 3, 1)
    f = lambda x: np.asarray(x, dtype=np.float64).reshape(1)
    P = stress(Fp, f(c), f(d), f(E), f(nu), f(Om), law)[:, :, 0]
    K = tangent(Fp, f(c), f(d), f(E), f(nu), f(Om), law)[:, :, 0].reshape(3, 3, 3, 3)
    return P, K


def laminate_solution(Fbar, axis, phi, matA, matB, tol=1e-15, max_iter=50):
    """matA / matB: dicts with scalars E, nu, Omega, c, d (and optionally
    the law).  Returns (F_A, F_B, a)."""
    Fbar = np.asarray(Fbar, dtype=np.float64)
    n = axis
    e = np.zeros(3)
    e[n] = 1.0
    a = np.zeros(3)
    for _ in range(max_iter):
        FA = Fbar + (1.0 - phi) * np.outer(a, e)
        FB = Fbar - phi * np.outer(a, e)
        PA, KA = _pt(FA, matA["c"], matA["d"], matA["E"], matA["nu"], matA["Omega"], law_of(matA))
        PB, KB = _pt(FB, matB["c"], matB["d"], matB["E"], matB["nu"], matB["Omega"], law_of(matB))
        res = PA[:, n] - PB[:, n]
        scale = max(np.abs(PA).max(), np.abs(PB).max(), 1e-300)
        if np.abs(res).max() <= tol * scale:
            break
        Jm = (1.0 - phi) * KA[:, n, :, n] + phi * KB[:, n, :, n]
        a = a - np.linalg.solve(Jm, res)
    FA = Fbar + (1.0 - phi) * np.outer(a, e)
    FB = Fbar - phi * np.outer(a, e)
    return FA, FB, a
