"""Effective stiffness of many RVEs with the batched solver (fg_batch_*).

The six macroscopic load cases F = I + eps E^(k) (k = 11, 22, 33, 23, 13, 12,
shear cases symmetric) give the columns of the 6x6 Voigt stiffness
C_eff[:, k] = voigt(sym <P>^(k)) / eps: at small eps the first Piola-Kirchhoff
stress equals the Cauchy stress to O(eps), and the shear cases apply an
engineering shear strain of eps.  Every solve runs in the HIP library.
"""
from __future__ import annotations

import numpy as np

from .fgfft import Batch, make_opts

VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def six_load_cases(eps):
    out = []
    for i, j in VOIGT:
        E = np.zeros((3, 3))
        E[i, j] += 0.5
        E[j, i] += 0.5
        out.append(np.eye(3) + eps * E)
    return out


def voigt_stiffness(P_cases, eps):
    """P_cases: (6, 3, 3) mean stresses of the six load cases -> (6, 6)."""
    C = np.zeros((6, 6))
    for k in range(6):
        S = 0.5 * (P_cases[k] + P_cases[k].T)
        C[:, k] = [S[i, j] for i, j in VOIGT]
    return C / eps


def effective_stiffness(rves, eps=1e-3, precision="fp64", opts=None, graph_ticks=16, stream=None):
    """rves: list of dicts with shape, spacing and device tensors E, nu,
    Omega (and optionally c).  Returns (C_eff [n_rve, 6, 6], per-item stats,
    P_avg [n_rve, 6, 3, 3])."""
    b = Batch([r["shape"] for r in rves], [r["spacing"] for r in rves], 6, precision, stream=stream)
    try:
        for k, r in enumerate(rves):
            b.set_material(k, r["E"], r["nu"], r["Omega"], r.get("c"))
        P, stats, _ = b.newton_solve(six_load_cases(eps), opts or make_opts(), graph_ticks=graph_ticks)
    finally:
        b.close()
    C = np.stack([voigt_stiffness(P[k], eps) for k in range(len(rves))])
    return C, stats, P
