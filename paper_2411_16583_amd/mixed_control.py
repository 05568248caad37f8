"""Mixed macroscopic stress/strain control of Alg. 1 (Sec. 3.1: the full
Fbar prescribed, or combined with macroscopic stress conditions).

Some components of Fbar are prescribed and the others are free, with the
homogenised stress <P> prescribed in the free ones.  The discrete solution is
the state of Alg. 1 at the Fbar whose free components make <P> match.  Here
it is reached by an outer Newton iteration on those free components z:

    R(z) = <P>(Fbar(z))_free - Pbar_free,
    J    = d<P>_free / dz      (fg_homogenized_tangent, one solve per free
                                component at the current converged state),
    z   <- z - J^-1 R,

each step one strain-controlled Newton solve of Alg. 1 at Fbar(z) from the
previous state (the fluctuation is kept).  Every solve runs in the HIP
library; this module only sequences them.
"""
from __future__ import annotations

import numpy as np

from .fgfft import FG_E_NOCONV, FgError, make_opts


def newton_solve_mixed(plan, F_macro, stress_mask, P_target, opts=None, tol_stress=1e-12, max_outer=30,
                       tangent_opts=None):
    """F_macro: 3x3, the prescribed components (mask False) and the start of
    the free ones; stress_mask: 3x3 booleans, True where <P>_ij = P_target_ij
    is prescribed.  Stops when |<P> - P_target| over the masked components
    is <= tol_stress |<P>|.  Returns (Fbar, stats)."""
    mask = np.asarray(stress_mask, dtype=bool).reshape(3, 3)
    free = [int(k) for k in np.flatnonzero(mask.ravel())]
    Fbar = np.asarray(F_macro, dtype=np.float64).reshape(3, 3).copy()
    Pt = np.asarray(P_target, dtype=np.float64).reshape(3, 3)
    opts = opts or make_opts(1e-12, 1e-12)
    topts = tangent_opts or make_opts(opts.tol_newton, opts.tol_lin)
    st = dict(outer=0, newton=[], tangent_solves=0, stress_err=[])
    for it in range(max_outer + 1):
        st["newton"].append(plan.newton_solve(Fbar, opts))
        Pm = plan.homogenized_stress()
        R = np.array([Pm.ravel()[k] - Pt.ravel()[k] for k in free])
        err = float(np.max(np.abs(R))) / max(float(np.max(np.abs(Pm))), 1e-300) if free else 0.0
        st["stress_err"].append(err)
        if err <= tol_stress:
            st["outer"] = it
            return Fbar, st
        if it == max_outer:
            break
        J = np.empty((len(free), len(free)))
        for b, kb in enumerate(free):
            E = np.zeros(9)
            E[kb] = 1.0
            T = plan.homogenized_tangent(E.reshape(3, 3), topts).ravel()
            st["tangent_solves"] += 1
            J[:, b] = [T[ka] for ka in free]
        dz = np.linalg.solve(J, -R)
        for b, kb in enumerate(free):
            Fbar.flat[kb] += dz[b]
    raise FgError(FG_E_NOCONV, f"mixed control: stress error {st['stress_err'][-1]:.3e} after {max_outer} steps")
