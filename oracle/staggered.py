"""Global staggered scheme (Sec. 3.2 Global problem, Alg. 4).

Per time step:
  1. F <- F_t + dFbar (the macroscopic increment; fluctuation kept).
  2. Chemistry once, with F and d of the previous step (Alg. 3).
  3. Repeat: mechanics (Alg. 1) with (c, d^k) -> F^{k+1}; history and PFF
     (Alg. 2) with the new stress -> d^{k+1}; stop when the equilibrium
     residual (eq. (31)) recomputed with d^{k+1} is <= tol_nw.

Beyond the paper (its stated approximation removed): chemistry="coupled"
solves the Fick step inside the loop, from c_t with the current F^k and
d^k, before each mechanics solve, and the loop also requires the
concentration to have settled, ||c^{k+1} - c^k|| <= tol_chem ||c_t||.

Readings of the paper taken here: Alg. 4 tests "tol_mech" but declares
tol_nw; we use tol_nw.  Alg. 4 sets no cap on the staggered iterations; we
stop after 100 and report it (during damage growth the loop converges
linearly, at a rate near 0.75 per iteration when a ligament is half broken,
so 20 are too few).  The history
is updated as H <- max(H, D_f) at every PFF call, so staggered iterates
count as intermediate states.
"""
from __future__ import annotations

import numpy as np

from .chemistry import fick_step
from .fracture import pff_solve, update_history
from .mechanics import NoConvergence, err_denominator, newton_solve, norm, residual_rhs, uniform_field


class StaggeredNoConvergence(NoConvergence):
    """The staggered loop used max_stag iterations without reaching tol_nw;
    ``result`` holds (F, c, d, H, stats) of the last iterate."""

    def __init__(self, result):
        st = result[-1]
        super().__init__(f"staggered loop: err_res {st['err_res']:.3e} after {st['stag_iters']} iterations")
        self.result = result


def staggered_step(F, c, d, H, Fbar_new, Fbar_old, mat, dt=None, cdot_B=None,
                   chemistry=True, tol_newton=1e-8, tol_lin=1e-10, tol_chem=1e-8,
                   tol_pff=1e-10, max_stag=100, raise_on_noconv=True, jacobian="mu_c"):
    """One time step of Alg. 4; returns (F, c, d, H, stats), stats["converged"]
    telling whether err_res <= tol_newton was reached.  Without convergence in
    max_stag iterations StaggeredNoConvergence is raised (or, with
    raise_on_noconv=False, the result is returned with converged False)."""
    shape = mat["shape"]
    spacing = mat["spacing"]
    F = F + uniform_field(np.asarray(Fbar_new) - np.asarray(Fbar_old), shape)
    st = dict(newton=[], pff_iters=[], stag_iters=0, chem=None, converged=False, chem_coupled=[])
    coupled = chemistry == "coupled"
    c_t = c
    if chemistry and not coupled:
        c, chem = fick_step(c, F, d, cdot_B, dt, mat, tol_chem=tol_chem, tol_lin=tol_lin, jacobian=jacobian)
        st["chem"] = chem
    den = None if coupled else err_denominator(Fbar_new, c, d, mat, spacing)
    for k in range(max_stag):
        dc_rel = 0.0
        if coupled:
            c_prev = c
            c, chem = fick_step(c_t, F, d, cdot_B, dt, mat, tol_chem=tol_chem, tol_lin=tol_lin, jacobian=jacobian)
            st["chem_coupled"].append(chem)
            st["chem"] = chem
            dc_rel = norm(c - c_prev) / norm(c_t)
            den = err_denominator(Fbar_new, c, d, mat, spacing)
        F, ns = newton_solve(F, Fbar_new, c, d, mat, spacing,
                             tol_newton=tol_newton, tol_lin=tol_lin)
        st["newton"].append(ns)
        H = update_history(H, F, c, mat)
        d, n = pff_solve(H, mat["gc"], mat["lc"], spacing, tol=tol_pff)
        st["pff_iters"].append(n)
        GP, _ = residual_rhs(F, c, d, mat, spacing)
        err = norm(GP) / den
        st["stag_iters"] = k + 1
        st["err_res"] = err
        st["dc_rel"] = dc_rel
        if err <= tol_newton and (not coupled or (k > 0 and dc_rel <= tol_chem)):
            st["converged"] = True
            break
    if not st["converged"] and raise_on_noconv:
        raise StaggeredNoConvergence((F, c, d, H, st))
    return F, c, d, H, st
