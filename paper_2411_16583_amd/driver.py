"""Staggered time stepping (Alg. 4) on top of the C ABI.

Per time step: the macroscopic increment and one Fick step with the fields
of the previous step (Alg. 3), then mechanics (Alg. 1) and phase field
(Alg. 2) alternate until the equilibrium residual (eq. (31)) recomputed with
the new damage is <= tol_newton (at most ``max_stag`` times).  Every solver
call runs in the HIP library; this module only sequences them.

chemistry="coupled" removes the paper's once-per-step approximation: each
staggered iteration first re-solves the Fick step from c_t with the current
F and d, and the loop also waits for the concentration to settle
(||c^{k+1} - c^k|| <= tol_chem ||c_t||).  jacobian="full" uses the fully
implicit Newton linearisation of the Fick step (fick_step_full).
"""
from __future__ import annotations

from .fgfft import FG_E_NOCONV, FgError, make_opts


class StaggeredNoConvergence(FgError):
    """The staggered loop of Alg. 4 used its ``max_stag`` iterations without
    reaching err_res <= tol_newton.  ``stats`` holds the step's statistics;
    the plan's state holds the last iterate."""

    def __init__(self, stats):
        super().__init__(FG_E_NOCONV, f"staggered loop: err_res {stats['err_res']:.3e} after "
                                      f"{stats['stag_iters']} iterations")
        self.stats = stats


def staggered_step(plan, F_macro, dt=None, cdot_B=None, chemistry=True, tol_newton=1e-8, tol_lin=1e-10,
                   tol_chem=1e-8, tol_pff=1e-10, max_stag=100, max_lin=20000, raise_on_noconv=True,
                   jacobian="mu_c"):
    """One time step; returns a stats dict (``converged`` tells whether the
    staggered loop met its tolerance).  The plan's state (F, c, d, H) is
    updated in place.  When the loop does not converge within ``max_stag``
    iterations, StaggeredNoConvergence is raised (or, with
    raise_on_noconv=False, the stats are returned with converged=False)."""
    st = dict(chem=None, newton=[], pff=[], stag_iters=0, err_res=None, converged=False, chem_coupled=[])
    plan.apply_macro(F_macro)  # F^0 = F_t + dFbar (Alg. 1, first line)
    coupled = chemistry == "coupled"
    chem_opts = make_opts(tol_chem, tol_lin, 50, max_lin)
    if chemistry and not coupled:
        # chemistry once per step, with the new macroscopic F and the damage of
        # the previous step
        st["chem"] = plan.fick_step(dt, cdot_B, chem_opts, jacobian=jacobian)
    c = plan._keep.get("c") if coupled else None
    if coupled:
        import torch

        c_t = c.clone()
        nct = float(torch.linalg.vector_norm(c_t).item())
    for k in range(max_stag):
        dc_rel = 0.0
        if coupled:
            c_prev = c.clone()
            c.copy_(c_t)
            st["chem"] = plan.fick_step(dt, cdot_B, chem_opts, jacobian=jacobian)
            st["chem_coupled"].append(st["chem"])
            dc_rel = float(torch.linalg.vector_norm(c - c_prev).item()) / nct
        st["newton"].append(plan.newton_solve(F_macro, make_opts(tol_newton, tol_lin, 50, max_lin)))
        st["pff"].append(plan.pff_solve(make_opts(tol_newton, tol_pff, 50, max_lin)))
        err = plan.residual(F_macro)
        st["stag_iters"] = k + 1
        st["err_res"] = err
        st["dc_rel"] = dc_rel
        if err <= tol_newton and (not coupled or (k > 0 and dc_rel <= tol_chem)):
            st["converged"] = True
            break
    if not st["converged"] and raise_on_noconv:
        raise StaggeredNoConvergence(st)
    return st
