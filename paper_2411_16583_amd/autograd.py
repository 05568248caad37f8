"""Differentiable homogenised stress: <P>(log E, Omega) of the equilibrium
state under a prescribed macroscopic F, with the backward pass by the adjoint
CG of the C ABI (fg_adjoint_gradient).

    P = homogenized_stress(plan, logE, Omega, nu, F_macro)   # (3, 3) tensor
    P[0, 0].backward()   # fills logE.grad and Omega.grad (voxel fields)

The forward pass runs Newton-CG (Alg. 1) from F = I plus the macroscopic
increment; the backward pass solves the adjoint system on the same operator
and evaluates (W + lam) : dP/dtheta per voxel.  Both run in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from .fgfft import make_opts


class _HomogenizedStress(torch.autograd.Function):
    @staticmethod
    def forward(ctx, logE, Omega, plan, nu, F_macro, c, d, opts, material):
        E = torch.exp(logE).contiguous()
        Om = Omega.contiguous()
        plan.set_material(E, nu, Om, material.get("D"), material.get("sigma_max"),
                          gc=material.get("gc", 1.0), lc=material.get("lc", 1.0),
                          RT=material.get("RT", 2478.957), c_max=material.get("c_max", 3e4))
        shape = tuple(logE.shape)
        F = torch.zeros((9,) + shape, dtype=torch.float64, device=logE.device)
        F[0] = 1.0
        F[4] = 1.0
        F[8] = 1.0
        plan.set_state(F, c, d, None)
        plan.newton_solve(np.asarray(F_macro, dtype=np.float64), opts)
        P = torch.tensor(plan.homogenized_stress(), dtype=torch.float64)
        ctx.plan, ctx.opts, ctx.shape = plan, opts, shape
        ctx.keep = (E, Om, F, c, d)
        return P

    @staticmethod
    def backward(ctx, grad_P):
        plan = ctx.plan
        dev = ctx.keep[0].device
        gE = torch.empty(ctx.shape, dtype=torch.float64, device=dev)
        gO = torch.empty(ctx.shape, dtype=torch.float64, device=dev)
        plan.adjoint_gradient(grad_P.detach().cpu().numpy().astype(np.float64), gE, gO, ctx.opts)
        return gE, gO, None, None, None, None, None, None, None


def homogenized_stress(plan, logE, Omega, nu, F_macro, c=None, d=None, opts=None, material=None):
    """<P> (3x3, float64 CPU tensor) as a differentiable function of the
    voxel fields logE and Omega (float64 device tensors of the plan's grid)."""
    opts = opts or make_opts(1e-10, 1e-12)
    material = material or {}
    if c is None:
        c = torch.zeros_like(logE)
    if d is None:
        d = torch.zeros_like(logE)
    return _HomogenizedStress.apply(logE, Omega, plan, nu, F_macro, c.contiguous(), d.contiguous(), opts, material)
