"""Helpers shared by the GPU tests (device tensors from numpy, plan setup)."""
import numpy as np
import torch

from paper_2411_16583_amd import Plan

DEV = torch.device("cuda:0")


def dt(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), dtype=torch.float64, device=DEV)


def host(t, shape=None):
    a = t.detach().cpu().numpy()
    return a.reshape(shape) if shape is not None else a


def plan_for(work, precision="fp64", with_chem=False):
    plan = Plan(work["shape"], work["spacing"], precision, law=work.get("law", "neo_hookean"))
    mats = dict(E=dt(work["E"]), nu=dt(work["nu"]), Omega=dt(work["Omega"]),
                D=dt(work["D"]), sigma_max=dt(work["sigma_max"]))
    plan.set_material(mats["E"], mats["nu"], mats["Omega"], mats["D"], mats["sigma_max"],
                      gc=work["gc"], lc=work["lc"], RT=work["RT"], c_max=work["c_max"])
    plan._mats = mats
    return plan


def rel(a, b, ref=None):
    ref = b if ref is None else ref
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(ref)), 1e-300))
