"""The damage ramp of the polydisperse workload at full resolution: the
48^3 window around the gap between spheres 12 and 55 (where damage starts),
20 load increments of the staggered scheme (Alg. 4 without chemistry:
mechanics and phase field alternated to err_res <= 1e-8), threshold stress
0.25 E, through the C ABI, against the oracle's ramp stored by
tests/golden/make_polydisperse_window48_ramp.py.

FP64: every increment with the oracle's staggered count, and max d, ||d||,
||F - Fbar||, max H and <P> within 1e-10 (relative; absolute 1e-12 while d
and H are zero); F, d and H at 512 seeded voxels after increments 12, 16
and 20 within 1e-10.  Mixed form (single-precision CG operator, Newton
refined in double precision): the same quantities within 1e-6, except the
sampled history H, within 1e-5: H = gc/(2 lc) D_f with D_f = sum
(sigma_i / sigma_max)^2 - 1 near its threshold turns a relative difference
of the stress into a relative difference of D_f larger by
2 (sigma / sigma_max)^2 / D_f (measured: F 7e-9 and d 3e-7 give H 1.2e-6
at increment 16).
"""
import json
import os

import numpy as np
import pytest
import torch

import synth
from paper_2411_16583_amd.driver import staggered_step
from tests.gpu_util import dt, host, plan_for

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _err(a, b):
    return abs(a - b) / abs(b) if b != 0 else abs(a)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_window48_damage_ramp_matches_oracle(precision, tol):
    with open(os.path.join(HERE, "golden", "polydisperse_window48_ramp.json")) as f:
        gold = json.load(f)
    w = synth.polydisperse_window(n=48, strength_ratio=gold["strength_ratio"])
    shape = w["shape"]
    plan = plan_for(w, precision)
    F = dt(np.broadcast_to(np.eye(3).reshape(9, 1, 1, 1), (9,) + shape))
    c, d, H = dt(w["c0"]), dt(w["d0"]), dt(np.zeros(shape))
    plan.set_state(F, c, d, H)
    vox = np.asarray(gold["voxels"])
    worst = 0.0
    for k, (Fbar, g) in enumerate(zip(w["loads"], gold["increments"])):
        st = staggered_step(plan, Fbar, chemistry=False, max_stag=gold["max_stag"], tol_newton=gold["tol_newton"],
                            tol_lin=gold["tol_lin"], tol_pff=gold["tol_pff"])
        Fu = torch.as_tensor(np.asarray(Fbar).reshape(9, 1, 1, 1), device=F.device)
        vals = dict(d_max=float(d.max().item()), d_norm=float(torch.linalg.vector_norm(d).item()),
                    F_dev=float(torch.linalg.vector_norm(F - Fu).item()), H_max=float(H.max().item()))
        errs = [_err(vals[q], g[q]) for q in vals]
        Pm = plan.homogenized_stress().ravel()
        errs.append(float(np.max(np.abs(Pm - np.asarray(g["P_avg"]))) / np.max(np.abs(g["P_avg"]))))
        worst = max(worst, max(errs))
        print(f"{precision} increment {k + 1}: stag {st['stag_iters']} (oracle {g['stag']}), d_max "
              f"{vals['d_max']:.4f}, worst rel {max(errs):.2e}", flush=True)
        if precision == "fp64":
            assert st["stag_iters"] == g["stag"], (k, st["stag_iters"], g["stag"])
        assert max(errs) <= tol, (k, errs)
        snap = gold["snapshots"].get(str(k + 1))
        if snap:
            Fg = host(F).reshape(9, -1)[:, vox]
            Fo = np.asarray(snap["F"])
            ub = np.asarray(Fbar).reshape(9, 1)
            eF = np.linalg.norm(Fg - Fo) / np.linalg.norm(Fo - ub)
            ed = np.linalg.norm(host(d).ravel()[vox] - snap["d"]) / max(np.linalg.norm(snap["d"]), 1e-300)
            eH = np.linalg.norm(host(H).ravel()[vox] - snap["H"]) / max(np.linalg.norm(snap["H"]), 1e-300)
            print(f"  samples after increment {k + 1}: F {eF:.2e}, d {ed:.2e}, H {eH:.2e}", flush=True)
            assert eF <= tol and ed <= tol and eH <= (tol if precision == "fp64" else 1e-5)
    plan.close()
