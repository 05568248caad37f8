"""The coupled path over a whole trajectory: the 32^3 twin of the
chemo-mechanical particle workload (ellipsoid 10/8/7 voxels in a compliant
buffer, inward flux on its inner shell, dt = 5 s, 200 steps of Alg. 4: one
Fick step, then mechanics and phase field to tol_nw), through the C ABI,
against the oracle's trajectory stored by tests/golden/make_particle32_200.py.

Every step: the same staggered and Fick Newton iteration counts, and the
mean concentration, ||c - c0||, ||F - I||, max d and <P> within 1e-9 of the
oracle's.  After the last step: c, d, H and F at 512 seeded voxels within
1e-9 (c relative to the sampled c - c0, F to the sampled F - I, d and H
relative to their sampled norms, or absolutely 1e-12 while they are zero).
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


def _rel(a, b, ref):
    return abs(a - b) / max(abs(ref), 1e-300)


def test_particle32_trajectory_matches_oracle():
    with open(os.path.join(HERE, "golden", "particle32_200.json")) as f:
        gold = json.load(f)
    w = synth.particle_workload(n=32)
    shape = w["shape"]
    plan = plan_for(w)
    eye = np.eye(3)
    F = dt(np.broadcast_to(eye.reshape(9, 1, 1, 1), (9,) + shape))
    c, d, H = dt(w["c0"]), dt(w["d0"]), dt(np.zeros(shape))
    plan.set_state(F, c, d, H)
    cdot = dt(w["cdot_B"])
    c0 = torch.as_tensor(w["c0"], device=c.device)
    I9 = torch.as_tensor(eye.reshape(9, 1, 1, 1), device=F.device)
    worst = 0.0
    for k, g in enumerate(gold["steps"]):
        st = staggered_step(plan, eye, dt=w["dt"], cdot_B=cdot)
        assert st["stag_iters"] == g["stag"], (k, st["stag_iters"], g["stag"])
        assert st["chem"]["newton_iters"] == g["fick_newton"], (k, st["chem"]["newton_iters"], g["fick_newton"])
        c_mean = float(c.mean().item())
        c_dev = float(torch.linalg.vector_norm(c - c0).item())
        F_dev = float(torch.linalg.vector_norm(F - I9).item())
        d_max = float(d.max().item())
        Pm = plan.homogenized_stress().ravel()
        errs = [_rel(c_mean, g["c_mean"], g["c_mean"]), _rel(c_dev, g["c_dev"], g["c_dev"]),
                _rel(F_dev, g["F_dev"], g["F_dev"]),
                abs(d_max - g["d_max"]) / max(g["d_max"], 1e-3),
                float(np.max(np.abs(Pm - np.asarray(g["P_avg"]))) / max(np.max(np.abs(g["P_avg"])), 1e-300))]
        worst = max(worst, max(errs))
        assert max(errs) <= 1e-9, (k, errs)
        if k % 20 == 19:
            print(f"step {k + 1}: stag {st['stag_iters']} fick {st['chem']['newton_iters']} c_mean {c_mean:.8f} "
                  f"worst rel so far {worst:.2e}", flush=True)
    vox = np.asarray(gold["voxels"])
    cg_ = host(c).ravel()[vox]
    c0s = w["c0"].ravel()[vox]
    co = np.asarray(gold["c"])
    ec = np.linalg.norm(cg_ - co) / np.linalg.norm(co - c0s)
    Fg = host(F).reshape(9, -1)[:, vox]
    Fo = np.asarray(gold["F"])
    Is = eye.reshape(9, 1)
    eF = np.linalg.norm(Fg - Fo) / np.linalg.norm(Fo - Is)
    dg, do = host(d).ravel()[vox], np.asarray(gold["d"])
    Hg, Ho = host(H).ravel()[vox], np.asarray(gold["H"])
    ed = np.linalg.norm(dg - do) / np.linalg.norm(do) if np.linalg.norm(do) > 0 else np.max(np.abs(dg))
    eH = np.linalg.norm(Hg - Ho) / np.linalg.norm(Ho) if np.linalg.norm(Ho) > 0 else np.max(np.abs(Hg))
    print(f"after {len(gold['steps'])} steps: c {ec:.2e}, F {eF:.2e}, d {ed:.2e}, H {eH:.2e}", flush=True)
    assert ec <= 1e-9 and eF <= 1e-9
    assert ed <= (1e-9 if np.linalg.norm(do) > 0 else 1e-12)
    assert eH <= (1e-9 if np.linalg.norm(Ho) > 0 else 1e-12)
    plan.close()
