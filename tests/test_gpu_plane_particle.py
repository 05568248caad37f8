"""The 2-D particle of Sec. 5.1 on the GPU: its 64 x 64 twin (eq. (Gumbell)
Young's modulus and threshold stress, SVK law, Omega = 1.3, inward source on
the band) against the oracle's Alg. 4 step by step to the first damage of
0.05 (tests/golden/plane_particle64.json, written by
tests/golden/make_plane_particle64.py from the oracle only).  The 512 x 512
particle itself runs through the N1 passes of length 512 (their transforms
are checked against numpy and the oracle in tests/test_gpu_core.py)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import mechanics
from paper_2411_16583_amd.driver import staggered_step
from tests.gpu_util import dt, host, plan_for

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "plane_particle64.json")


def test_plane_particle_twin_matches_oracle():
    with open(GOLDEN) as f:
        rec = json.load(f)
    w = synth.plane_particle_workload(64)
    shape = w["shape"]
    plan = plan_for(w)
    F0 = mechanics.uniform_field(np.eye(3), shape)
    t = dict(F=dt(F0), c=dt(w["c0"]), d=dt(w["d0"]), H=dt(np.zeros(shape)))
    plan.set_state(t["F"], t["c"], t["d"], t["H"])
    cdot = dt(w["cdot_B"])
    print(f"plane particle twin: {len(rec['steps'])} steps", flush=True)
    for k, o in enumerate(rec["steps"]):
        st = staggered_step(plan, np.eye(3), dt=w["dt"], cdot_B=cdot, tol_lin=w["tol_lin"], jacobian=w["jacobian"],
                            max_stag=100, raise_on_noconv=False)
        c, d = host(t["c"], shape), host(t["d"], shape)
        F = host(t["F"], (3, 3) + shape)
        assert st["chem"]["newton_iters"] == o["fick_newton"], k
        if o["converged"]:
            assert st["converged"] and st["stag_iters"] == o["stag"], k
        assert abs(np.linalg.norm(c - w["c0"]) - o["c_dev"]) <= 1e-9 * o["c_dev"], k
        assert abs(np.linalg.norm(F - F0) - o["F_dev"]) <= 1e-6 * o["F_dev"], k
        assert abs(np.linalg.norm(d) - o["d_norm"]) <= 1e-6 * max(o["d_norm"], 1e-3), k
    at = np.unravel_index(int(np.argmax(d)), d.shape)
    assert [int(at[1]), int(at[2])] == rec["steps"][-1]["d_at"]
    assert d.max() >= rec["d_nucleation"]
    assert np.max(np.abs(d[0] - np.asarray(rec["d_final"]))) <= 1e-6
    # damage starts inside the particle, away from the swelling band
    cc = (shape[1] - 1) / 2
    r = np.hypot(at[1] - cc, at[2] - cc)
    assert r < 0.4 * shape[1] - 3 * max(1, round(6 * shape[1] / 512))
