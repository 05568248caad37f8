"""The adjoint form at its full size: 128^3 Gaussian-random-field workload,
L = <P_11> at F = I + 0.02 e1 (x) e1 (eq. (30) differentiated).

* The FP64 and mixed GPU gradients d L / d log E and d L / d Omega against
  the oracle's, stored by tests/golden/make_grf128_adjoint.py at 256 seeded
  voxels (FP64 1e-9, mixed 1e-6 relative over the sample), and the exact
  invariant sum_x dL/dlogE = L.
* Both against central finite differences by difference solves (the
  shifted Newton solve from the converged state with B = P of that state,
  one voxel's log E or Omega perturbed by +-eta) on the workload's 32
  seeded voxels: |g - fd| <= 1e-5 (|fd| + rms g).
"""
import json
import os

import numpy as np
import pytest
import torch

import synth
from paper_2411_16583_amd import make_opts
from tests.gpu_util import DEV, dt, host, plan_for

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
W11 = np.diag([1.0, 0.0, 0.0])


def _gold():
    with open(os.path.join(HERE, "golden", "grf128_adjoint.json")) as f:
        return json.load(f)


def _solve(w, precision):
    shape = w["shape"]
    plan = plan_for(w, precision)
    F = dt(np.broadcast_to(np.eye(3).reshape(9, 1, 1, 1), (9,) + shape))
    plan.set_state(F, dt(w["c0"]), dt(w["d0"]), dt(np.zeros(shape)))
    tn = 1e-12 if precision == "fp64" else 1e-10
    st = plan.newton_solve(w["loads"][0], make_opts(tn, 1e-12))
    gE = torch.empty(shape, dtype=torch.float64, device=DEV)
    gO = torch.empty(shape, dtype=torch.float64, device=DEV)
    sa = plan.adjoint_gradient(W11, gE, gO, make_opts(1e-12, 1e-12))
    L = float(plan.homogenized_stress()[0, 0])
    print(f"{precision} 128^3: newton {st['newton_iters']} cg {st['lin_history']}, adjoint cg "
          f"{sa['lin_iters_last']}, L {L:.9e}", flush=True)
    return plan, F, gE, gO, L


@pytest.fixture(scope="module")
def fd128():
    """FP64 base state, gradients and the 32 finite differences."""
    w = synth.grf_workload(n=128)
    shape = w["shape"]
    plan, F, gE, gO, L = _solve(w, "fp64")
    F0 = F.clone()
    P0 = torch.empty((9,) + shape, dtype=torch.float64, device=DEV)
    plan.stress(P0)
    m = plan._mats
    fd = {"logE": [], "Omega": []}
    # the difference problem's residual has a floor near 1e-8 of its start at
    # 128^3: P(F) - B carries the rounding of the stress, about 1e-16 of its
    # two ~G-sized terms that nearly cancel, at every one of the 1.9e7 values,
    # against a start set by one perturbed voxel.  Solved to 1e-6, the
    # difference of <P> is good to about 1e-6, below the 1e-5 bar of the check
    opts = make_opts(1e-6, 1e-8)
    for k, v in enumerate(int(x) for x in w["fd_voxels"]):
        for param, eta in (("logE", 1e-3), ("Omega", 1e-4)):
            dL = []
            for sgn in (1.0, -1.0):
                E = m["E"].clone()
                Om = m["Omega"].clone()
                if param == "logE":
                    E.view(-1)[v] *= float(np.exp(sgn * eta))
                else:
                    Om.view(-1)[v] += sgn * eta
                plan.set_material(E, m["nu"], Om, m["D"], m["sigma_max"], gc=w["gc"], lc=w["lc"], RT=w["RT"],
                                  c_max=w["c_max"])
                F.copy_(F0)
                plan.newton_solve_shifted(P0, opts)
                P1 = torch.empty_like(P0)
                plan.stress(P1)
                dL.append(float(torch.mean(P1[0] - P0[0]).item()))
            fd[param].append((dL[0] - dL[1]) / (2.0 * eta))
        if k % 8 == 7:
            print(f"finite differences: {k + 1} voxels done", flush=True)
    plan.close()
    return dict(w=w, gE=host(gE).ravel(), gO=host(gO).ravel(), L=L, fd=fd)


def _check(w, gE, gO, L, gold, fd, tol_oracle):
    vox = np.asarray(gold["voxels"])
    oE, oO = np.asarray(gold["dL_dlogE"]), np.asarray(gold["dL_dOmega"])
    eE = np.linalg.norm(gE[vox] - oE) / np.linalg.norm(oE)
    eO = np.linalg.norm(gO[vox] - oO) / np.linalg.norm(oO)
    print(f"  vs oracle (256 voxels): logE {eE:.2e}, Omega {eO:.2e}; L {abs(L - gold['L']) / abs(gold['L']):.2e}; "
          f"sum dL/dlogE - L {abs(gE.sum() - L) / abs(L):.2e}", flush=True)
    assert eE <= tol_oracle and eO <= tol_oracle
    assert abs(L - gold["L"]) <= tol_oracle * abs(gold["L"])
    assert abs(gE.sum() - L) <= 1e-9 * abs(L)
    fv = [int(x) for x in w["fd_voxels"]]
    rE, rO = np.sqrt(np.mean(gE ** 2)), np.sqrt(np.mean(gO ** 2))
    worst_E = max(abs(gE[v] - f) / (abs(f) + rE) for v, f in zip(fv, fd["logE"]))
    worst_O = max(abs(gO[v] - f) / (abs(f) + rO) for v, f in zip(fv, fd["Omega"]))
    print(f"  vs finite differences (32 voxels): worst logE {worst_E:.2e}, Omega {worst_O:.2e}", flush=True)
    assert worst_E <= 1e-5 and worst_O <= 1e-5


def test_adjoint128_fp64_matches_oracle_and_fd(fd128):
    gold = _gold()
    _check(fd128["w"], fd128["gE"], fd128["gO"], fd128["L"], gold, fd128["fd"], 1e-9)


def test_adjoint128_mixed_matches_oracle_and_fd(fd128):
    gold = _gold()
    w = fd128["w"]
    plan, F, gE, gO, L = _solve(w, "mixed")
    plan.close()
    _check(w, host(gE).ravel(), host(gO).ravel(), L, gold, fd128["fd"], 1e-6)
