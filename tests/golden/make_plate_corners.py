"""Write plate_corners.json: the oracle's Alg. 4 on the chemo-mechanical
plate of Sec. 4.3 (synth.plate_workload: 64 x 64 plane grid, SVK law,
Omega = 1.3, sigma_max = 50 MPa, inward source on the plate's one-voxel
boundary band, three times stronger on 20-voxel segments at one corner) for
each of the four flux corners, from c = 0.01, F = I, d = 0, step by step
until the damage first reaches 0.05 (nucleation) or 60 steps.  Chemistry
with the full Jacobian, CG tolerance 1e-6, staggered loop capped at 100
iterations (a step that does not converge is recorded as such and the run
goes on from its state).

Stored per corner and step: staggered iterations, converged or not, Fick
Newton iterations, ||c - c0||, ||d||, ||F - I||, max c, max d and the voxel
(i1, i2) of max d; and at the last step d on the 20 x 20 window of the plate
at the flux corner.
Calls only the oracle and the seeded input generators.

    python tests/golden/make_plate_corners.py      (a few minutes)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import mechanics, staggered  # noqa: E402

D_NUCLEATION = 0.05


def run_corner(corner):
    w = synth.plate_workload(corner=corner)
    shape = w["shape"]
    eye = np.eye(3)
    F0 = mechanics.uniform_field(eye, shape)
    F, c, d, H = F0.copy(), w["c0"].copy(), w["d0"].copy(), np.zeros(shape)
    steps = []
    for k in range(w["n_steps"]):
        F, c, d, H, st = staggered.staggered_step(F, c, d, H, eye, eye, w, dt=w["dt"], cdot_B=w["cdot_B"],
                                                  tol_lin=w["tol_lin"], jacobian=w["jacobian"], max_stag=100,
                                                  raise_on_noconv=False)
        at = np.unravel_index(int(np.argmax(d)), d.shape)
        steps.append(dict(
            stag=st["stag_iters"], converged=bool(st["converged"]), fick_newton=st["chem"]["newton_iters"],
            c_dev=float(np.linalg.norm(c - w["c0"])), d_norm=float(np.linalg.norm(d)),
            F_dev=float(np.linalg.norm(F - F0)), c_max=float(c.max()), d_max=float(d.max()),
            d_at=[int(at[1]), int(at[2])]))
        if d.max() >= D_NUCLEATION:
            break
    r, q = w["corner_site"]
    r0 = r - 19 if r > shape[1] // 2 else r
    q0 = q - 19 if q > shape[2] // 2 else q
    win = d[0, r0:r0 + 20, q0:q0 + 20]
    return dict(corner=corner, corner_site=list(w["corner_site"]), steps=steps, window=[r0, q0],
                d_window=[[float(v) for v in row] for row in win])


def main():
    t0 = time.time()
    out = dict(workload="plate n=64 (Sec. 4.3)", d_nucleation=D_NUCLEATION, corners=[])
    for corner in range(4):
        r = run_corner(corner)
        s = r["steps"][-1]
        print(f"corner {corner}: {len(r['steps'])} steps, d max {s['d_max']:.3f} at {s['d_at']} "
              f"(flux corner {r['corner_site']}) ({time.time() - t0:.0f} s)", flush=True)
        out["corners"].append(r)
    with open(os.path.join(HERE, "plate_corners.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
