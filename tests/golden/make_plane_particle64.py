"""Write plane_particle64.json: the oracle's Alg. 4 on the 64 x 64 twin of
the 2-D particle of Sec. 5.1 (synth.plane_particle_workload(64): disc of
0.8 of the side, Young's modulus and threshold stress drawn from
eq. (Gumbell) with m = 3, SVK law, Omega = 1.3, inward source on the band),
from c = 0.01, F = I, d = 0, step by step until the damage first reaches
0.05, with the chemistry's full Jacobian, CG tolerance 1e-6 and the
staggered loop capped at 100 iterations.

Stored per step: staggered iterations, converged or not, Fick Newton
iterations, ||c - c0||, ||d||, ||F - I||, max c, max d and the voxel of
max d; and d at the last step on the whole 64 x 64 plane (10 digits).
Calls only the oracle and the seeded input generators.

    python tests/golden/make_plane_particle64.py      (about a minute)
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


def main():
    t0 = time.time()
    w = synth.plane_particle_workload(64)
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
    s = steps[-1]
    print(f"{len(steps)} steps, d max {s['d_max']:.3f} at {s['d_at']} ({time.time() - t0:.0f} s)", flush=True)
    out = dict(workload="plane particle n=64 (Sec. 5.1 twin)", d_nucleation=D_NUCLEATION, steps=steps,
               d_final=[[float(f"{v:.9e}") for v in row] for row in d[0]])
    with open(os.path.join(HERE, "plane_particle64.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
