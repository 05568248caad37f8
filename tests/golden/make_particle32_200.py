"""Write particle32_200.json: the oracle's Alg. 4 (global staggered scheme:
one backward-Euler Fick step, then mechanics and phase field alternated to
tol_nw) over the 200 time steps of the 32^3 twin of the chemo-mechanical
particle workload (ellipsoid 10/8/7 voxels in a compliant buffer, inward
flux on the particle's inner shell, dt = 5 s, Omega = 0.03, sigma_max =
20 MPa), from c = 0.01, F = I, d = 0.

Stored: per step the staggered, Fick Newton and CG iteration counts, the
mean concentration, ||c - c0||, ||F - I||, max d, max H and <P>; after the
last step c, d, H and F at 512 seeded voxels and the full-field norms.
Calls only the oracle and the seeded input generators.

    python tests/golden/make_particle32_200.py     (about half an hour on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle.spectral as osp  # noqa: E402
import synth  # noqa: E402
from oracle import mechanics, staggered  # noqa: E402

N_SAMPLE = 512


def main():
    osp.WORKERS = min(4, os.cpu_count() or 1)
    t0 = time.time()
    w = synth.particle_workload(n=32)
    shape = w["shape"]
    eye = np.eye(3)
    F = mechanics.uniform_field(eye, shape)
    c, d, H = w["c0"].copy(), w["d0"].copy(), np.zeros(shape)
    steps = []
    for k in range(w["n_steps"]):
        F, c, d, H, st = staggered.staggered_step(F, c, d, H, eye, eye, w, dt=w["dt"], cdot_B=w["cdot_B"])
        Pm = mechanics.mean_stress(F, c, d, w)
        steps.append(dict(
            stag=st["stag_iters"], fick_newton=st["chem"]["newton_iters"], fick_cg=list(st["chem"]["lin_iters"]),
            newton=[s["newton_iters"] for s in st["newton"]], cg=[list(s["lin_iters"]) for s in st["newton"]],
            pff_cg=list(st["pff_iters"]), err_res=st["err_res"],
            c_mean=float(c.mean()), c_dev=float(np.linalg.norm(c - w["c0"])),
            F_dev=float(np.linalg.norm(F - mechanics.uniform_field(eye, shape))),
            d_max=float(d.max()), H_max=float(H.max()), P_avg=Pm.ravel().tolist()))
        if k % 10 == 9:
            print(f"step {k + 1}: stag {st['stag_iters']} fick {st['chem']['newton_iters']} c_mean {c.mean():.6f} "
                  f"d_max {d.max():.3e} ({time.time() - t0:.0f} s)", flush=True)
    rng = np.random.default_rng(241116583 + 22)
    vox = rng.choice(int(np.prod(shape)), size=N_SAMPLE, replace=False)
    Ff = F.reshape(9, -1)
    rec = dict(
        workload="particle n=32", n_steps=w["n_steps"], dt=w["dt"], steps=steps,
        voxels=[int(v) for v in vox],
        c=[float(c.ravel()[v]) for v in vox], d=[float(d.ravel()[v]) for v in vox],
        H=[float(H.ravel()[v]) for v in vox], F=[[float(Ff[k, v]) for v in vox] for k in range(9)],
        norm_c_dev=float(np.linalg.norm(c - w["c0"])), norm_d=float(np.linalg.norm(d)),
        norm_F_dev=float(np.linalg.norm(F - mechanics.uniform_field(eye, shape))),
    )
    with open(os.path.join(HERE, "particle32_200.json"), "w") as f:
        json.dump(rec, f)
    print(f"written ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
