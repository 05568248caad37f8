"""Write polydisperse_window48_ramp.json: the oracle's damage ramp on the
48^3 full-resolution window of the 256^3 polydisperse microstructure around
the gap between spheres 12 and 55 (synth.polydisperse_window): 20 load
increments Fbar = I + 0.0025 n e1 (x) e1, each one step of the global
staggered scheme (Alg. 4) without chemistry (mechanics and phase field
alternated to err_res <= 1e-8, at most 100 iterations), damage on, the
threshold stress sigma_max = 0.25 E.

Stored: per increment the staggered, Newton and CG iteration counts, err_res,
max d, ||d||, ||F - Fbar||, max H and <P>; after increments 12, 16 and 20, F,
d and H at 512 seeded voxels and the full-field norms.  Calls only the
oracle and the seeded input generators.

    python tests/golden/make_polydisperse_window48_ramp.py     (one to two hours on 8 cores)
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
SNAPSHOTS = (12, 16, 20)
STRENGTH = 0.25
MAX_STAG = 100


def main():
    osp.WORKERS = min(4, os.cpu_count() or 1)
    t0 = time.time()
    w = synth.polydisperse_window(n=48, strength_ratio=STRENGTH)
    shape = w["shape"]
    rng = np.random.default_rng(241116583 + 33)
    vox = rng.choice(int(np.prod(shape)), size=N_SAMPLE, replace=False)
    F = mechanics.uniform_field(np.eye(3), shape)
    c, d, H = w["c0"].copy(), w["d0"].copy(), np.zeros(shape)
    Fprev = np.eye(3)
    incs, snaps = [], {}
    for k, Fbar in enumerate(w["loads"]):
        F, c, d, H, st = staggered.staggered_step(F, c, d, H, Fbar, Fprev, w, chemistry=False, max_stag=MAX_STAG)
        Fprev = Fbar
        Pm = mechanics.mean_stress(F, c, d, w)
        Fu = mechanics.uniform_field(Fbar, shape)
        incs.append(dict(
            stag=st["stag_iters"], newton=[s["newton_iters"] for s in st["newton"]],
            cg=[list(s["lin_iters"]) for s in st["newton"]], pff_cg=list(st["pff_iters"]), err_res=st["err_res"],
            d_max=float(d.max()), d_norm=float(np.linalg.norm(d)), F_dev=float(np.linalg.norm(F - Fu)),
            H_max=float(H.max()), P_avg=Pm.ravel().tolist()))
        print(f"increment {k + 1}: stag {st['stag_iters']} d_max {d.max():.4f} ({time.time() - t0:.0f} s)", flush=True)
        if k + 1 in SNAPSHOTS:
            Ff = F.reshape(9, -1)
            snaps[str(k + 1)] = dict(
                F=[[float(Ff[q, v]) for v in vox] for q in range(9)], d=[float(d.ravel()[v]) for v in vox],
                H=[float(H.ravel()[v]) for v in vox], norm_F_dev=float(np.linalg.norm(F - Fu)),
                norm_d=float(np.linalg.norm(d)), norm_H=float(np.linalg.norm(H)))
    rec = dict(workload="polydisperse_window n=48 pair (12, 55)", gap=float(w["gap"]), strength_ratio=STRENGTH,
               max_stag=MAX_STAG, tol_newton=1e-8, tol_lin=1e-10, tol_pff=1e-10, voxels=[int(v) for v in vox],
               increments=incs, snapshots=snaps)
    with open(os.path.join(HERE, "polydisperse_window48_ramp.json"), "w") as f:
        json.dump(rec, f)
    print(f"written ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
