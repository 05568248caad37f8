"""Write grf128_adjoint.json: the oracle's adjoint gradient of L = <P_11>
with respect to log E and Omega on the 128^3 Gaussian-random-field workload
(correlation length 8 voxels; log E mean log(10 GPa), std 0.5; Omega mean
0.03, std 0.01; c = 0.5, nu = 0.3; F = I + 0.02 e1 (x) e1), at the 32 seeded
finite-difference voxels of the workload and 224 further seeded voxels,
with L, the oracle's iteration counts and the sums of both gradient fields.

The gradient follows eq. (30) differentiated (the adjoint reading of the
oracle's adjoint module): a converged Newton state (Alg. 1, tolerances
1e-12 / 1e-12), then one CG solve of the adjoint system.  Calls only the
oracle and the seeded input generators.

    python tests/golden/make_grf128_adjoint.py      (about half an hour on 8 cores)
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
from oracle import adjoint, mechanics  # noqa: E402

N_EXTRA = 224


def main():
    osp.WORKERS = os.cpu_count() or 1
    t0 = time.time()
    w = synth.grf_workload(n=128)
    Fbar = w["loads"][0]
    shape = w["shape"]
    F = mechanics.uniform_field(Fbar, shape)
    F, st = mechanics.newton_solve(F, Fbar, w["c0"], w["d0"], w, w["spacing"], tol_newton=1e-12, tol_lin=1e-12)
    print(f"newton {st['newton_iters']} cg {st['lin_iters']} ({time.time() - t0:.0f} s)", flush=True)
    gE, gO, it = adjoint.adjoint_gradient(F, w["c0"], w["d0"], w, tol_lin=1e-12)
    print(f"adjoint cg {it} ({time.time() - t0:.0f} s)", flush=True)
    L = float(mechanics.mean_stress(F, w["c0"], w["d0"], w)[0, 0])
    rng = np.random.default_rng(241116583 + 55)
    extra = rng.choice(int(np.prod(shape)), size=N_EXTRA, replace=False)
    vox = [int(v) for v in w["fd_voxels"]] + [int(v) for v in extra]
    gEf, gOf = gE.ravel(), gO.ravel()
    rec = dict(
        workload="grf n=128", Fbar=np.asarray(Fbar).tolist(), L=L,
        newton_iters=st["newton_iters"], newton_cg=st["lin_iters"], adjoint_cg=it,
        tol_newton=1e-12, tol_lin=1e-12,
        sum_dL_dlogE=float(gE.sum()), sum_dL_dOmega=float(gO.sum()),
        rms_dL_dlogE=float(np.sqrt(np.mean(gE ** 2))), rms_dL_dOmega=float(np.sqrt(np.mean(gO ** 2))),
        n_fd_voxels=len(w["fd_voxels"]), voxels=vox,
        dL_dlogE=[float(gEf[v]) for v in vox], dL_dOmega=[float(gOf[v]) for v in vox],
    )
    with open(os.path.join(HERE, "grf128_adjoint.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(f"written ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
