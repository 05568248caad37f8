"""Pins of oracle/adjoint.py (FD by difference solves, exact scaling
invariant, global-shift FD) and oracle/staggered.py (reduces to Alg. 1 without
damage and chemistry; mass identity and 0 <= d < 1 on a small particle)."""
import numpy as np

import synth
from oracle import adjoint, mechanics, staggered


def _grf_small(n=8):
    w = synth.grf_workload(n=n)
    F0 = mechanics.uniform_field(np.eye(3), w["shape"])
    Fbar = w["loads"][0]
    F = F0 + mechanics.uniform_field(Fbar - np.eye(3), w["shape"])
    F, _ = mechanics.newton_solve(F, Fbar, w["c0"], w["d0"], w, w["spacing"],
                                  tol_newton=1e-12, tol_lin=1e-12)
    return w, F


def test_adjoint_vs_finite_differences():
    w, F = _grf_small()
    gE, gO, _ = adjoint.adjoint_gradient(F, w["c0"], w["d0"], w, tol_lin=1e-12)
    rng = np.random.default_rng(50)
    vox = rng.integers(0, gE.size, size=3)
    for v in vox:
        fdE = adjoint.fd_gradient(F, w["c0"], w["d0"], w, int(v), "logE", 1e-3)
        fdO = adjoint.fd_gradient(F, w["c0"], w["d0"], w, int(v), "Omega", 1e-4)
        assert abs(gE.ravel()[v] - fdE) <= 1e-5 * (abs(fdE) + np.sqrt(np.mean(gE ** 2)))
        assert abs(gO.ravel()[v] - fdO) <= 1e-5 * (abs(fdO) + np.sqrt(np.mean(gO ** 2)))


def test_adjoint_scaling_invariant_and_global_shift():
    w, F = _grf_small()
    gE, gO, _ = adjoint.adjoint_gradient(F, w["c0"], w["d0"], w, tol_lin=1e-12)
    L = mechanics.mean_stress(F, w["c0"], w["d0"], w)[0, 0]
    # scaling every E by e^t scales P and leaves F unchanged: sum dL/dlogE = L
    assert abs(gE.sum() - L) < 1e-9 * abs(L)
    # d/dt L(Omega + t) by a well-conditioned global FD
    eta = 1e-4
    vals = []
    for s in (1, -1):
        m = dict(w)
        m["Omega"] = w["Omega"] + s * eta
        Fs, _ = mechanics.newton_solve(F.copy(), w["loads"][0], w["c0"], w["d0"], m, w["spacing"],
                                       tol_newton=1e-12, tol_lin=1e-12)
        vals.append(mechanics.mean_stress(Fs, w["c0"], w["d0"], m)[0, 0])
    fd = (vals[0] - vals[1]) / (2 * eta)
    assert abs(gO.sum() - fd) < 1e-6 * abs(fd)


def test_staggered_reduces_to_mechanics_without_damage():
    w = synth.inclusion_workload(n=8, n_inc=1)
    shape = w["shape"]
    F0 = mechanics.uniform_field(np.eye(3), shape)
    Fbar = w["loads"][0]
    F1, c1, d1, H1, st = staggered.staggered_step(F0, w["c0"], w["d0"], np.zeros(shape), Fbar,
                                                 np.eye(3), w, chemistry=False)
    F2, _ = mechanics.newton_solve(F0 + mechanics.uniform_field(Fbar - np.eye(3), shape), Fbar,
                                   w["c0"], w["d0"], w, w["spacing"])
    assert st["stag_iters"] == 1
    assert np.array_equal(F1, F2)
    assert np.all(d1 == 0.0)


def test_particle_twin_mass_and_bounds():
    w = synth.particle_workload(n=16, n_steps=1, dt=20.0, q_in=4e-10, sigma_max=0.8e6)
    shape = w["shape"]
    F = mechanics.uniform_field(np.eye(3), shape)
    c, d, H = w["c0"].copy(), w["d0"].copy(), np.zeros(shape)
    for step in range(1):
        c_prev = c.copy()
        F, c, d, H, st = staggered.staggered_step(F, c, d, H, np.eye(3), np.eye(3), w,
                                                  dt=w["dt"], cdot_B=w["cdot_B"])
        assert abs(c.sum() - c_prev.sum() - w["dt"] * w["cdot_B"].sum()) < 1e-9 * c.sum()
        assert np.all(d >= 0.0) and np.all(d < 1.0)
    assert np.max(H) > 0.0 and np.max(d) > 0.0


def test_coupled_chemistry_reduces_to_once_per_step_without_coupling():
    """With no swelling (Omega = 0) and no damage the mechanics does not
    depend on c and F stays F_t: solving the chemistry inside the loop gives
    exactly the concentration of the once-per-step scheme."""
    w = synth.particle_workload(n=8, n_steps=1, dt=20.0, sigma_max=1e30)
    w["Omega"] = np.zeros(w["shape"])
    shape = w["shape"]
    F0 = mechanics.uniform_field(np.eye(3), shape)
    args = (F0, w["c0"].copy(), w["d0"].copy(), np.zeros(shape), np.eye(3), np.eye(3), w)
    _, ca, _, _, sa = staggered.staggered_step(*args, dt=w["dt"], cdot_B=w["cdot_B"])
    _, cb, _, _, sb = staggered.staggered_step(*args, dt=w["dt"], cdot_B=w["cdot_B"], chemistry="coupled",
                                               jacobian="full")
    assert sb["stag_iters"] == 2 and sb["dc_rel"] == 0.0
    assert np.max(np.abs(ca - cb)) <= 1e-14


def test_coupled_chemistry_solves_fick_with_final_fields():
    """The coupled step's concentration solves the Fick equation (eq. (43))
    with the step's final F and d (to the Newton and loop tolerances), which
    the once-per-step scheme's does not (it uses F of the start of the
    step)."""
    from oracle import chemistry as ch

    w = synth.particle_workload(n=8, n_steps=1, dt=20.0, sigma_max=1e30)
    shape = w["shape"]
    F0 = mechanics.uniform_field(np.eye(3), shape)
    c_t = w["c0"].copy()
    args = (F0, c_t.copy(), w["d0"].copy(), np.zeros(shape), np.eye(3), np.eye(3), w)
    res = {}
    for mode in (True, "coupled"):
        F, c, d, H, st = staggered.staggered_step(*args, dt=w["dt"], cdot_B=w["cdot_B"], chemistry=mode,
                                                  jacobian="full", tol_chem=1e-11)
        f = ch.residual(c, c_t, F, d, w["cdot_B"], w["dt"], w)
        res[mode] = np.linalg.norm(f) / np.linalg.norm(c - c_t)
    assert res["coupled"] <= 1e-9
    assert res[True] >= 1e3 * res["coupled"]
