"""Oracle on plane grids (N0 = 1, the 2-D problems of Sec. 4.3 and 5.1).

A plane grid is one voxel thick along axis 0 and periodic, so every
difference along axis 0 vanishes and the solution is the plane-strain one
(F_00 held at its macroscopic value).  Pins that do not use the oracle's own
formulas:
* a prismatic cell (the same plane repeated along axis 0) has a solution
  that does not vary along axis 0 and equals the plane grid's solution, for
  the mechanics (Alg. 1), the phase field (Alg. 2) and Fick's step (Alg. 3);
* a laminate along an in-plane axis has the exact piecewise-uniform
  solution of the laminate construction (the same rank-one jumps as in 3-D);
* the phase-field plane crack across an in-plane axis has the closed-form
  discrete profile.
"""
import numpy as np
import pytest

import synth
from oracle import chemistry, fracture, laminate, mechanics



def _tile(a, n0):
    return np.broadcast_to(a, a.shape[:-3] + (n0,) + a.shape[-2:]).copy()


def test_plane_mechanics_equals_prismatic_cell():
    n = 12
    w1 = synth.plane_inclusion_workload(n, n_inc=2)
    w4 = synth.plane_inclusion_workload(n, n_inc=2, thickness=4)
    F1, s1 = mechanics.solve_increments(w1, tol_newton=1e-12, tol_lin=1e-13)
    F4, s4 = mechanics.solve_increments(w4, tol_newton=1e-12, tol_lin=1e-13)
    Fbar = w1["loads"][-1]
    fl = np.max(np.abs(F1 - Fbar.reshape(3, 3, 1, 1, 1)))
    assert fl > 1e-4
    # no variation along axis 0 in the prismatic cell
    assert np.max(np.abs(F4 - F4[:, :, :1])) <= 1e-12 * fl
    assert np.max(np.abs(F4[:, :, :1] - F1)) <= 1e-11 * fl
    # plane strain: F_00 stays at its macroscopic value, F_0a = F_a0 = 0
    assert np.max(np.abs(F1[0, 0] - Fbar[0, 0])) <= 1e-14
    assert np.max(np.abs(F1[0, 1:])) <= 1e-14 and np.max(np.abs(F1[1:, 0])) <= 1e-14


@pytest.mark.parametrize("axis", [1, 2])
def test_plane_laminate_exact(axis):
    shape = [1, 8, 8]
    shape[axis] = 12
    shape = tuple(shape)
    work = synth.homogeneous_workload(shape, (0.1, 1.2, 0.9))
    mask = synth.laminate_mask(shape, axis, 5.0 / 12.0)
    matA = dict(E=80e9, nu=0.21, Omega=0.03, c=0.2, d=0.3)
    matB = dict(E=9e9, nu=0.34, Omega=0.0, c=0.0, d=0.0)
    work["E"] = np.where(mask, matA["E"], matB["E"])
    work["nu"] = np.where(mask, matA["nu"], matB["nu"])
    work["Omega"] = np.where(mask, matA["Omega"], matB["Omega"])
    c = np.where(mask, matA["c"], matB["c"])
    d = np.where(mask, matA["d"], matB["d"])
    Fbar = np.eye(3) + np.array([[0.01, 0.0, 0.0], [0.0, -0.01, 0.02], [0.0, 0.015, 0.03]])
    FA, FB, a = laminate.laminate_solution(Fbar, axis, 5.0 / 12.0, matA, matB)
    F = mechanics.uniform_field(Fbar, shape)
    Fn, st = mechanics.newton_solve(F, Fbar, c, d, work, work["spacing"], tol_newton=1e-13, tol_lin=1e-14)
    exact = np.where(mask[None, None], FA.reshape(3, 3, 1, 1, 1), FB.reshape(3, 3, 1, 1, 1))
    assert np.max(np.abs(Fn - exact)) <= 1e-12 * np.max(np.abs(exact - F))
    assert np.linalg.norm(a) > 1e-3


@pytest.mark.parametrize("axis", [1, 2])
def test_plane_crack_profile_on_plane_grid(axis):
    n = 64
    shape = [1, 4, 4]
    shape[axis] = n
    h = 0.05
    gc, lc, H0 = 2.0, 2 * h, 40.0
    H = np.zeros(shape)
    sl = [slice(None)] * 3
    sl[axis] = 0
    H[tuple(sl)] = H0
    d, _ = fracture.pff_solve(H, gc, lc, (h, h, h), tol=1e-14)
    prof, _ = fracture.plane_crack_profile(n, h, lc, gc, H0)
    line = np.moveaxis(d, axis, 0)[:, 0, 1]
    assert np.max(np.abs(line - prof)) < 1e-12 * prof.max()


def test_plane_phase_field_and_fick_equal_prismatic_cell():
    rng = np.random.default_rng(7)
    n = 16
    shape1 = (1, n, n)
    H = 5.0 * rng.random(shape1) ** 4
    sp = (0.1, 0.1, 0.1)
    d1, _ = fracture.pff_solve(H, 1.0, 0.2, sp, tol=1e-13)
    d4, _ = fracture.pff_solve(_tile(H, 4), 1.0, 0.2, sp, tol=1e-13)
    assert np.max(np.abs(d4 - _tile(d1, 4))) <= 1e-12
    w1 = synth.homogeneous_workload(shape1, (0.1, 1.0, 1.0), Omega=0.05, D=1e-14)
    w1["D"] = np.where(rng.random(shape1) < 0.5, 1e-14, 3e-15)
    w4 = synth.homogeneous_workload((4, n, n), (0.4, 1.0, 1.0), Omega=0.05, D=1e-14)
    w4["D"] = _tile(w1["D"], 4)
    c_t = 0.3 + 0.2 * rng.random(shape1)
    F_t = mechanics.uniform_field(np.eye(3), shape1) + 0.01 * rng.standard_normal((3, 3) + shape1)
    F_t[0, 1:] = 0.0
    F_t[1:, 0] = 0.0
    d_t = 0.2 * rng.random(shape1)
    src = np.where(rng.random(shape1) < 0.1, 1e-3, 0.0)
    c1, s1 = chemistry.fick_step(c_t, F_t, d_t, src, 10.0, w1)
    c4, s4 = chemistry.fick_step(_tile(c_t, 4), _tile(F_t, 4), _tile(d_t, 4), _tile(src, 4), 10.0, w4)
    assert s1["newton_iters"] == s4["newton_iters"]
    assert np.max(np.abs(c4 - _tile(c1, 4))) <= 1e-12 * np.max(np.abs(c1 - c_t))
