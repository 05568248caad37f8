"""Pins of oracle/mechanics.py: dense brute force on 4^3, uniform field,
exact laminate, averaging / Hill-Mandel invariants, homogenisation bounds."""
import numpy as np
import pytest

import synth
from oracle import constitutive as cm
from oracle import dense, laminate, mechanics, spectral


def small_two_phase(shape=(4, 4, 4), seed=20):
    rng = np.random.default_rng(seed)
    mask = rng.random(shape) < 0.4
    work = synth.homogeneous_workload(shape, 1.0)
    work["E"] = np.where(mask, 60e9, 10e9)
    work["nu"] = np.where(mask, 0.22, 0.33)
    work["c0"] = 0.3 * rng.random(shape)
    work["Omega"] = 0.05 * rng.random(shape)
    work["d0"] = 0.2 * rng.random(shape)
    return work


def test_matvec_equals_dense_operator():
    work = small_two_phase()
    shape, sp = work["shape"], work["spacing"]
    rng = np.random.default_rng(21)
    F = mechanics.uniform_field(np.eye(3), shape) + 0.05 * rng.standard_normal((3, 3) + shape)
    K = cm.tangent(F, work["c0"], work["d0"], work["E"], work["nu"], work["Omega"])
    A = dense.projector_dense(shape, sp) @ dense.tangent_blockdiag(K)
    X = rng.standard_normal((3, 3) + shape)
    y = mechanics.operator(K, X, sp)
    yd = (A @ X.ravel()).reshape(y.shape)
    assert np.max(np.abs(y - yd)) <= 1e-13 * np.max(np.abs(yd))


def test_cg_and_newton_equal_dense_solves():
    work = small_two_phase()
    shape, sp = work["shape"], work["spacing"]
    Fbar = np.eye(3) + np.array([[0.02, 0.003, 0], [0, -0.004, 0.001], [0.002, 0, 0.005]])
    F = mechanics.uniform_field(Fbar, shape)
    c, d = work["c0"], work["d0"]
    G = dense.projector_dense(shape, sp)
    # one linear solve: CG vs dense least squares restricted to range(G)
    K = cm.tangent(F, c, d, work["E"], work["nu"], work["Omega"])
    GP, _ = mechanics.residual_rhs(F, c, d, work, sp)
    b = -GP
    from oracle.krylov import cg
    x, it, _ = cg(lambda X: mechanics.operator(K, X, sp), b, 1e-13, 5000)
    A = G @ dense.tangent_blockdiag(K) @ G
    xd = np.linalg.lstsq(A, b.ravel(), rcond=1e-12)[0]
    xd = G @ xd
    assert np.max(np.abs(x.ravel() - xd)) <= 1e-10 * np.max(np.abs(xd))
    # full Newton vs a dense Newton written with the dense projector
    Fn, st = mechanics.newton_solve(F.copy(), Fbar, c, d, work, sp, tol_newton=1e-12, tol_lin=1e-13)
    Fd = F.ravel().copy()
    for _ in range(30):
        P = cm.stress(Fd.reshape(F.shape), c, d, work["E"], work["nu"], work["Omega"])
        r = -(G @ P.ravel())
        if np.linalg.norm(r) < 1e-14 * np.linalg.norm(P):
            break
        Kd = cm.tangent(Fd.reshape(F.shape), c, d, work["E"], work["nu"], work["Omega"])
        A = G @ dense.tangent_blockdiag(Kd) @ G
        Fd = Fd + G @ np.linalg.lstsq(A, r, rcond=1e-12)[0]
    fl = (Fd.reshape(F.shape) - F)
    assert np.linalg.norm(Fn - Fd.reshape(F.shape)) <= 1e-10 * np.linalg.norm(fl)


def test_uniform_field_is_exact_without_iterations():
    work = synth.homogeneous_workload((8, 6, 4), (1.0, 0.8, 0.5), Omega=0.04)
    work["c0"] = np.full(work["shape"], 0.3)
    work["d0"] = np.full(work["shape"], 0.1)
    Fbar = np.eye(3) + np.array([[0.03, 0.01, 0], [0.0, -0.01, 0.02], [0.005, 0, 0.0]])
    F = mechanics.uniform_field(Fbar, work["shape"])
    Fn, st = mechanics.newton_solve(F.copy(), Fbar, work["c0"], work["d0"], work, work["spacing"])
    assert st["newton_iters"] == 0
    assert st["err_history"][0] == 0.0
    assert np.array_equal(Fn, F)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laminate_exact(axis):
    shape = [8, 8, 8]
    shape[axis] = 12
    shape = tuple(shape)
    work = synth.homogeneous_workload(shape, (1.0, 1.2, 0.9))
    mask = synth.laminate_mask(shape, axis, 5.0 / 12.0)
    matA = dict(E=80e9, nu=0.21, Omega=0.03, c=0.2, d=0.3)
    matB = dict(E=9e9, nu=0.34, Omega=0.0, c=0.0, d=0.0)
    work["E"] = np.where(mask, matA["E"], matB["E"])
    work["nu"] = np.where(mask, matA["nu"], matB["nu"])
    work["Omega"] = np.where(mask, matA["Omega"], matB["Omega"])
    c = np.where(mask, matA["c"], matB["c"])
    d = np.where(mask, matA["d"], matB["d"])
    Fbar = np.eye(3) + np.array([[0.04, 0.01, -0.02], [0.015, -0.01, 0.0], [0.0, 0.02, 0.01]])
    FA, FB, a = laminate.laminate_solution(Fbar, axis, 5.0 / 12.0, matA, matB)
    F = mechanics.uniform_field(Fbar, shape)
    Fn, st = mechanics.newton_solve(F, Fbar, c, d, work, work["spacing"], tol_newton=1e-13, tol_lin=1e-14)
    exact = np.where(mask[None, None], FA.reshape(3, 3, 1, 1, 1), FB.reshape(3, 3, 1, 1, 1))
    assert np.max(np.abs(Fn - exact)) <= 1e-12 * np.max(np.abs(exact - F))
    assert np.linalg.norm(a) > 1e-3


def test_inclusion_invariants():
    """<F> = Fbar, Hill-Mandel <P F~^T> = 0, <P> Fbar^T symmetric."""
    work = synth.inclusion_workload(n=12, n_inc=2)
    F, stats = mechanics.solve_increments(work)
    Fbar = work["loads"][-1]
    mean = F.reshape(3, 3, -1).mean(axis=-1)
    assert np.max(np.abs(mean - Fbar)) < 1e-14
    P = cm.stress(F, work["c0"], work["d0"], work["E"], work["nu"], work["Omega"])
    Ft = F - Fbar.reshape(3, 3, 1, 1, 1)
    hm = np.einsum("ijabc,kjabc->ik", P, Ft) / F[0, 0].size
    Pm = P.reshape(3, 3, -1).mean(axis=-1)
    assert np.max(np.abs(hm)) < 1e-9 * np.max(np.abs(Pm)) * np.max(np.abs(Ft))
    tau = Pm @ Fbar.T
    assert np.max(np.abs(tau - tau.T)) < 1e-8 * np.max(np.abs(tau))
    for st in stats:
        assert st["err_history"][-1] <= 1e-8


def test_effective_stiffness_bounds_and_symmetry():
    """Small-strain C_eff of a two-phase RVE: symmetric and between the
    Reuss and Voigt bounds in the energy sense; phi = 0 gives the matrix."""
    work = synth.inclusion_workload(n=8)
    eps = 1e-4
    shape = work["shape"]
    Ceff = np.zeros((6, 6))
    idx = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    plus, minus = synth.six_load_cases(eps), synth.six_load_cases(-eps)
    for k in range(6):
        Pm = []
        for Fbar in (plus[k], minus[k]):
            F = mechanics.uniform_field(Fbar, shape)
            F, _ = mechanics.newton_solve(F, Fbar, work["c0"], work["d0"], work, work["spacing"],
                                          tol_newton=1e-10, tol_lin=1e-12)
            Pm.append(mechanics.mean_stress(F, work["c0"], work["d0"], work))
        for a, (i, j) in enumerate(idx):
            Ceff[a, k] = 0.5 * ((Pm[0] - Pm[1])[i, j] + (Pm[0] - Pm[1])[j, i]) / (2 * eps)
    # the shear cases impose engineering shear strain eps, so Ceff is in
    # Voigt notation with engineering shears (C_44 = G for an isotropic phase)
    assert np.max(np.abs(Ceff - Ceff.T)) < 1e-4 * np.max(np.abs(Ceff))

    def C_iso(E, nu):
        lam = E * nu / ((1 + nu) * (1 - 2 * nu))
        G = E / (2 * (1 + nu))
        C = np.zeros((6, 6))
        C[:3, :3] = lam
        C[np.arange(3), np.arange(3)] += 2 * G
        C[np.arange(3, 6), np.arange(3, 6)] = G
        return C

    Cs = [C_iso(E, nu) for E, nu in zip(work["E"].ravel(), work["nu"].ravel())]
    voigt = np.mean(Cs, axis=0)
    reuss = np.linalg.inv(np.mean([np.linalg.inv(C) for C in Cs], axis=0))
    rng = np.random.default_rng(22)
    for _ in range(20):
        e = rng.standard_normal(6)
        q = e @ Ceff @ e
        assert e @ reuss @ e * (1 - 1e-6) <= q <= e @ voigt @ e * (1 + 1e-6)


def _converged(work, Fbar, tol=1e-13):
    shape = work["shape"]
    F = mechanics.uniform_field(Fbar, shape)
    F, _ = mechanics.newton_solve(F, Fbar, work["c0"], work["d0"], work, work["spacing"], tol_newton=tol,
                                  tol_lin=1e-13)
    return F


def test_homogenized_tangent_matches_finite_differences_and_is_symmetric():
    """d<P>/dFbar : W by one linearised solve equals the central difference
    of <P> between two converged Newton solves at Fbar +- h W, and
    W1 : C_eff : W2 = W2 : C_eff : W1 (major symmetry at equilibrium)."""
    work = small_two_phase(shape=(6, 4, 8), seed=22)
    Fbar = np.eye(3) + np.array([[0.01, 0.002, 0.0], [0.0, -0.004, 0.001], [0.003, 0.0, 0.006]])
    F = _converged(work, Fbar)
    rng = np.random.default_rng(23)
    W1, W2 = rng.standard_normal((3, 3)), rng.standard_normal((3, 3))
    T1, _ = mechanics.homogenized_tangent(F, work["c0"], work["d0"], work, W1)
    T2, _ = mechanics.homogenized_tangent(F, work["c0"], work["d0"], work, W2)
    h = 1e-6
    Pp = mechanics.mean_stress(_converged(work, Fbar + h * W1), work["c0"], work["d0"], work)
    Pm = mechanics.mean_stress(_converged(work, Fbar - h * W1), work["c0"], work["d0"], work)
    fd = (Pp - Pm) / (2 * h)
    assert np.max(np.abs(T1 - fd)) <= 1e-6 * np.max(np.abs(fd))
    assert abs(np.sum(W1 * T2) - np.sum(W2 * T1)) <= 1e-10 * abs(np.sum(W1 * T2))


def test_homogenized_tangent_of_homogeneous_cell_is_local_tangent():
    shape = (4, 6, 4)
    work = synth.homogeneous_workload(shape, 1.0, E=30e9, nu=0.27, Omega=0.02)
    work["c0"] = np.full(shape, 0.4)
    work["d0"] = np.full(shape, 0.1)
    Fbar = np.eye(3) + np.array([[0.02, 0.0, 0.01], [0.0, -0.01, 0.0], [0.005, 0.0, 0.01]])
    F = mechanics.uniform_field(Fbar, shape)
    W = np.arange(9.0).reshape(3, 3) / 10.0
    T, it = mechanics.homogenized_tangent(F, work["c0"], work["d0"], work, W)
    K = cm.tangent(F[:, :, :1, :1, :1], work["c0"][:1, :1, :1], work["d0"][:1, :1, :1], work["E"][:1, :1, :1],
                   work["nu"][:1, :1, :1], work["Omega"][:1, :1, :1])
    ref = (K.reshape(9, 9) @ W.reshape(9)).reshape(3, 3)
    assert it == 0
    assert np.max(np.abs(T - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_mixed_projection_is_symmetric_idempotent():
    shape, sp = (4, 6, 4), (0.3, 0.2, 0.25)
    rng = np.random.default_rng(24)
    mask = np.zeros((3, 3), bool)
    mask[1, 1] = mask[2, 2] = mask[0, 2] = True
    A, B = rng.standard_normal((3, 3) + shape), rng.standard_normal((3, 3) + shape)
    GA = mechanics.project_mixed(A, mask, sp)
    assert np.max(np.abs(mechanics.project_mixed(GA, mask, sp) - GA)) <= 1e-13 * np.max(np.abs(GA))
    assert abs(np.sum(GA * B) - np.sum(A * mechanics.project_mixed(B, mask, sp))) <= 1e-12 * np.sum(np.abs(GA * B))
    # the strain-controlled components keep zero mean
    m = GA.reshape(3, 3, -1).mean(-1)
    assert np.max(np.abs(m[~mask])) <= 1e-14 * np.max(np.abs(GA))


def test_mixed_control_homogeneous_uniaxial_stress_exact():
    """Uniform material, Fbar_11 = 1.01 prescribed, <P>_22 = <P>_33 = 0
    (other components strain-controlled at the identity): the solution is
    the uniform F = diag(1.01, s, s) with P_22(s) = 0 of the Neo-Hookean
    law, from a scalar Newton written here from P = G F + (lam ln J - G) F^-T."""
    shape = (4, 4, 6)
    E, nu = 20e9, 0.3
    work = synth.homogeneous_workload(shape, 1.0, E=E, nu=nu)
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    G = E / (2 * (1 + nu))
    s = 1.0
    for _ in range(60):
        f = G * s + (lam * np.log(1.01 * s * s) - G) / s
        df = G + (2 * lam / s) / s - (lam * np.log(1.01 * s * s) - G) / s ** 2
        s -= f / df
    mask = np.zeros((3, 3), bool)
    mask[1, 1] = mask[2, 2] = True
    Fbar = np.diag([1.01, 1.0, 1.0])
    F, st = mechanics.newton_solve_mixed(mechanics.uniform_field(Fbar, shape), Fbar, mask, np.zeros((3, 3)),
                                         work["c0"], work["d0"], work, work["spacing"], tol_newton=1e-13)
    exact = mechanics.uniform_field(np.diag([1.01, s, s]), shape)
    assert np.max(np.abs(F - exact)) <= 1e-13
    Pm = mechanics.mean_stress(F, work["c0"], work["d0"], work)
    assert abs(Pm[1, 1]) <= 1e-3 and abs(Pm[2, 2]) <= 1e-3  # Pa, against P_11 ~ 2e8


def test_mixed_control_recovers_the_strain_controlled_state():
    """Solve with Fbar* prescribed, record <P>*; then prescribe <P>_22, <P>_33
    = <P>*_22, <P>*_33 with Fbar_22 = Fbar_33 = 1 as the start: the mixed
    solve lands on Fbar* and on the same field."""
    work = small_two_phase(shape=(6, 4, 8), seed=25)
    Fs = np.eye(3) + np.diag([0.008, -0.003, 0.002])
    Fs[0, 1] = 0.001
    F1 = _converged(work, Fs)
    P1 = mechanics.mean_stress(F1, work["c0"], work["d0"], work)
    mask = np.zeros((3, 3), bool)
    mask[1, 1] = mask[2, 2] = True
    F0 = Fs.copy()
    F0[1, 1] = F0[2, 2] = 1.0
    F2, st = mechanics.newton_solve_mixed(mechanics.uniform_field(F0, work["shape"]), F0, mask, P1, work["c0"],
                                          work["d0"], work, work["spacing"], tol_newton=1e-13, tol_lin=1e-13)
    fl = F1 - mechanics.uniform_field(Fs, work["shape"])
    assert np.max(np.abs(F2.reshape(3, 3, -1).mean(-1) - Fs)) <= 1e-12
    assert np.max(np.abs(F2 - F1)) <= 1e-10 * np.max(np.abs(fl))
