"""Pins of the oracle's Saint-Venant-Kirchhoff law (Sec. 2.1 eqs. (3) [Ee],
(4) [psie0], (11)-(12) [Pderivada, pristine], with the swelling split of
eq. (2) and the degradation g(d) = (1 - d)^2), independent of its formulas:

* P = g dpsi_0/dF: the energy is a quartic polynomial in F at fixed c, so the
  five-point central difference of the energy is exact up to rounding;
  likewise K = dP/dF (P is cubic in F);
* isotropic Hooke's law with the same (E, nu) in the small-strain limit;
* uniaxial stretch without swelling worked by hand: E_11 = (l^2 - 1)/2,
  P_11 = l (lambda + 2G) E_11, P_22 = P_33 = lambda E_11;
* free swelling F = (1 + Omega c)^{1/3} I is stress free;
* frame indifference P(QF) = Q P(F), sigma(QF) = Q sigma(F) Q^T;
* mu_e = d psi_e / dc and its slope by differences in c; dP/dOmega by
  differences in Omega and dP/dlog E = P;
* the exact laminate solution through the FFT Newton solve with this law.
"""
import numpy as np
import pytest

import synth
from oracle import chemistry as ch
from oracle import constitutive as cm
from oracle import fracture, laminate, mechanics


def _fields(rng, n=6, amp=0.15):
    F = np.eye(3)[:, :, None] + amp * rng.standard_normal((3, 3, n))
    c = 0.1 + 0.5 * rng.random(n)
    d = 0.4 * rng.random(n)
    E = 5e9 + 20e9 * rng.random(n)
    nu = 0.1 + 0.3 * rng.random(n)
    Om = 0.3 * rng.random(n)
    return F, c, d, E, nu, Om


def _five_point(f, x, h):
    return (-f(x + 2 * h) + 8 * f(x + h) - 8 * f(x - h) + f(x - 2 * h)) / (12 * h)


def _rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


def test_stress_is_energy_derivative_and_tangent_is_stress_derivative():
    rng = np.random.default_rng(400)
    F, c, d, E, nu, Om = _fields(rng)
    g = (1 - d) ** 2
    P = cm.stress(F, c, d, E, nu, Om, "svk")
    K = cm.tangent(F, c, d, E, nu, Om, "svk")
    h = 1e-3
    for i in range(3):
        for j in range(3):
            def psi(t):
                Fp = F.copy()
                Fp[i, j] += t
                return g * cm.svk_energy(Fp, c, E, nu, Om)

            def Pcol(t):
                Fp = F.copy()
                Fp[i, j] += t
                return cm.stress(Fp, c, d, E, nu, Om, "svk").reshape(9, -1)

            assert np.max(np.abs(_five_point(psi, 0.0, h) - P[i, j])) <= 1e-9 * np.max(np.abs(P))
            assert np.max(np.abs(_five_point(Pcol, 0.0, h) - K[:, 3 * i + j])) <= 1e-9 * np.max(np.abs(K))


def test_hooke_limit():
    rng = np.random.default_rng(401)
    E, nu = np.array([12e9]), np.array([0.27])
    lam, G = cm.lame(E, nu)
    H = rng.standard_normal((3, 3))
    for eps in (1e-4, 1e-6):
        F = (np.eye(3) + eps * H)[:, :, None]
        P = cm.stress(F, np.zeros(1), np.zeros(1), E, nu, np.zeros(1), "svk")[:, :, 0]
        e = 0.5 * (H + H.T)
        hooke = lam[0] * np.trace(e) * np.eye(3) + 2 * G[0] * e
        assert np.max(np.abs(P / eps - hooke)) <= 20 * eps * np.max(np.abs(hooke))


def test_uniaxial_stretch_by_hand():
    E, nu = np.array([15e9]), np.array([0.3])
    lam, G = cm.lame(E, nu)
    for l in (0.8, 1.05, 1.3):
        F = np.diag([l, 1.0, 1.0])[:, :, None]
        P = cm.stress(F, np.zeros(1), np.zeros(1), E, nu, np.zeros(1), "svk")[:, :, 0]
        E11 = 0.5 * (l * l - 1)
        ref = np.diag([l * (lam[0] + 2 * G[0]) * E11, lam[0] * E11, lam[0] * E11])
        assert np.max(np.abs(P - ref)) <= 1e-15 * np.max(np.abs(ref)) * 10


def test_free_swelling_is_stress_free_and_frame_indifference():
    rng = np.random.default_rng(402)
    c = np.array([0.4]) * np.ones(4)
    Om = np.array([0.25, 1.3, 0.05, 0.7])
    F = np.einsum("ij,k->ijk", np.eye(3), (1 + Om * c) ** (1 / 3))
    P = cm.stress(F, c, np.zeros(4), np.full(4, 15e9), np.full(4, 0.3), Om, "svk")
    assert np.max(np.abs(P)) <= 1e-14 * 15e9  # rounding of (1 + Omega c)^{1/3} cubed
    F, c, d, E, nu, Om = _fields(rng)
    Q = _rotation(rng)
    P = cm.stress(F, c, d, E, nu, Om, "svk")
    PQ = cm.stress(np.einsum("ik,kj...->ij...", Q, F), c, d, E, nu, Om, "svk")
    assert np.max(np.abs(PQ - np.einsum("ik,kj...->ij...", Q, P))) <= 1e-13 * np.max(np.abs(P))
    s = fracture.effective_cauchy(F, c, E, nu, Om, "svk")
    sQ = fracture.effective_cauchy(np.einsum("ik,kj...->ij...", Q, F), c, E, nu, Om, "svk")
    assert np.max(np.abs(sQ - np.einsum("ik,kl...,jl->ij...", Q, s, Q))) <= 1e-13 * np.max(np.abs(s))
    assert np.max(np.abs(s - np.swapaxes(s, 0, 1))) <= 1e-13 * np.max(np.abs(s))
    # sigma is the push-forward of the undegraded P: J sigma = P_0 F^T
    J = np.linalg.det(np.moveaxis(F, -1, 0))
    P0 = cm.stress(F, c, np.zeros_like(d), E, nu, Om, "svk")
    assert np.max(np.abs(J * s - np.einsum("ik...,jk...->ij...", P0, F))) <= 1e-13 * np.max(np.abs(P0))


def test_chemical_potential_and_slope_by_differences():
    rng = np.random.default_rng(403)
    shape = (2, 2, 2)
    w = synth.homogeneous_workload(shape, 1.0, E=15e9, Omega=0.3)
    w["law"] = "svk"
    F = mechanics.uniform_field(np.eye(3), shape) + 0.05 * rng.standard_normal((3, 3) + shape)
    c = 0.2 + 0.3 * rng.random(shape)
    d = 0.3 * rng.random(shape)
    g = (1 - d) ** 2
    mu_e = ch.chemical_potential(c, F, d, w) - w["RT"] * np.log(c / (1 - c))
    psi = lambda t: g * cm.svk_energy(F, c + t, w["E"], w["nu"], w["Omega"])
    fd = _five_point(psi, 0.0, 1e-4) / w["c_max"]
    assert np.max(np.abs(mu_e - fd)) <= 1e-8 * np.max(np.abs(fd))
    mue = lambda t: ch.chemical_potential(c + t, F, d, w) - w["RT"] * np.log((c + t) / (1 - c - t))
    slope = ch.elastic_potential_slope(c, F, d, w)
    fd = _five_point(mue, 0.0, 1e-4)
    assert np.max(np.abs(slope - fd)) <= 1e-7 * np.max(np.abs(fd))


def test_parameter_derivatives_by_differences():
    rng = np.random.default_rng(404)
    F, c, d, E, nu, Om = _fields(rng)
    P, dP = cm.stress_param_derivatives(F, c, d, E, nu, Om, "svk")
    fd = _five_point(lambda t: cm.stress(F, c, d, E, nu, Om + t, "svk"), 0.0, 1e-4)
    assert np.max(np.abs(dP - fd)) <= 1e-8 * np.max(np.abs(fd))
    fdE = _five_point(lambda t: cm.stress(F, c, d, E * np.exp(t), nu, Om, "svk"), 0.0, 1e-4)
    assert np.max(np.abs(P - fdE)) <= 1e-8 * np.max(np.abs(P))


@pytest.mark.parametrize("axis", [0, 2])
def test_laminate_exact_svk(axis):
    shape = [8, 8, 8]
    shape[axis] = 12
    shape = tuple(shape)
    work = synth.homogeneous_workload(shape, (1.0, 1.2, 0.9))
    work["law"] = "svk"
    mask = synth.laminate_mask(shape, axis, 5.0 / 12.0)
    matA = dict(E=80e9, nu=0.21, Omega=0.3, c=0.2, d=0.3, law="svk")
    matB = dict(E=9e9, nu=0.34, Omega=0.0, c=0.0, d=0.0, law="svk")
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
    # the laminate with the Neo-Hookean law differs (the law is really used)
    FA2, _, _ = laminate.laminate_solution(Fbar, axis, 5.0 / 12.0, dict(matA, law="neo_hookean"),
                                           dict(matB, law="neo_hookean"))
    assert np.max(np.abs(FA2 - FA)) > 1e-4 * np.max(np.abs(FA - Fbar))
