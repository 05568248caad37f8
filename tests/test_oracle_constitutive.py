"""Pins of oracle/constitutive.py: P = dpsi/dF and K = dP/dF by finite
differences of an energy written out here from its definition, Hooke limit,
stress-free swelling, degradation, objectivity."""
import numpy as np

from oracle import constitutive as cm


def energy(F, c, d, E, nu, Om):
    """psi = (1-d)^2 psi_0(F / (1 + Om c)^{1/3}), compressible Neo-Hookean."""
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    G = E / (2 * (1 + nu))
    Fe = F / (1 + Om * c) ** (1.0 / 3.0)
    Ce = Fe.T @ Fe
    lnJ = np.log(np.linalg.det(Fe))
    return (1 - d) ** 2 * (G / 2 * (np.trace(Ce) - 3) - G * lnJ + lam / 2 * lnJ ** 2)


def one(x):
    return np.asarray([x], dtype=np.float64)


def P_of(F, c, d, E, nu, Om):
    return cm.stress(F.reshape(3, 3, 1), one(c), one(d), one(E), one(nu), one(Om))[:, :, 0]


def K_of(F, c, d, E, nu, Om):
    return cm.tangent(F.reshape(3, 3, 1), one(c), one(d), one(E), one(nu), one(Om))[:, :, 0]


def rand_F(rng, amp=0.2):
    return np.eye(3) + amp * rng.standard_normal((3, 3))


PARAMS = dict(c=0.37, d=0.21, E=12e9, nu=0.27, Om=0.08)


def test_stress_is_energy_derivative():
    rng = np.random.default_rng(10)
    for _ in range(5):
        F = rand_F(rng)
        P = P_of(F, **PARAMS)
        h = 1e-6
        Pfd = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                Fp, Fm = F.copy(), F.copy()
                Fp[i, j] += h
                Fm[i, j] -= h
                Pfd[i, j] = (energy(Fp, **PARAMS) - energy(Fm, **PARAMS)) / (2 * h)
        assert np.max(np.abs(P - Pfd)) <= 1e-7 * np.max(np.abs(P))


def test_tangent_is_stress_derivative_and_major_symmetric():
    rng = np.random.default_rng(11)
    for _ in range(5):
        F = rand_F(rng)
        K = K_of(F, **PARAMS)
        h = 1e-6
        Kfd = np.zeros((9, 9))
        for k in range(3):
            for l in range(3):
                Fp, Fm = F.copy(), F.copy()
                Fp[k, l] += h
                Fm[k, l] -= h
                Kfd[:, 3 * k + l] = ((P_of(Fp, **PARAMS) - P_of(Fm, **PARAMS)) / (2 * h)).ravel()
        assert np.max(np.abs(K - Kfd)) <= 1e-7 * np.max(np.abs(K))
        assert np.max(np.abs(K - K.T)) <= 1e-12 * np.max(np.abs(K))


def test_hooke_limit():
    E, nu = 10e9, 0.3
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    G = E / (2 * (1 + nu))
    K = K_of(np.eye(3), 0.0, 0.0, E, nu, 0.0).reshape(3, 3, 3, 3)
    I = np.eye(3)
    C = lam * np.einsum("ij,kl->ijkl", I, I) + G * (np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I))
    assert np.max(np.abs(K - C)) <= 1e-6
    assert np.max(np.abs(P_of(np.eye(3), 0.0, 0.0, E, nu, 0.0))) == 0.0


def test_free_swelling_is_stress_free_and_degradation_scales():
    c, Om = 0.4, 0.05
    s = (1 + Om * c) ** (1.0 / 3.0)
    P = P_of(s * np.eye(3), c, 0.0, 10e9, 0.3, Om)
    assert np.max(np.abs(P)) < 1e-6 * 10e9 * 1e-9 + 1e-3
    rng = np.random.default_rng(12)
    F = rand_F(rng)
    P0 = P_of(F, 0.3, 0.0, 10e9, 0.3, 0.02)
    P1 = P_of(F, 0.3, 0.4, 10e9, 0.3, 0.02)
    assert np.allclose(P1, 0.36 * P0, rtol=1e-14, atol=0)


def test_objectivity():
    rng = np.random.default_rng(13)
    F = rand_F(rng)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    P = P_of(F, **PARAMS)
    PQ = P_of(Q @ F, **PARAMS)
    assert np.max(np.abs(PQ - Q @ P)) < 1e-12 * np.max(np.abs(P))


def test_parameter_derivatives_fd():
    rng = np.random.default_rng(14)
    F = rand_F(rng)
    p = dict(PARAMS)
    P, dOm = cm.stress_param_derivatives(F.reshape(3, 3, 1), one(p["c"]), one(p["d"]),
                                         one(p["E"]), one(p["nu"]), one(p["Om"]))
    h = 1e-7
    Pp = P_of(F, p["c"], p["d"], p["E"], p["nu"], p["Om"] + h)
    Pm = P_of(F, p["c"], p["d"], p["E"], p["nu"], p["Om"] - h)
    assert np.max(np.abs(dOm[:, :, 0] - (Pp - Pm) / (2 * h))) < 1e-6 * np.max(np.abs(dOm))
    Ep = P_of(F, p["c"], p["d"], p["E"] * np.exp(h), p["nu"], p["Om"])
    Em = P_of(F, p["c"], p["d"], p["E"] * np.exp(-h), p["nu"], p["Om"])
    assert np.max(np.abs(P[:, :, 0] - (Ep - Em) / (2 * h))) < 1e-6 * np.max(np.abs(P))
