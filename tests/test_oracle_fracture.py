"""Pins of oracle/fracture.py: uniform-H closed form, exact 1-D plane-crack
profile and its exp(-|x|/l_c) limit, driving-force special cases."""
import numpy as np
import pytest

from oracle import fracture, spectral


def test_uniform_history_closed_form_one_iteration():
    shape, sp = (8, 6, 4), (0.1, 0.1, 0.2)
    gc, lc = 1.3, 0.2
    H = np.full(shape, 7.5)
    d, it = fracture.pff_solve(H, gc, lc, sp, tol=1e-12)
    exact = 2 * 7.5 / (gc / lc + 2 * 7.5)
    assert np.max(np.abs(d - exact)) < 1e-14
    assert it == 1


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_plane_crack_profile(axis):
    n = 64
    shape = [4, 4, 4]
    shape[axis] = n
    h = 0.05
    sp = (h, h, h)
    gc, lc, H0 = 2.0, 2 * h, 40.0
    H = np.zeros(shape)
    sl = [slice(None)] * 3
    sl[axis] = 0
    H[tuple(sl)] = H0
    d, _ = fracture.pff_solve(H, gc, lc, sp, tol=1e-14)
    prof, rho = fracture.plane_crack_profile(n, h, lc, gc, H0)
    line = np.moveaxis(d, axis, 0)[:, 1, 2]
    assert np.max(np.abs(line - prof)) < 1e-12 * prof.max()
    assert np.all(d >= 0) and np.all(d < 1)
    # the discrete decay rate tends to exp(-h/l_c) as h/l_c -> 0
    assert abs(rho - 0.6096117967977924) < 1e-12  # l_c = 2h: rho + 1/rho = 2.25
    for ratio in (8, 32, 128):
        t = 2.0 + 1.0 / ratio ** 2
        r = 0.5 * (t - np.sqrt(t * t - 4))
        assert abs(np.log(r) * ratio + 1) < 1.0 / ratio ** 2


def test_operator_stencil_form():
    shape, sp = (6, 8, 4), (0.3, 0.2, 0.25)
    rng = np.random.default_rng(30)
    d = rng.random(shape)
    H = rng.random(shape)
    gc, lc = 1.1, 0.4
    A = fracture.pff_operator(d, H, gc, lc, sp)
    lap = np.zeros(shape)
    for ax in range(3):
        lap += (np.roll(d, 1, ax) + np.roll(d, -1, ax) - 2 * d) / sp[ax] ** 2
    ref = (gc / lc + 2 * H) * d - gc * lc * lap
    assert np.max(np.abs(A - ref)) < 1e-12 * np.abs(ref).max()


def _rot(seed):
    Q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    return Q


def test_driving_force_cases():
    smax = 10.0
    # hydrostatic compression: no driving force
    sig = -5.0 * np.eye(3)
    assert fracture.driving_force(sig.reshape(3, 3, 1), smax)[0] == 0.0
    # uniaxial tension above threshold in a rotated frame
    Q = _rot(31)
    sig = Q @ np.diag([25.0, 0.0, -3.0]) @ Q.T
    Df = fracture.driving_force(sig.reshape(3, 3, 1), smax)[0]
    assert abs(Df - ((25.0 / smax) ** 2 - 1.0)) < 1e-12
    # below threshold
    sig = Q @ np.diag([5.0, 4.0, 3.0]) @ Q.T
    assert fracture.driving_force(sig.reshape(3, 3, 1), smax)[0] == 0.0
    # three positive principal stresses: sum of squares = Frobenius norm^2
    sig = Q @ np.diag([15.0, 12.0, 9.0]) @ Q.T
    Df = fracture.driving_force(sig.reshape(3, 3, 1), smax)[0]
    assert abs(Df - (np.sum(sig * sig) / smax ** 2 - 1)) < 1e-12


def test_effective_cauchy_limits():
    F = (1 + 0.03 * 0.2) ** (1 / 3) * np.eye(3)
    s = fracture.effective_cauchy(F.reshape(3, 3, 1), np.array([0.2]), np.array([10e9]),
                                  np.array([0.3]), np.array([0.03]))
    assert np.max(np.abs(s)) < 1e-3
    eps = 1e-7
    F = np.eye(3)
    F[0, 0] += eps
    s = fracture.effective_cauchy(F.reshape(3, 3, 1), np.array([0.0]), np.array([10e9]),
                                  np.array([0.3]), np.array([0.0]))[:, :, 0]
    E, nu = 10e9, 0.3
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    G = E / (2 * (1 + nu))
    assert abs(s[0, 0] / eps - (lam + 2 * G)) < 1e-5 * (lam + 2 * G)
    assert abs(s[1, 1] / eps - lam) < 1e-5 * (lam + 2 * G)


def test_effective_cauchy_is_push_forward_of_undegraded_stress():
    """sigma = J^-1 (P / g) F^T (the Cauchy stress of the undegraded law,
    reading A6 of eq. (8)), with P from the pinned constitutive stress, at
    random finite F (J far from 1), concentration, swelling and damage; the
    result is symmetric and objective: sigma(Q F) = Q sigma(F) Q^T."""
    from oracle import constitutive as cm

    rng = np.random.default_rng(3111)
    n = 40
    F = np.eye(3)[:, :, None] + 0.25 * rng.standard_normal((3, 3, n))
    J = np.linalg.det(np.moveaxis(F, 2, 0))
    F[:, :, J < 0.2] = np.eye(3)[:, :, None] * 1.3  # keep det F well positive
    c = rng.uniform(0.0, 0.9, n)
    Om = rng.uniform(0.0, 1.3, n)
    E = rng.uniform(5e9, 2e11, n)
    nu = rng.uniform(0.1, 0.45, n)
    d = rng.uniform(0.0, 0.9, n)
    sig = fracture.effective_cauchy(F, c, E, nu, Om)
    P = cm.stress(F, c, d, E, nu, Om)
    J = np.linalg.det(np.moveaxis(F, 2, 0))
    ref = np.einsum("ik...,jk...->ij...", P / (1 - d) ** 2, F) / J
    scale = np.max(np.abs(ref), axis=(0, 1))
    assert np.max(np.abs(sig - ref) / scale) <= 1e-12
    assert np.max(np.abs(sig - np.swapaxes(sig, 0, 1)) / scale) <= 1e-12
    Q = _rot(3112)
    sigQ = fracture.effective_cauchy(np.einsum("ik,kj...->ij...", Q, F), c, E, nu, Om)
    rotated = np.einsum("ik,kl...,jl->ij...", Q, sig, Q)
    assert np.max(np.abs(sigQ - rotated) / scale) <= 1e-12
