"""Pins of oracle/chemistry.py: uniform update, mass identity (eq. (25)),
single Fourier mode decay, the dmu-form PCG against a dense solve of the
literal dc Jacobian, mu_e against a finite difference of the energy."""
import numpy as np

import synth
from oracle import chemistry as ch
from oracle import spectral
from oracle.mechanics import uniform_field


def chem_work(shape=(8, 8, 8), length=1e-6, Omega=0.0, D=1e-14):
    w = synth.homogeneous_workload(shape, length, E=15e9, nu=0.3, Omega=Omega, D=D)
    return w


def test_uniform_concentration_and_source():
    w = chem_work()
    shape = w["shape"]
    c = np.full(shape, 0.2)
    cdot = np.full(shape, 3e-3)
    F = uniform_field(np.eye(3), shape)
    c1, st = ch.fick_step(c, F, w["d0"], cdot, 2.0, w)
    assert np.max(np.abs(c1 - (0.2 + 2.0 * 3e-3))) < 1e-15
    assert st["newton_iters"] >= 1


def test_mass_identity_heterogeneous():
    w = chem_work(Omega=0.0)
    shape = w["shape"]
    rng = np.random.default_rng(40)
    w["D"] = np.where(rng.random(shape) < 0.5, 1e-14, 1e-16)
    c = 0.05 + 0.3 * rng.random(shape)
    cdot = np.where(rng.random(shape) < 0.2, 4e-3, 0.0)
    F = uniform_field(np.eye(3), shape) + 0.01 * rng.standard_normal((3, 3) + shape)
    d = 0.3 * rng.random(shape)
    c1, st = ch.fick_step(c, F, d, cdot, 5.0, w)
    assert abs(c1.sum() - c.sum() - 5.0 * cdot.sum()) < 1e-10 * c.sum()


def test_single_mode_decay():
    """c = c0 + a sin(2 pi m x/L): per-step amplitude factor
    1/(1 + dt 0.9 D lambda(q)).  The nonlinearity of mu_c only feeds the
    second harmonic, so the error in the first mode is O(a^2): it drops by
    4 when a halves."""
    n = 16
    w = chem_work(shape=(n, 4, 4), length=(1e-6, 0.25e-6, 0.25e-6), D=1e-14)
    shape, sp = w["shape"], w["spacing"]
    x = (np.arange(n) + 0.5) / n
    c0, m, dt = 0.3, 2, 0.5
    q = 2 * np.pi * m / n
    lam = (2 / sp[0]) ** 2 * np.sin(q / 2) ** 2
    factor = 1.0 / (1.0 + dt * 0.9 * 1e-14 * lam)
    errs = []
    for a in (1e-3, 5e-4):
        c = c0 + a * np.sin(2 * np.pi * m * x)[:, None, None] * np.ones(shape)
        F = uniform_field(np.eye(3), shape)
        c1, _ = ch.fick_step(c, F, w["d0"], np.zeros(shape), dt, w, tol_chem=1e-13, tol_lin=1e-14)
        amp = 2 * np.mean((c1[:, 0, 0] - c0) * np.sin(2 * np.pi * m * x))
        errs.append(abs(amp / a - factor))
    assert errs[0] < 1e-5 * factor
    assert 3.6 < errs[0] / errs[1] < 4.4


def test_dmu_form_equals_literal_dc_jacobian():
    w = chem_work(shape=(4, 4, 4), Omega=0.05)
    shape = w["shape"]
    rng = np.random.default_rng(41)
    w["D"] = 1e-14 * (0.5 + rng.random(shape))
    c_t = 0.1 + 0.5 * rng.random(shape)
    F = uniform_field(np.eye(3), shape) + 0.02 * rng.standard_normal((3, 3) + shape)
    d = 0.4 * rng.random(shape)
    cdot = 1e-3 * rng.random(shape)
    dt = 20.0
    dc_dense = ch.literal_newton_increment_dense(c_t, c_t, F, d, cdot, dt, w)
    # first Newton increment of the PCG dmu form
    Q = ch.flux_coefficient(c_t, F, d, w)
    f = ch.residual(c_t, c_t, F, d, cdot, dt, w, Q)
    wv = ch.potential_slope(c_t, w["RT"])
    from oracle.krylov import pcg
    lam = spectral.laplacian_symbol(shape, w["spacing"])
    dmu, it, _ = pcg(lambda x: x / wv + dt * ch.div_Q_grad(x, Q, w["spacing"]),
                     lambda r: r, -f, 1e-14, 2000)
    assert np.max(np.abs(dmu / wv - dc_dense)) < 1e-10 * np.max(np.abs(dc_dense))


def test_elastic_potential_is_energy_derivative():
    """mu_e * c_max = d psi_e / d c at fixed F (FD of the energy written out)."""
    rng = np.random.default_rng(42)
    E, nu, Om, dmg = 15e9, 0.3, 0.06, 0.2
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    G = E / (2 * (1 + nu))

    def psi_e(F, c):
        Fe = F / (1 + Om * c) ** (1 / 3)
        lnJ = np.log(np.linalg.det(Fe))
        return (1 - dmg) ** 2 * (G / 2 * (np.trace(Fe.T @ Fe) - 3) - G * lnJ + lam / 2 * lnJ ** 2)

    F = np.eye(3) + 0.05 * rng.standard_normal((3, 3))
    c = 0.4
    w = dict(RT=2000.0, E=np.array([E]), nu=np.array([nu]), Omega=np.array([Om]), c_max=3e4)
    mu = ch.chemical_potential(np.array([c]), F.reshape(3, 3, 1), np.array([dmg]), w)[0]
    mu_c = 2000.0 * np.log(c / (1 - c))
    h = 1e-6
    fd = (psi_e(F, c + h) - psi_e(F, c - h)) / (2 * h)
    assert abs((mu - mu_c) * 3e4 - fd) < 1e-6 * abs(fd)


def test_div_grad_is_minus_seven_point_laplacian():
    shape, sp = (6, 4, 8), (0.2, 0.3, 0.1)
    rng = np.random.default_rng(43)
    v = rng.standard_normal(shape)
    I = np.broadcast_to(np.eye(3).reshape(3, 3, 1, 1, 1), (3, 3) + shape)
    lhs = ch.div_Q_grad(v, I, sp)
    lap = np.zeros(shape)
    for ax in range(3):
        lap += (np.roll(v, 1, ax) + np.roll(v, -1, ax) - 2 * v) / sp[ax] ** 2
    assert np.max(np.abs(lhs - lap)) < 1e-12 * np.abs(lap).max()


def test_elastic_potential_slope_is_derivative_of_mu_e():
    """d(mu_e / c_max)/dc of the fully implicit Jacobian against a central
    difference of mu - mu_c in c, at random finite F, damage and swelling
    coefficients up to the plate's 1.3."""
    rng = np.random.default_rng(44)
    n = 30
    F = np.eye(3)[:, :, None] + 0.08 * rng.standard_normal((3, 3, n))
    c = rng.uniform(0.05, 0.9, n)
    d = rng.uniform(0.0, 0.8, n)
    w = dict(RT=2478.0, E=rng.uniform(5e9, 3e10, n), nu=rng.uniform(0.2, 0.4, n), Omega=rng.uniform(0.0, 1.3, n),
             c_max=3e4)
    h = 1e-6
    mue = lambda cc: ch.chemical_potential(cc, F, d, w) - w["RT"] * np.log(cc / (1 - cc))
    fd = (mue(c + h) - mue(c - h)) / (2 * h)
    slope = ch.elastic_potential_slope(c, F, d, w)
    assert np.max(np.abs(slope - fd) / (np.abs(fd) + 1e-3 * np.max(np.abs(fd)))) < 1e-6


def test_full_jacobian_newton_increment_is_dense_fd_newton_step():
    """The first increment of the fully implicit Newton step (the dmu-form
    PCG with d mu/dc including the elastic part) equals the Newton step of
    the residual of eq. (43) with its Jacobian assembled densely by central
    differences of that residual (4^3 grid, strong swelling coupling)."""
    w = chem_work(shape=(4, 4, 4), Omega=1.3)
    shape = w["shape"]
    rng = np.random.default_rng(45)
    w["D"] = 1e-14 * (0.5 + rng.random(shape))
    c_t = 0.1 + 0.5 * rng.random(shape)
    F = uniform_field(np.eye(3), shape) + 0.02 * rng.standard_normal((3, 3) + shape)
    d = 0.3 * rng.random(shape)
    cdot = 1e-3 * rng.random(shape)
    dt = 20.0
    c1, st = ch.fick_step(c_t, F, d, cdot, dt, w, tol_chem=1e30, tol_lin=1e-14, jacobian="full")
    assert st["newton_iters"] == 1
    n = c_t.size
    f0 = ch.residual(c_t, c_t, F, d, cdot, dt, w)
    J = np.empty((n, n))
    eps = 1e-7
    for k in range(n):
        e = np.zeros(n)
        e[k] = eps
        e = e.reshape(shape)
        J[:, k] = ((ch.residual(c_t + e, c_t, F, d, cdot, dt, w) - ch.residual(c_t - e, c_t, F, d, cdot, dt, w))
                   / (2 * eps)).ravel()
    dc = np.linalg.solve(J, -f0.ravel()).reshape(shape)
    assert np.max(np.abs((c1 - c_t) - dc)) < 1e-6 * np.max(np.abs(dc))


def test_full_jacobian_same_solution_quadratic_convergence():
    """Both linearisations solve the same equation f(c) = 0: the fully
    implicit step lands on the same concentration, in fewer Newton
    iterations, with quadratic contraction of the increments (swelling
    coefficient 0.1 at a deformation near the free swelling of c = 0.35;
    measured 5 Newton iterations against 26)."""
    w = chem_work(shape=(8, 8, 8), Omega=0.1)
    shape = w["shape"]
    rng = np.random.default_rng(46)
    c_t = 0.2 + 0.3 * rng.random(shape)
    F = uniform_field(np.eye(3), shape) * (1 + 0.1 * 0.35) ** (1 / 3) + 0.01 * rng.standard_normal((3, 3) + shape)
    d = 0.2 * rng.random(shape)
    cdot = np.where(rng.random(shape) < 0.2, 4e-3, 0.0)
    ca, sa = ch.fick_step(c_t, F, d, cdot, 20.0, w, tol_chem=1e-12, tol_lin=1e-13)
    cb, sb = ch.fick_step(c_t, F, d, cdot, 20.0, w, tol_chem=1e-12, tol_lin=1e-13, jacobian="full")
    assert np.max(np.abs(ca - cb)) < 1e-11
    assert sb["newton_iters"] < sa["newton_iters"]
    h = sb["dc_history"]
    assert all(h[k + 1] <= 10.0 * h[k] ** 2 / h[0] for k in range(len(h) - 1) if h[k] > 1e-9)
