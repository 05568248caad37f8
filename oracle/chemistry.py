"""Chemical problem (Sec. 2.2 eqs. (13)-(22); Sec. 3.2 Chemical problem,
eqs. (37)-(50); Alg. 3 "Chemical diffusion problem").

Backward-Euler, semi-implicit step (eq. (42) [ChemDTsolve]) with residual
(eq. (43) [Chemresidualfc])
    f(c) = c + dt div[ M(d_t) c_t (1 - c_t) C_t^-1 grad mu(c) ] - dt cdot_B - c_t,
mobility M(d) = -D/RT (0.9 (1-d)^2 + 0.1 d^2) (eq. (20)),
chemical potential mu = mu_c + mu_e, mu_c = RT log(c/(1-c)) (eq. (17)).
Newton from c^0 = c_t, c^{i+1} = c^i + dc (eq. (47)), stopped when
||dc|| / ||c_t|| < tol_chem (eq. (48)).

The operators are applied in Fourier space as in eqs. (49)-(50): grad by the
forward-difference frequencies xi_j = (e^{i q_j} - 1)/h_j, div by the
backward-difference frequencies -conj(xi_j) (their adjoint, so that
div grad is the 7-point Laplacian).

Readings of the paper taken here:
* M(d) literal: the effective diffusivity at d = 0 is 0.9 D.
* mu_e is re-derived from the chosen energy (the printed eq. (18) is
  garbled):  mu_e = dpsi_e/dc = -g Omega / (3 (1 + Omega c))
  [ G (tr C_e - 3) + 3 lambda ln J_e ]  (J/m^3), divided by c_max (mol/m^3)
  to give J/mol before adding to mu_c.  For the Saint-Venant-Kirchhoff law
  (E_e = (s^-2 C - I)/2, dE_e/dc = -Omega/(3a) (2 E_e + I), a = 1 + Omega c):
  mu_e = -g Omega / (3a) [ 2 lambda tr^2 E_e + 4 G E_e:E_e + (3 lambda + 2 G) tr E_e ].
* The Newton linearisation keeps only mu_c (as eq. (45) does):
      dmu_c/dc = w = RT (1/c + 1/(1 - c)),
  and the linear step is solved for dmu = w dc with the SPD operator
      B(dmu) = dmu / w + dt div[ M c_t (1-c_t) C_t^-1 grad dmu ] = -f(c),
  then dc = dmu / w (identical to the dc of the literal Jacobian; pinned on
  tiny grids against a dense solve of eq. (45) in dc form).
* Preconditioner (the paper gives none for this problem): the
  constant-coefficient inverse F^-1[ F(.) / (mean(1/w) + dt abar lambda(q)) ]
  with abar = mean(tr(-M c_t(1-c_t) C_t^-1)) / 3.
* C_t = F^T F of the stored deformation, d_t the stored damage (chemistry is
  solved once per step with the fields of the previous step, Sec. 3.2
  Global problem).

Fully implicit variant (beyond the paper's stated approximation): with
``jacobian="full"`` the Newton linearisation also keeps the elastic part,
d mu/dc = w + d(mu_e / c_max)/dc, so the step converges quadratically; the
equation f(c) = 0 and hence its solution are unchanged.  The staggered
driver can then call the step inside its loop with the current F and d
(staggered.staggered_step(chemistry="coupled")).
"""
from __future__ import annotations

import numpy as np

from .constitutive import DomainError, det_and_inv_transpose, green_lagrange_elastic, lame, law_of, swelling_factors
from .krylov import pcg
from .spectral import forward_difference_symbol, irfft3, laplacian_symbol, rfft3


def chemical_potential(c, F, d, mat):
    """mu(c) = mu_c + mu_e / c_max (J/mol)."""
    if np.any(c <= 0.0) or np.any(c >= 1.0):
        raise DomainError("c outside (0, 1)")
    RT = mat["RT"]
    mu_c = RT * np.log(c / (1.0 - c))
    lam, G = lame(mat["E"], mat["nu"])
    Om = mat["Omega"]
    g = (1.0 - d) ** 2
    a, s2inv = swelling_factors(c, Om)
    if law_of(mat) == "svk":
        t, q = _svk_invariants(F, c, Om)
        mu_e = -g * Om / (3.0 * a) * (2.0 * lam * t * t + 4.0 * G * q + (3.0 * lam + 2.0 * G) * t)
        return mu_c + mu_e / mat["c_max"]
    J, _ = det_and_inv_transpose(F)
    lnJe = np.log(J) - np.log(a)
    trC = np.einsum("ij...,ij...->...", F, F)
    mu_e = -g * Om / (3.0 * a) * (G * (trC * s2inv - 3.0) + 3.0 * lam * lnJe)
    return mu_c + mu_e / mat["c_max"]


def _svk_invariants(F, c, Omega):
    """(tr E_e, E_e : E_e) of the elastic Green-Lagrange strain."""
    Ee = green_lagrange_elastic(F, c, Omega)
    return np.einsum("ii...->...", Ee), np.einsum("ij...,ij...->...", Ee, Ee)


def elastic_potential_slope(c, F, d, mat):
    """d(mu_e / c_max)/dc at fixed F and d (J/mol per unit c), from the
    mu_e above with a = 1 + Omega c:
        d mu_e/dc = g Omega^2 / (3 a^2) [ (5/3) G a^(-2/3) tr C - 3 G
                                           + 3 lambda (ln J_e + 1) ]."""
    lam, G = lame(mat["E"], mat["nu"])
    Om = mat["Omega"]
    g = (1.0 - d) ** 2
    a, s2inv = swelling_factors(c, Om)
    if law_of(mat) == "svk":
        # with t = tr E_e, q = E_e:E_e, T = 2 lambda t^2 + 4 G q + (3 lambda + 2 G) t:
        # d mu_e/dc = g Omega^2 / (3 a^2) [ T + ((4 lambda t + 3 lambda + 2 G)(2 t + 3)
        #                                        + 8 G (2 q + t)) / 3 ]
        t, q = _svk_invariants(F, c, Om)
        T = 2.0 * lam * t * t + 4.0 * G * q + (3.0 * lam + 2.0 * G) * t
        dT = ((4.0 * lam * t + 3.0 * lam + 2.0 * G) * (2.0 * t + 3.0) + 8.0 * G * (2.0 * q + t)) / 3.0
        return g * Om * Om / (3.0 * a * a) * (T + dT) / mat["c_max"]
    J, _ = det_and_inv_transpose(F)
    lnJe = np.log(J) - np.log(a)
    trC = np.einsum("ij...,ij...->...", F, F)
    dmue = g * Om * Om / (3.0 * a * a) * ((5.0 / 3.0) * G * s2inv * trC - 3.0 * G + 3.0 * lam * (lnJe + 1.0))
    return dmue / mat["c_max"]


def mobility(d, D, RT):
    """M(d) of eq. (20) (negative)."""
    return -D / RT * (0.9 * (1.0 - d) ** 2 + 0.1 * d * d)


def flux_coefficient(c_t, F_t, d_t, mat):
    """Q = M(d_t) c_t (1 - c_t) C_t^-1, shape (3, 3, ...) (negative definite)."""
    Fl = np.moveaxis(F_t, (0, 1), (-2, -1))
    C = np.swapaxes(Fl, -1, -2) @ Fl
    Cinv = np.moveaxis(np.linalg.inv(C), (-2, -1), (0, 1))
    return mobility(d_t, mat["D"], mat["RT"]) * c_t * (1.0 - c_t) * Cinv


def grad(v, spacing):
    """Forward-difference gradient via its symbol, shape (3, ...)."""
    xi = forward_difference_symbol(v.shape, spacing)
    vh = rfft3(v)
    return np.stack([irfft3(xi[j] * vh, v.shape) for j in range(3)])


def div(w, spacing):
    """Backward-difference divergence (minus the adjoint of grad)."""
    shape = w.shape[1:]
    xi = forward_difference_symbol(shape, spacing)
    acc = 0.0
    for j in range(3):
        acc = acc - np.conj(xi[j]) * rfft3(w[j])
    return irfft3(acc, shape)


def div_Q_grad(v, Q, spacing):
    """div[ Q grad v ] with a voxel-wise 3x3 coefficient Q."""
    g = grad(v, spacing)
    return div(np.einsum("jk...,k...->j...", Q, g), spacing)


def residual(c, c_t, F_t, d_t, cdot_B, dt, mat, Q=None):
    """f(c) of eq. (43)."""
    if Q is None:
        Q = flux_coefficient(c_t, F_t, d_t, mat)
    mu = chemical_potential(c, F_t, d_t, mat)
    return c + dt * div_Q_grad(mu, Q, mat["spacing"]) - dt * cdot_B - c_t


def potential_slope(c, RT):
    """w = d mu_c / dc = RT (1/c + 1/(1 - c))."""
    return RT * (1.0 / c + 1.0 / (1.0 - c))


def fick_step(c_t, F_t, d_t, cdot_B, dt, mat, tol_chem=1e-8, tol_lin=1e-10,
              max_newton=50, maxit_lin=10000, fixed_lin=None, jacobian="mu_c"):
    """Alg. 3: one backward-Euler step.  Returns (c_{t+dt}, stats).
    jacobian="mu_c": the paper's linearisation (eq. (45)); "full": also
    the elastic part of d mu/dc (see the module docstring)."""
    spacing = mat["spacing"]
    Q = flux_coefficient(c_t, F_t, d_t, mat)
    lam = laplacian_symbol(c_t.shape, spacing)
    abar = float(np.mean(-(Q[0, 0] + Q[1, 1] + Q[2, 2]))) / 3.0
    norm_ct = float(np.sqrt(np.sum(c_t * c_t)))
    c = c_t.copy()
    lin_iters, rel = [], []
    for it in range(max_newton):
        f = residual(c, c_t, F_t, d_t, cdot_B, dt, mat, Q)
        w = potential_slope(c, mat["RT"])
        if jacobian == "full":
            w = w + elastic_potential_slope(c, F_t, d_t, mat)
            if np.any(w <= 0.0):
                raise DomainError("d mu / dc <= 0: the full Jacobian is not SPD")
        winv_mean = float(np.mean(1.0 / w))

        def B(x):
            return x / w + dt * div_Q_grad(x, Q, spacing)

        def M(r):
            return irfft3(rfft3(r) / (winv_mean + dt * abar * lam), r.shape)

        fixed = None if fixed_lin is None else fixed_lin[it]
        dmu, n, _ = pcg(B, M, -f, tol_lin, maxit_lin, fixed_iters=fixed)
        dc = dmu / w
        c = c + dc
        lin_iters.append(n)
        r = float(np.sqrt(np.sum(dc * dc))) / norm_ct
        rel.append(r)
        if r < tol_chem:
            return c, dict(newton_iters=it + 1, lin_iters=lin_iters, dc_history=rel)
    raise RuntimeError("Fick Newton did not converge")


def literal_newton_increment_dense(c, c_t, F_t, d_t, cdot_B, dt, mat):
    """One Newton increment dc of eq. (46) with the Jacobian of eq. (45)
    assembled as a dense (non-symmetric) matrix in dc form and solved by LU.
    Tiny grids only (pins the dmu-form PCG)."""
    shape = c.shape
    n = c.size
    Q = flux_coefficient(c_t, F_t, d_t, mat)
    w = potential_slope(c, mat["RT"])
    f = residual(c, c_t, F_t, d_t, cdot_B, dt, mat, Q)
    Jm = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        e = e.reshape(shape)
        Jm[:, k] = (e + dt * div_Q_grad(w * e, Q, mat["spacing"])).ravel()
    return np.linalg.solve(Jm, -f.ravel()).reshape(shape)
