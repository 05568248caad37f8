"""Phase-field fracture (Sec. 2.1 eqs. (5)-(8); Sec. 3.2 Fracture problem,
eqs. (32)-(36), Alg. 2 "Phase Field Fracture problem").

Driving force: principal-stress criterion (eq. (8) [SigDrivingForce])
    D_f = < sum_i ( <sigma_i> / sigma_max )^2 - 1 >,
history (eq. (7) [Hist]) H = max over time of the driving force.
PFF equation rearranged (eq. (32)):
    [g_c/l_c + 2H] d - g_c l_c Lap d = 2H,
as a linear map A(d) = b (eqs. (34), (35)) solved by CG with the
constant-coefficient preconditioner (eq. (36))
    P(.) = F^{-1}{ F(.) / (g_c/l_c + 2 Hbar + xi.xi g_c l_c) },
Hbar = mean(H).

Readings of the paper taken here:
* xi.xi is the forward/backward finite-difference symbol
  lambda(q) = sum_j (2/h_j)^2 sin^2(q_j/2) (7-point Laplacian).
* H carries the factor g_c/(2 l_c):  H = max(H_old, g_c/(2 l_c) D_f), which
  makes eq. (6) read  d - l_c^2 Lap d = (1 - d) max D_f.
* sigma is the effective (undegraded) Cauchy stress
      sigma = J^-1 [ G (b/s^2 - I) + lambda ln J_e I ],  b = F F^T,
  for the Neo-Hookean law, and sigma = J^-1 s^-2 F S F^T (the push-forward
  of the undegraded P = s^-2 F S) for the Saint-Venant-Kirchhoff law.
* Alg. 2's printed operator drops the factor d; it is [g_c/l_c + 2H] d.
"""
from __future__ import annotations

import numpy as np

from .constitutive import det_and_inv_transpose, lame, law_of, svk_second_piola, swelling_factors
from .krylov import pcg
from .spectral import irfft3, laplacian_symbol, rfft3


def effective_cauchy(F, c, E, nu, Omega, law="neo_hookean"):
    """Undegraded Cauchy stress, shape (3, 3, ...)."""
    if law == "svk":
        _, s2inv = swelling_factors(c, Omega)
        J, _ = det_and_inv_transpose(F)
        S = svk_second_piola(F, c, E, nu, Omega)
        return s2inv * np.einsum("ik...,kl...,jl...->ij...", F, S, F) / J
    lam, G = lame(E, nu)
    a, s2inv = swelling_factors(c, Omega)
    J, _ = det_and_inv_transpose(F)
    lnJe = np.log(J) - np.log(a)
    b = np.einsum("ik...,jk...->ij...", F, F)
    I = np.eye(3).reshape((3, 3) + (1,) * (F.ndim - 2))
    return (G * s2inv * b + (lam * lnJe - G) * I) / J


def principal_stresses(sigma):
    """Eigenvalues of the symmetric stress (LAPACK eigvalsh), shape (3, ...)."""
    sl = np.moveaxis(sigma, (0, 1), (-2, -1))
    sl = 0.5 * (sl + np.swapaxes(sl, -1, -2))
    ev = np.linalg.eigvalsh(sl)
    return np.moveaxis(ev, -1, 0)


def driving_force(sigma, sigma_max):
    """D_f of eq. (8)."""
    ev = principal_stresses(sigma)
    pos = np.maximum(ev, 0.0)
    return np.maximum(np.sum((pos / sigma_max) ** 2, axis=0) - 1.0, 0.0)


def update_history(H_old, F, c, mat):
    """H <- max(H_old, g_c/(2 l_c) D_f(sigma(F)))."""
    sig = effective_cauchy(F, c, mat["E"], mat["nu"], mat["Omega"], law_of(mat))
    Df = driving_force(sig, mat["sigma_max"])
    return np.maximum(H_old, mat["gc"] / (2.0 * mat["lc"]) * Df)


def pff_operator(d, H, gc, lc, spacing):
    """A(d) of eq. (34), with the Laplacian applied through its symbol."""
    lam = laplacian_symbol(d.shape, spacing)
    return (gc / lc + 2.0 * H) * d + gc * lc * irfft3(lam * rfft3(d), d.shape)


def pff_preconditioner(v, Hbar, gc, lc, spacing):
    """P of eq. (36)."""
    lam = laplacian_symbol(v.shape, spacing)
    return irfft3(rfft3(v) / (gc / lc + 2.0 * Hbar + lam * gc * lc), v.shape)


def pff_solve(H, gc, lc, spacing, tol=1e-10, maxit=10000, fixed_iters=None):
    """Alg. 2: solve A(d) = 2H by preconditioned CG.  Returns (d, iters)."""
    Hbar = float(np.mean(H))
    b = 2.0 * H
    d, it, _ = pcg(lambda x: pff_operator(x, H, gc, lc, spacing),
                   lambda r: pff_preconditioner(r, Hbar, gc, lc, spacing),
                   b, tol, maxit, fixed_iters=fixed_iters)
    return d, it


def plane_crack_profile(n, h, lc, gc, H0):
    """Exact discrete solution of eq. (32) on a periodic line of n voxels when
    H = H0 on voxel 0 and 0 elsewhere (used as a pin):
        d_i = A (rho^|i| + rho^(n-|i|)),  rho + 1/rho = 2 + h^2/l_c^2,
    with A from the balance at i = 0."""
    t = 2.0 + h * h / (lc * lc)
    rho = 0.5 * (t - np.sqrt(t * t - 4.0))
    i = np.arange(n)
    k = np.minimum(i, n - i)
    shape_fun = rho ** k + rho ** (n - k)
    f0, f1 = shape_fun[0], shape_fun[1]
    # (gc/lc + 2 H0) d0 - gc lc (2 d1 - 2 d0)/h^2 = 2 H0
    coef = (gc / lc + 2.0 * H0) * f0 - gc * lc * (2.0 * f1 - 2.0 * f0) / (h * h)
    A = 2.0 * H0 / coef
    return A * shape_fun, rho
