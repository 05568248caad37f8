"""Pointwise constitutive law (Sec. 2 and Sec. 2.1).

Kinematics: F = F_e F_c (eq. (1)), F_c = (1 + Omega c)^{1/3} I (eq. (2)).
Damage degrades the elastic energy by g(d) = (1 - d)^2 (eq. (9)) and
P = dpsi_e/dF (eq. (11)), P(F, c, d) = (1 - d)^2 P_0(F_e) (eq. (27)).

Readings of the paper taken here:
* The hyperelastic law is the compressible Neo-Hookean energy
      psi_0(F_e) = G/2 (tr C_e - 3) - G ln J_e + lambda/2 (ln J_e)^2,
  C_e = F_e^T F_e, J_e = det F_e, with Lame constants (lambda, G) from
  (E, nu).  It linearises to isotropic Hooke's law with the same E, nu.
* The energy is per reference volume, psi(F) = g psi_0(F / s) with
  s = (1 + Omega c)^{1/3}, so by the chain rule
      P = g [ G s^-2 F + (lambda ln J_e - G) F^-T ],
      ln J_e = ln det F - ln(1 + Omega c),
  and the tangent K = dP/dF is, with A = F^-T,
      K_ijkl = g [ G s^-2 d_ik d_jl + lambda A_ij A_kl
                   + (G - lambda ln J_e) A_il A_kj ].
  (Derivation: d(F^-T)_ij / dF_kl = -A_il A_kj and d ln J / dF_kl = A_kl.)

The paper's own law, Saint-Venant-Kirchhoff (Sec. 2.1 eqs. (3) [Ee], (4)
[psie0], (12) [pristine]), is the second law here (law="svk"):
      E_e = (F_e^T F_e - I) / 2 = (s^-2 C - I) / 2,   C = F^T F,
      psi_0 = lambda/2 tr^2 E_e + G tr(E_e^2),   S = lambda tr E_e I + 2 G E_e,
and with the same energy-per-reference-volume reading psi(F) = g psi_0(F/s):
      P = g s^-2 F S,
  which is eq. (12) exactly when Omega c = 0.  Its tangent, from
  dE_e = s^-2 sym(F^T dF):
      K : X = g s^-2 [ X S + s^-2 F (lambda tr(F^T X) I + 2 G sym(F^T X)) ],
      K_ijkl = g s^-2 [ d_ik S_lj + s^-2 (lambda F_ij F_kl + G (F F^T)_ik d_jl
                                          + G F_il F_kj) ].
Every function taking a law accepts "neo_hookean" (the default) or "svk".

Tensors are stored with the two tensor indices first: F has shape
(3, 3, N0, N1, N2) and F[i, j] = F_ij.  K is returned as a 9 x 9 matrix per
voxel, K[3i+j, 3k+l] = K_ijkl.
"""
from __future__ import annotations

import numpy as np


class DomainError(ValueError):
    """det F <= 0, or a logarithm of a non-positive argument."""


def lame(E, nu):
    """Lame constants (lambda, G) from Young's modulus and Poisson ratio."""
    G = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return lam, G


def _to_last(T):
    return np.moveaxis(T, (0, 1), (-2, -1))


def _to_first(T):
    return np.moveaxis(T, (-2, -1), (0, 1))


def det_and_inv_transpose(F):
    """det F and F^-T by LAPACK (numpy.linalg), F of shape (3, 3, ...)."""
    Fl = _to_last(F)
    J = np.linalg.det(Fl)
    if np.any(J <= 0.0):
        raise DomainError("det F <= 0")
    Finv = np.linalg.inv(Fl)
    return J, _to_first(np.swapaxes(Finv, -1, -2))


def swelling_factors(c, Omega):
    """(1 + Omega c), s^-2 = (1 + Omega c)^{-2/3}."""
    a = 1.0 + Omega * c
    if np.any(a <= 0.0):
        raise DomainError("1 + Omega c <= 0")
    return a, a ** (-2.0 / 3.0)


LAWS = ("neo_hookean", "svk")


def law_of(mat):
    """The law named by a material dict (key "law", default Neo-Hookean)."""
    law = mat.get("law", "neo_hookean") if hasattr(mat, "get") else "neo_hookean"
    if law not in LAWS:
        raise ValueError(f"unknown law {law!r}")
    return law


def green_lagrange_elastic(F, c, Omega):
    """E_e = (s^-2 F^T F - I) / 2 (eq. (3) with F_e = F / s), shape (3, 3, ...)."""
    _, s2inv = swelling_factors(c, Omega)
    C = np.einsum("ki...,kj...->ij...", F, F)
    I = np.eye(3).reshape((3, 3) + (1,) * (F.ndim - 2))
    return 0.5 * (s2inv * C - I)


def svk_energy(F, c, E, nu, Omega):
    """Undegraded SVK energy psi_0(F_e) = lambda/2 tr^2 E_e + G tr(E_e^2) (eq. (4))."""
    lam, G = lame(E, nu)
    Ee = green_lagrange_elastic(F, c, Omega)
    tr = np.einsum("ii...->...", Ee)
    return 0.5 * lam * tr * tr + G * np.einsum("ij...,ji...->...", Ee, Ee)


def svk_second_piola(F, c, E, nu, Omega):
    """S = lambda tr E_e I + 2 G E_e (the bracket of eq. (12))."""
    lam, G = lame(E, nu)
    Ee = green_lagrange_elastic(F, c, Omega)
    tr = np.einsum("ii...->...", Ee)
    I = np.eye(3).reshape((3, 3) + (1,) * (F.ndim - 2))
    return lam * tr * I + 2.0 * G * Ee


def stress(F, c, d, E, nu, Omega, law="neo_hookean"):
    """First Piola-Kirchhoff stress P (eq. (27) with the A1/A2 reading; with
    law="svk", eqs. (11)-(12) with the swelling of eq. (2))."""
    g = (1.0 - d) ** 2
    if law == "svk":
        _, s2inv = swelling_factors(c, Omega)
        S = svk_second_piola(F, c, E, nu, Omega)
        return g * s2inv * np.einsum("ik...,kj...->ij...", F, S)
    lam, G = lame(E, nu)
    a, s2inv = swelling_factors(c, Omega)
    J, A = det_and_inv_transpose(F)
    lnJe = np.log(J) - np.log(a)
    return g * (G * s2inv * F + (lam * lnJe - G) * A)


def tangent(F, c, d, E, nu, Omega, law="neo_hookean"):
    """Tangent K = dP/dF (eq. (30), the K under it) as a 9x9 matrix per voxel,
    shape (9, 9, N0, N1, N2)."""
    if law == "svk":
        return _svk_tangent(F, c, d, E, nu, Omega)
    lam, G = lame(E, nu)
    g = (1.0 - d) ** 2
    a, s2inv = swelling_factors(c, Omega)
    J, A = det_and_inv_transpose(F)
    lnJe = np.log(J) - np.log(a)
    I = np.eye(3)
    extra = F.shape[2:]
    K = (
        np.einsum("ik,jl->ijkl", I, I).reshape((3, 3, 3, 3) + (1,) * len(extra))
        * (g * G * s2inv)
        + np.einsum("ij...,kl...->ijkl...", A, A) * (g * lam)
        + np.einsum("il...,kj...->ijkl...", A, A) * (g * (G - lam * lnJe))
    )
    return K.reshape((9, 9) + extra)


def _svk_tangent(F, c, d, E, nu, Omega):
    lam, G = lame(E, nu)
    g = (1.0 - d) ** 2
    _, s2inv = swelling_factors(c, Omega)
    S = svk_second_piola(F, c, E, nu, Omega)
    I = np.eye(3)
    extra = F.shape[2:]
    FFt = np.einsum("im...,km...->ik...", F, F)
    K = (
        np.einsum("ik,lj...->ijkl...", I, S)
        + s2inv * (
            lam * np.einsum("ij...,kl...->ijkl...", F, F)
            + G * np.einsum("ik...,jl->ijkl...", FFt, I)
            + G * np.einsum("il...,kj...->ijkl...", F, F)
        )
    ) * (g * s2inv)
    return K.reshape((9, 9) + extra)


def apply_tangent(K, X):
    """(K : X)_ij = K_ijkl X_kl with K as (9, 9, ...) and X as (3, 3, ...)."""
    extra = X.shape[2:]
    Y = np.einsum("ab...,b...->a...", K, X.reshape((9,) + extra))
    return Y.reshape((3, 3) + extra)


def stress_param_derivatives(F, c, d, E, nu, Omega, law="neo_hookean"):
    """dP/d(log E) and dP/dOmega at fixed F (used by the adjoint).

    Both Lame constants are proportional to E, and P is linear in them, so
    dP/dlogE = P.  With s^-2 = (1+Omega c)^{-2/3} and
    ln J_e = ln J - ln(1 + Omega c):
        dP/dOmega = g [ -(2/3) G c (1+Omega c)^{-5/3} F
                        - lambda c / (1 + Omega c) F^-T ].
    """
    if law == "svk":
        # with a = 1 + Omega c: d(s^-2)/dOmega = -(2c / 3a) s^-2 and
        # dE_e/dOmega = -(c / 3a)(2 E_e + I), so
        # dP/dOmega = g s^-2 F [ -(2c / 3a) S + lambda tr(dE) I + 2 G dE ]
        lam, G = lame(E, nu)
        g = (1.0 - d) ** 2
        a, s2inv = swelling_factors(c, Omega)
        Ee = green_lagrange_elastic(F, c, Omega)
        S = svk_second_piola(F, c, E, nu, Omega)
        I = np.eye(3).reshape((3, 3) + (1,) * (F.ndim - 2))
        dE = -(c / (3.0 * a)) * (2.0 * Ee + I)
        dS = lam * np.einsum("ii...->...", dE) * I + 2.0 * G * dE
        inner = -(2.0 * c / (3.0 * a)) * S + dS
        P = stress(F, c, d, E, nu, Omega, law)
        return P, g * s2inv * np.einsum("ik...,kj...->ij...", F, inner)
    lam, G = lame(E, nu)
    g = (1.0 - d) ** 2
    a, s2inv = swelling_factors(c, Omega)
    J, A = det_and_inv_transpose(F)
    P = stress(F, c, d, E, nu, Omega)
    dP_dOm = g * (-(2.0 / 3.0) * G * c * a ** (-5.0 / 3.0) * F - lam * c / a * A)
    return P, dP_dOm
