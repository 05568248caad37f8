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


def stress(F, c, d, E, nu, Omega):
    """First Piola-Kirchhoff stress P (eq. (27) with the A1/A2 reading)."""
    lam, G = lame(E, nu)
    g = (1.0 - d) ** 2
    a, s2inv = swelling_factors(c, Omega)
    J, A = det_and_inv_transpose(F)
    lnJe = np.log(J) - np.log(a)
    return g * (G * s2inv * F + (lam * lnJe - G) * A)


def tangent(F, c, d, E, nu, Omega):
    """Tangent K = dP/dF (eq. (30), the K under it) as a 9x9 matrix per voxel,
    shape (9, 9, N0, N1, N2)."""
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


def apply_tangent(K, X):
    """(K : X)_ij = K_ijkl X_kl with K as (9, 9, ...) and X as (3, 3, ...)."""
    extra = X.shape[2:]
    Y = np.einsum("ab...,b...->a...", K, X.reshape((9,) + extra))
    return Y.reshape((3, 3) + extra)


def stress_param_derivatives(F, c, d, E, nu, Omega):
    """dP/d(log E) and dP/dOmega at fixed F (used by the adjoint).

    Both Lame constants are proportional to E, and P is linear in them, so
    dP/dlogE = P.  With s^-2 = (1+Omega c)^{-2/3} and
    ln J_e = ln J - ln(1 + Omega c):
        dP/dOmega = g [ -(2/3) G c (1+Omega c)^{-5/3} F
                        - lambda c / (1 + Omega c) F^-T ].
    """
    lam, G = lame(E, nu)
    g = (1.0 - d) ** 2
    a, s2inv = swelling_factors(c, Omega)
    J, A = det_and_inv_transpose(F)
    P = stress(F, c, d, E, nu, Omega)
    dP_dOm = g * (-(2.0 / 3.0) * G * c * a ** (-5.0 / 3.0) * F - lam * c / a * A)
    return P, dP_dOm
