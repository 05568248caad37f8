"""Discrete frequencies and spectral symbols (Sec. 3.2, "FFT resolution
algorithms"; Mechanical Equilibrium subsection).

Fields are voxel-centred on an N0 x N1 x N2 periodic grid with spacing h_j;
the discrete Fourier transform is taken over the three spatial axes
(numpy/scipy ``rfftn`` convention, half spectrum on the last axis).  The
paper replaces continuum frequencies by finite-difference ("modified")
frequencies; for mechanics it uses the rotated scheme of Willot.  We read the
rotated scheme as the 8-corner finite-difference gradient (nodal
displacement at voxel corners, gradient at the voxel centre), whose symbol is

    k_j = (1/(4 h_j)) (e^{i q_j} - 1) prod_{l != j} (1 + e^{i q_l})
        = i r_j e^{i (q_0 + q_1 + q_2)/2},
    r_j = (2/h_j) sin(q_j/2) prod_{l != j} cos(q_l/2),

with q_j = 2 pi m_j / N_j.  cos(q_l/2) is set to an exact zero at
m_l = N_l/2 (detected by index, never by a floating-point cosine).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

WORKERS = -1  # all host threads for the library FFT

AXES = (-3, -2, -1)


def rfft3(f):
    """Forward real DFT over the last three axes (unnormalised)."""
    return sfft.rfftn(f, axes=AXES, workers=WORKERS)


def irfft3(F, shape):
    """Inverse of :func:`rfft3` (normalised by 1/N)."""
    return sfft.irfftn(F, s=tuple(shape), axes=AXES, workers=WORKERS)


def _axis_indices(shape):
    n0, n1, n2 = shape
    m0 = np.arange(n0)
    m1 = np.arange(n1)
    m2 = np.arange(n2 // 2 + 1)
    return m0, m1, m2


def half_angle_sin_cos(m, n):
    """sin(pi m / n), cos(pi m / n) with exact zeros at m = 0 (sin) and
    m = n/2 (cos)."""
    m = np.asarray(m)
    s = np.sin(np.pi * m / n)
    c = np.cos(np.pi * m / n)
    s = np.where(m == 0, 0.0, s)
    if n % 2 == 0:
        c = np.where(m == n // 2, 0.0, c)
    return s, c


def _bcast(v, ax):
    shape = [1, 1, 1]
    shape[ax] = v.size
    return v.reshape(shape)


def rotated_vector(shape, spacing):
    """Real vector r(q) of the rotated scheme on the half spectrum,
    shape (3, N0, N1, N2//2+1)."""
    ms = _axis_indices(shape)
    s, c = [], []
    for ax in range(3):
        sa, ca = half_angle_sin_cos(ms[ax], shape[ax])
        s.append(_bcast(sa, ax))
        c.append(_bcast(ca, ax))
    r = []
    for j in range(3):
        val = (2.0 / spacing[j]) * s[j]
        for l in range(3):
            if l != j:
                val = val * c[l]
        r.append(np.broadcast_to(val, (shape[0], shape[1], shape[2] // 2 + 1)))
    return np.stack(r)


def rotated_symbol(shape, spacing):
    """Complex symbol k_j of the 8-corner gradient, directly from its
    definition with exponentials (used only by pins)."""
    ms = _axis_indices(shape)
    e = [_bcast(np.exp(2j * np.pi * ms[ax] / shape[ax]), ax) for ax in range(3)]
    out = []
    for j in range(3):
        val = (e[j] - 1.0) / (4.0 * spacing[j])
        for l in range(3):
            if l != j:
                val = val * (1.0 + e[l])
        out.append(np.broadcast_to(val, (shape[0], shape[1], shape[2] // 2 + 1)))
    return np.stack(out)


def laplacian_symbol(shape, spacing):
    """lambda(q) = sum_j (2/h_j)^2 sin^2(q_j/2): symbol of minus the 7-point
    Laplacian (the forward-and-backward finite-difference frequencies)."""
    ms = _axis_indices(shape)
    lam = 0.0
    for ax in range(3):
        s, _ = half_angle_sin_cos(ms[ax], shape[ax])
        lam = lam + _bcast((2.0 / spacing[ax]) ** 2 * s * s, ax)
    return np.broadcast_to(lam, (shape[0], shape[1], shape[2] // 2 + 1)).copy()


def forward_difference_symbol(shape, spacing):
    """xi_j = (e^{i q_j} - 1)/h_j: symbol of the periodic forward difference."""
    ms = _axis_indices(shape)
    out = []
    for j in range(3):
        v = (np.exp(2j * np.pi * ms[j] / shape[j]) - 1.0) / spacing[j]
        out.append(np.broadcast_to(_bcast(v, j), (shape[0], shape[1], shape[2] // 2 + 1)))
    return np.stack(out)


def project(A, spacing):
    """Compatibility projection  G * A  = F^{-1}[ G^ : F[A] ]  (eq. (28)
    [mapping G], eq. (30) [mechanicalsolve]).

    A has shape (3, 3, N0, N1, N2).  In Fourier space the projector onto
    compatible (gradient) fields is G^_{ijkl} = delta_ik r_l r_j / |r|^2 (so
    (G^:A^)_ij = A^_il r_l r_j / |r|^2), and G^ = 0 where r = 0 (q = 0 and the
    frequencies with two or more components equal to pi).
    """
    shape = A.shape[2:]
    r = rotated_vector(shape, spacing)
    r2 = np.sum(r * r, axis=0)
    inv = np.zeros_like(r2)
    nz = r2 > 0.0
    inv[nz] = 1.0 / r2[nz]
    Ah = rfft3(A)
    Zh = np.einsum("il...,l...,j...->ij...", Ah, r, r) * inv
    return irfft3(Zh, shape)
