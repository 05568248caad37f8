"""The five seeded workloads (material fields, state and load schedules).

Workloads (grid sizes are defaults; every builder takes a size so that the
same generator makes the small twins used for parity):

* ``inclusion``   16^3 unit cell, centred sphere r = 4 voxels, stiff inclusion
                  (100 GPa / 0.25) in a 10 GPa / 0.3 matrix, macro F = I +
                  0.01 e1 (x) e1 in 5 increments, no damage, no chemistry.
* ``particle``    128^3, L = 15 um, one ellipsoidal particle (semi-axes
                  40/32/28 voxels, 15 GPa, D = 1e-14 m^2/s, Omega = 0.03) in a
                  compliant buffer (E = 1e-3 E_p), constant inward flux on a
                  one-voxel inner shell, 200 backward-Euler steps, AT2 damage.
* ``polydisperse`` 256^3 unit cell, 60 RSA spheres, radii U(10, 24) voxels,
                  contrast 20, macro stretch ramped to 1.05 in 20 increments.
* ``batch``       48 two-phase RVEs with N in {32, 48, 64, 96}, Boolean spheres
                  r = N/8 at volume fraction U(0.1, 0.4), 6 load cases.
* ``grf``         128^3 Gaussian random fields for log E and Omega.

SI units throughout (Pa, m, s, J/mol).  The concentration c is a normalised
mole fraction in (0, 1).
"""
from __future__ import annotations

import numpy as np

from .microstructure import (
    SEED_BASE,
    boolean_spheres,
    ellipsoid_mask,
    gaussian_random_field,
    inner_shell,
    rng_for,
    rsa_spheres,
    sphere_mask,
)

__all__ = [
    "GAS_R",
    "Workload",
    "uniaxial_schedule",
    "six_load_cases",
    "inclusion_workload",
    "particle_workload",
    "polydisperse_workload",
    "polydisperse_window",
    "batch_workloads",
    "grf_workload",
    "homogeneous_workload",
    "plane_inclusion_workload",
    "in_plane_schedule",
    "plate_workload",
    "gumbel_field",
    "plane_particle_workload",
]

GAS_R = 8.314462618  # J / (mol K)


class Workload(dict):
    """Plain dict with attribute access.

    Keys: shape, spacing, E, nu, Omega, D, sigma_max (voxel fields, float64),
    gc, lc, RT, c_max (scalars), c0, d0 (initial fields), loads (list of 3x3
    macro F), plus workload-specific extras.
    """

    __getattr__ = dict.__getitem__


def uniaxial_schedule(total_strain, n_inc):
    """F_n = I + (n / n_inc) * total_strain * e1 (x) e1, n = 1..n_inc."""
    out = []
    for n in range(1, n_inc + 1):
        F = np.eye(3)
        F[0, 0] += total_strain * n / n_inc
        out.append(F)
    return out


def in_plane_schedule(total_strain, n_inc, axis=1):
    """F_n = I + (n / n_inc) * total_strain * e_a (x) e_a, a = axis (an
    in-plane axis of a plane grid (1, N1, N2): 1 or 2)."""
    out = []
    for n in range(1, n_inc + 1):
        F = np.eye(3)
        F[axis, axis] += total_strain * n / n_inc
        out.append(F)
    return out


def six_load_cases(eps):
    """F = I + eps * E^(k) for the 6 Voigt directions 11, 22, 33, 23, 13, 12
    (shear directions symmetrised, (a (x) b + b (x) a)/2)."""
    pairs = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    out = []
    for i, j in pairs:
        E = np.zeros((3, 3))
        E[i, j] += 0.5
        E[j, i] += 0.5
        out.append(np.eye(3) + eps * E)
    return out


def _base(shape, length):
    shape = tuple(int(n) for n in shape)
    if np.isscalar(length):
        length = (float(length),) * 3
    spacing = tuple(float(L) / n for L, n in zip(length, shape))
    return shape, spacing


def homogeneous_workload(shape=(8, 8, 8), length=1.0, E=10e9, nu=0.3, Omega=0.0,
                         D=1e-14, sigma_max=1e30):
    shape, spacing = _base(shape, length)
    one = np.ones(shape)
    return Workload(
        name="homogeneous", shape=shape, spacing=spacing,
        E=E * one, nu=nu * one, Omega=Omega * one, D=D * one,
        sigma_max=sigma_max * one, gc=1.0, lc=2.0 * spacing[0],
        RT=GAS_R * 298.15, c_max=3.0e4,
        c0=np.zeros(shape), d0=np.zeros(shape), loads=uniaxial_schedule(0.01, 1),
    )


def inclusion_workload(n=16, radius=None, n_inc=5, total_strain=0.01):
    """Centred spherical inclusion in a unit cell (deterministic)."""
    shape, spacing = _base((n, n, n), 1.0)
    if radius is None:
        radius = 4.0 * n / 16.0
    inc = sphere_mask(shape, radius)
    E = np.where(inc, 100e9, 10e9)
    nu = np.where(inc, 0.25, 0.3)
    return Workload(
        name="inclusion", shape=shape, spacing=spacing, phase=inc,
        E=E, nu=nu, Omega=np.zeros(shape), D=np.full(shape, 1e-14),
        sigma_max=np.full(shape, 1e30), gc=1.0, lc=2.0 * spacing[0],
        RT=GAS_R * 298.15, c_max=3.0e4,
        c0=np.zeros(shape), d0=np.zeros(shape),
        loads=uniaxial_schedule(total_strain, n_inc),
        tol_newton=1e-8, tol_lin=1e-10,
    )


def plane_inclusion_workload(n=32, radius=None, n_inc=3, total_strain=0.01, thickness=1):
    """Plane (2-D) twin of the inclusion workload: a grid (thickness, n, n)
    of unit in-plane size, a centred circular inclusion (a cylinder through
    the thickness) of radius n/4, stiff inclusion in a compliant matrix as in
    the 3-D case, in-plane uniaxial stretch along axis 1.  With thickness 1
    it is a 2-D plan; with thickness > 1 the same cell is a prismatic 3-D
    grid whose solution does not vary along axis 0."""
    shape = (int(thickness), int(n), int(n))
    h = 1.0 / n
    spacing = (h, h, h)
    if radius is None:
        radius = n / 4.0
    inc = sphere_mask((1, n, n), radius)
    inc = np.broadcast_to(inc, shape).copy()
    E = np.where(inc, 100e9, 10e9)
    nu = np.where(inc, 0.25, 0.3)
    return Workload(
        name="plane_inclusion", shape=shape, spacing=spacing, phase=inc,
        E=E, nu=nu, Omega=np.zeros(shape), D=np.full(shape, 1e-14),
        sigma_max=np.full(shape, 1e30), gc=1.0, lc=2.0 * h,
        RT=GAS_R * 298.15, c_max=3.0e4,
        c0=np.zeros(shape), d0=np.zeros(shape),
        loads=in_plane_schedule(total_strain, n_inc),
        tol_newton=1e-8, tol_lin=1e-10,
    )


def plate_workload(n=64, corner=0, plate=40, corner_len=20, n_steps=60, dt=1.0, q_edge=1e-3, q_corner=3e-3,
                   law="svk", buffer_E=1e-2):
    """The chemo-mechanical plate of Sec. 4.3 (Table of Sec. 4.3): a plane
    grid (1, n, n) of side 0.008 mm (voxel 1.25e-4 mm, also the thickness),
    a homogeneous plate (E = 15 GPa, nu = 0.3, Omega = 1.3, D = 1e-9 mm^2/s,
    sigma_max = 50 MPa, l_c = 2 voxels) in a buffer with small stiffness and
    diffusivity and no swelling, an inward source on the plate's one-voxel
    boundary band (delta L = 1 voxel), stronger near one corner.

    Readings (the figure that fixes the geometry is not available, the units
    of the printed fluxes do not fit a normalised concentration, and two of
    the table's values do not let this discretisation run):
    * the plate is the centred plate x plate square (40 of 64 voxels, its
      corners near 0.2 L and 0.8 L, where the paper's stress concentrates);
    * the source rates are q_edge and q_corner per second in normalised
      concentration, in the band voxels; q_corner covers the band voxels
      within corner_len voxels of the plate corner `corner` (0: high i1 and
      high i2, then 90-degree turns: the fields of corner k are those of
      corner 0 turned k times by numpy.rot90 over (i1, i2));
    * q_corner / q_edge = 3 over 20-voxel corner segments (the paper: 1.5,
      extent not given): the forward-difference flux of eqs. (49)-(50) puts
      the plate's mobility on the faces from its upper band into the buffer
      and the buffer's on the faces below its lower band, so the lower bands
      keep more of their source; with the ratio 1.5 the tension near the
      (low, low) corner (0.97 sigma_max) stays above that near the flux
      corner (0.75) and damage starts there whatever the flux corner;
    * the buffer's stiffness is buffer_E E = 1e-2 E (table: 1e-5 E): the
      swollen, compressed one-voxel band on a softer foundation makes the
      Newton system indefinite (negative geometric stiffness of the
      compressed band; p.Kp < 0 in the first step for two of the four
      corners at 1e-3 E), and at 1e-5 E the CG also reaches its rounding
      floor (relative residual 8e-8, incompatible direction at 7e-8) before
      tol_lin; the buffer's diffusivity is 1e-5 D as in the table;
    * c_0 = 1e-2 (the initial concentration of Sec. 4.1), dt = 1 s;
    * g_c / l_c as printed (2e-3 / 2.5e-4) enters only as the scale of H,
      which cancels in the phase-field equation d - l_c^2 Lap d = (1 - d) D_f
      (history reading), so g_c = 8 l_c here;
    * the law is the paper's Saint-Venant-Kirchhoff law; F_macro = I (the
      compliant buffer lets the plate deform freely); the chemistry is
      solved with the full Jacobian (the mu_c-only Newton of Alg. 3 stalls
      at Omega = 1.3).
    """
    shape = (1, int(n), int(n))
    h = 0.008e-3 / n
    spacing = (h, h, h)
    lo = (n - plate) // 2
    hi = lo + plate
    part = np.zeros((n, n), dtype=bool)
    part[lo:hi, lo:hi] = True
    band = part.copy()
    band[lo + 1:hi - 1, lo + 1:hi - 1] = False
    near = np.zeros((n, n), dtype=bool)
    near[hi - corner_len:hi, hi - corner_len:hi] = True  # corner 0: high i1, high i2
    rate = np.where(band, q_edge, 0.0)
    rate = np.where(band & near, q_corner, rate)
    rate = np.rot90(rate, k=corner).copy()
    corner_mask = np.zeros((n, n), dtype=bool)
    corner_mask[hi - 1, hi - 1] = True
    site = tuple(int(v) for v in np.argwhere(np.rot90(corner_mask, k=corner))[0])  # plate corner of the flux
    part3 = part[None]
    Ep, Dp = 15e9, 1e-15
    E = np.where(part3, Ep, buffer_E * Ep)
    D = np.where(part3, Dp, 1e-5 * Dp)
    Omega = np.where(part3, 1.3, 0.0)
    lc = 2.0 * h
    return Workload(
        name="plate", shape=shape, spacing=spacing, phase=part3, corner=corner, law=law,
        E=E, nu=np.full(shape, 0.3), Omega=Omega, D=D, sigma_max=np.full(shape, 50e6),
        gc=8.0 * lc, lc=lc, RT=GAS_R * 298.15, c_max=3.0e4,
        c0=np.full(shape, 1e-2), d0=np.zeros(shape), cdot_B=rate[None].copy(),
        dt=dt, n_steps=n_steps, loads=[np.eye(3)] * n_steps, jacobian="full",
        tol_newton=1e-8, tol_lin=1e-6, tol_chem=1e-8,
        corner_site=site,
    )


def gumbel_field(shape, mean_value, m, rng):
    """Per-voxel property of eq. (Gumbell): value_i = mean_value *
    log(1 / (1 - omega_i))^(1/m), omega_i uniform in (0, 1), one draw per voxel.
    (log(1/(1 - omega)) is a unit exponential, so value / mean_value follows
    a Weibull law of shape m and unit scale, mean Gamma(1 + 1/m).)"""
    omega = rng.random(shape)
    return mean_value * np.log(1.0 / (1.0 - omega)) ** (1.0 / m)


def plane_particle_workload(n=512, n_steps=400, dt=2.0, q_in=8e-4, sigma_max=160e6, m=3.0, delta_l=None,
                            void=1e-2, law="svk", seed_offset=51):
    """The 2-D circular particle of Sec. 5.1 (Table of Sec. 5.1): a plane grid
    (1, n, n) of side 16 um with a centred disc of diameter 12.8 um, Young's
    modulus and threshold stress drawn per voxel from eq. (Gumbell) (m = 3)
    around E_mat = 15 GPa and sigma_max, nu = 0.3, Omega = 1.3,
    D = 1e-9 mm^2/s, a void with E and D scaled by `void` (table: 1e-5) and no
    swelling, and an inward source q_in on the particle's band of delta_l
    voxels (6 at n = 512, scaled with n).

    Readings: the text gives sigma_max = 100 MPa and l_c = 1.25e-4 mm, the
    table 160 MPa and 2.325e-4 mm; the table's sigma_max and the text's l_c
    (4 voxels at n = 512; at least 2 voxels in the coarser twins) are taken.  The source q_in is a
    rate per second in normalised concentration on the band (the printed
    8e-5 mol/mm^3/s does not fit c in (0, 1)); q_in = 8e-4 / s with
    dt = 2 s starts damage after about 20 steps in the 64 x 64 twin;
    c_0 = 1e-2; g_c = 2 l_c (g_c only scales H, which cancels in the
    phase-field equation).  The void's stiffness and diffusivity are scaled
    by void = 1e-2 (table: 1e-5): at 1e-5 and 1e-3 the swollen, compressed
    band on the softer void makes the first Newton system indefinite (the CG
    breaks down, p.Kp < 0, in the 64 x 64 twin), as for the plate of
    Sec. 4.3.  Chemistry with the full Jacobian, CG tolerance 1e-6.  Seeded
    from the workload's own offset; at n < 512 the same recipe at lower
    resolution (a twin, not a crop).
    """
    shape = (1, int(n), int(n))
    h = 16e-6 / n
    spacing = (h, h, h)
    if delta_l is None:
        delta_l = max(1, int(round(6 * n / 512)))
    centre = (n - 1) / 2.0
    i1, i2 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    r = np.hypot(i1 - centre, i2 - centre)
    radius = 0.5 * 0.8 * n
    part = r <= radius
    band = part & (r > radius - delta_l)
    rng = rng_for(seed_offset)
    Eg = gumbel_field((n, n), 15e9, m, rng)
    Sg = gumbel_field((n, n), sigma_max, m, rng)
    part3, band3 = part[None], band[None]
    E = np.where(part3, Eg[None], void * 15e9)
    smax = np.where(part3, Sg[None], sigma_max)
    Dp = 1e-15
    D = np.where(part3, Dp, void * Dp)
    lc = max(1.25e-7, 2.0 * h)  # the text's 1.25e-4 mm (4 voxels at n = 512), at least 2 voxels
    return Workload(
        name="plane_particle", shape=shape, spacing=spacing, phase=part3, band=band3, law=law,
        E=E, nu=np.full(shape, 0.3), Omega=np.where(part3, 1.3, 0.0), D=D, sigma_max=smax,
        gc=2.0 * lc, lc=lc, RT=GAS_R * 298.15, c_max=3.0e4,
        c0=np.full(shape, 1e-2), d0=np.zeros(shape), cdot_B=np.where(band3, q_in, 0.0),
        dt=dt, n_steps=n_steps, loads=[np.eye(3)] * n_steps, jacobian="full",
        tol_newton=1e-8, tol_lin=1e-6, tol_chem=1e-8,
    )


def particle_workload(n=128, n_steps=200, dt=5.0, q_in=4.0e-10, sigma_max=20e6):
    """Chemo-mechanical particle: ellipsoid in a compliant buffer with an inward
    flux on its one-voxel inner shell.  Sizes scale with n / 128."""
    shape, spacing = _base((n, n, n), 15e-6)
    s = n / 128.0
    part = ellipsoid_mask(shape, (40.0 * s, 32.0 * s, 28.0 * s))
    shell = inner_shell(part)
    Ep, Dp = 15e9, 1e-14
    E = np.where(part, Ep, 1e-3 * Ep)
    nu = np.full(shape, 0.3)
    Omega = np.where(part, 0.03, 0.0)
    D = np.where(part, Dp, 1e-5 * Dp)
    h = spacing[0]
    cdot_B = np.where(shell, q_in / h, 0.0)
    return Workload(
        name="particle", shape=shape, spacing=spacing, phase=part, shell=shell,
        E=E, nu=nu, Omega=Omega, D=D, sigma_max=np.full(shape, sigma_max),
        gc=1.0, lc=2.0 * h, RT=GAS_R * 298.15, c_max=3.0e4,
        c0=np.full(shape, 1e-2), d0=np.zeros(shape), cdot_B=cdot_B,
        dt=dt, n_steps=n_steps, loads=[np.eye(3)] * n_steps,
        tol_newton=1e-8, tol_lin=1e-10, tol_chem=1e-8,
    )


def polydisperse_workload(n=256, n_spheres=60, n_inc=20, total_strain=0.05,
                          strength_ratio=0.25):
    """Periodic RSA spheres (radii U(10, 24) voxels at 256^3, scaled with
    n / 256), spheres 200 GPa, matrix 10 GPa, nu = 0.3.  The threshold
    stress is proportional to stiffness, sigma_max = strength_ratio E
    (default 0.25: 2.5 GPa in the matrix, 50 GPa in the spheres), so that
    damage starts in the second half of the stretch ramp, in the matrix
    ligament of the narrowest gap aligned with the stretch (about ten times
    the mean strain there).  With 0.04 E that ligament damages from the
    second increment and a crack runs through the matrix at 1 % stretch."""
    shape, spacing = _base((n, n, n), 1.0)
    s = n / 256.0
    rng = rng_for(3)
    inc, centres, radii = rsa_spheres(shape, n_spheres, 10.0 * s, 24.0 * s, rng)
    E = np.where(inc, 200e9, 10e9)
    return Workload(
        name="polydisperse", shape=shape, spacing=spacing, phase=inc,
        centres=centres, radii=radii,
        E=E, nu=np.full(shape, 0.3), Omega=np.zeros(shape),
        D=np.full(shape, 1e-14), sigma_max=strength_ratio * E,
        gc=1.0, lc=2.0 * spacing[0], RT=GAS_R * 298.15, c_max=3.0e4,
        c0=np.zeros(shape), d0=np.zeros(shape),
        loads=uniaxial_schedule(total_strain, n_inc),
        tol_newton=1e-8, tol_lin=1e-10,
    )


def polydisperse_window(n=48, pair=(12, 55), strength_ratio=0.25, n_inc=20, total_strain=0.05):
    """An n^3 window of the 256^3 polydisperse microstructure (same voxels,
    same materials, same load ramp), centred on the surface gap between the
    two given spheres (by default the gap most aligned with the stretch
    axis among the narrowest, where damage starts), taken as a periodic cell
    of its own: the full-resolution twin of the damage ramp."""
    full = polydisperse_workload(n=256, strength_ratio=strength_ratio, n_inc=n_inc, total_strain=total_strain)
    C, R = full["centres"], full["radii"]
    i, j = pair
    L = np.array([256.0] * 3)
    d = C[j] - C[i]
    d = d - L * np.round(d / L)
    dist = float(np.sqrt(np.sum(d * d)))
    gap = dist - R[i] - R[j]
    mid = (C[i] + d * (R[i] + 0.5 * gap) / dist) % 256.0
    lo = np.floor(mid - n / 2).astype(int)
    sub = np.ix_(*[np.arange(lo[a], lo[a] + n) % 256 for a in range(3)])
    w = Workload(full)
    for k in ("E", "nu", "Omega", "D", "sigma_max", "c0", "d0", "phase"):
        w[k] = np.ascontiguousarray(full[k][sub])
    w.update(name="polydisperse_window", shape=(n, n, n), gap=gap, window_origin=lo.tolist())
    return w


def batch_workloads(n_items=48, sizes=(32, 48, 64, 96), eps=1e-3):
    """Two-phase RVEs: grid size ~ uniform over ``sizes``, Boolean spheres of
    radius N/8 up to a volume fraction ~ U(0.1, 0.4); materials as the
    inclusion workload; 6 load cases each."""
    rng = rng_for(4)
    items = []
    for k in range(n_items):
        n = int(rng.choice(np.asarray(sizes)))
        phi = float(rng.uniform(0.1, 0.4))
        shape, spacing = _base((n, n, n), 1.0)
        inc = boolean_spheres(shape, n / 8.0, phi, rng)
        items.append(Workload(
            name="batch_item", index=k, shape=shape, spacing=spacing,
            phase=inc, target_fraction=phi,
            E=np.where(inc, 100e9, 10e9), nu=np.where(inc, 0.25, 0.3),
            Omega=np.zeros(shape), D=np.full(shape, 1e-14),
            sigma_max=np.full(shape, 1e30), gc=1.0, lc=2.0 * spacing[0],
            RT=GAS_R * 298.15, c_max=3.0e4,
            c0=np.zeros(shape), d0=np.zeros(shape),
            loads=six_load_cases(eps),
        ))
    return items


def grf_workload(n=128, corr_len=8.0):
    """Gaussian random fields for log-stiffness and swelling coefficient."""
    shape, spacing = _base((n, n, n), 1.0)
    rng = rng_for(5)
    g1 = gaussian_random_field(shape, corr_len * n / 128.0, rng)
    g2 = gaussian_random_field(shape, corr_len * n / 128.0, rng)
    logE = np.log(10e9) + 0.5 * g1
    F = np.eye(3)
    F[0, 0] += 0.02
    return Workload(
        name="grf", shape=shape, spacing=spacing,
        E=np.exp(logE), nu=np.full(shape, 0.3), Omega=0.03 + 0.01 * g2,
        D=np.full(shape, 1e-14), sigma_max=np.full(shape, 1e30),
        gc=1.0, lc=2.0 * spacing[0], RT=GAS_R * 298.15, c_max=3.0e4,
        c0=np.full(shape, 0.5), d0=np.zeros(shape), loads=[F],
        fd_voxels=rng.integers(0, int(np.prod(shape)), size=32),
        tol_newton=1e-8, tol_lin=1e-10,
    )
