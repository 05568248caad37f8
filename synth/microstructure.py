"""Voxel phase maps and random fields on periodic grids.

All geometry is evaluated on voxel centres x_i = (i + 1/2) h, i.e. in voxel
units a voxel i is "inside" a body when its centre (i + 0.5) is.  Spheres and
ellipsoids wrap periodically (minimum image).  Every generator takes an
explicit numpy Generator so that both sides of a parity test see identical
inputs.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "SEED_BASE",
    "rng_for",
    "voxel_centres",
    "sphere_mask",
    "ellipsoid_mask",
    "rsa_spheres",
    "boolean_spheres",
    "inner_shell",
    "laminate_mask",
    "gaussian_random_field",
]

#: Base seed: the arXiv identifier of the paper.  Workload k uses SEED_BASE + k.
SEED_BASE = 241116583


def rng_for(offset: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + int(offset))


def voxel_centres(shape):
    """Voxel-centre coordinates in voxel units, one 1-D array per axis."""
    return [np.arange(n, dtype=np.float64) + 0.5 for n in shape]


def _min_image(d, n):
    return d - n * np.round(d / n)


def sphere_mask(shape, radius, centre=None):
    """Periodic ball of the given radius (voxel units) around ``centre``."""
    return ellipsoid_mask(shape, (radius, radius, radius), centre)


def ellipsoid_mask(shape, semi_axes, centre=None):
    """Axis-aligned periodic ellipsoid; a voxel is inside iff its centre is
    (sum_j ((x_j - c_j)/a_j)^2 <= 1)."""
    shape = tuple(int(n) for n in shape)
    if centre is None:
        centre = [n / 2.0 for n in shape]
    xs = voxel_centres(shape)
    acc = np.zeros(shape, dtype=np.float64)
    for ax in range(3):
        d = _min_image(xs[ax] - centre[ax], shape[ax]) / float(semi_axes[ax])
        bshape = [1, 1, 1]
        bshape[ax] = shape[ax]
        acc = acc + (d * d).reshape(bshape)
    return acc <= 1.0


def _stamp_ball(mask, centre, radius):
    """OR a periodic ball into ``mask`` (in place), touching only its box."""
    shape = mask.shape
    idx = []
    d2 = 0.0
    for ax in range(3):
        lo = int(np.floor(centre[ax] - radius - 1))
        hi = int(np.ceil(centre[ax] + radius + 1))
        rng = np.arange(lo, hi + 1)
        d = (rng + 0.5) - centre[ax]
        bshape = [1, 1, 1]
        bshape[ax] = rng.size
        d2 = d2 + (d * d).reshape(bshape)
        idx.append(np.mod(rng, shape[ax]))
    inside = d2 <= radius * radius
    sub = mask[np.ix_(*idx)]
    mask[np.ix_(*idx)] = sub | inside


def rsa_spheres(shape, n_spheres, r_min, r_max, rng, max_tries=200000):
    """Random sequential addition of non-overlapping periodic spheres.

    Radii ~ U(r_min, r_max), centres ~ U([0, N)^3) (voxel units); a candidate
    is rejected when its minimum-image centre distance to an accepted sphere
    is not larger than the sum of the radii.
    Returns (mask, centres (k,3), radii (k,)).
    """
    shape = tuple(int(n) for n in shape)
    centres, radii = [], []
    tries = 0
    while len(radii) < n_spheres:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("RSA did not place all spheres")
        r = rng.uniform(r_min, r_max)
        c = rng.uniform(0.0, 1.0, size=3) * np.asarray(shape, dtype=np.float64)
        ok = True
        for c2, r2 in zip(centres, radii):
            d = _min_image(c - c2, np.asarray(shape, dtype=np.float64))
            if np.sqrt(np.sum(d * d)) <= r + r2:
                ok = False
                break
        if ok:
            centres.append(c)
            radii.append(r)
    mask = np.zeros(shape, dtype=bool)
    for c, r in zip(centres, radii):
        _stamp_ball(mask, c, r)
    return mask, np.asarray(centres), np.asarray(radii)


def boolean_spheres(shape, radius, target_fraction, rng, max_spheres=100000):
    """Overlapping (Boolean) periodic spheres of one radius, added until the
    voxel fraction reaches ``target_fraction``."""
    shape = tuple(int(n) for n in shape)
    mask = np.zeros(shape, dtype=bool)
    k = 0
    while mask.mean() < target_fraction:
        c = rng.uniform(0.0, 1.0, size=3) * np.asarray(shape, dtype=np.float64)
        _stamp_ball(mask, c, radius)
        k += 1
        if k > max_spheres:
            raise RuntimeError("Boolean model did not reach the fraction")
    return mask


def inner_shell(mask):
    """Voxels of ``mask`` with at least one of their 6 face neighbours outside
    (periodic neighbours)."""
    out = np.zeros_like(mask)
    for ax in range(3):
        for s in (1, -1):
            out |= mask & ~np.roll(mask, s, axis=ax)
    return out


def laminate_mask(shape, axis, fraction):
    """Layer normal to ``axis``: True for index < round(fraction * N_axis)."""
    shape = tuple(int(n) for n in shape)
    k = int(round(fraction * shape[axis]))
    idx = np.arange(shape[axis]) < k
    bshape = [1, 1, 1]
    bshape[axis] = shape[axis]
    return np.broadcast_to(idx.reshape(bshape), shape).copy()


def gaussian_random_field(shape, corr_len, rng):
    """Zero-mean, unit-sample-std Gaussian field with covariance
    exp(-r^2 / (2 l^2)) (l in voxels): white noise filtered by
    exp(-|k|^2 l^2 / 4) in Fourier space."""
    shape = tuple(int(n) for n in shape)
    w = rng.standard_normal(shape)
    W = np.fft.rfftn(w, axes=(0, 1, 2))
    k2 = 0.0
    for ax, n in enumerate(shape):
        if ax == 2:
            k = 2.0 * np.pi * np.fft.rfftfreq(n)
        else:
            k = 2.0 * np.pi * np.fft.fftfreq(n)
        bshape = [1, 1, 1]
        bshape[ax] = k.size
        k2 = k2 + (k * k).reshape(bshape)
    g = np.fft.irfftn(W * np.exp(-k2 * corr_len * corr_len / 4.0), s=shape, axes=(0, 1, 2))
    g = g - g.mean()
    return g / g.std()
