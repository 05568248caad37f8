"""Inputs of the Sec. 5.1 particle: eq. (Gumbell) draws and the disc geometry.

value = mean * log(1 / (1 - omega))^(1/m) with omega uniform: log(1/(1 -
omega)) is a unit exponential, so value / mean follows the Weibull law of
shape m and unit scale (mean Gamma(1 + 1/m)); checked against scipy's
distribution by a Kolmogorov-Smirnov test and against the closed-form mean.
"""
import math

import numpy as np
from scipy import stats

import synth


def test_gumbel_draws_follow_weibull_law():
    rng = np.random.default_rng(7)
    m = 3.0
    v = synth.gumbel_field((200000,), 15e9, m, rng) / 15e9
    ks = stats.kstest(v, stats.weibull_min(c=m).cdf)
    assert ks.pvalue > 1e-3
    mean = math.gamma(1 + 1 / m)
    sd = math.sqrt(math.gamma(1 + 2 / m) - mean ** 2)
    assert abs(v.mean() - mean) <= 4 * sd / math.sqrt(v.size)
    assert np.all(v > 0)


def test_plane_particle_geometry():
    for n in (64, 512):
        w = synth.plane_particle_workload(n)
        assert w["shape"] == (1, n, n)
        frac = w["phase"].mean()
        assert abs(frac - math.pi * 0.4 ** 2) <= 4.0 / n  # disc of diameter 0.8 L
        dl = max(1, round(6 * n / 512))
        c = (n - 1) / 2
        i1, i2 = np.nonzero(w["band"][0])
        r = np.hypot(i1 - c, i2 - c)
        assert r.min() > 0.4 * n - dl and r.max() <= 0.4 * n
        assert np.all(w["cdot_B"][w["band"]] > 0) and np.all(w["cdot_B"][~w["band"]] == 0)
        # the void is softer and does not swell
        assert np.all(w["Omega"][~w["phase"]] == 0) and np.all(w["E"][~w["phase"]] == 1e-2 * 15e9)
    w = synth.plane_particle_workload(512)
    assert abs(w["lc"] / w["spacing"][1] - 4.0) < 1e-12
