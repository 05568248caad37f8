"""Host-side logic that needs no GPU: effective-stiffness assembly, the tile
autotuner's choice and cache (against a stand-in for the library's timing
calls), and the benchmark's byte-model arithmetic."""
import ctypes
import json
import os

import numpy as np
import pytest

import synth
from paper_2411_16583_amd import autotune, homogenize


def test_load_cases_match_generator():
    for a, b in zip(homogenize.six_load_cases(1e-3), synth.six_load_cases(1e-3)):
        assert np.array_equal(a, b)


def test_voigt_stiffness_of_isotropic_linear_response():
    """For P = lambda tr(e) I + 2 mu e with e = F - I (exact for a linear
    law), the assembled matrix is the isotropic Voigt stiffness with
    engineering shear: C_44 = C_55 = C_66 = mu."""
    lam, mu, eps = 3.7, 1.9, 1e-3
    P = []
    for F in homogenize.six_load_cases(eps):
        e = F - np.eye(3)
        P.append(lam * np.trace(e) * np.eye(3) + 2 * mu * e)
    C = homogenize.voigt_stiffness(np.array(P), eps)
    ref = np.zeros((6, 6))
    ref[:3, :3] = lam
    ref[[0, 1, 2], [0, 1, 2]] = lam + 2 * mu
    ref[[3, 4, 5], [3, 4, 5]] = mu
    assert np.allclose(C, ref, rtol=0, atol=1e-12)


def test_voigt_stiffness_symmetrises_the_stress():
    eps = 1e-3
    P = np.zeros((6, 3, 3))
    P[5, 0, 1] = 2e-3  # only the (0, 1) entry of the shear case
    C = homogenize.voigt_stiffness(P, eps)
    assert C[5, 5] == pytest.approx(1.0)  # (P01 + P10) / 2 / eps


class FakeLib:
    """Stand-in for the tile calls of libfgfft: candidates per pass and a
    timing table; records what the tuner sets."""

    def __init__(self, cands, times):
        self.cands, self.times = cands, times
        self.timed = []
        self.set = None

    def fg_plan_tile_candidates(self, handle, which, out, cap):
        c = self.cands[which]
        for k in range(min(cap, len(c))):
            out[k] = c[k]
        return len(c)

    def fg_plan_time_pass(self, handle, which, tile, reps, ms_ref):
        self.timed.append((which, tile))
        ms_ref._obj.value = self.times[(which, tile)]
        return 0

    def fg_plan_set_tiles(self, handle, arr):
        self.set = list(arr)
        return 0

    def fg_last_error(self, handle):
        return b""


def test_tuner_picks_fastest_and_caches(tmp_path):
    cands = {0: [2, 4, 8], 1: [4, 8, 4 | 0x10000, 8 | 0x10000]}
    times = {(0, 2): 3.0, (0, 4): 1.0, (0, 8): 2.0,
             (1, 4): 5.0, (1, 8): 4.0, (1, 4 | 0x10000): 4.5, (1, 8 | 0x10000): 3.5}
    lib = FakeLib(cands, times)
    path = str(tmp_path / "tiles.json")
    rep = autotune.tune_handle(None, (16, 32, 64), 1, 0, path, reps=3, lib=lib, arch="gfx950")
    assert lib.set == [4, 8 | 0x10000, 0, 0]
    assert rep["axis_f64"][0] == 4 and rep["zproj_f64"][0] == 8 | 0x10000
    assert len(lib.timed) == 7
    cache = json.load(open(path))
    assert cache["gfx950|16x32x64|items=1|axis_f64"]["tile"] == 4
    # second call: from the cache, nothing timed
    lib2 = FakeLib(cands, times)
    rep2 = autotune.tune_handle(None, (16, 32, 64), 1, 0, path, reps=3, lib=lib2, arch="gfx950")
    assert lib2.timed == [] and lib2.set == lib.set
    assert all(v[1] is None for v in rep2.values())
    # another grid or item count is tuned separately; force re-times
    lib3 = FakeLib(cands, times)
    autotune.tune_handle(None, (16, 32, 64), 6, 0, path, reps=3, lib=lib3, arch="gfx950")
    assert len(lib3.timed) == 7
    lib4 = FakeLib(cands, times)
    autotune.tune_handle(None, (16, 32, 64), 1, 0, path, reps=3, lib=lib4, arch="gfx950", force=True)
    assert len(lib4.timed) == 7


def test_tuner_ignores_stale_cache_entries(tmp_path):
    """A cached tile that is no longer a candidate is re-timed."""
    path = str(tmp_path / "tiles.json")
    json.dump({"gfx950|8x8x8|items=1|axis_f64": {"tile": 64}}, open(path, "w"))
    lib = FakeLib({0: [1, 2], 1: [1]}, {(0, 1): 2.0, (0, 2): 1.0, (1, 1): 1.0})
    autotune.tune_handle(None, (8, 8, 8), 1, 0, path, lib=lib, arch="gfx950")
    assert lib.set[0] == 2 and (0, 1) in lib.timed


def test_mixed_plans_tune_four_passes(tmp_path):
    cands = {w: [1] for w in range(4)}
    times = {(w, 1): 1.0 for w in range(4)}
    lib = FakeLib(cands, times)
    rep = autotune.tune_handle(None, (8, 8, 8), 1, 1, str(tmp_path / "t.json"), lib=lib, arch="gfx950")
    assert set(rep) == {"axis_f64", "zproj_f64", "axis_f32", "zproj_f32"}


def test_bench_byte_model_and_roofline():
    import bench

    N = 256 ** 3
    # words per voxel per CG iteration of the kernels on the path
    assert sum(bench.WORDS_PER_VOXEL[k] for k in ("front", "axis", "zproj", "axis3", "c2r3", "grad")) == 81
    prof = {k: (0.0, 0) for k in ["front", "r2c", "axis", "zproj", "c2r", "cg_update", "finalize", "constitutive",
                                  "zscalar", "axis3", "c2r3", "grad"]}
    prof["front"] = (1693.2 * 10 / 1e3, 10)  # 10 launches of 1693.2 us
    prof["axis"] = (0.4402 * 10, 10)
    r = bench.roofline(dict(prof=prof), N, 8)
    assert r["kernel"] == "front"
    assert r["bytes_per_launch"] == 36 * 8 * N
    assert r["achieved"] == pytest.approx(36 * 8 * N / 1693.2e-6 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-3)
    assert set(r["per_class"]) == {"front", "axis"}


@pytest.mark.parametrize("L", [1, 3, 6, 8, 12, 96, 256])
def test_two_point_stencil_identity_of_the_n0_pass(L):
    """The identity the N0 projection pass rests on: with sz = (2/h) sin(pi k/L),
    cz = cos(pi k/L) and q = 2 pi k / L (the same k for every factor),
    e^{i q/2} (sz X0 + cz X1) is the DFT of the two-point stencil
    c[n] = (x1[n] + x1[n+1]) / 2 - i (x0[n+1] - x0[n]) / h (periodic), so one
    forward transform replaces two.  Checked with numpy's FFT on random
    complex data, odd lengths and L = 1 included."""
    rng = np.random.default_rng(L)
    h = 0.37
    x0 = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    x1 = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    k = np.arange(L)
    a = np.pi * k / L
    sz, cz = (2.0 / h) * np.sin(a), np.cos(a)
    lhs = np.exp(1j * a) * (sz * np.fft.fft(x0) + cz * np.fft.fft(x1))
    c = 0.5 * (x1 + np.roll(x1, -1)) - 1j * (np.roll(x0, -1) - x0) / h
    assert np.allclose(np.fft.fft(c), lhs, rtol=0, atol=1e-12 * max(1.0, np.abs(lhs).max()))
