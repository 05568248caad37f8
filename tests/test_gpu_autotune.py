"""Tile autotuner of the column passes: every valid tile gives bit-identical
results (the tile groups columns, the per-column arithmetic is unchanged),
the tuner picks a valid tile per pass and caches it, and a tuned batch solves
to the same bits as an untuned one."""
import numpy as np
import pytest
import torch

import synth
from paper_2411_16583_amd import Batch, FgError, Plan, make_opts
from paper_2411_16583_amd.autotune import candidates, tune_plan
from paper_2411_16583_amd.fgfft import FG_E_ARG
from tests.gpu_util import DEV, dt, host, plan_for

pytestmark = pytest.mark.gpu

SHAPE = (16, 32, 64)


def test_every_tile_gives_identical_projection():
    print(f"tiles fp64 {SHAPE}", flush=True)
    work = synth.homogeneous_workload(SHAPE, 1.0)
    plan = plan_for(work)
    x = dt(np.random.default_rng(7).standard_normal((9,) + SHAPE))
    y0 = torch.empty_like(x)
    plan.project(x, y0)
    ref = host(y0)
    for w in (0, 1):
        cands = candidates(plan.handle, w)
        widths = [c & 0xFFFF for c in cands]
        assert cands and all(b & (b - 1) == 0 for b in widths)
        assert (w == 1) == any(c & 0x10000 for c in cands)  # ky-major order: projection pass only
        for b in cands:
            tiles = [0, 0, 0, 0]
            tiles[w] = b
            plan.set_tiles(tiles)
            y = torch.empty_like(x)
            plan.project(x, y)
            assert np.array_equal(host(y), ref), (w, b)
    plan.close()


def test_every_fp32_tile_gives_identical_operator():
    print(f"tiles fp32 {SHAPE}", flush=True)
    work = synth.inclusion_workload(n=16)
    shape = work["shape"]
    plan = plan_for(work, "mixed")
    F = dt(np.broadcast_to((np.eye(3) * 1.01).reshape(3, 3, 1, 1, 1), (3, 3) + shape).copy())
    plan.set_state(F)
    x = dt(np.random.default_rng(8).standard_normal((9,) + shape))
    y0 = torch.empty_like(x)
    plan.apply_operator(x, y0)
    ref = host(y0)
    for w in (2, 3):
        for b in candidates(plan.handle, w):
            tiles = [0, 0, 0, 0]
            tiles[w] = b
            plan.set_tiles(tiles)
            y = torch.empty_like(x)
            plan.apply_operator(x, y)
            assert np.array_equal(host(y), ref), (w, b)
    plan.close()


def test_invalid_tile_rejected():
    plan = Plan(SHAPE, (1.0, 1.0, 1.0))
    with pytest.raises(FgError) as ei:
        plan.set_tiles([3, 0, 0, 0])
    assert ei.value.code == FG_E_ARG
    with pytest.raises(FgError):
        plan.set_tiles([0, 64, 0, 0])  # 64 does not divide N2 / 2 = 32
    plan.close()


def test_tuner_picks_valid_tiles_and_caches(tmp_path):
    print("tune plan", flush=True)
    cache = str(tmp_path / "tiles.json")
    plan = Plan((64, 64, 128), (1.0, 1.0, 1.0), "mixed")
    rep = tune_plan(plan, cache, reps=3)
    assert set(rep) == {"axis_f64", "zproj_f64", "axis_f32", "zproj_f32"}
    tiles = plan.tiles()
    for w, name in enumerate(["axis_f64", "zproj_f64", "axis_f32", "zproj_f32"]):
        assert tiles[w] == rep[name][0] and tiles[w] in candidates(plan.handle, w)
        assert rep[name][1] is not None and all(t > 0 for t in rep[name][1].values())
    plan2 = Plan((64, 64, 128), (1.0, 1.0, 1.0), "mixed")
    rep2 = tune_plan(plan2, cache, reps=3)
    assert all(v[1] is None for v in rep2.values())  # from the cache, no timing
    assert plan2.tiles() == tiles
    plan.close()
    plan2.close()


def test_tuned_batch_identical(tmp_path):
    print("tune batch", flush=True)
    rng = synth.rng_for(41)
    shapes = [(16, 16, 16), (8, 16, 32)]
    rves = []
    for shape in shapes:
        inc = synth.microstructure.boolean_spheres(shape, min(shape) / 5.0, 0.3, rng)
        rves.append(dict(shape=shape, spacing=tuple(1.0 / n for n in shape), E=np.where(inc, 100e9, 10e9),
                         nu=np.where(inc, 0.25, 0.3), Omega=np.zeros(shape)))
    loads = synth.six_load_cases(1e-3)[:2]
    out = []
    for tuned in (False, True):
        b = Batch([r["shape"] for r in rves], [r["spacing"] for r in rves], len(loads))
        for k, r in enumerate(rves):
            b.set_material(k, dt(r["E"]), dt(r["nu"]), dt(r["Omega"]))
        if tuned:
            b.autotune(str(tmp_path / "tiles.json"), reps=2)
        P, stats, _ = b.newton_solve(loads, make_opts(1e-10, 1e-12), graph_ticks=4)
        out.append(P)
        b.close()
    assert np.array_equal(out[0], out[1])
