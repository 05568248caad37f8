"""Tile autotuner for the column passes of the 3-D transform.

The complex pass along N1 and the N0 pass fused with the projection
(eq. (28)) process `tile` adjacent kx columns per workgroup.  The best tile
trades workgroup size against LDS per workgroup (occupancy) and depends on
the grid, the item count of a batch and the precision, so it is measured:
every valid tile of each pass is timed on the plan itself
(fg_plan_time_pass, HIP events) and the fastest is kept.  Results are cached
in a JSON file keyed by (GPU architecture, grid, items, pass), so a later
plan of the same shape takes the cached choice without timing.  The tile
changes the grouping of columns only, never the arithmetic, so results are
bit-identical for every tile.
"""
from __future__ import annotations

import ctypes
import json
import os
import tempfile

from .fgfft import FG_MIXED, FG_OK, FgError, load_library

CACHE_ENV = "FGFFT_TILE_CACHE"
PASS_NAMES = ["axis_f64", "zproj_f64", "axis_f32", "zproj_f32"]


def default_cache_path():
    p = os.environ.get(CACHE_ENV)
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "fgfft", "tiles.json")


def _arch():
    import torch

    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, cache):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".tiles", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates(handle, which, lib=None):
    lib = lib or load_library()
    n = lib.fg_plan_tile_candidates(handle, which, None, 0)
    if n < 0:
        raise FgError(1, "fg_plan_tile_candidates")
    out = (ctypes.c_int * max(n, 1))()
    lib.fg_plan_tile_candidates(handle, which, out, n)
    return list(out[:n])


def time_pass(handle, which, tile, reps=10, lib=None):
    lib = lib or load_library()
    ms = ctypes.c_double()
    st = lib.fg_plan_time_pass(handle, which, int(tile), int(reps), ctypes.byref(ms))
    if st != FG_OK:
        raise FgError(st, f"fg_plan_time_pass({which}, {tile}): {lib.fg_last_error(handle).decode()}")
    return ms.value


def get_tiles(handle, lib=None):
    lib = lib or load_library()
    t = (ctypes.c_int * 4)()
    lib.fg_plan_get_tiles(handle, t)
    return list(t)


def tune_handle(handle, grid, nitems, precision, cache_path=None, reps=10, lib=None, arch=None, force=False):
    """Tune one plan handle (a plan or a batch group); returns a dict
    {pass name: (tile, timings or None when cached)}."""
    lib = lib or load_library()
    arch = arch or _arch()
    path = cache_path or default_cache_path()
    cache = _load(path)
    passes = [0, 1] + ([2, 3] if precision == FG_MIXED else [])
    tiles = [0, 0, 0, 0]
    report = {}
    dirty = False
    for w in passes:
        key = f"{arch}|{grid[0]}x{grid[1]}x{grid[2]}|items={nitems}|{PASS_NAMES[w]}"
        cands = candidates(handle, w, lib)
        hit = cache.get(key)
        if hit is not None and not force and hit.get("tile") in cands:
            tiles[w] = int(hit["tile"])
            report[PASS_NAMES[w]] = (tiles[w], None)
            continue
        times = {b: time_pass(handle, w, b, reps, lib) for b in cands}
        best = min(times, key=times.get)
        tiles[w] = best
        cache[key] = {"tile": best, "ms": {str(b): round(t, 5) for b, t in times.items()}}
        report[PASS_NAMES[w]] = (best, times)
        dirty = True
    st = lib.fg_plan_set_tiles(handle, (ctypes.c_int * 4)(*tiles))
    if st != FG_OK:
        raise FgError(st, "fg_plan_set_tiles")
    if dirty:
        _store(path, cache)
    return report


def tune_plan(plan, cache_path=None, reps=10, force=False):
    from .fgfft import PRECISIONS

    return tune_handle(plan.handle, plan.grid, 1, PRECISIONS[plan.precision], cache_path, reps, plan.lib,
                       force=force)


def tune_batch(batch, cache_path=None, reps=10, force=False):
    """Tune every grid group of a batch (each group's plan handle)."""
    from .fgfft import PRECISIONS

    lib = batch.lib
    out = []
    for g in range(batch.n_groups):
        h = lib.fg_batch_plan(batch.handle, g)
        grid = (ctypes.c_int * 3)()
        nit = ctypes.c_int()
        lib.fg_batch_group_info(batch.handle, g, grid, ctypes.byref(nit))
        out.append(tune_handle(ctypes.c_void_p(h), tuple(grid), nit.value, PRECISIONS[batch.precision], cache_path,
                               reps, lib, force=force))
    return out
