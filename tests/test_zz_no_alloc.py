"""The allocation-free projection (fg_project_noalloc, through the C ABI)
against fg_project of a plan on the same grid: two calls in a row, the
second on a smaller grid, both within the double-precision bar of the
projection (1e-13 relative); in place; an oversized grid is refused."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from paper_2411_16583_amd import fgfft
from tests.gpu_util import DEV, dt, host, plan_for, rel

pytestmark = pytest.mark.gpu


def _call(grid, spacing, x, y):
    lib = fgfft.load_library()
    g = (ctypes.c_int * 3)(*grid)
    h = (ctypes.c_double * 3)(*spacing)
    return lib.fg_project_noalloc(g, h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_project_noalloc_matches_project_on_two_calls():
    rng = np.random.default_rng(7071)
    for shape, lengths in [((48, 32, 64), (1.0, 0.8, 1.3)), ((16, 24, 12), (0.5, 0.7, 0.4))]:
        print(f"noalloc shape={shape}", flush=True)
        work = synth.homogeneous_workload(shape, lengths)
        spacing = work["spacing"]
        x = dt(rng.standard_normal((9,) + shape))
        x0 = x.clone()
        y_ref = torch.empty_like(x)
        plan = plan_for(work)
        plan.project(x, y_ref)
        y = torch.full_like(x, np.nan)
        assert _call(shape, spacing, x, y) == fgfft.FG_OK
        torch.cuda.synchronize()
        e = rel(host(y), host(y_ref))
        print(f"  rel to fg_project {e:.2e}", flush=True)
        assert e <= 1e-13
        assert torch.equal(x, x0)
        # in place (y = x)
        assert _call(shape, spacing, x, x) == fgfft.FG_OK
        torch.cuda.synchronize()
        assert rel(host(x), host(y_ref)) <= 1e-13
        plan.close()


def test_project_noalloc_refuses_oversized_and_bad_grids():
    x = torch.zeros(9 * 4 * 4 * 4, dtype=torch.float64, device=DEV)
    # 128^3 needs 9 N doubles = 144 MiB of spectrum, beyond the 64 MiB array
    assert _call((128, 128, 128), (1.0, 1.0, 1.0), x, x) == fgfft.FG_E_SIZE
    assert _call((16, 16, 10), (1.0, 1.0, 1.0), x, x) == fgfft.FG_E_SIZE
    assert _call((4, 4, 4), (1.0, -1.0, 1.0), x, x) == fgfft.FG_E_ARG
