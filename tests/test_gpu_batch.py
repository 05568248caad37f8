"""Batched form of Alg. 1 (fg_batch_*): RVEs of different grids times load
cases, all items solved together with per-item masking.

Parity: every item against the plain loop over (RVE, case) — the oracle's
Newton solve (FP64, <= 1e-10 relative to the fluctuation) and the single-item
GPU plan (<= 1e-10); the mixed batch against the FP64 batch (<= 1e-6).  The
captured graph and the direct launches run the same kernels in the same
order, so their results are compared bit for bit, as are two items with the
same RVE and load case in different positions of one launch.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import mechanics
from paper_2411_16583_amd import Batch, FgError, make_opts
from paper_2411_16583_amd.fgfft import FG_E_STATE
from tests.gpu_util import DEV, dt, host, rel

pytestmark = pytest.mark.gpu

EPS = 1e-3
# uniaxial 11, shear 12 and the zero load (F = I: converged at once, P = 0)
CASES = [synth.six_load_cases(EPS)[0], synth.six_load_cases(EPS)[5], np.eye(3)]
# ragged grids; RVE 3 repeats RVE 1 (same grid and material)
GRIDS = [(16, 16, 16), (8, 8, 8), (12, 12, 12), (8, 8, 8), (8, 12, 16)]


def make_rves():
    rng = synth.rng_for(40)
    rves = []
    for k, shape in enumerate(GRIDS):
        if k == 3:
            rves.append(rves[1])
            continue
        inc = synth.microstructure.boolean_spheres(shape, min(shape) / 6.0, 0.25, rng)
        spacing = tuple(1.0 / n for n in shape)
        rves.append(dict(shape=shape, spacing=spacing, E=np.where(inc, 100e9, 10e9),
                         nu=np.where(inc, 0.25, 0.3), Omega=np.zeros(shape)))
    return rves


def make_batch(rves, precision="fp64"):
    b = Batch([r["shape"] for r in rves], [r["spacing"] for r in rves], len(CASES), precision)
    for k, r in enumerate(rves):
        b.set_material(k, dt(r["E"]), dt(r["nu"]), dt(r["Omega"]))
    return b


def batch_fields(b, rves):
    out = {}
    for k, r in enumerate(rves):
        for lc in range(len(CASES)):
            F = torch.empty(9 * int(np.prod(r["shape"])), dtype=torch.float64, device=DEV)
            out[k, lc] = host(b.state(k, lc, F), (3, 3) + r["shape"])
    return out


OPTS = dict(tol_newton=1e-10, tol_lin=1e-12, max_newton=20, max_lin=5000)


@pytest.fixture(scope="module")
def rves():
    return make_rves()


@pytest.fixture(scope="module")
def fp64_eager(rves):
    print("batch fp64 eager", flush=True)
    b = make_batch(rves)
    assert b.n_groups == 4
    P, stats, st = b.newton_solve(CASES, make_opts(**OPTS), graph_ticks=0)
    F = batch_fields(b, rves)
    b.close()
    return P, stats, F


def test_batch_items_match_oracle_loop(rves, fp64_eager):
    """Each (RVE, case) item against the oracle's own Newton solve from the
    same uniform start (the plain loop over items)."""
    P, stats, F = fp64_eager
    for k, r in enumerate(rves):
        if k in (0, 3):
            continue  # 16^3 is covered by the single-plan comparison; RVE 3 repeats RVE 1
        c0 = np.zeros(r["shape"])
        for lc, Fbar in enumerate(CASES):
            print(f"oracle rve={k} shape={r['shape']} case={lc}", flush=True)
            Fo, so = mechanics.newton_solve(mechanics.uniform_field(Fbar, r["shape"]), Fbar, c0, c0, r,
                                            r["spacing"], tol_newton=1e-10, tol_lin=1e-12)
            s = stats[k * len(CASES) + lc]
            assert s["newton_iters"] == so["newton_iters"]
            if lc == 2:
                assert s["newton_iters"] == 0 and np.all(P[k, lc] == 0.0)
                continue
            fl = Fo - mechanics.uniform_field(Fbar, r["shape"])
            assert rel(F[k, lc], Fo, fl) <= 1e-10
            Po = mechanics.mean_stress(Fo, c0, c0, r)
            assert rel(P[k, lc], Po) <= 1e-10


def test_batch_items_match_single_plans(rves, fp64_eager):
    """Each item against a single-item GPU plan solved from F = I."""
    from tests.gpu_util import plan_for

    P, stats, F = fp64_eager
    for k, r in enumerate(rves):
        work = dict(r, D=np.full(r["shape"], 1e-14), sigma_max=np.full(r["shape"], 1e30), gc=1.0, lc=0.1,
                    RT=2478.957, c_max=3.0e4)
        for lc, Fbar in enumerate(CASES):
            print(f"single rve={k} case={lc}", flush=True)
            plan = plan_for(work)
            Fs = dt(mechanics.uniform_field(np.eye(3), r["shape"]))
            plan.set_state(Fs)
            s1 = plan.newton_solve(Fbar, make_opts(**OPTS))
            Ps = plan.homogenized_stress()
            s = stats[k * len(CASES) + lc]
            assert s["newton_iters"] == s1["newton_iters"]
            if lc == 2:
                assert np.all(Ps == 0.0) and np.all(P[k, lc] == 0.0)
                continue
            fl = host(Fs, (3, 3) + r["shape"]) - mechanics.uniform_field(Fbar, r["shape"])
            assert rel(F[k, lc], host(Fs, (3, 3) + r["shape"]), fl) <= 1e-10
            assert rel(P[k, lc], Ps) <= 1e-10
            assert s["err_res"] <= 1e-10
            plan.close()


def test_batch_repeated_rve_identical(fp64_eager):
    """Same RVE and case at two positions of one launch: identical bits."""
    P, stats, F = fp64_eager
    for lc in range(len(CASES)):
        assert np.array_equal(F[1, lc], F[3, lc])
        assert np.array_equal(P[1, lc], P[3, lc])


def test_batch_graph_equals_eager(rves, fp64_eager):
    """One captured graph (5 steps per replay, replayed until every item has
    finished, twice with direct work between the solves) against the direct
    launches: bit-identical states, stresses and iteration counts."""
    P0, stats0, F0 = fp64_eager
    b = make_batch(rves)
    for rep in range(2):
        print(f"batch graph solve {rep}", flush=True)
        P, stats, st = b.newton_solve(CASES, make_opts(**OPTS), graph_ticks=5)
        F = batch_fields(b, rves)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 16, device=DEV, dtype=torch.float64).sum().item()  # eager work between solves
        assert np.isfinite(junk)
        assert np.array_equal(P, P0)
        for key in F0:
            assert np.array_equal(F[key], F0[key]), key
        for s, s0 in zip(stats, stats0):
            assert s["newton_iters"] == s0["newton_iters"]
            assert s["lin_iters_total"] == s0["lin_iters_total"]
    b.close()


@pytest.mark.parametrize("every,ticks", [(3, 0), (4, 8)])
def test_batch_schedule_does_not_change_results(rves, fp64_eager, every, ticks):
    """The Newton step every k-th step (direct launches or graph): the same
    bits, iteration counts unchanged."""
    P0, stats0, F0 = fp64_eager
    b = make_batch(rves)
    b.set_schedule(every)
    P, stats, st = b.newton_solve(CASES, make_opts(**OPTS), graph_ticks=ticks)
    F = batch_fields(b, rves)
    b.close()
    assert np.array_equal(P, P0)
    for key in F0:
        assert np.array_equal(F[key], F0[key]), key
    for s, s0 in zip(stats, stats0):
        assert s["newton_iters"] == s0["newton_iters"] and s["lin_iters_total"] == s0["lin_iters_total"]


def test_batch_mixed_matches_fp64(rves, fp64_eager):
    """Mixed form of the batch (FP32 CG operator, FP64 Newton residual)."""
    P0, stats0, F0 = fp64_eager
    b = make_batch(rves, "mixed")
    P, stats, st = b.newton_solve(CASES, make_opts(**OPTS), graph_ticks=8)
    F = batch_fields(b, rves)
    b.close()
    for k, r in enumerate(rves):
        for lc, Fbar in enumerate(CASES):
            s = stats[k * len(CASES) + lc]
            assert s["err_res"] <= 1e-10
            if lc == 2:
                continue
            fl = F0[k, lc] - mechanics.uniform_field(Fbar, r["shape"])
            e = rel(F[k, lc], F0[k, lc], fl)
            print(f"mixed rve={k} case={lc} newton {s['newton_iters']} rel {e:.2e}", flush=True)
            assert e <= 1e-6
            assert rel(P[k, lc], P0[k, lc]) <= 1e-6


def test_batch_needs_material(rves):
    b = Batch([r["shape"] for r in rves], [r["spacing"] for r in rves], len(CASES))
    with pytest.raises(FgError) as ei:
        b.newton_solve(CASES, make_opts(**OPTS))
    assert ei.value.code == FG_E_STATE
    b.close()
