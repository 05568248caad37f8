"""GPU adjoint (d<P_11>/d(log E, Omega), derived from eq. (30)) against the
oracle's adjoint, finite differences by difference solves and the exact
scaling invariant sum_x dL/dlogE = L; and the torch.autograd wrapper."""
import numpy as np
import pytest
import torch

import synth
from oracle import adjoint, mechanics
from paper_2411_16583_amd import Plan, make_opts
from paper_2411_16583_amd.autograd import homogenized_stress
from tests.gpu_util import DEV, dt, host, plan_for, rel

pytestmark = pytest.mark.gpu


def _converged(n):
    w = synth.grf_workload(n=n)
    Fbar = w["loads"][0]
    F = mechanics.uniform_field(Fbar, w["shape"])
    F, _ = mechanics.newton_solve(F, Fbar, w["c0"], w["d0"], w, w["spacing"], tol_newton=1e-12, tol_lin=1e-12)
    return w, F


@pytest.mark.parametrize("n", [8, 16])
def test_adjoint_matches_oracle_and_invariant(n):
    w, F = _converged(n)
    shape = w["shape"]
    plan = plan_for(w)
    Ft = dt(mechanics.uniform_field(np.eye(3), shape))
    plan.set_state(Ft, dt(w["c0"]), dt(w["d0"]), dt(np.zeros(shape)))
    plan.newton_solve(w["loads"][0], make_opts(1e-12, 1e-12))
    gE = torch.empty(shape, dtype=torch.float64, device=DEV)
    gO = torch.empty(shape, dtype=torch.float64, device=DEV)
    W = np.zeros((3, 3))
    W[0, 0] = 1.0
    st = plan.adjoint_gradient(W, gE, gO, make_opts(1e-12, 1e-12))
    oE, oO, it = adjoint.adjoint_gradient(F, w["c0"], w["d0"], w, tol_lin=1e-12)
    print(f"adjoint n={n}: cg gpu {st['lin_iters_last']} oracle {it}", flush=True)
    assert rel(host(gE), oE) <= 1e-9
    assert rel(host(gO), oO) <= 1e-9
    L = plan.homogenized_stress()[0, 0]
    assert abs(host(gE).sum() - L) <= 1e-9 * abs(L)


def test_adjoint_vs_finite_differences():
    w, F = _converged(8)
    shape = w["shape"]
    plan = plan_for(w)
    plan.set_state(dt(mechanics.uniform_field(np.eye(3), shape)), dt(w["c0"]), dt(w["d0"]), dt(np.zeros(shape)))
    plan.newton_solve(w["loads"][0], make_opts(1e-12, 1e-12))
    gE = torch.empty(shape, dtype=torch.float64, device=DEV)
    gO = torch.empty(shape, dtype=torch.float64, device=DEV)
    W = np.zeros((3, 3))
    W[0, 0] = 1.0
    plan.adjoint_gradient(W, gE, gO, make_opts(1e-12, 1e-12))
    gE, gO = host(gE).ravel(), host(gO).ravel()
    rng = np.random.default_rng(300)
    for v in rng.integers(0, gE.size, size=3):
        fdE = adjoint.fd_gradient(F, w["c0"], w["d0"], w, int(v), "logE", 1e-3)
        fdO = adjoint.fd_gradient(F, w["c0"], w["d0"], w, int(v), "Omega", 1e-4)
        assert abs(gE[v] - fdE) <= 1e-5 * (abs(fdE) + np.sqrt(np.mean(gE ** 2)))
        assert abs(gO[v] - fdO) <= 1e-5 * (abs(fdO) + np.sqrt(np.mean(gO ** 2)))


def test_autograd_wrapper_matches_c_abi():
    w, F = _converged(8)
    shape = w["shape"]
    plan = Plan(shape, w["spacing"], "fp64")
    logE = dt(np.log(w["E"])).requires_grad_(True)
    Om = dt(w["Omega"]).requires_grad_(True)
    P = homogenized_stress(plan, logE, Om, dt(w["nu"]), w["loads"][0], c=dt(w["c0"]),
                           material=dict(gc=w["gc"], lc=w["lc"], RT=w["RT"], c_max=w["c_max"]))
    Po = mechanics.mean_stress(F, w["c0"], w["d0"], w)
    assert np.max(np.abs(P.detach().numpy() - Po)) <= 1e-10 * np.abs(Po).max()
    P[0, 0].backward()
    oE, oO, _ = adjoint.adjoint_gradient(F, w["c0"], w["d0"], w, tol_lin=1e-12)
    assert rel(host(logE.grad), oE) <= 1e-8
    assert rel(host(Om.grad), oO) <= 1e-8


@pytest.mark.parametrize("n", [8, 16])
def test_mixed_adjoint_matches_oracle_and_invariant(n):
    """Mixed plan: Newton and the adjoint refined in double precision around
    single-precision CG corrections; gradients within the mixed-form bound
    (1e-6) of the oracle, and the scaling invariant."""
    w, F = _converged(n)
    shape = w["shape"]
    plan = plan_for(w, "mixed")
    plan.set_state(dt(mechanics.uniform_field(np.eye(3), shape)), dt(w["c0"]), dt(w["d0"]), dt(np.zeros(shape)))
    plan.newton_solve(w["loads"][0], make_opts(1e-10, 1e-12))
    gE = torch.empty(shape, dtype=torch.float64, device=DEV)
    gO = torch.empty(shape, dtype=torch.float64, device=DEV)
    W = np.zeros((3, 3))
    W[0, 0] = 1.0
    st = plan.adjoint_gradient(W, gE, gO, make_opts(1e-12, 1e-12))
    oE, oO, it = adjoint.adjoint_gradient(F, w["c0"], w["d0"], w, tol_lin=1e-12)
    eE, eO = rel(host(gE), oE), rel(host(gO), oO)
    print(f"mixed adjoint n={n}: refinements {st['newton_iters']} cg {st['lin_iters_total']} "
          f"relres {st['lin_relres']:.1e} rel logE {eE:.1e} Omega {eO:.1e}", flush=True)
    assert st["newton_iters"] >= 1 and st["lin_relres"] <= 1e-12
    assert eE <= 1e-6 and eO <= 1e-6
    L = plan.homogenized_stress()[0, 0]
    assert abs(host(gE).sum() - L) <= 1e-9 * abs(L)


def test_mixed_adjoint_vs_finite_differences():
    w, F = _converged(8)
    shape = w["shape"]
    plan = plan_for(w, "mixed")
    plan.set_state(dt(mechanics.uniform_field(np.eye(3), shape)), dt(w["c0"]), dt(w["d0"]), dt(np.zeros(shape)))
    plan.newton_solve(w["loads"][0], make_opts(1e-10, 1e-12))
    gE = torch.empty(shape, dtype=torch.float64, device=DEV)
    gO = torch.empty(shape, dtype=torch.float64, device=DEV)
    W = np.zeros((3, 3))
    W[0, 0] = 1.0
    plan.adjoint_gradient(W, gE, gO, make_opts(1e-12, 1e-12))
    gE, gO = host(gE).ravel(), host(gO).ravel()
    rng = np.random.default_rng(301)
    for v in rng.integers(0, gE.size, size=3):
        fdE = adjoint.fd_gradient(F, w["c0"], w["d0"], w, int(v), "logE", 1e-3)
        fdO = adjoint.fd_gradient(F, w["c0"], w["d0"], w, int(v), "Omega", 1e-4)
        assert abs(gE[v] - fdE) <= 1e-5 * (abs(fdE) + np.sqrt(np.mean(gE ** 2)))
        assert abs(gO[v] - fdO) <= 1e-5 * (abs(fdO) + np.sqrt(np.mean(gO ** 2)))


def test_autograd_wrapper_mixed_plan():
    w, F = _converged(8)
    shape = w["shape"]
    plan = Plan(shape, w["spacing"], "mixed")
    logE = dt(np.log(w["E"])).requires_grad_(True)
    Om = dt(w["Omega"]).requires_grad_(True)
    P = homogenized_stress(plan, logE, Om, dt(w["nu"]), w["loads"][0], c=dt(w["c0"]),
                           material=dict(gc=w["gc"], lc=w["lc"], RT=w["RT"], c_max=w["c_max"]))
    Po = mechanics.mean_stress(F, w["c0"], w["d0"], w)
    assert np.max(np.abs(P.detach().numpy() - Po)) <= 1e-6 * np.abs(Po).max()
    P[0, 0].backward()
    oE, oO, _ = adjoint.adjoint_gradient(F, w["c0"], w["d0"], w, tol_lin=1e-12)
    assert rel(host(logE.grad), oE) <= 1e-6
    assert rel(host(Om.grad), oO) <= 1e-6
