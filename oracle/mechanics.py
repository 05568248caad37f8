"""Finite-strain Fourier-Galerkin equilibrium (Sec. 3.1 and Sec. 3.2,
Mechanical Equilibrium; Alg. 1 "Mechanical problem").

Unknown: the periodic fluctuation of F = Fbar + F~ (eq. (23)), <F> = Fbar
(eq. (24)).  Discrete system (eq. (30) [mechanicalsolve]):
    F^{-1}[ G^ : F[ K : dF ] ] = - F^{-1}[ G^ : F[ P(F) ] ],
linearised by Newton-Raphson with a CG inner solve for the zero-mean
correction dF, stopped on the equilibrium residual (eq. (31)
[mechresiduum])
    err_res = || G*P(F) || / || G*P(Fbar) ||.

Reading A8: the normaliser is max(||G*P(Fbar)||, 1e-14 ||P(Fbar)||, 1e-300),
which is finite for a homogeneous cell (where G*P(Fbar) = 0 exactly).
Reading A21: each load increment starts from F^0 = F_t + dFbar (Alg. 1,
first line), i.e. the previous fluctuation is kept.
Reading A31 (numerical): the CG right-hand side is projected a second time,
b = -G*(G*P).  G is idempotent, so this is the same vector in exact
arithmetic, but the FFT rounding of the first projection (~1e-16 ||P||) is
not compatible; once ||G*P|| falls to ~1e-8 ||P|| that inconsistent part
exceeds the CG tolerance and CG on G K diverges.  err_res uses the first
projection, as eq. (31) defines it.
"""
from __future__ import annotations

import numpy as np

from .constitutive import apply_tangent, law_of, stress, tangent
from .krylov import cg
from .spectral import project


class NoConvergence(RuntimeError):
    pass


def norm(a):
    return float(np.sqrt(np.sum(a * a)))


def uniform_field(Fbar, shape):
    return np.broadcast_to(np.asarray(Fbar, dtype=np.float64).reshape(3, 3, 1, 1, 1),
                           (3, 3) + tuple(shape)).copy()


def operator(K, X, spacing):
    """The Fourier-Galerkin operator  X -> F^{-1}[ G^ : F[ K : X ] ]."""
    return project(apply_tangent(K, X), spacing)


def residual_rhs(F, c, d, mat, spacing):
    """Equilibrium residual of eq. (30)/(31): returns (G*P(F), P)."""
    P = stress(F, c, d, mat["E"], mat["nu"], mat["Omega"], law_of(mat))
    return project(P, spacing), P


def err_denominator(Fbar, c, d, mat, spacing):
    shape = np.shape(c)
    Pbar = stress(uniform_field(Fbar, shape), c, d, mat["E"], mat["nu"], mat["Omega"], law_of(mat))
    GP = project(Pbar, spacing)
    return max(norm(GP), 1e-14 * norm(Pbar), 1e-300)


def newton_solve(F, Fbar, c, d, mat, spacing, tol_newton=1e-8, tol_lin=1e-10,
                 max_newton=50, max_lin=20000, fixed_lin=None):
    """Alg. 1 from the given initial iterate F (the caller has already added
    the macroscopic increment).  ``fixed_lin``: optional list of CG iteration
    counts, one per Newton iteration (parity runs with matched counts).

    Returns (F, stats) with stats = dict(newton_iters, lin_iters (list),
    err_history (list), den).
    """
    den = err_denominator(Fbar, c, d, mat, spacing)
    lin_iters, errs = [], []
    it = 0
    while True:
        GP, P = residual_rhs(F, c, d, mat, spacing)
        err = norm(GP) / den
        errs.append(err)
        if err <= tol_newton:
            break
        if it >= max_newton:
            raise NoConvergence("Newton did not converge")
        b = -project(GP, spacing)
        K = tangent(F, c, d, mat["E"], mat["nu"], mat["Omega"], law_of(mat))
        fixed = None if fixed_lin is None else fixed_lin[it]
        dF, n, _ = cg(lambda X: operator(K, X, spacing), b, tol_lin, max_lin,
                      fixed_iters=fixed)
        lin_iters.append(n)
        F = F + dF
        it += 1
    return F, dict(newton_iters=it, lin_iters=lin_iters, err_history=errs, den=den)


def solve_increments(work, loads=None, F=None, c=None, d=None, **kw):
    """Apply the load schedule (list of macro F) increment by increment,
    each increment by :func:`newton_solve` from F_t + dFbar.  Returns
    (F, list of per-increment stats)."""
    shape = work["shape"]
    loads = work["loads"] if loads is None else loads
    c = work["c0"] if c is None else c
    d = work["d0"] if d is None else d
    Fprev = np.eye(3)
    F = uniform_field(Fprev, shape) if F is None else F
    stats = []
    for Fbar in loads:
        F = F + uniform_field(np.asarray(Fbar) - Fprev, shape)
        F, st = newton_solve(F, Fbar, c, d, work, work["spacing"], **kw)
        stats.append(st)
        Fprev = np.asarray(Fbar)
    return F, stats


def mean_stress(F, c, d, mat):
    """Homogenised (voxel-mean) first Piola-Kirchhoff stress <P>."""
    P = stress(F, c, d, mat["E"], mat["nu"], mat["Omega"], law_of(mat))
    return P.reshape(3, 3, -1).mean(axis=-1)


def homogenized_tangent(F, c, d, mat, W, tol_lin=1e-12, maxit=20000):
    """The homogenised tangent applied to a macroscopic direction W (3x3):
    d<P>/dFbar : W at the converged state F.  A uniform change W of Fbar
    changes the fluctuation by the compatible, zero-mean dF solving the
    linearised equilibrium of eq. (30),
        G*(K : dF) = -G*(K : W),
    and then d<P> = <K : (W + dF)>.  Returns (3x3 array, CG iterations)."""
    spacing = mat["spacing"]
    shape = F.shape[2:]
    K = tangent(F, c, d, mat["E"], mat["nu"], mat["Omega"], law_of(mat))
    Wf = uniform_field(W, shape)
    b = -project(project(apply_tangent(K, Wf), spacing), spacing)
    dF, it, _ = cg(lambda X: operator(K, X, spacing), b, tol_lin, maxit)
    T = apply_tangent(K, Wf + dF)
    return T.reshape(3, 3, -1).mean(axis=-1), it


def project_mixed(A, mask, spacing):
    """Projection of the mixed macroscopic control: the compatibility
    projection of eq. (28) on the fluctuation, plus, at zero frequency, the
    mean of the stress-controlled components (mask: 3x3 booleans, True where
    <P>_ij is prescribed and Fbar_ij is free).  Idempotent and symmetric,
    like the projection itself."""
    shape = A.shape[2:]
    m = np.asarray(mask, dtype=np.float64).reshape(3, 3, 1, 1, 1)
    mean = A.reshape(3, 3, -1).mean(axis=-1).reshape(3, 3, 1, 1, 1)
    return project(A, spacing) + np.broadcast_to(m * mean, (3, 3) + tuple(shape))


def newton_solve_mixed(F, Fbar, mask, Pbar, c, d, mat, spacing, tol_newton=1e-8, tol_lin=1e-10, max_newton=50,
                       max_lin=20000):
    """Alg. 1 under mixed macroscopic control (Sec. 3.1: Fbar prescribed in
    some components, <P> in the others; reading of the cited mixed-control
    approach as the zero-frequency extension of the projection): the mean of
    F is Fbar where mask is False (the caller's F already has it) and free
    where mask is True; there <P> = Pbar is required.  Residual
        R = G_m*(P) - mask Pbar,   G_m = project_mixed,
    normalised by its value at the entry state; Newton with CG on
    X -> G_m*(K : X) (self-adjoint on the range of G_m).  Returns (F, stats)."""
    m = np.asarray(mask, dtype=np.float64).reshape(3, 3, 1, 1, 1)
    target = m * np.asarray(Pbar, dtype=np.float64).reshape(3, 3, 1, 1, 1)
    shape = F.shape[2:]
    lin_iters, errs = [], []
    den = None
    it = 0
    while True:
        P = stress(F, c, d, mat["E"], mat["nu"], mat["Omega"], law_of(mat))
        R = project_mixed(P, mask, spacing) - np.broadcast_to(target, (3, 3) + tuple(shape))
        nr = norm(R)
        if den is None:
            den = max(nr, 1e-14 * norm(P), 1e-300)
        err = nr / den
        errs.append(err)
        if err <= tol_newton:
            break
        if it >= max_newton:
            raise NoConvergence("mixed-control Newton did not converge")
        b = -project_mixed(R, mask, spacing)
        K = tangent(F, c, d, mat["E"], mat["nu"], mat["Omega"], law_of(mat))
        dF, n, _ = cg(lambda X: project_mixed(apply_tangent(K, X), mask, spacing), b, tol_lin, max_lin)
        lin_iters.append(n)
        F = F + dF
        it += 1
    return F, dict(newton_iters=it, lin_iters=lin_iters, err_history=errs, den=den)
