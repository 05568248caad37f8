"""ctypes binding of libfgfft.so (include/fgfft.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides device memory (the workspace and the fields are CUDA/HIP
tensors owned by the caller) and the stream.  The library is loaded from the
package directory; importing this module on a machine where it is missing
raises immediately (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfgfft.so")

FG_OK, FG_E_ARG, FG_E_SIZE, FG_E_HIP, FG_E_NOCONV, FG_E_BREAKDOWN, FG_E_DOMAIN, FG_E_STATE = range(8)
FG_FP64, FG_MIXED = 0, 1
PRECISIONS = {"fp64": FG_FP64, "mixed": FG_MIXED}
FG_LAW_NEO_HOOKE, FG_LAW_SVK = 0, 1
LAWS = {"neo_hookean": FG_LAW_NEO_HOOKE, "svk": FG_LAW_SVK}

# Every function declared in include/fgfft.h.
EXPORTED = [
    "fg_plan_create", "fg_plan_workspace_bytes", "fg_plan_set_workspace", "fg_set_law", "fg_set_material",
    "fg_set_state", "fg_apply_macro", "fg_newton_solve", "fg_newton_solve_shifted", "fg_newton_linear_begin", "fg_cg_iterate",
    "fg_adjoint_gradient", "fg_homogenized_tangent", "fg_residual", "fg_homogenized_stress", "fg_stress",
    "fg_apply_operator", "fg_project", "fg_project_noalloc", "fg_project_grad", "fg_fft_r2c", "fg_fft_c2r", "pff_solve", "fick_step", "fick_step_full",
    "fg_batch_create", "fg_batch_workspace_bytes", "fg_batch_groups", "fg_batch_set_workspace",
    "fg_batch_set_material", "fg_batch_newton_solve", "fg_batch_state", "fg_batch_last_error", "fg_batch_destroy",
    "fg_batch_plan", "fg_batch_group_info", "fg_batch_set_schedule", "fg_plan_tile_candidates", "fg_plan_set_tiles", "fg_plan_get_tiles",
    "fg_plan_time_pass",
    "fg_profile_begin", "fg_profile_end", "fg_profile_passes", "fg_status_string", "fg_last_error",
    "fg_plan_destroy",
]
PASS_NAMES = ["front", "r2c", "axis", "zproj", "c2r", "cg_update", "finalize", "constitutive", "zscalar", "axis3",
              "c2r3", "grad"]


class SolverOpts(ctypes.Structure):
    _fields_ = [
        ("tol_newton", ctypes.c_double),
        ("tol_lin", ctypes.c_double),
        ("max_newton", ctypes.c_int),
        ("max_lin", ctypes.c_int),
        ("fixed_lin", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("newton_iters", ctypes.c_int),
        ("lin_iters_total", ctypes.c_int),
        ("lin_iters_last", ctypes.c_int),
        ("n_history", ctypes.c_int),
        ("err_res", ctypes.c_double),
        ("lin_relres", ctypes.c_double),
        ("err_history", ctypes.c_double * 64),
        ("lin_history", ctypes.c_int * 64),
    ]

    def to_dict(self):
        n = min(self.n_history, 64)
        return dict(
            newton_iters=self.newton_iters,
            lin_iters_total=self.lin_iters_total,
            lin_iters_last=self.lin_iters_last,
            err_res=self.err_res,
            lin_relres=self.lin_relres,
            err_history=list(self.err_history[:n]),
            lin_history=list(self.lin_history[: min(self.newton_iters, 64)]) if self.newton_iters else
            list(self.lin_history[:n]),
        )


class FgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def load_library(path=LIB_PATH):
    """Load libfgfft.so and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2411_16583_amd.build`")
    lib = ctypes.CDLL(path)
    vp, c_int, c_double, c_size = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    dptr = ctypes.c_void_p
    sig = {
        "fg_plan_create": ([ctypes.POINTER(c_int), ctypes.POINTER(c_double), c_int, vp, ctypes.POINTER(vp)], c_int),
        "fg_plan_workspace_bytes": ([vp], c_size),
        "fg_plan_set_workspace": ([vp, vp, c_size], c_int),
        "fg_set_law": ([vp, c_int], c_int),
        "fg_set_material": ([vp, dptr, dptr, dptr, dptr, dptr, c_double, c_double, c_double, c_double], c_int),
        "fg_set_state": ([vp, dptr, dptr, dptr, dptr], c_int),
        "fg_apply_macro": ([vp, ctypes.POINTER(c_double)], c_int),
        "fg_newton_solve": ([vp, ctypes.POINTER(c_double), ctypes.POINTER(SolverOpts), ctypes.POINTER(Stats)], c_int),
        "fg_newton_solve_shifted": ([vp, dptr, ctypes.POINTER(SolverOpts), ctypes.POINTER(Stats)], c_int),
        "fg_newton_linear_begin": ([vp, ctypes.POINTER(c_double), ctypes.POINTER(c_double)], c_int),
        "fg_cg_iterate": ([vp, c_int, c_int, ctypes.POINTER(Stats)], c_int),
        "fg_adjoint_gradient": ([vp, ctypes.POINTER(c_double), dptr, dptr, ctypes.POINTER(SolverOpts),
                                 ctypes.POINTER(Stats)], c_int),
        "fg_homogenized_tangent": ([vp, ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                    ctypes.POINTER(SolverOpts), ctypes.POINTER(Stats)], c_int),
        "fg_residual": ([vp, ctypes.POINTER(c_double), ctypes.POINTER(c_double)], c_int),
        "fg_homogenized_stress": ([vp, ctypes.POINTER(c_double)], c_int),
        "fg_stress": ([vp, dptr], c_int),
        "fg_apply_operator": ([vp, dptr, dptr], c_int),
        "fg_project": ([vp, dptr, dptr], c_int),
        "fg_project_grad": ([vp, dptr, dptr], c_int),
        "fg_project_noalloc": ([ctypes.POINTER(c_int), ctypes.POINTER(c_double), dptr, dptr, vp], c_int),
        "fg_fft_r2c": ([vp, dptr, c_int], c_int),
        "fg_fft_c2r": ([vp, dptr, c_int], c_int),
        "pff_solve": ([vp, ctypes.POINTER(SolverOpts), ctypes.POINTER(Stats)], c_int),
        "fick_step": ([vp, c_double, dptr, ctypes.POINTER(SolverOpts), ctypes.POINTER(Stats)], c_int),
        "fick_step_full": ([vp, c_double, dptr, ctypes.POINTER(SolverOpts), ctypes.POINTER(Stats)], c_int),
        "fg_profile_begin": ([vp], c_int),
        "fg_profile_passes": ([vp, ctypes.c_uint], c_int),
        "fg_profile_end": ([vp, ctypes.POINTER(c_double), ctypes.POINTER(ctypes.c_long)], c_int),
        "fg_status_string": ([c_int], ctypes.c_char_p),
        "fg_last_error": ([vp], ctypes.c_char_p),
        "fg_plan_destroy": ([vp], None),
        "fg_batch_create": ([c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_double), c_int, c_int, vp,
                             ctypes.POINTER(vp)], c_int),
        "fg_batch_workspace_bytes": ([vp], c_size),
        "fg_batch_groups": ([vp], c_int),
        "fg_batch_set_workspace": ([vp, vp, c_size], c_int),
        "fg_batch_set_material": ([vp, c_int, dptr, dptr, dptr, dptr], c_int),
        "fg_batch_newton_solve": ([vp, ctypes.POINTER(c_double), ctypes.POINTER(SolverOpts), c_int,
                                   ctypes.POINTER(c_double), ctypes.POINTER(Stats)], c_int),
        "fg_batch_state": ([vp, c_int, c_int, dptr], c_int),
        "fg_batch_last_error": ([vp], ctypes.c_char_p),
        "fg_batch_destroy": ([vp], None),
        "fg_batch_plan": ([vp, c_int], vp),
        "fg_batch_set_schedule": ([vp, c_int], c_int),
        "fg_batch_group_info": ([vp, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int)], c_int),
        "fg_plan_tile_candidates": ([vp, c_int, ctypes.POINTER(c_int), c_int], c_int),
        "fg_plan_set_tiles": ([vp, ctypes.POINTER(c_int)], c_int),
        "fg_plan_get_tiles": ([vp, ctypes.POINTER(c_int)], c_int),
        "fg_plan_time_pass": ([vp, c_int, c_int, c_int, ctypes.POINTER(c_double)], c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t):
    """Device pointer of a contiguous float64 CUDA tensor (or None)."""
    if t is None:
        return None
    import torch

    if not t.is_cuda:
        raise ValueError("fields must be device tensors")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("fields must be contiguous float64 tensors")
    return ctypes.c_void_p(t.data_ptr())


def _mat9(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(9))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def project_noalloc(grid, spacing, x, y, stream=None):
    """fg_project_noalloc: y = G * x on the given grid without a plan (the
    library's fixed device array holds the tables and the spectrum)."""
    import torch

    lib = load_library()
    if stream is None:
        stream = torch.cuda.current_stream()
    g = (ctypes.c_int * 3)(*[int(n) for n in grid])
    h = (ctypes.c_double * 3)(*[float(v) for v in spacing])
    st = lib.fg_project_noalloc(g, h, _ptr(x), _ptr(y), ctypes.c_void_p(stream.cuda_stream))
    if st != FG_OK:
        raise FgError(st, f"fg_project_noalloc{tuple(grid)}: {lib.fg_status_string(st).decode()}")
    return y


def make_opts(tol_newton=1e-8, tol_lin=1e-10, max_newton=50, max_lin=20000, fixed_lin=0):
    return SolverOpts(tol_newton, tol_lin, max_newton, max_lin, fixed_lin)


class Plan:
    """One grid / precision / stream.  Holds references to every tensor it
    was given so that their memory outlives the plan's use of it."""

    def __init__(self, grid, spacing, precision="fp64", stream=None, device="cuda", law="neo_hookean"):
        import torch

        if law not in LAWS:
            raise ValueError(f"unknown law {law!r}; one of {sorted(LAWS)}")
        self.lib = load_library()
        self.law = law
        self.grid = tuple(int(n) for n in grid)
        self.spacing = tuple(float(h) for h in spacing)
        self.N = int(np.prod(self.grid))
        self.precision = precision
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        g = (ctypes.c_int * 3)(*self.grid)
        h = (ctypes.c_double * 3)(*self.spacing)
        out = ctypes.c_void_p()
        st = self.lib.fg_plan_create(g, h, PRECISIONS[precision], ctypes.c_void_p(stream.cuda_stream),
                                     ctypes.byref(out))
        if st != FG_OK:
            raise FgError(st, f"fg_plan_create{self.grid}: {self.lib.fg_status_string(st).decode()}")
        self.handle = out
        if law != "neo_hookean":
            self._check(self.lib.fg_set_law(self.handle, LAWS[law]), "fg_set_law")
        nbytes = int(self.lib.fg_plan_workspace_bytes(self.handle))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self._check(self.lib.fg_plan_set_workspace(self.handle, ctypes.c_void_p(self.workspace.data_ptr()),
                                                    nbytes), "fg_plan_set_workspace")
        self._keep = {}

    def _check(self, st, what):
        if st != FG_OK:
            msg = self.lib.fg_last_error(self.handle).decode() if self.handle else ""
            raise FgError(st, f"{what}: {self.lib.fg_status_string(st).decode()}: {msg}")

    def close(self):
        if getattr(self, "handle", None):
            self.lib.fg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_material(self, E, nu, Omega, D=None, sigma_max=None, gc=1.0, lc=1.0, RT=2478.957, c_max=3.0e4):
        self._keep.update(E=E, nu=nu, Omega=Omega, D=D, sigma_max=sigma_max)
        self._check(self.lib.fg_set_material(self.handle, _ptr(E), _ptr(nu), _ptr(Omega), _ptr(D), _ptr(sigma_max),
                                             gc, lc, RT, c_max), "fg_set_material")

    def set_state(self, F, c=None, d=None, H=None):
        self._keep.update(F=F, c=c, d=d, H=H)
        self._check(self.lib.fg_set_state(self.handle, _ptr(F), _ptr(c), _ptr(d), _ptr(H)), "fg_set_state")

    def newton_solve(self, F_macro, opts=None, raise_on_error=True):
        opts = opts or make_opts()
        a, p = _mat9(F_macro)
        stats = Stats()
        st = self.lib.fg_newton_solve(self.handle, p, ctypes.byref(opts), ctypes.byref(stats))
        if raise_on_error:
            self._check(st, "fg_newton_solve")
        d = stats.to_dict()
        d["status"] = st
        return d

    def newton_solve_shifted(self, B, opts=None):
        """Newton on G*(P(F) - B) = 0 from the current F (difference solves)."""
        opts = opts or make_opts()
        stats = Stats()
        self._check(self.lib.fg_newton_solve_shifted(self.handle, _ptr(B), ctypes.byref(opts), ctypes.byref(stats)),
                    "fg_newton_solve_shifted")
        return stats.to_dict()

    def newton_linear_begin(self, F_macro):
        """P, tangent and the CG right-hand side of one Newton correction at
        the current F; returns err_res (eq. (31))."""
        a, p = _mat9(F_macro)
        out = ctypes.c_double()
        self._check(self.lib.fg_newton_linear_begin(self.handle, p, ctypes.byref(out)), "fg_newton_linear_begin")
        return out.value

    def cg_iterate(self, n, apply=False):
        """Exactly n more CG iterations of the open Newton system; apply=True
        then adds the CG iterate to F and closes the system."""
        stats = Stats()
        self._check(self.lib.fg_cg_iterate(self.handle, int(n), 1 if apply else 0, ctypes.byref(stats)),
                    "fg_cg_iterate")
        return dict(iters=stats.lin_iters_last, relres=stats.lin_relres)

    def adjoint_gradient(self, dL_dPavg, g_logE=None, g_Omega=None, opts=None):
        """Per-voxel d L / d log E and d L / d Omega of L = sum w_ij <P_ij> into
        the given device tensors (N doubles each)."""
        opts = opts or make_opts()
        a, p = _mat9(dL_dPavg)
        stats = Stats()
        self._check(self.lib.fg_adjoint_gradient(self.handle, p, _ptr(g_logE), _ptr(g_Omega), ctypes.byref(opts),
                                                 ctypes.byref(stats)), "fg_adjoint_gradient")
        return stats.to_dict()

    def homogenized_tangent(self, W, opts=None):
        """d<P>/dFbar : W at the current converged state (3x3 array)."""
        opts = opts or make_opts()
        a, p = _mat9(W)
        out = (ctypes.c_double * 9)()
        stats = Stats()
        self._check(self.lib.fg_homogenized_tangent(self.handle, p, out, ctypes.byref(opts), ctypes.byref(stats)),
                    "fg_homogenized_tangent")
        return np.array(out[:]).reshape(3, 3)

    def apply_macro(self, F_macro):
        a, p = _mat9(F_macro)
        self._check(self.lib.fg_apply_macro(self.handle, p), "fg_apply_macro")

    def residual(self, F_macro):
        a, p = _mat9(F_macro)
        out = ctypes.c_double()
        self._check(self.lib.fg_residual(self.handle, p, ctypes.byref(out)), "fg_residual")
        return out.value

    def homogenized_stress(self):
        out = (ctypes.c_double * 9)()
        self._check(self.lib.fg_homogenized_stress(self.handle, out), "fg_homogenized_stress")
        return np.array(out[:]).reshape(3, 3)

    def stress(self, out):
        self._check(self.lib.fg_stress(self.handle, _ptr(out)), "fg_stress")
        return out

    def apply_operator(self, x, y):
        self._check(self.lib.fg_apply_operator(self.handle, _ptr(x), _ptr(y)), "fg_apply_operator")
        return y

    def project(self, x, y):
        self._check(self.lib.fg_project(self.handle, _ptr(x), _ptr(y)), "fg_project")
        return y

    def project_grad(self, x, y):
        self._check(self.lib.fg_project_grad(self.handle, _ptr(x), _ptr(y)), "fg_project_grad")
        return y

    def fft_r2c(self, data, ncomp):
        self._check(self.lib.fg_fft_r2c(self.handle, _ptr(data), int(ncomp)), "fg_fft_r2c")
        return data

    def fft_c2r(self, data, ncomp):
        self._check(self.lib.fg_fft_c2r(self.handle, _ptr(data), int(ncomp)), "fg_fft_c2r")
        return data

    def pff_solve(self, opts=None, raise_on_error=True):
        opts = opts or make_opts()
        stats = Stats()
        st = self.lib.pff_solve(self.handle, ctypes.byref(opts), ctypes.byref(stats))
        if raise_on_error:
            self._check(st, "pff_solve")
        d = stats.to_dict()
        d["status"] = st
        return d

    def autotune(self, cache_path=None, reps=10, force=False):
        """Pick the tile widths of the column passes by timing them on this
        plan (cached per architecture, grid and pass)."""
        from .autotune import tune_plan

        return tune_plan(self, cache_path, reps, force)

    def tiles(self):
        from .autotune import get_tiles

        return get_tiles(self.handle, self.lib)

    def set_tiles(self, tiles):
        self._check(self.lib.fg_plan_set_tiles(self.handle, (ctypes.c_int * 4)(*[int(t) for t in tiles])),
                    "fg_plan_set_tiles")

    def profile_begin(self, passes=None):
        """Start timing the kernel classes named in passes (PASS_NAMES;
        default: all of them)."""
        mask = 0xFFFFFFFF if passes is None else sum(1 << PASS_NAMES.index(p) for p in passes)
        self._check(self.lib.fg_profile_passes(self.handle, mask), "fg_profile_passes")
        self._check(self.lib.fg_profile_begin(self.handle), "fg_profile_begin")

    def profile_end(self):
        n = len(PASS_NAMES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_long * n)()
        self._check(self.lib.fg_profile_end(self.handle, ms, cnt), "fg_profile_end")
        return {name: (ms[k], cnt[k]) for k, name in enumerate(PASS_NAMES)}

    def fick_step(self, dt, cdot_B=None, opts=None, raise_on_error=True, jacobian="mu_c"):
        """Alg. 3 (jacobian="mu_c", the paper's linearisation) or its fully
        implicit form (jacobian="full", fick_step_full)."""
        opts = opts or make_opts()
        stats = Stats()
        self._keep["cdot_B"] = cdot_B
        fn = self.lib.fick_step_full if jacobian == "full" else self.lib.fick_step
        st = fn(self.handle, float(dt), _ptr(cdot_B), ctypes.byref(opts), ctypes.byref(stats))
        if raise_on_error:
            self._check(st, "fick_step")
        d = stats.to_dict()
        d["status"] = st
        return d


class Batch:
    """Batched Newton solves (fg_batch_*): RVEs of any supported grids times
    macroscopic load cases.  Owns its workspace tensor; material arrays are
    copied into the batch by set_material."""

    def __init__(self, grids, spacings, n_cases, precision="fp64", stream=None, device="cuda"):
        import torch

        self.lib = load_library()
        self.grids = [tuple(int(n) for n in g) for g in grids]
        self.spacings = [tuple(float(h) for h in s) for s in spacings]
        if len(self.grids) != len(self.spacings) or not self.grids:
            raise ValueError("one grid and one spacing per RVE")
        self.n_rve = len(self.grids)
        self.n_cases = int(n_cases)
        self.precision = precision
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        g = (ctypes.c_int * (3 * self.n_rve))(*[n for gr in self.grids for n in gr])
        h = (ctypes.c_double * (3 * self.n_rve))(*[x for sp in self.spacings for x in sp])
        out = ctypes.c_void_p()
        st = self.lib.fg_batch_create(self.n_rve, g, h, self.n_cases, PRECISIONS[precision],
                                      ctypes.c_void_p(stream.cuda_stream), ctypes.byref(out))
        if st != FG_OK:
            raise FgError(st, f"fg_batch_create: {self.lib.fg_status_string(st).decode()}")
        self.handle = out
        nbytes = int(self.lib.fg_batch_workspace_bytes(self.handle))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self._check(self.lib.fg_batch_set_workspace(self.handle, ctypes.c_void_p(self.workspace.data_ptr()),
                                                     nbytes), "fg_batch_set_workspace")

    @property
    def n_groups(self):
        return int(self.lib.fg_batch_groups(self.handle))

    def _check(self, st, what):
        if st != FG_OK:
            msg = self.lib.fg_batch_last_error(self.handle).decode() if self.handle else ""
            raise FgError(st, f"{what}: {self.lib.fg_status_string(st).decode()}: {msg}")

    def close(self):
        if getattr(self, "handle", None):
            self.lib.fg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_material(self, rve, E, nu, Omega, c=None):
        self._check(self.lib.fg_batch_set_material(self.handle, int(rve), _ptr(E), _ptr(nu), _ptr(Omega), _ptr(c)),
                    "fg_batch_set_material")

    def newton_solve(self, F_macro, opts=None, graph_ticks=16, raise_on_error=True):
        """Solve every (RVE, case) item.  F_macro: n_cases 3x3 tensors.
        Returns (P_avg [n_rve, n_cases, 3, 3], list of per-item stats dicts
        (rve-major), status)."""
        opts = opts or make_opts()
        Fm = np.ascontiguousarray(np.asarray(F_macro, dtype=np.float64).reshape(self.n_cases * 9))
        P = np.zeros(self.n_rve * self.n_cases * 9)
        stats = (Stats * (self.n_rve * self.n_cases))()
        dp = ctypes.POINTER(ctypes.c_double)
        st = self.lib.fg_batch_newton_solve(self.handle, Fm.ctypes.data_as(dp), ctypes.byref(opts), int(graph_ticks),
                                            P.ctypes.data_as(dp), stats)
        if raise_on_error:
            self._check(st, "fg_batch_newton_solve")
        return P.reshape(self.n_rve, self.n_cases, 3, 3), [s.to_dict() for s in stats], st

    def set_schedule(self, newton_every):
        self._check(self.lib.fg_batch_set_schedule(self.handle, int(newton_every)), "fg_batch_set_schedule")

    def autotune(self, cache_path=None, reps=10, force=False):
        from .autotune import tune_batch

        return tune_batch(self, cache_path, reps, force)

    def state(self, rve, lcase, out):
        self._check(self.lib.fg_batch_state(self.handle, int(rve), int(lcase), _ptr(out)), "fg_batch_state")
        return out
