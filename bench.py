"""Benchmark: voxel CG-iterations per second of the Fourier-Galerkin hot path
at 256^3 (double precision and the mixed form) and the HBM-roofline fraction
of the dominant kernel, on one MI355X.

Workload: the polydisperse microstructure (256^3 unit cell, 60 seeded RSA
spheres with radii U(10, 24) voxels, stiffness contrast 20) at the state of
its first load increment (macroscopic stretch 1.0025 along e1).  One "step"
is one CG iteration of the linear system of the first Newton correction
(eq. (30) with the tangent at F = Fbar): the matvec (fused contraction and
N2 transform, N1 pass, N0 pass with the projection, inverse passes of the
potential) and the CG updates and FP64 reductions.  Warmup iterations run
first, untimed; then exactly --steps iterations are timed between two
device synchronisations.  The system is assembled before the warmup.

value = voxels x timed CG iterations / wall time of those iterations (FP64).
The mixed form's figures are reported alongside, together with one complete
Newton solve of the increment in each form (end-to-end time to Newton 1e-8,
CG 1e-10, and the mixed form's field error against the FP64 solution).
The roofline object refers to the kernel class with the largest time in the
warmup (the fused front kernel); its average launch duration comes from HIP
events taken by the kernel launches themselves during the timed iterations.

    python bench.py [--gpus 1] [--steps 40] [--warmup 5] [--n 256] [--no-cpu]
    python bench.py --ramp [--steps 2] [--warmup 1]   (staggered load increments with damage)
    python bench.py --batch [--batch-items 48] [--graph-ticks 16]   (batched form)
    python bench.py --coupled [--steps 3] [--warmup 1]   (coupled path, particle 128^3)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

# Algorithmic bytes per voxel and launch for each kernel class of the
# mechanics CG iteration, in words of the working precision (9-component
# fields; the spectrum occupies the same bytes as the real field).
WORDS_PER_VOXEL = {
    "front": 36,      # read rho, pi, xi (9) + state (12); write xi, pi (6), spectrum (9)
    "axis": 15,       # N1 pass of the 9-component spectrum: read 9, write 6 (2 merged fields per row)
    "zproj": 9,       # N0 pass + projection to the potential: read 6, write 3
    "axis3": 6,       # inverse N1 pass of the potential: read 3, write 3
    "c2r3": 6,        # inverse N2 pass of the potential: read 3, write 3
    "grad": 9,        # rho -= alpha U and |D rho|^2: read U 3 + rho 3, write rho 3
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps: CG iterations (default 40); load increments with --ramp, time steps with "
                         "--coupled (default 2 / 3)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (default 5; 1 with --ramp, "
                                                                 "--coupled)")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--forms", default="fp64,mixed")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--ramp", action="store_true",
                    help="staggered load increments of the polydisperse ramp (Newton-CG, history, phase field) "
                         "instead of CG iterations at the first increment")
    ap.add_argument("--first-increment", type=int, default=1,
                    help="--ramp: run the increments before this one untimed first (to reach a damaged state)")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the end-to-end Newton solve of the increment after the timed iterations")
    ap.add_argument("--batch", action="store_true",
                    help="the batched form instead: 48 ragged RVEs x 6 load cases (effective stiffness), batched "
                         "FP64 and mixed against the 288 single-item FP64 solves")
    ap.add_argument("--coupled", action="store_true",
                    help="the coupled path instead: staggered steps (Fick, Newton-CG, phase field) of the 128^3 "
                         "particle workload, FP64 and mixed")
    ap.add_argument("--chemistry", choices=["once", "coupled"], default="once",
                    help="--coupled: chemistry once per step (the paper) or inside the staggered loop")
    ap.add_argument("--jacobian", choices=["mu_c", "full"], default="mu_c",
                    help="--coupled: Fick Newton linearisation of the paper (mu_c) or fully implicit")
    ap.add_argument("--plane-particle", action="store_true",
                    help="the 2-D particle of Sec. 5.1 (512 x 512 plane grid, eq. (Gumbell) fields, SVK law): "
                         "staggered time steps until the damage has spread, a record line (not the headline)")
    ap.add_argument("--pp-n", type=int, default=512, help="grid side of --plane-particle")
    ap.add_argument("--batch-items", type=int, default=48)
    ap.add_argument("--graph-ticks", type=int, default=16)
    ap.add_argument("--newton-every", type=int, default=4,
                    help="batched form: the Newton step in every k-th step (graph_ticks a multiple of k)")
    ap.add_argument("--no-sequential", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 9 N doubles device-to-device 3 times (a plain copy kernel of known size, "
                         "for scaling HBM counters)")
    args = ap.parse_args()
    long_steps = args.ramp or args.coupled
    if args.steps is None:
        args.steps = (3 if args.coupled else 2) if long_steps else 40
    if args.warmup is None:
        args.warmup = 1 if long_steps else 5
    if args.steps < 1 or args.warmup < 0:
        ap.error("--steps must be >= 1 and --warmup >= 0")
    return args


def new_plan(work, form):
    """Plan, material and state (F = I, c = d = H = 0) of a workload on cuda:0."""
    import torch

    from paper_2411_16583_amd import Plan

    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    shape = work["shape"]
    plan = Plan(shape, work["spacing"], form)
    mats = [t(work[k]) for k in ("E", "nu", "Omega", "D", "sigma_max")]
    plan.set_material(*mats, gc=work["gc"], lc=work["lc"], RT=work["RT"], c_max=work["c_max"])
    F = torch.zeros((9,) + shape, dtype=torch.float64, device=dev)
    F[0] = 1.0
    F[4] = 1.0
    F[8] = 1.0
    c = torch.zeros(shape, dtype=torch.float64, device=dev)
    d = torch.zeros(shape, dtype=torch.float64, device=dev)
    H = torch.zeros(shape, dtype=torch.float64, device=dev)
    plan.set_state(F, c, d, H)
    return plan, F


def run_cg_form(work, form, steps, warmup, solve=True):
    """The benchmark step: CG iterations of the first Newton correction of
    the first load increment.  Warmup iterations (every kernel class timed
    with HIP events: the per-class breakdown) come first; then exactly
    `steps` iterations are timed (events only on the dominant class, taken by
    its launches).  Afterwards, untimed by the step clock, one complete Newton
    solve of the increment from F = I (end-to-end time and iteration counts);
    its F is returned for the accuracy comparison between the forms."""
    import torch

    from paper_2411_16583_amd import make_opts

    plan, F = new_plan(work, form)
    Fbar = work["loads"][0]
    plan.apply_macro(Fbar)
    err0 = plan.newton_linear_begin(Fbar)
    plan.profile_begin()
    if warmup > 0:
        plan.cg_iterate(warmup)
    torch.cuda.synchronize()
    prof_all = plan.profile_end()
    timed = [k for k in WORDS_PER_VOXEL if prof_all[k][1] > 0]
    dominant = max(timed, key=lambda k: prof_all[k][0]) if timed else "front"
    plan.profile_begin(passes=[dominant])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = plan.cg_iterate(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = plan.profile_end()
    print(f"[{form}] {steps} CG iterations (after {warmup} warmup) in {elapsed * 1e3:.2f} ms, "
          f"err_res before the correction {err0:.3e}, ||r||/||b|| {it['relres']:.3e}", flush=True)
    out = dict(elapsed=elapsed, cg_iters=steps, prof=prof, prof_all=prof_all, relres=it["relres"], err0=err0)
    if solve:
        F.zero_()
        F[0] = 1.0
        F[4] = 1.0
        F[8] = 1.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = plan.newton_solve(Fbar, make_opts(tol_newton=1e-8, tol_lin=1e-10, max_newton=50, max_lin=20000))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        Pm = plan.homogenized_stress()
        print(f"[{form}] Newton solve of the increment: {el:.3f} s, newton {st['newton_iters']}, "
              f"cg {st['lin_history']}, err_res {st['err_res']:.2e}", flush=True)
        out.update(solve=dict(seconds=el, newton_iters=st["newton_iters"], cg_iters=st["lin_iters_total"],
                              cg_history=st["lin_history"], err_res=st["err_res"], P_avg=Pm), F=F)
    plan.close()
    return out


def run_ramp_form(work, form, steps, warmup, first=1):
    """Staggered load increments (Alg. 4 without chemistry) of the ramp:
    increments 1 .. first - 1 untimed (silently), then warmup increments
    with every kernel class timed, then `steps` timed increments.  An
    increment whose staggered loop does not converge raises (it is not
    timed as a step)."""
    import torch

    from paper_2411_16583_amd.driver import staggered_step

    loads = work["loads"]
    if first - 1 + warmup + steps > len(loads):
        raise SystemExit(f"increments up to {first - 1 + warmup + steps} requested; the ramp has {len(loads)}")
    plan, F = new_plan(work, form)
    for k in range(first - 1):
        st = staggered_step(plan, loads[k], chemistry=False)
        print(f"[{form}] increment {k + 1} (untimed): staggered {st['stag_iters']}", flush=True)
    loads = loads[first - 1:]
    # warm-up increments: HIP events around every kernel class (the per-class
    # breakdown); timed increments: events around the dominant class only
    # (the roofline kernel), since the event records of all classes cost a
    # few % of the step
    plan.profile_begin()
    for k in range(warmup):
        st = staggered_step(plan, loads[k], chemistry=False)
        print(f"[{form}] warmup increment {first + k}: newton {[s['newton_iters'] for s in st['newton']]} "
              f"cg {[s['lin_history'] for s in st['newton']]}", flush=True)
    torch.cuda.synchronize()
    prof_all = plan.profile_end()
    timed = [k for k in WORDS_PER_VOXEL if prof_all[k][1] > 0]
    dominant = max(timed, key=lambda k: prof_all[k][0]) if timed else "front"
    plan.profile_begin(passes=[dominant])
    cg_iters = 0
    newton_iters = 0
    t0 = time.perf_counter()
    for k in range(warmup, warmup + steps):
        st = staggered_step(plan, loads[k], chemistry=False)
        its = sum(s["lin_iters_total"] for s in st["newton"])
        cg_iters += its
        newton_iters += sum(s["newton_iters"] for s in st["newton"])
        print(f"[{form}] increment {first + k}: staggered {st['stag_iters']}, newton "
              f"{[s['newton_iters'] for s in st['newton']]} cg {[s['lin_history'] for s in st['newton']]} "
              f"err {st['err_res']:.2e}", flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = plan.profile_end()
    Pm = plan.homogenized_stress()
    plan.close()
    return dict(elapsed=elapsed, cg_iters=cg_iters, newton_iters=newton_iters, prof=prof, prof_all=prof_all,
                P11=float(Pm[0, 0]))


def measured_traffic(kernel, word_bytes):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (profiles/*_traffic.json), or None when the kernel's
    sources changed since those counters were taken."""
    import hashlib

    form = {8: "fp64", 4: "fp32"}.get(word_bytes)
    path = os.path.join(ROOT, "profiles", f"front_polydisperse256_{form}_traffic.json")
    if kernel != "front" or form is None or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec["source_files"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def roofline(res, N, word_bytes):
    """Roofline record of the dominant kernel class from the timed region's
    events (res["prof"]); per_class from the warm-up's events of every class
    (res["prof_all"]) when there were any."""
    prof = res["prof"]
    warm = res.get("prof_all")
    cands = {k: prof[k] for k in WORDS_PER_VOXEL if prof[k][1] > 0}
    name = max(cands, key=lambda k: cands[k][0])
    ms, launches = cands[name]
    avg_s = ms / 1e3 / launches
    bytes_per_launch = WORDS_PER_VOXEL[name] * word_bytes * N
    achieved = bytes_per_launch / avg_s / 1e9
    traffic = measured_traffic(name, word_bytes) if N == 256 ** 3 else None
    return dict(kernel=name, bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                avg_launch_us=round(avg_s * 1e6, 2), launches=launches,
                bytes_per_launch=bytes_per_launch,
                per_class=per_class(warm if warm and any(n > 0 for _, n in warm.values()) else prof, N,
                                    word_bytes))


def per_class(prof, N, word_bytes):
    """Per kernel class: total ms, counted launches, mean us per launch and,
    for the CG-iteration classes, algorithmic GB/s."""
    out = {}
    for k, (ms, n) in prof.items():
        if n <= 0:
            continue
        avg = ms / n
        d = {"ms": round(ms, 2), "launches": int(n), "avg_us": round(1e3 * avg, 1)}
        if k in WORDS_PER_VOXEL:
            d["GB/s"] = round(WORDS_PER_VOXEL[k] * word_bytes * N / (avg * 1e-3) / 1e9, 1)
        out[k] = d
    return out


def cpu_baseline(work, iters):
    """The oracle's CG iterations on the same 256^3 increment-1 state
    (timed: the iterations only; K is built first, untimed)."""
    import oracle.spectral as osp
    from oracle import constitutive as cm
    from oracle import mechanics
    from oracle.krylov import dot

    threads = min(16, os.cpu_count() or 1)
    osp.WORKERS = threads
    shape = work["shape"]
    Fbar = work["loads"][0]
    F = mechanics.uniform_field(Fbar, shape)
    c, d = work["c0"], work["d0"]
    GP, _ = mechanics.residual_rhs(F, c, d, work, work["spacing"])
    b = -osp.project(GP, work["spacing"])
    K = cm.tangent(F, c, d, work["E"], work["nu"], work["Omega"])
    print("cpu baseline: oracle tangent and right-hand side built", flush=True)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = dot(r, r)
    t0 = time.perf_counter()
    for _ in range(iters):
        Ap = mechanics.operator(K, p, work["spacing"])
        alpha = rr / dot(p, Ap)
        x += alpha * p
        r -= alpha * Ap
        rr_new = dot(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        print(f"cpu baseline: iteration done at {time.perf_counter() - t0:.1f} s", flush=True)
    el = time.perf_counter() - t0
    N = int(np.prod(shape))
    return dict(value=N * iters / el, unit="voxel*CG-iter/s", cores=threads, kind="oracle",
                sample=f"{iters} CG iterations of the oracle's Newton-CG at {shape[0]}^3, increment-1 state "
                       f"(numpy/scipy float64, scipy.fft workers={threads}, einsum single-threaded), "
                       f"{el:.1f} s")


def run_batch(args):
    """Batched form: every (RVE, load case) item to tol_newton 1e-8 / CG 1e-10
    from the reference state; batched FP64 and mixed (one captured graph per
    form, warm solve first), then the same 288 solves one at a time with
    single-item FP64 plans.  value = item solves per second of the batched
    FP64 form."""
    import torch

    import synth
    from paper_2411_16583_amd import Batch, Plan, make_opts
    from paper_2411_16583_amd.homogenize import voigt_stiffness

    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    items = synth.batch_workloads(args.batch_items)
    eps = 1e-3
    loads = items[0]["loads"]
    ncase = len(loads)
    Ns = [int(np.prod(w["shape"])) for w in items]
    sizes = sorted(set(w["shape"][0] for w in items))
    print(f"batch workload: {len(items)} RVEs, sizes {[(n, sum(w['shape'][0] == n for w in items)) for n in sizes]}, "
          f"{sum(Ns)} voxels, built in {time.perf_counter() - t0:.1f} s", flush=True)
    opts = make_opts(tol_newton=1e-8, tol_lin=1e-10, max_newton=50, max_lin=20000)
    out = {}
    for form in ("fp64", "mixed"):
        b = Batch([w["shape"] for w in items], [w["spacing"] for w in items], ncase, form)
        for k, w in enumerate(items):
            b.set_material(k, t(w["E"]), t(w["nu"]), t(w["Omega"]))
        b.set_schedule(args.newton_every)
        b.newton_solve(loads, opts, graph_ticks=args.graph_ticks)  # warm: graph capture, first touch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P, stats, _ = b.newton_solve(loads, opts, graph_ticks=args.graph_ticks)
        el = time.perf_counter() - t0
        vi = sum(Ns[i // ncase] * s["lin_iters_total"] for i, s in enumerate(stats))
        out[form] = dict(elapsed=el, P=P, voxel_iters=vi, groups=b.n_groups,
                         newton=[s["newton_iters"] for s in stats], cg=sum(s["lin_iters_total"] for s in stats),
                         err_max=max(s["err_res"] for s in stats))
        print(f"[batch {form}] {el:.3f} s, {b.n_groups} groups, CG iterations {out[form]['cg']}, "
              f"Newton {min(out[form]['newton'])}..{max(out[form]['newton'])}, max err_res {out[form]['err_max']:.1e}",
              flush=True)
        b.close()
        del b
        torch.cuda.empty_cache()
    seq = None
    if not args.no_sequential:
        plans = []
        for w in items:
            pl = Plan(w["shape"], w["spacing"], "fp64")
            mats = [t(w[k]) for k in ("E", "nu", "Omega")]
            pl.set_material(*mats, None, None, gc=1.0, lc=1.0, RT=1.0, c_max=1.0)
            F = torch.zeros((9,) + w["shape"], dtype=torch.float64, device=dev)
            pl.set_state(F)
            plans.append((pl, mats, F))
        Pseq = np.zeros((len(items), ncase, 3, 3))
        cg = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, (pl, mats, F) in enumerate(plans):
            for lc, Fm in enumerate(loads):
                F.zero_()
                F[0] = 1.0
                F[4] = 1.0
                F[8] = 1.0
                s = pl.newton_solve(Fm, opts)
                cg += s["lin_iters_total"]
                Pseq[k, lc] = pl.homogenized_stress()
        el = time.perf_counter() - t0
        seq = dict(elapsed=el, P=Pseq, cg=cg)
        print(f"[sequential fp64] {el:.3f} s for {len(items) * ncase} solves, CG iterations {cg}", flush=True)
        for pl, _, _ in plans:
            pl.close()
    ref = seq["P"] if seq else out["fp64"]["P"]
    Cref = np.stack([voigt_stiffness(ref[k], eps) for k in range(len(items))])

    def cdiff(P):
        C = np.stack([voigt_stiffness(P[k], eps) for k in range(len(items))])
        return float(np.max(np.abs(C - Cref)) / np.max(np.abs(Cref)))

    nsolve = len(items) * ncase
    f64, mx = out["fp64"], out["mixed"]
    line = {
        "metric": "batched effective-stiffness solves/s (48 ragged RVEs x 6 load cases, Newton 1e-8)",
        "value": nsolve / f64["elapsed"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": 1e3 * f64["elapsed"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{len(items)} Boolean-sphere RVEs, N ~ U{{32,48,64,96}}, phi ~ U(0.1,0.4), "
                               f"contrast 10, 6 load cases eps = 1e-3, from the reference state",
                   "voxels": sum(Ns), "graph_ticks": args.graph_ticks, "newton_every": args.newton_every,
                   "groups": f64["groups"]},
        "batched_fp64": dict(seconds=round(f64["elapsed"], 4), cg_iters=f64["cg"],
                             voxel_cg_iters_per_s=f64["voxel_iters"] / f64["elapsed"],
                             C_eff_rel_diff=cdiff(f64["P"]) if seq else 0.0),
        "batched_mixed": dict(seconds=round(mx["elapsed"], 4), cg_iters=mx["cg"],
                              voxel_cg_iters_per_s=mx["voxel_iters"] / mx["elapsed"],
                              C_eff_rel_diff=cdiff(mx["P"]), speedup_vs_batched_fp64=f64["elapsed"] / mx["elapsed"]),
    }
    if seq:
        line["sequential_fp64"] = dict(seconds=round(seq["elapsed"], 4), cg_iters=seq["cg"],
                                       speedup_batched_fp64=seq["elapsed"] / f64["elapsed"],
                                       speedup_batched_mixed=seq["elapsed"] / mx["elapsed"])
    print(json.dumps(line), flush=True)


def run_coupled(args):
    """Coupled path: time steps of Alg. 4 on the particle workload (inward
    flux on the particle's inner shell, swelling, damage), each step one
    backward-Euler Fick step, then Newton-CG and the phase-field PCG
    alternating until the equilibrium residual with the new damage is below
    tol.  value = time steps per second (FP64); the mixed form runs the same
    steps, and the final c, d and F of both forms are compared."""
    import torch

    import synth
    from paper_2411_16583_amd import Plan
    from paper_2411_16583_amd.driver import staggered_step

    n = args.n if args.n != 256 else 128
    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    work = synth.particle_workload(n=n)
    shape = work["shape"]
    N = int(np.prod(shape))
    res, fields = {}, {}
    for form in ("fp64", "mixed"):
        plan = Plan(shape, work["spacing"], form)
        mats = [t(work[k]) for k in ("E", "nu", "Omega", "D", "sigma_max")]
        plan.set_material(*mats, gc=work["gc"], lc=work["lc"], RT=work["RT"], c_max=work["c_max"])
        F = torch.zeros((9,) + shape, dtype=torch.float64, device=dev)
        F[0] = 1.0
        F[4] = 1.0
        F[8] = 1.0
        c, d, H = t(work["c0"]), t(work["d0"]), torch.zeros(shape, dtype=torch.float64, device=dev)
        plan.set_state(F, c, d, H)
        cdot = t(work["cdot_B"])
        kw = dict(dt=work["dt"], cdot_B=cdot, chemistry=True if args.chemistry == "once" else "coupled",
                  jacobian=args.jacobian)
        for k in range(args.warmup):
            staggered_step(plan, work["loads"][k], **kw)
        torch.cuda.synchronize()
        plan.profile_begin()
        cg = pcg = chem = stag = chem_newton = 0
        t0 = time.perf_counter()
        for k in range(args.warmup, args.warmup + args.steps):
            st = staggered_step(plan, work["loads"][k], **kw)
            cg += sum(s_["lin_iters_total"] for s_ in st["newton"])
            pcg += sum(s_["lin_iters_last"] for s_ in st["pff"])
            chem += sum(ch_["lin_iters_total"] for ch_ in (st["chem_coupled"] or [st["chem"]]))
            chem_newton += sum(ch_["newton_iters"] for ch_ in (st["chem_coupled"] or [st["chem"]]))
            stag += st["stag_iters"]
            print(f"[coupled {form}] step {k + 1}: staggered {st['stag_iters']}, newton CG "
                  f"{[s_['lin_iters_total'] for s_ in st['newton']]}, pff {[s_['lin_iters_last'] for s_ in st['pff']]}, "
                  f"fick {st['chem']['newton_iters']} Newton / {st['chem']['lin_iters_total']} PCG, "
                  f"err {st['err_res']:.1e}", flush=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = plan.profile_end()
        res[form] = dict(elapsed=el, cg=cg, pcg=pcg, chem=chem, chem_newton=chem_newton, stag=stag, prof=prof)
        fields[form] = (c.cpu().numpy(), d.cpu().numpy(), F.cpu().numpy())
        plan.close()
        del F, c, d, H, mats, cdot
        torch.cuda.empty_cache()

    def rdiff(a, b, ref):
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(ref), 1e-300))

    cf, df, Ff = fields["fp64"]
    cm_, dm, Fm = fields["mixed"]
    c0 = work["c0"]
    eye = np.eye(3).reshape(9, 1, 1, 1)
    f64, mx = res["fp64"], res["mixed"]
    line = {
        "metric": f"coupled staggered time steps/s (particle {n}^3: Fick BE + Newton-CG + phase-field PCG)",
        "value": args.steps / f64["elapsed"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * f64["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"particle {n}^3 (ellipsoid 40/32/28 voxels at 128^3, buffer 1e-3 E), flux "
                               f"4e-10 m/s on the inner shell, dt = {work['dt']} s, Omega = 0.03, sigma_max = 20 MPa",
                   "voxels": N, "chemistry": args.chemistry, "fick_jacobian": args.jacobian},
        "fp64": dict(cg_iters=f64["cg"], pff_pcg_iters=f64["pcg"], fick_pcg_iters=f64["chem"],
                     fick_newton_iters=f64["chem_newton"],
                     staggered_iters=f64["stag"], per_class=per_class(f64["prof"], N, 8),
                     voxel_cg_iters_per_s=N * f64["cg"] / f64["elapsed"]),
        "mixed": dict(ms_per_step=1e3 * mx["elapsed"] / args.steps, cg_iters=mx["cg"], pff_pcg_iters=mx["pcg"],
                      fick_pcg_iters=mx["chem"], staggered_iters=mx["stag"],
                      speedup_per_step=f64["elapsed"] / mx["elapsed"],
                      rel_diff_c=rdiff(cm_, cf, cf - c0), rel_diff_d=rdiff(dm, df, df) if np.any(df) else 0.0,
                      rel_diff_F=rdiff(Fm, Ff, Ff - eye)),
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the hot path here is single-GPU "
              "(a sharded multi-GPU form is not implemented)", file=sys.stderr)
        sys.exit(2)
    import synth

    if args.batch:
        run_batch(args)
        return
    if args.coupled:
        run_coupled(args)
        return
    if args.plane_particle:
        run_plane_particle(args)
        return
    t0 = time.perf_counter()
    work = synth.polydisperse_workload(n=args.n)
    N = int(np.prod(work["shape"]))
    print(f"workload polydisperse {work['shape']} built in {time.perf_counter() - t0:.1f} s, "
          f"inclusion fraction {work['phase'].mean():.3f}", flush=True)
    if args.copy_calibration:
        import torch

        a = torch.ones(9 * N, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"copy calibration: 3 copies of {9 * N * 8} bytes", flush=True)
        del a, b
    forms = args.forms.split(",")
    if args.ramp:
        run_ramp(args, work, forms, N)
    else:
        run_cg(args, work, forms, N)


def run_plane_particle(args):
    """--plane-particle: the 2-D particle of Sec. 5.1 at full size (512 x 512
    plane grid, Young's modulus and threshold stress from eq. (Gumbell),
    SVK law, Omega = 1.3, source on the 6-voxel band), FP64, staggered time
    steps (Alg. 4, full chemistry Jacobian, CG tolerance 1e-6, staggered loop
    capped at 100 iterations) until 2 % of the particle has d > 0.9 or
    --steps steps (default 400).  Prints a record line: the step where the
    damage first reaches 0.05 and its radius, and at the end the damaged
    voxels' radii (the paper: damage starts at random points, more likely
    near the particle centre, and spreads to fracture)."""
    import torch

    import synth
    from paper_2411_16583_amd import Plan
    from paper_2411_16583_amd.driver import staggered_step

    n_steps = args.steps or 400
    w = synth.plane_particle_workload(args.pp_n)
    shape = w["shape"]
    n = shape[1]
    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    plan = Plan(shape, w["spacing"], "fp64", law=w["law"])
    mats = [t(w[k]) for k in ("E", "nu", "Omega", "D", "sigma_max")]
    plan.set_material(*mats, gc=w["gc"], lc=w["lc"], RT=w["RT"], c_max=w["c_max"])
    F = torch.zeros((9,) + shape, dtype=torch.float64, device=dev)
    F[0] = F[4] = F[8] = 1.0
    c, d, H = t(w["c0"]), t(w["d0"]), torch.zeros(shape, dtype=torch.float64, device=dev)
    plan.set_state(F, c, d, H)
    cdot = t(w["cdot_B"])
    phase = torch.as_tensor(w["phase"], device=dev)
    n_part = int(phase.sum().item())
    ctr = (n - 1) / 2.0
    radius = 0.4 * n
    from paper_2411_16583_amd import FgError

    steps, nucleation, stop = [], None, None
    t0 = time.perf_counter()
    for k in range(n_steps):
        ts = time.perf_counter()
        try:
            st = staggered_step(plan, np.eye(3), dt=w["dt"], cdot_B=cdot, tol_lin=w["tol_lin"],
                                jacobian=w["jacobian"], max_stag=100, raise_on_noconv=False)
        except FgError as e:  # e.g. the CG's breakdown once cracked voxels make the operator singular
            stop = f"step {k + 1}: {e}"
            print(f"stopped at {stop}", flush=True)
            break
        torch.cuda.synchronize()
        dmax = float(d.max().item())
        cg = sum(sum(x["lin_history"]) for x in st["newton"])
        steps.append(dict(stag=st["stag_iters"], converged=st["converged"], cg=cg, d_max=dmax,
                          ms=1e3 * (time.perf_counter() - ts)))
        if nucleation is None and dmax >= 0.05:
            at = np.unravel_index(int(torch.argmax(d).item()), shape)
            nucleation = dict(step=k + 1, r_over_R=float(np.hypot(at[1] - ctr, at[2] - ctr) / radius))
        broken = int(((d > 0.9) & phase).sum().item())
        if k % 20 == 19 or broken >= 0.02 * n_part:
            print(f"step {k + 1}: stag {st['stag_iters']} cg {cg} d max {dmax:.3f} broken {broken} "
                  f"({time.perf_counter() - t0:.1f} s)", flush=True)
        if broken >= 0.02 * n_part:
            break
    elapsed = time.perf_counter() - t0
    dh = d.cpu().numpy()[0]
    i1, i2 = np.nonzero((dh > 0.5) & w["phase"][0])
    rr = np.hypot(i1 - ctr, i2 - ctr) / radius
    line = {
        "metric": "plane particle of Sec. 5.1: staggered steps to fracture (record, not the headline)",
        "value": len(steps) / elapsed,  # steps completed
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": len(steps),
        "warmup": 0,
        "ms_per_step": 1e3 * elapsed / len(steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plane particle {n} x {n} (disc 0.8 L, eq. (Gumbell) E and sigma_max, m = 3, "
                               f"SVK, Omega = 1.3, source on the {max(1, round(6 * n / 512))}-voxel band, "
                               f"dt = {w['dt']} s)", "voxels": n * n},
        "nucleation": nucleation,
        "stopped": stop,
        "damaged_d_gt_0.5": dict(voxels=int(rr.size), fraction_of_particle=float(rr.size / n_part),
                                 r_over_R_quartiles=[float(q) for q in np.quantile(rr, [0.25, 0.5, 0.75])]
                                 if rr.size else None,
                                 inner_half_radius_fraction=float(np.mean(rr < 0.5)) if rr.size else None),
        "stag_iters_total": int(sum(s["stag"] for s in steps)),
        "steps_not_converged": int(sum(not s["converged"] for s in steps)),
        "cg_iters_total": int(sum(s["cg"] for s in steps)),
    }
    print(json.dumps(line), flush=True)


def field_error(Fa, Fb, Fbar):
    """||Fa - Fb|| / ||Fb - Fbar|| (relative to the fluctuation) and the
    largest absolute difference, computed on the device."""
    import torch

    ub = torch.as_tensor(np.asarray(Fbar, dtype=np.float64).reshape(9, 1, 1, 1), device=Fb.device)
    num = torch.linalg.vector_norm(Fa - Fb).item()
    den = torch.linalg.vector_norm(Fb - ub).item()
    return num / max(den, 1e-300), torch.max(torch.abs(Fa - Fb)).item()


def run_cg(args, work, forms, N):
    """Default mode: CG iterations of the first Newton correction (see the
    module docstring), FP64 as the headline value and mixed beside it."""
    import torch

    res = {}
    errors = {}
    F64 = None
    for form in forms:
        try:
            res[form] = run_cg_form(work, form, args.steps, args.warmup, solve=not args.no_solve)
        except Exception as e:  # report a failing form instead of dropping the line
            if form == forms[0]:
                raise
            errors[form] = repr(e)
            print(f"[{form}] failed: {e!r}", flush=True)
            continue
        F = res[form].pop("F", None)
        if form == "fp64":
            F64 = F
        elif F is not None and F64 is not None:
            res[form]["F_err"] = field_error(F, F64, work["loads"][0])
        del F
        torch.cuda.empty_cache()
    main_form = "fp64" if "fp64" in res else forms[0]
    r0 = res[main_form]
    value = N * r0["cg_iters"] / r0["elapsed"]

    def solve_rec(r):
        if "solve" not in r:
            return None
        sv = r["solve"]
        return dict(seconds=round(sv["seconds"], 4), newton_iters=sv["newton_iters"], cg_iters=sv["cg_iters"],
                    cg_history=sv["cg_history"], err_res=sv["err_res"],
                    voxel_cg_iters_per_s=N * sv["cg_iters"] / sv["seconds"], P11=float(sv["P_avg"][0, 0]))

    line = {
        "metric": "voxel*CG-iters/s at 256^3 (FP64 vs mixed) + % of HBM roofline",
        "value": value,
        "unit": "voxel*CG-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r0["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_form == "fp64" else "f32/f64",
        "data": "synthetic",
        "config": {"workload": f"polydisperse RVE {args.n}^3 (60 RSA spheres r~U(10,24) vox, contrast 20), "
                               f"first load increment F = I + 0.0025 e1(x)e1; step = one CG iteration of the "
                               f"first Newton correction",
                   "voxels": N, "step": "CG iteration", "relres_after_steps": r0["relres"]},
        "roofline": roofline(r0, N, 8 if main_form == "fp64" else 4),
    }
    if solve_rec(r0):
        line["newton_solve"] = solve_rec(r0)
    for form in forms:
        if form == main_form:
            continue
        if form in errors:
            line[form] = dict(error=errors[form])
            continue
        r = res[form]
        v = N * r["cg_iters"] / r["elapsed"]
        rec = dict(value=v, ms_per_step=1e3 * r["elapsed"] / args.steps, speedup_per_cg_iter=v / value,
                   relres_after_steps=r["relres"], roofline=roofline(r, N, 4))
        sv = solve_rec(r)
        if sv:
            rec["newton_solve"] = sv
            if "solve" in r0:
                rec["speedup_newton_solve_at_equal_accuracy"] = r0["solve"]["seconds"] / r["solve"]["seconds"]
                P0 = r0["solve"]["P_avg"]
                rec["rel_diff_Pavg_vs_fp64"] = float(np.linalg.norm(r["solve"]["P_avg"] - P0) / np.linalg.norm(P0))
            if "F_err" in r:
                rec["rel_diff_F_vs_fp64"] = r["F_err"][0]
                rec["max_abs_diff_F_vs_fp64"] = r["F_err"][1]
        line[form] = rec
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(work, args.cpu_iters)
    print(json.dumps(line), flush=True)


def run_ramp(args, work, forms, N):
    """--ramp: staggered load increments (Newton-CG, history, phase field)."""
    res = {}
    for form in forms:
        res[form] = run_ramp_form(work, form, args.steps, args.warmup, args.first_increment)
    main_form = "fp64" if "fp64" in res else forms[0]
    r0 = res[main_form]
    value = N * r0["cg_iters"] / r0["elapsed"]
    line = {
        "metric": "voxel*CG-iters/s at 256^3 over staggered load increments (damage on)",
        "value": value,
        "unit": "voxel*CG-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r0["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_form == "fp64" else "f32/f64",
        "data": "synthetic",
        "config": {"workload": f"polydisperse RVE {args.n}^3, load increments "
                               f"{args.first_increment + args.warmup}..{args.first_increment - 1 + args.warmup + args.steps}"
                               f" of the stretch ramp (sigma_max = 0.25 E), damage on, chemistry off; "
                               f"step = one staggered load increment",
                   "voxels": N, "cg_iters": r0["cg_iters"], "newton_iters": r0["newton_iters"]},
        "roofline": roofline(r0, N, 8 if main_form == "fp64" else 4),
    }
    for form in forms:
        if form == main_form:
            continue
        r = res[form]
        v = N * r["cg_iters"] / r["elapsed"]
        line[form] = dict(value=v, ms_per_step=1e3 * r["elapsed"] / args.steps, cg_iters=r["cg_iters"],
                          newton_iters=r["newton_iters"], speedup_per_cg_iter=v / value,
                          speedup_per_step=r0["elapsed"] / r["elapsed"],
                          rel_diff_P11_vs_fp64=abs(r["P11"] - r0["P11"]) / abs(r0["P11"]),
                          roofline=roofline(r, N, 4))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
