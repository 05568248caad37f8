/*
 * fgfft: Fourier-Galerkin chemo-mechanical solver core for MI355X (gfx950).
 *
 * C ABI of the hot path of Zarzoso, Roque, Montero-Chacon, Segurado, "An FFT
 * based chemo-mechanical framework with fracture" (arXiv:2411.16583): the
 * matrix-free operator  y = F^-1[ G^ : F[ K : x ] ]  applied by conjugate
 * gradients inside the finite-strain Newton iteration (Sec. 3.2, eq. (30),
 * Alg. 1), the preconditioned CG of the phase-field equation (eqs. (32)-(36),
 * Alg. 2) and the backward-Euler Fick step (eqs. (42)-(50), Alg. 3).
 *
 * Conventions shared by every call
 * --------------------------------
 * Grid: N0 x N1 x N2 voxels on a periodic box, spacing h[3] (metres), N2 the
 * fastest axis, N = N0 N1 N2.  Supported sizes: N0, N1 in {4, 6, 8, 12, 16,
 * 24, 32, 48, 64, 96, 128, 256}, and also N0 = 1 and N1 = 512; N2 = 2 M with
 * M in {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256}.  Others return
 * FG_E_SIZE.
 * N0 = 1 is a plane (the 2-D problems of Sec. 4.3 and 5.1): the box is one
 * voxel thick and periodic along axis 0, so every difference along axis 0
 * vanishes and F_00 stays at its macroscopic value (plane strain, with the
 * out-of-plane stretch prescribed by F_macro).
 * Fields: device pointers, double precision, component-major.  A scalar field
 * is N doubles in C order (index (i0 N1 + i1) N2 + i2); a 3x3 tensor field is
 * 9 such planes, plane 3 i + j holding the ij component (row-major tensor
 * index, so F_ij = du_i / dX_j).  Tensors passed by value (F_macro, P_avg)
 * are host arrays of 9 doubles, row-major.
 * Memory: every field, material array and the workspace is owned by the
 * caller (for example PyTorch tensors) and must stay valid until it is
 * replaced or the plan is destroyed.  The library allocates no device
 * memory; it owns only the opaque plan, a little pinned host memory for
 * scalar read-backs, and the fixed device array of fg_project_noalloc that
 * is part of its code object.
 * Streams: all device work is issued on the stream given at plan creation
 * (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream; NULL is the
 * default stream).  Calls that return solver statistics synchronise that
 * stream; fg_fft_* and fg_apply_operator do not.
 * Errors: every call returns an fg_status; nothing throws across the ABI.
 * Arguments are validated before any device work is issued; on error the
 * device state is unchanged unless the description says otherwise.
 * fg_last_error returns a message for the last failing call on a plan.
 */
#ifndef FGFFT_H
#define FGFFT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fg_plan fg_plan;
typedef struct fg_batch fg_batch;

typedef enum {
  FG_OK = 0,
  FG_E_ARG = 1,       /* null pointer, bad value                         */
  FG_E_SIZE = 2,      /* unsupported grid size or workspace too small    */
  FG_E_HIP = 3,       /* a HIP runtime call failed                       */
  FG_E_NOCONV = 4,    /* Newton / Krylov iteration limit reached         */
  FG_E_BREAKDOWN = 5, /* p.Ap <= 0 inside CG (operator not SPD)          */
  FG_E_DOMAIN = 6,    /* det F <= 0, 1 + Omega c <= 0 or c outside (0,1) */
  FG_E_STATE = 7      /* workspace, material or state not set            */
} fg_status;

/* FG_FP64: everything in double precision.
 * FG_MIXED: the CG operator (tangent state, FFTs, CG vectors) in single
 * precision with double-precision dot products; the Newton residual, the
 * stress and F stay double, so Newton refines to the double tolerance. */
typedef enum { FG_FP64 = 0, FG_MIXED = 1 } fg_precision;

/* Material law of a plan (fg_set_law).
 * FG_LAW_NEO_HOOKE: compressible Neo-Hookean energy psi_0 = G/2 (tr C_e - 3)
 *   - G ln J_e + lambda/2 (ln J_e)^2 (the default).
 * FG_LAW_SVK: the paper's Saint-Venant-Kirchhoff energy (Sec. 2.1 eqs. (3),
 *   (4), (12)): psi_0 = lambda/2 tr^2 E_e + G tr(E_e^2), E_e = (F_e^T F_e -
 *   I)/2.  Both take F_e = F (1 + Omega c)^{-1/3} (eq. (2)), the degradation
 *   g(d) = (1 - d)^2 and the energy per reference volume, so that for SVK
 *   P = g (1 + Omega c)^{-2/3} F S(E_e), eq. (12) when Omega c = 0.  The law
 *   sets the stress, the CG operator's tangent, the effective Cauchy stress
 *   of the driving force, the elastic chemical potential and the adjoint's
 *   parameter derivatives. */
typedef enum { FG_LAW_NEO_HOOKE = 0, FG_LAW_SVK = 1 } fg_law;

typedef struct {
  double tol_newton; /* err_res tolerance (eq. (31)), e.g. 1e-8           */
  double tol_lin;    /* CG tolerance ||r|| <= tol ||b||, e.g. 1e-10       */
  int max_newton;    /* Newton iteration limit, e.g. 50                   */
  int max_lin;       /* CG iteration limit per solve                      */
  int fixed_lin;     /* > 0: run exactly this many CG iterations per solve
                        (tol_lin ignored); used for matched-count parity   */
} fg_solver_opts;

typedef struct {
  int newton_iters;    /* Newton corrections applied                      */
  int lin_iters_total; /* CG iterations summed over the Newton loop       */
  int lin_iters_last;  /* CG iterations of the last linear solve          */
  int n_history;       /* entries used in err_history                     */
  double err_res;      /* final equilibrium residual (eq. (31))           */
  double lin_relres;   /* final ||r|| / ||b|| of the last linear solve    */
  double err_history[64]; /* err_res before each Newton correction       */
  int lin_history[64];    /* CG iterations of each Newton correction      */
} fg_stats;

/* Create a plan for an N0 x N1 x N2 periodic grid with spacing h (Sec. 3.2:
 * voxel grid, DFT over the three axes).  grid: 3 ints, spacing: 3 doubles
 * (host).  stream: hipStream_t or NULL.  *out receives the plan.
 * Errors: FG_E_ARG (null pointers, h <= 0), FG_E_SIZE (unsupported size). */
fg_status fg_plan_create(const int grid[3], const double spacing[3], fg_precision prec,
                         void* stream, fg_plan** out);

/* Bytes of device workspace the plan needs (0 for a null plan). */
size_t fg_plan_workspace_bytes(const fg_plan* plan);

/* Hand the plan a caller-owned device buffer of at least
 * fg_plan_workspace_bytes bytes, 256-byte aligned.  The plan writes its
 * transform and symbol tables into it (asynchronously on the plan stream).
 * Errors: FG_E_ARG, FG_E_SIZE (too small), FG_E_HIP. */
fg_status fg_plan_set_workspace(fg_plan* plan, void* dev, size_t bytes);

/* Choose the plan's material law (fg_law).  Call before
 * fg_plan_workspace_bytes / fg_plan_set_workspace: the SVK tangent state
 * takes 18 words per voxel instead of 12, so the workspace size depends on
 * the law.  Batch plans use the Neo-Hookean law only.
 * Errors: FG_E_ARG (unknown law, null plan, a batch group), FG_E_STATE (the
 * workspace is already set). */
fg_status fg_set_law(fg_plan* plan, int law);

/* Material fields (Sec. 2; Table of Sec. 4.3 for the kind of data): Young's
 * modulus E (Pa), Poisson ratio nu, swelling coefficient Omega (eq. (2)),
 * diffusivity D (m^2/s, eq. (20)) and threshold stress sigma_max (Pa,
 * eq. (8)); device arrays of N doubles each (D and sigma_max may be NULL if
 * the chemistry / fracture calls are not used).  Scalars: fracture
 * toughness gc (J/m^2), length scale lc (m) (eq. (5)), RT (J/mol) and the
 * concentration scale c_max (mol/m^3) that converts the elastic chemical
 * potential to J/mol.  Errors: FG_E_ARG. */
fg_status fg_set_material(fg_plan* plan, const double* E, const double* nu, const double* Omega,
                          const double* D, const double* sigma_max, double gc, double lc, double RT,
                          double c_max);

/* State fields, updated in place by the solvers: F (9 N, the deformation
 * gradient, Sec. 3.1 eq. (23)), c (N, concentration in (0,1)), d (N, phase
 * field), H (N, history of eq. (7)).  c, d and H may be NULL for pure
 * mechanics (then c = d = 0).  Errors: FG_E_ARG. */
fg_status fg_set_state(fg_plan* plan, double* F, double* c, double* d, double* H);

/* Alg. 1 "Mechanical problem": add the macroscopic increment
 * F_macro - <F> to F (F^0 = F_t + dFbar, the fluctuation is kept) and run
 * Newton with a CG inner solve of eq. (30) until err_res (eq. (31),
 * normalised by ||G*P(F_macro)||) <= tol_newton.  F_macro: host, 9 doubles.
 * stats may be NULL.  Errors: FG_E_STATE, FG_E_NOCONV (F holds the last
 * iterate), FG_E_BREAKDOWN, FG_E_DOMAIN, FG_E_HIP. */
fg_status fg_newton_solve(fg_plan* plan, const double F_macro[9], const fg_solver_opts* opts,
                          fg_stats* stats);

/* Alg. 1 for the shifted equilibrium G*[P(F) - B] = 0 (eqs. (30), (31) with
 * P replaced by P - B), from the current F: no macroscopic increment is
 * applied and every correction has zero mean, so <F> is kept.  err_res is
 * ||G*(P(F) - B)|| normalised by its value at the entry state.  B: device,
 * 9 N doubles, caller-owned.  With B = P(F0; theta) of a converged state F0
 * and a perturbed material theta', this is the difference solve of a finite
 * difference: the base residual cancels exactly, and the solve is accurate
 * relative to the (small) difference problem.  Errors as fg_newton_solve. */
fg_status fg_newton_solve_shifted(fg_plan* plan, const double* B, const fg_solver_opts* opts, fg_stats* stats);

/* One Newton correction of Alg. 1 split in two calls, for callers that run
 * the CG iterations of eq. (30) themselves (a stopping rule of their own, or
 * timing the CG loop alone).
 * fg_newton_linear_begin evaluates P and the tangent at the current F (the
 * macroscopic increment is NOT applied), writes err_res of eq. (31)
 * (normalised by ||G*P(F_macro)|| as in fg_newton_solve) to *err_res (host,
 * may be NULL) and starts CG on G*(K : dF) = -G*P from dF = 0.  F_macro:
 * host, 9 doubles.  Synchronises.  Errors: FG_E_STATE, FG_E_DOMAIN,
 * FG_E_HIP.
 * fg_cg_iterate continues that CG by exactly n iterations (n >= 0; no
 * tolerance test, the iterations are those fg_newton_solve runs).  With
 * apply != 0 it then adds the CG iterate dF to F (double precision) and the
 * system is closed.  Any other call on the plan that uses its workspace also
 * closes it; fg_cg_iterate on a closed system returns FG_E_STATE.  stats (may
 * be NULL): lin_iters_last = CG iterations of this system so far,
 * lin_relres = ||r|| / ||b||.  Synchronises.  Errors: FG_E_ARG (n < 0),
 * FG_E_STATE, FG_E_BREAKDOWN (p.Ap <= 0; the system stays open but cannot
 * advance), FG_E_HIP. */
fg_status fg_newton_linear_begin(fg_plan* plan, const double F_macro[9], double* err_res);
fg_status fg_cg_iterate(fg_plan* plan, int n, int apply, fg_stats* stats);

/* Add the macroscopic increment F_macro - <F> to F (the first line of
 * Alg. 1, F^0 = F_t + dFbar; Sec. 3.2 Global problem: the chemistry of a step
 * sees the new macroscopic F).  F_macro: host, 9 doubles.  Synchronises.
 * fg_newton_solve performs the same update itself. */
fg_status fg_apply_macro(fg_plan* plan, const double F_macro[9]);

/* Adjoint sensitivity of L = sum_ij w_ij <P_ij> at the current, converged
 * state (eq. (30) differentiated: the equilibrium operator is self-adjoint
 * on compatible fields): solves G*(K : lam) = -G*(K : W) (W the uniform
 * field w = dL_dPavg, host, 9 doubles) to ||r|| <= opts->tol_lin ||b||, then
 * writes
 *   dL_dlogE[x]  = (W + lam(x)) : P(x) / N,
 *   dL_dOmega[x] = (W + lam(x)) : dP/dOmega(x) / N
 * (device, N doubles each, either may be NULL).  FG_FP64 plans solve by CG
 * in double precision.  FG_MIXED plans refine lam in double precision:
 * each step solves for a correction by CG with the single-precision
 * operator (relative tolerance max(1e-5, what is left)) and recomputes the
 * residual with the double-precision tangent.  stats: lin_iters_last,
 * lin_relres (final ||r|| / ||b||); mixed plans also lin_iters_total and
 * newton_iters = number of refinements.  Errors: FG_E_STATE, FG_E_NOCONV,
 * FG_E_BREAKDOWN, FG_E_DOMAIN, FG_E_HIP. */
fg_status fg_adjoint_gradient(fg_plan* plan, const double dL_dPavg[9], double* dL_dlogE, double* dL_dOmega,
                              const fg_solver_opts* opts, fg_stats* stats);

/* Homogenised tangent of the current, converged state applied to a
 * macroscopic direction W (host, 9 doubles): T_out = d<P>/dFbar : W (host,
 * 9 doubles).  A uniform change W of Fbar changes the fluctuation by the
 * compatible, zero-mean dF solving the linearised equilibrium of eq. (30),
 * G*(K : dF) = -G*(K : W) (one CG solve with the operator of the Newton
 * step, to ||r|| <= opts->tol_lin ||b||), and T_out = <K : (W + dF)>.  By the
 * major symmetry of K this is the adjoint system of fg_adjoint_gradient with
 * dL_dPavg = W, and mixed plans refine it in double precision the same way.
 * Used for mixed macroscopic stress/strain control (the Jacobian of the
 * prescribed stress components with respect to the free strain components)
 * and for effective stiffnesses.  stats as fg_adjoint_gradient.  Errors:
 * FG_E_STATE, FG_E_NOCONV, FG_E_BREAKDOWN, FG_E_DOMAIN, FG_E_HIP. */
fg_status fg_homogenized_tangent(fg_plan* plan, const double W[9], double T_out[9], const fg_solver_opts* opts,
                                 fg_stats* stats);

/* Equilibrium residual of the current state (eq. (31)) with respect to the
 * macroscopic F_macro (host, 9 doubles): *err_res (host).  Synchronises. */
fg_status fg_residual(fg_plan* plan, const double F_macro[9], double* err_res);

/* Homogenised first Piola-Kirchhoff stress <P> of the current state (Sec.
 * 3.1): P_avg, host, 9 doubles.  Synchronises. */
fg_status fg_homogenized_stress(fg_plan* plan, double P_avg[9]);

/* First Piola-Kirchhoff stress field of the current state into P (device,
 * 9 N doubles, caller-owned).  Errors: FG_E_DOMAIN (checked after a sync). */
fg_status fg_stress(fg_plan* plan, double* P);

/* One application of the operator of eq. (30) with the tangent of the
 * current state: y = F^-1[ G^ : F[ K(F) : x ] ]  (x, y: device, 9 N doubles,
 * may not alias).  In FG_MIXED plans the contraction and the transforms
 * run in single precision.  Does not synchronise. */
fg_status fg_apply_operator(fg_plan* plan, const double* x, double* y);

/* Compatibility projection y = F^-1[ G^ : F[x] ] (eq. (28)), double
 * precision (x, y: device, 9 N doubles; y may equal x).  Does not sync. */
fg_status fg_project(fg_plan* plan, const double* x, double* y);

/* The same projection computed as the CG iteration computes it: the N0
 * pass reduces the 9-component spectrum to the 3-component potential
 * U = -i e^{i Phi} (A r) / |r|^2 (Phi = (q0 + q1 + q2) / 2), only U is
 * transformed back, and y = D U with D the corner-difference stencil of the
 * rotated scheme (its symbol is i e^{-i Phi} r).  Double precision; x, y:
 * device, 9 N doubles (y may equal x).  Does not synchronise. */
fg_status fg_project_grad(fg_plan* plan, const double* x, double* y);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * projection of fg_project, y = F^-1[ G^ : F[x] ] (eq. (28)), without a plan
 * or workspace.  grid: 3 ints, spacing: 3 doubles (host), as for
 * fg_plan_create; x, y: device, 9 N doubles, caller-owned (y may equal x);
 * stream: hipStream_t or NULL.  Its transform tables and its spectral work
 * buffer (9 N doubles) live in a fixed 64 MiB + 64 KiB array that the
 * library holds on every device it runs on until the process ends, so the
 * call allocates nothing; grids with 9 N doubles beyond 64 MiB (N above
 * 932067 voxels, e.g. 96^3 fits, 128^3 does not) return FG_E_SIZE before any
 * device work.  Every call on a device shares that device's array (each call
 * rewrites all of it before reading it): calls that overlap on one device,
 * on different streams or host threads, race.  Double precision; the
 * result equals fg_project's to rounding.  Does not synchronise.
 * Errors: FG_E_ARG, FG_E_SIZE, FG_E_HIP. */
fg_status fg_project_noalloc(const int grid[3], const double spacing[3], const double* x, double* y, void* stream);

/* 3-D real transform of ncomp scalar fields, double precision, in place:
 * fg_fft_r2c turns ncomp real fields (ncomp N doubles) into the packed half
 * spectrum (the same bytes: ncomp x N0 x N1 x N2/2 complex, where the kx = 0
 * entry of each (kz, ky) line holds the real DC-plane value in .x and the
 * real Nyquist-plane value in .y only after the N2 pass; after all three
 * passes kx = 0 holds A + i B with A, B the 2-D spectra of the kx = 0 and
 * kx = N2/2 planes).  fg_fft_c2r is its exact inverse including the 1/N
 * normalisation.  Diagnostic entry points (parity of the transform). */
fg_status fg_fft_r2c(fg_plan* plan, double* data, int ncomp);
fg_status fg_fft_c2r(fg_plan* plan, double* data, int ncomp);

/* Phase-field problem (Alg. 2): update the history H <- max(H, gc/(2 lc)
 * D_f(sigma)) from the current F and c (eqs. (7), (8), effective Cauchy
 * stress), then solve [gc/lc + 2H] d - gc lc Lap d = 2H (eq. (32)) for d by
 * CG with the preconditioner of eq. (36), to ||r|| <= tol_lin ||b||.
 * stats: lin_iters_last, lin_relres.  Errors: FG_E_STATE, FG_E_NOCONV,
 * FG_E_BREAKDOWN, FG_E_HIP. */
fg_status pff_solve(fg_plan* plan, const fg_solver_opts* opts, fg_stats* stats);

/* Backward-Euler Fick step (Alg. 3, eq. (42)): Newton on
 * f(c) = c - c_t + dt div[M(d) c_t(1-c_t) C^-1 grad mu(c)] - dt cdot_B with
 * the linear step solved by preconditioned CG in dmu = w dc (w = RT(1/c +
 * 1/(1-c))); stops when ||dc|| / ||c_t|| < tol_newton.  Uses the stored F
 * and d.  cdot_B: device, N doubles (source of eq. (37)/(40)), may be NULL.
 * Errors: FG_E_STATE, FG_E_DOMAIN (c leaves (0,1)), FG_E_NOCONV,
 * FG_E_BREAKDOWN, FG_E_HIP. */
fg_status fick_step(fg_plan* plan, double dt, const double* cdot_B, const fg_solver_opts* opts,
                    fg_stats* stats);

/* Fully implicit form of fick_step: the same backward-Euler equation
 * f(c) = 0 (eq. (43)), with the Newton linearisation of eq. (45) extended by
 * the elastic part of the chemical potential, d mu/dc = RT (1/c + 1/(1-c))
 * + d(mu_e / c_max)/dc at the stored F and d, so Newton converges
 * quadratically to the same c (the paper linearises mu_c only).  The
 * linear step stays SPD PCG in dmu while d mu/dc > 0; a voxel where it is not
 * returns FG_E_DOMAIN.  Arguments, outputs and errors as fick_step. */
fg_status fick_step_full(fg_plan* plan, double dt, const double* cdot_B, const fg_solver_opts* opts,
                         fg_stats* stats);

/* ---------------------------------------------------------------------
 * Batched form of Alg. 1: n_rve RVEs (each with its own grid, spacing and
 * material) times n_cases macroscopic load cases, every (RVE, case) pair an
 * independent Newton solve started from the undeformed reference state with
 * F = F_macro[case] uniform.  Items of one grid share every kernel launch
 * (item-major fields, converged items masked on the device); each grid runs
 * on a stream of its own, forked from and joined into a batch stream that
 * the library creates (default priority).  With graph_ticks > 0 the solve
 * replays one captured hipGraph holding graph_ticks steps of every item (a
 * step is one CG iteration, or the Newton update, residual test and new
 * right-hand side once the item's CG has ended); the host reads one counter
 * per group between replays.  With graph_ticks = 0 the same steps are
 * launched directly, 8 per read-back; both give identical results.
 * Pure mechanics: d = 0, the chemistry enters only through a fixed c. */

/* grids: 3 ints per RVE, spacings: 3 doubles per RVE (host).  stream: the
 * caller's stream, on which the inputs of fg_batch_set_material and the
 * outputs are ordered.  Errors: FG_E_ARG, FG_E_SIZE, FG_E_HIP. */
fg_status fg_batch_create(int n_rve, const int* grids, const double* spacings, int n_cases, fg_precision prec,
                          void* stream, fg_batch** out);
/* Device workspace bytes (all groups: plans, item-major material copies,
 * F of every item, control blocks), and the number of grid groups. */
size_t fg_batch_workspace_bytes(const fg_batch* batch);
int fg_batch_groups(const fg_batch* batch);
/* Caller-owned, 256-byte aligned device buffer of at least
 * fg_batch_workspace_bytes.  Synchronises.  Errors: FG_E_ARG, FG_E_SIZE. */
fg_status fg_batch_set_workspace(fg_batch* batch, void* dev, size_t bytes);
/* Material of RVE rve (device, N_rve doubles each; c may be NULL for c = 0):
 * copied into the batch for each load case, so the caller's buffers may be
 * reused on return.  Errors: FG_E_ARG, FG_E_STATE (no workspace). */
fg_status fg_batch_set_material(fg_batch* batch, int rve, const double* E, const double* nu, const double* Omega,
                                const double* c);
/* Solve every item: F_macro host, 9 n_cases doubles (case-major); P_avg
 * host, 9 n_rve n_cases doubles ((rve n_cases + case) 9 + ij), may be NULL;
 * stats host, n_rve n_cases entries in the same order, may be NULL (the
 * histories hold the first 32 Newton iterations).  Returns the status of
 * the first failing item (FG_E_NOCONV, FG_E_BREAKDOWN, FG_E_DOMAIN) with its
 * index in fg_batch_last_error; every item's outputs are written anyway. */
fg_status fg_batch_newton_solve(fg_batch* batch, const double* F_macro, const fg_solver_opts* opts, int graph_ticks,
                                double* P_avg, fg_stats* stats);
/* Schedule of the batched solve: the Newton step (with its masked launches
 * over every item of every group) runs in every newton_every-th step of the
 * sequence, 1 <= newton_every <= 64 (default 1); an item whose CG has ended
 * waits for the next such step.  graph_ticks must then be a multiple of
 * newton_every.  Results do not depend on the schedule.  Errors: FG_E_ARG. */
fg_status fg_batch_set_schedule(fg_batch* batch, int newton_every);
/* Copy F of item (rve, lcase) into F (device, 9 N_rve doubles). */
fg_status fg_batch_state(fg_batch* batch, int rve, int lcase, double* F);
const char* fg_batch_last_error(const fg_batch* batch);
void fg_batch_destroy(fg_batch* batch);

/* Group g of a batch (items of one grid) as a plan handle owned by the
 * batch: only the tile calls below accept it (others return FG_E_ARG) and
 * fg_plan_destroy ignores it.  NULL for a bad index. */
fg_plan* fg_batch_plan(fg_batch* batch, int group);
/* Grid (3 ints) and item count of group g; 0, or -1 for a bad index. */
int fg_batch_group_info(const fg_batch* batch, int group, int grid[3], int* nitems);

/* ---------------------------------------------------------------------
 * Tile widths of the two column passes, for the autotuner: the complex
 * pass along N1 and the N0 pass fused with the projection of eq. (28) work
 * on `tile` adjacent kx columns per workgroup.  Pass index `which`:
 * 0 = N1 pass FP64, 1 = N0 projection pass FP64, 2 = N1 pass FP32,
 * 3 = N0 projection pass FP32 (the single-precision passes run in FG_MIXED
 * plans).  Valid tiles are powers of two dividing N2/2 with (threads per
 * line) x tile <= 256 and the LDS of the workgroup within 64 KiB; 0 selects
 * the built-in choice (the largest valid tile, ky-major for the projection
 * passes).  Results do not depend on
 * the tile: every column is transformed by the same arithmetic.  A tile of
 * the projection passes (1, 3) may carry FG_TILE_KY_MAJOR: its workgroups are
 * then ordered ky fastest instead of kx tile fastest.  A tile of the
 * single-precision N1 pass (2) may carry FG_TILE_COLUMN_PAIRS: each thread
 * then owns two adjacent columns (one 16-byte access; tile / 2 x threads per
 * line <= 256). */
enum { FG_TILE_KY_MAJOR = 0x10000, FG_TILE_COLUMN_PAIRS = 0x20000 };
/* Valid tiles of pass `which` into out[cap] (ascending, then for the
 * projection passes the same widths with FG_TILE_KY_MAJOR); returns how many
 * there are (may exceed cap), -1 on bad arguments. */
int fg_plan_tile_candidates(const fg_plan* plan, int which, int* out, int cap);
/* Set the four tiles (0 = built-in).  Errors: FG_E_ARG (invalid tile; the
 * plan keeps its previous tiles). */
fg_status fg_plan_set_tiles(fg_plan* plan, const int tiles[4]);
/* The four tiles in use (built-in choice resolved). */
fg_status fg_plan_get_tiles(const fg_plan* plan, int tiles[4]);
/* Mean time in milliseconds of one launch of pass `which` with `tile`
 * (0 = built-in) over all items of the plan, from reps launches after one
 * warm-up, HIP events on the plan stream.  Overwrites the plan's spectral
 * work buffer (state and material are untouched).  Synchronises.
 * Errors: FG_E_ARG (bad pass or tile, FP32 pass on an FG_FP64 plan),
 * FG_E_STATE (no workspace), FG_E_HIP. */
fg_status fg_plan_time_pass(fg_plan* plan, int which, int tile, int reps, double* ms);

/* Kernel classes timed by fg_profile_*: */
enum {
  FG_PASS_FRONT = 0,        /* CG front: x, p updates, K:p, p.Kp, N2 pass  */
  FG_PASS_R2C = 1,          /* real-to-complex pass along N2 (residuals)   */
  FG_PASS_AXIS = 2,         /* complex pass along N1 (forward and inverse) */
  FG_PASS_ZPROJ = 3,        /* N0 pass fused with the projection           */
  FG_PASS_C2R = 4,          /* N2 complex-to-real pass (9 components)      */
  FG_PASS_CG_UPDATE = 5,    /* vector updates of the scalar PCGs           */
  FG_PASS_FINALIZE = 6,     /* one-block reductions of the Krylov scalars  */
  FG_PASS_CONSTITUTIVE = 7, /* stress and tangent state                    */
  FG_PASS_ZSCALAR = 8,      /* N0 pass fused with a scalar symbol          */
  FG_PASS_AXIS3 = 9,        /* inverse N1 pass of the 3-component potential */
  FG_PASS_C2R3 = 10,        /* inverse N2 pass of the potential            */
  FG_PASS_GRAD = 11,        /* residual update rho -= a U and |D rho|^2    */
  FG_NPASS = 12
};

/* Time every launch of each kernel class with a HIP event pair on the plan
 * stream, from fg_profile_begin until fg_profile_end, which synchronises and
 * returns the summed milliseconds ms[FG_NPASS] and the number of launches
 * launches[FG_NPASS] per class (host arrays).  Launches of the CG loop that
 * found the solve already converged (they exit at once, a few microseconds)
 * are not counted in launches[].  Measurement support for the benchmark;
 * adds two event records per launch while enabled. */
fg_status fg_profile_begin(fg_plan* plan);
fg_status fg_profile_end(fg_plan* plan, double ms[], long launches[]);

/* Restrict the timing to the kernel classes whose bit (1 << FG_PASS_*) is
 * set in mask (default: all); the others then cost no event records.  Not
 * while profiling is on.  Errors: FG_E_ARG. */
fg_status fg_profile_passes(fg_plan* plan, unsigned mask);

const char* fg_status_string(fg_status s);
const char* fg_last_error(const fg_plan* plan);
void fg_plan_destroy(fg_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* FGFFT_H */
