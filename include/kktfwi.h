/*
 * kktfwi.h - C ABI of the MI355X (gfx950) full-space Gauss-Newton KKT solver for
 * 2-D frequency-domain acoustic full-waveform inversion with PML
 * (Malovichko, Orazbayev, Khokhlov, "Iterative PDE-constrained optimization for
 * seismic full-waveform inversion", arXiv 2204.06489).
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Pointers are DEVICE pointers owned by the caller unless marked [host].  The
 *   library never keeps a caller pointer after the call returns; gamma and the
 *   acquisition arrays are copied.
 * - Complex numbers are interleaved (re, im): c128 = two doubles, c64 = two floats.
 * - Wavefields are [K][nz][nx] row-major (x fastest).  Node (i, j) is at
 *   x = i*h, z = j*h; the listed nx x nz nodes include the PML strips and the
 *   field is zero outside them (U = 0 on the boundary, Section 2).
 * - The control is the squared slowness on the core (non-PML) nodes,
 *   [nz - 2 npml][nx - 2 npml] row-major; Ng = (nx - 2 npml)(nz - 2 npml).
 * - Packed KKT vectors xi = (du, ds, lambda) are
 *   [ du_0 .. du_{K-1} | ds | lambda_0 .. lambda_{K-1} ], length 2*K*nx*nz + Ng,
 *   c128 (the stacking of eq. partitioned_system_matrix, Section 5).
 * - All device work is ordered on the problem's HIP stream.  Calls that return
 *   statistics (helmholtz_solve, newton_step, helmholtz_adjoint_gradient, the
 *   factorisation) synchronise that stream before returning; kkt_apply and
 *   precond_apply are asynchronous.
 * - Errors are returned as kf_status; no exception crosses the ABI.  Argument
 *   validation happens before any HIP call; the message of the last failure on
 *   the calling thread is kf_last_error().  On KF_ENOCONV the outputs hold the
 *   last iterate and the statistics are filled; after any other error the
 *   outputs are unspecified.
 * - One problem is used by one host thread at a time.
 */
#ifndef KKTFWI_H
#define KKTFWI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kf_problem kf_problem;

typedef enum {
  KF_OK = 0,
  KF_EINVAL = 1,      /* invalid argument (null pointer, eps <= 0, node off the grid, ...) */
  KF_ESHAPE = 2,      /* inconsistent sizes */
  KF_ENOMEM = 3,      /* device allocation failed */
  KF_EHIP = 4,        /* a HIP runtime call failed */
  KF_ENOCONV = 5,     /* iteration limit reached before the tolerance */
  KF_EBREAKDOWN = 6,  /* Krylov breakdown (zero or non-finite Arnoldi norm) */
  KF_ENAN = 7,        /* non-finite residual */
  KF_ESTATE = 8       /* call needs state that is not set (e.g. no background field) */
} kf_status;

/* Arithmetic of Helmholtz block solves. */
typedef enum {
  KF_C128 = 0,   /* complex128 buffers, FP64 factors: direct solve to rounding */
  KF_C64 = 1,    /* complex64 buffers and factors (FP32 arithmetic and accumulation) */
  KF_MIXED = 2   /* complex128 buffers; complex64 factors inside FP64 iterative
                    refinement until the relative residual meets rtol */
} kf_prec;

/* Preconditioner of the KKT system (Section 5). */
typedef enum {
  KF_PC_EXACT = 0,     /* eq. precond: A and A^* solved exactly (FP64 factors) */
  KF_PC_INEXACT = 1,   /* eq. precond_approx: A replaced by A~ = the complex64
                          factorisation of A (one sweep per block solve) */
  KF_PC_MULTIGRID = 2  /* eq. precond_approx with A~^-1 = BiCGStab on A preconditioned by
                          one shifted-Laplacian multigrid V-cycle, stopped at the inner
                          tolerance of kf_set_multigrid (Section 5's suggested A~) */
} kf_pc;

/* Problem description (Sections 2-4).  Arrays marked [host] are copied. */
typedef struct {
  int32_t nx, nz;          /* grid nodes including the PML strips (>= 3 each) */
  double h;                /* grid spacing, metres (> 0) */
  int32_t npml;            /* PML width in cells on all four sides (0 <= 2 npml < min(nx, nz)) */
  double pml_r0;           /* design reflection of the quadratic PML profile, 0 < r0 < 1 */
  double pml_cref;         /* reference speed of the PML profile, m/s (> 0) */
  double omega;            /* circular frequency 2 pi f, rad/s (> 0) */
  int32_t K;               /* number of sources (>= 1) */
  const int32_t *src_ix;   /* [host][K] source node columns; f_k = e_src / h^2 (unit point source) */
  const int32_t *src_iz;   /* [host][K] source node rows */
  int32_t nrec;            /* receivers per source (>= 1); the same nodes for every source */
  const int32_t *rec_ix;   /* [host][nrec] receiver node columns (Dirac receivers on nodes) */
  const int32_t *rec_iz;   /* [host][nrec] receiver node rows */
  const double *w;         /* [host][K][nrec] real receiver weights W_k, or NULL for W = I */
  double eps;              /* L = eps * I on the control (> 0; the preconditioner needs L^-1) */
  int32_t reg_on_update;   /* 0: b_s = -eps s_n (eq. KKT); 1: b_s = 0, i.e. the -L s_n := 0
                              variant of the multi-frequency experiment (Section 6) */
} kf_desc;

typedef struct {
  double rtol;             /* relative residual target of one Newton-step KKT solve */
  int32_t restart;         /* FGMRES restart length m (1..200) */
  int32_t maxit;           /* total outer iteration limit */
  int32_t pc;              /* kf_pc */
  int32_t fwd_prec;        /* kf_prec of the background forward solve u_n = A^-1 f (C128 or MIXED) */
  double fwd_rtol;         /* tolerance of that solve when fwd_prec = KF_MIXED */
  int32_t misfit_after;    /* 1: also solve A(gamma_{n+1}) u = f and report the new misfit */
  double reorth_eta;       /* Gram-Schmidt of the Arnoldi steps: after the first classical pass
                              w' = w - V V^* w a second pass runs when |w'| < reorth_eta |w|
                              (0 <= reorth_eta <= 1; 1: always, i.e. CGS2; 1/sqrt 2: the
                              Daniel-Gragg-Kaufman-Stewart test; 0: never).  One pass leaves the
                              new vector orthogonal to about eps |w| / |w'|, so 0.1 keeps the
                              basis orthogonal to ~1e-15 while skipping the pass whenever the
                              cancellation is mild; FGMRES's true residual at each restart and
                              at exit checks the result either way. */
  int32_t outer;           /* KF_OUTER_FGMRES (restarted flexible GMRES, 2 restart + 1 packed
                              vectors) or KF_OUTER_BICGSTAB (right-preconditioned BiCGStab, the
                              Conclusions' memory-lean alternative: nine packed vectors, two
                              preconditioner applications and KKT matvecs per iteration, a
                              fixed preconditioner assumed; restart and reorth_eta unused) */
} kf_newton_opts;
typedef enum { KF_OUTER_FGMRES = 0, KF_OUTER_BICGSTAB = 1 } kf_outer;

typedef struct {
  int32_t outer_iters;     /* FGMRES iterations taken */
  int32_t restarts;        /* completed restart cycles */
  double rel_res;          /* true ||b - M xi|| / ||b|| at exit (recomputed with kkt_apply) */
  double rel_res_hist[512];/* FGMRES residual estimate per iteration (first 512) */
  double misfit_before;    /* ||d - Q u_n|| / ||d|| */
  double misfit_after;     /* ||d - Q u_{n+1}|| / ||d|| (if requested, else -1) */
  double phi_before;       /* 1/2 sum_k ||W_k (d_k - Q u_k)||^2 */
  double ds_imag_ratio;    /* ||Im ds|| / ||ds|| */
  double t_factor_ms;      /* time in the block factorisation(s) */
  double t_forward_ms;     /* background forward solve */
  double t_precond_ms;     /* preconditioner applications */
  double t_matvec_ms;      /* kkt_apply calls */
  double t_orth_ms;        /* orthogonalisation, Givens, updates */
  double t_total_ms;       /* whole call */
  int32_t fwd_refine_iters;/* refinement sweeps of the forward solve (KF_MIXED) */
  int32_t reorth_passes;   /* Arnoldi steps that needed the second Gram-Schmidt pass */
} kf_newton_stats;

typedef struct {
  int32_t iters;           /* sweeps (1 for a direct solve; refinement steps for KF_MIXED) */
  double rel_res_max;      /* max over sources of ||rhs_k - A x_k|| / ||rhs_k|| (computed
                              when rtol > 0 or the precision is KF_MIXED, else -1) */
} kf_solve_stats;

/* Library version string. */
const char *kf_version(void);
/* Message of the last failed call on this thread ("" if none). */
const char *kf_last_error(void);

/* Create a problem: validates and copies the description and gamma ([nz][nx] FP64, host
 * or device: `gamma_on_device` says which), allocates device state and builds the PML
 * coefficients (Section 2).  `hip_stream` is a hipStream_t (NULL = default stream).
 * Every gamma entry must be finite (checked on the host, or by a device reduction for a
 * device gamma): otherwise KF_EINVAL and no problem is created. */
kf_status kf_create(const kf_desc *desc, const double *gamma, int32_t gamma_on_device,
                    void *hip_stream, kf_problem **out);
kf_status kf_destroy(kf_problem *p);
/* Replace gamma (device pointer, [nz][nx]); invalidates the factorisation and u_n.
 * The entries are checked by a device reduction first (the call synchronises the
 * stream): a NaN or inf gives KF_EINVAL and leaves the problem's gamma, factors and
 * u_n as they were, so no non-finite value reaches the factorisation. */
kf_status kf_set_gamma(kf_problem *p, const double *gamma);
/* Read gamma back into a device buffer [nz][nx]. */
kf_status kf_get_gamma(kf_problem *p, double *gamma_out);
/* Set the background fields u_n (c128 [K][nz][nx], device) used by P = omega^2 diag(u_n)
 * in kkt_apply and precond_apply (eq. P). */
kf_status kf_set_background(kf_problem *p, const void *u_n);
/* Copy u_n out (c128 [K][nz][nx], device). */
kf_status kf_get_background(kf_problem *p, void *u_n_out);
/* Change the stream used by subsequent calls. */
kf_status kf_set_stream(kf_problem *p, void *hip_stream);
/* Shape of the block solver (any time; a change invalidates the factorisation).
 * chunks: the grid columns are cut into `chunks` pieces by chunks - 1 separator columns;
 * every piece is factorised and swept independently and a block-tridiagonal system on
 * the separators (their Schur complement, solved by block cyclic reduction in about
 * log2(chunks) levels) joins them, so more chunks means more parallel work and shorter
 * sequential sweeps, plus more reduction levels and correction work.  1 <= chunks <=
 * min(64, (nx + 1) / 2); 0 picks round(1.6 sqrt(nx)) (1 below nx = 32).
 * sources_per_group: right-hand sides per workgroup in the block solves, 1, 2, 4 or 8
 * (0 = 1; FP64 solves use at most 4).  Results do not depend on either beyond rounding. */
kf_status kf_set_solver_shape(kf_problem *p, int32_t chunks, int32_t sources_per_group);
kf_status kf_get_solver_shape(kf_problem *p, int32_t *chunks /*[host]*/, int32_t *sources_per_group /*[host]*/);
/* Autotuner of the solver shape: for chunk counts around the automatic choice (and 1),
 * then for the counts within 2 of the best of those, it builds the factorisation (FP64, plus the complex64 copy when prec = KF_C64), and for
 * each sources_per_group it times forward and adjoint block solves of all K sources
 * (complex64 sweeps with c128 I/O when prec = KF_C64, as in the inexact preconditioner;
 * FP64 otherwise) with HIP events on the problem's stream.  The score of a shape is
 * t_factor + solves_per_factor * t_solve; the best is set on the problem and remembered
 * for the process, keyed by (nx, nz, K, prec): later kf_create calls of that size start
 * from it.  A solve after the call rebuilds the factorisation if the chosen shape was not
 * the last one measured.  table (may be
 * NULL) receives up to table_len measured entries, n_table their number. */
typedef struct {
  int32_t chunks, sources_per_group;
  double t_factor_ms, t_solve_ms, score_ms;
} kf_tune_entry;
kf_status kf_autotune(kf_problem *p, int32_t prec, double solves_per_factor, kf_tune_entry *table /*[host]*/,
                      int32_t table_len, int32_t *n_table /*[host], may be NULL*/);
/* Build the block factorisation of A(gamma, omega) now (it is otherwise built on the first
 * solve that needs it).  `which`: bit 0 = FP64 factors, bit 1 = complex64 copy. */
kf_status kf_factor(kf_problem *p, int32_t which, double *t_ms /*[host], may be NULL*/);

/* y = A x or y = A^H x for all K sources (the 5-point PML Helmholtz operator of Section 2,
 * eq. Au=f).  x, y: [K][nz][nx] c128 (prec KF_C128) or c64 (KF_C64). Asynchronous. */
kf_status kf_stencil_apply(kf_problem *p, int32_t adjoint, int32_t prec, const void *x, void *y);

/* Solve A x_k = rhs_k (adjoint = 0) or A^H x_k = rhs_k (adjoint = 1) for all K sources:
 * the K independent block solves of the stacked forward problem (Section 2, eq. helmholtz).
 * prec: kf_prec.  rhs and x may alias.  rtol is the refinement target for KF_MIXED
 * (ignored otherwise, except that rtol > 0 makes the call report the residual).
 * maxit bounds the refinement sweeps.  Returns KF_ENOCONV if KF_MIXED misses rtol. */
kf_status helmholtz_solve(kf_problem *p, int32_t adjoint, int32_t prec, const void *rhs, void *x,
                          double rtol, int32_t maxit, kf_solve_stats *st /*[host], may be NULL*/);

/* y = M xi with the KKT matrix of eq. KKT,
 *   M = [[F, 0, A^*], [0, L, -P^*], [A, -P, 0]],  F_k = Q^T W_k^2 Q,  P_k = omega^2 diag(u_k) E,
 * applied matrix-free (needs kf_set_background or a previous newton_step).  xi, y: packed
 * c128 (no aliasing).  Asynchronous. */
kf_status kkt_apply(kf_problem *p, const void *xi, void *y);

/* kkt_apply for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and
 * result as kkt_apply (up to the order of the sum over source groups), but the source
 * groups' parts of the control row live in a file-scope device array of
 * KF_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends, instead of the
 * problem's buffer.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine); the problem, xi and y are the caller's.  A control row of more than
 * KF_NOALLOC_SCRATCH_BYTES / 16 nodes gives KF_ESHAPE; fewer source groups are used when
 * the array holds fewer than kkt_apply would take.  Calls on one GPU share the array:
 * calls that overlap (different streams or threads) race.  Asynchronous. */
#define KF_NOALLOC_SCRATCH_BYTES (64u << 20)
kf_status kkt_apply_noalloc(kf_problem *p, const void *xi, void *y);

/* z = P^-1 y for the block-triangular preconditioner of eq. precond (pc = KF_PC_EXACT) or
 * eq. precond_approx (KF_PC_INEXACT):
 *   z_lam = A^-* y_u;  z_s = (y_s + P^* z_lam) / eps;  z_u = A^-1 (y_lam + P z_s).
 * y, z packed c128 (no aliasing).  Asynchronous. */
kf_status precond_apply(kf_problem *p, int32_t pc, const void *y, void *z);

/* One full-space Gauss-Newton step (Sections 3-5):
 *   u_n = A(gamma_n)^-1 f;  r_k = d_k - Q u_k;  b = [Q^T W^2 r ; -eps s_n or 0 ; 0];
 *   solve M xi = b by right-preconditioned flexible GMRES to ||b - M xi|| <= rtol ||b||;
 *   gamma_{n+1} = gamma_n + Re(ds) on the core (PML values unchanged).
 * d_obs: [K][nrec] c128 device.  xi_out: packed c128 device or NULL.  gamma_next: device
 * [nz][nx] receiving gamma_{n+1}, or NULL.  update_in_place = 1 also makes gamma_{n+1} the
 * problem's gamma (for the next step); with 0 the problem keeps gamma_n, so kkt_apply and
 * precond_apply still describe the system that was solved.  u_n stays available as the
 * background (kf_get_background).  Returns KF_ENOCONV (outputs and stats filled) if
 * maxit is reached first. */
kf_status newton_step(kf_problem *p, const void *d_obs, const kf_newton_opts *opts /*[host]*/,
                      void *xi_out, double *gamma_next, int32_t update_in_place,
                      kf_newton_stats *st /*[host], may be NULL*/);

/* Frequency continuation (Section 6, the frequency sweep: the frequencies are
 * inverted one after another from low to high, each starting from the model the
 * previous one reached, with its own eps, i.e. the eps ramp).  problems[0..n) share
 * the grid (nx, nz, h, npml; KF_ESHAPE otherwise) and are ordered by frequency;
 * steps[q] >= 0 full Newton steps (newton_step with opts, gamma updated in place) run
 * on problem q from the gamma problem q-1 ended with (problem 0 starts from its own).
 * d_obs[q] is problem q's data ([K][nrec] c128 device).  gamma_out: device [nz][nx]
 * receiving the final gamma, or NULL.  st: [host] array of sum(steps) entries, the
 * statistics of every step in order, or NULL.  The first failing step's status is
 * returned (its statistics filled); later problems are then not touched. */
kf_status newton_continuation(kf_problem *const *problems /*[host][n]*/, int32_t n,
                              const void *const *d_obs /*[host][n]*/, const int32_t *steps /*[host][n]*/,
                              const kf_newton_opts *opts /*[host]*/, double *gamma_out,
                              kf_newton_stats *st /*[host], may be NULL*/);

/* One Newton step (newton_step with opts) on each of n independent problems (e.g. one
 * per frequency on its own grid, Section 6's multi-frequency setting) at once: for the
 * call every problem runs on a stream of its own, created here, driven by a host thread
 * of its own, so that the launches of one problem's latency-bound phases (block-solve
 * chains, reduction levels, host round trips of its Krylov iteration) overlap the
 * other problems' work.  Each problem computes exactly what newton_step computes alone.
 * problems: [host][n] distinct problems, 1 <= n <= 16; d_obs: [host][n], problem q's
 * data ([K][nrec] c128 device); xi_out, gamma_next: [host][n] arrays of newton_step's
 * outputs (the arrays or their entries may be NULL); st: [host][n] statistics or NULL.
 * The call first waits for the work already queued on the problems' own streams and
 * gives them their streams back before it returns; no other call may use these
 * problems meanwhile.  Every problem is stepped whatever the others return.  Returns
 * the first status other than KF_OK and KF_ENOCONV in problem order (kf_last_error
 * names the problem), else KF_ENOCONV if a problem reached maxit, else KF_OK. */
kf_status newton_step_concurrent(kf_problem *const *problems /*[host][n]*/, int32_t n,
                                 const void *const *d_obs /*[host][n]*/, const kf_newton_opts *opts /*[host]*/,
                                 void *const *xi_out /*[host][n] or NULL*/,
                                 double *const *gamma_next /*[host][n] or NULL*/, int32_t update_in_place,
                                 kf_newton_stats *st /*[host][n], may be NULL*/);

/* ---- reduced-space Gauss-Newton by conjugate gradients (Section 3) ----
 * The step the paper compares the full-space method with (Table 1 "CG"): with
 * u_n = A(gamma_n)^-1 f and r_k = d_k - Q u_k, CG on the normal equations
 *   H ds = g,  H = eps I + sum_k J_k^* W_k^2 J_k,  g = sum_k J_k^* W_k^2 r_k - eps s_n
 * (eqs. normal_system_discrete2 and normal_system_discrete_sum; the -eps s_n term is
 * dropped with reg_on_update, as in the KKT right-hand side), J_k = Q A^-1 P_k.  Every
 * Hessian product is one forward and one adjoint block solve of all K sources (the
 * solves the paper counts per CG iteration), P_k v and P^* lambda in between.  CG stops
 * at ||H ds - g|| <= rtol ||g|| (E_cg of Section 6); the true E_cg is recomputed at
 * exit.  real_constrained = 1 solves the real-constrained step instead: ds real with
 * Re(H) ds = Re(g), the normal equations of the GN problem over real updates (the real
 * model takes Re(ds) of the complex-linear step otherwise). */
typedef struct {
  double rtol;             /* CG stopping tolerance on ||H ds - g|| / ||g|| */
  int32_t maxit;           /* CG iteration limit */
  int32_t solve_prec;      /* the block solves of each Hessian product: KF_C128 (FP64 factors)
                              or KF_MIXED (complex64 factors in FP64 refinement to solve_rtol) */
  double solve_rtol;       /* refinement target when solve_prec = KF_MIXED */
  int32_t real_constrained;/* 1: real ds with Re(H) ds = Re(g) */
  int32_t fwd_prec;        /* background solve: KF_C128 or KF_MIXED (to fwd_rtol) */
  double fwd_rtol;
} kf_cg_opts;
typedef struct {
  int32_t iters;           /* CG iterations (Hessian products) */
  int32_t solves;          /* batched block solves of all K sources, gradient and check included */
  double rel_res;          /* ||H ds - g|| / ||g|| by the CG recurrence at exit */
  double true_rel_res;     /* the same recomputed with one more Hessian product */
  double rel_res_hist[512];/* recurrence residual per iteration (first 512) */
  double misfit_before;    /* ||d - Q u_n|| / ||d|| */
  double phi_before;       /* 1/2 sum_k ||W_k (d_k - Q u_k)||^2 */
  double t_factor_ms, t_forward_ms, t_cg_ms, t_total_ms;
} kf_cg_stats;
/* ds_out: [Ng] c128 device or NULL; gamma_next / update_in_place as in newton_step.
 * Returns KF_ENOCONV (outputs and stats filled) if maxit is reached first. */
kf_status rsgn_cg_step(kf_problem *p, const void *d_obs, const kf_cg_opts *opts /*[host]*/, void *ds_out,
                       double *gamma_next, int32_t update_in_place, kf_cg_stats *st /*[host], may be NULL*/);

/* Reduced gradient through the forward solve (Section 3, gradient; Section 4, eq. tmp2):
 * for u = A(gamma)^-1 f and grad_u = dl/dRe(u) + i dl/dIm(u) (both [K][nz][nx], c128 or
 * c64 per prec), computes mu = A^-H grad_u and
 *   grad_gamma[j][i] = omega^2 sum_k Re(conj(mu_k) X_i Z_j u_k)     ([nz][nx], FP64),
 * which on the core equals omega^2 sum_k Re(conj(mu_k) u_k).  Synchronous. */
kf_status helmholtz_adjoint_gradient(kf_problem *p, int32_t prec, const void *u, const void *grad_u,
                                     double *grad_gamma);

/* ---- shifted-Laplacian multigrid: the inexact block solver of KF_PC_MULTIGRID ----
 * Section 5 names the shifted-Laplacian preconditioner, inverted approximately by
 * multigrid, as the better A~ for eq. precond_approx; the paper gives no details.  The
 * library takes: the shifted operator M = A(gamma (1 + i beta)); levels by standard
 * coarsening of the vertex grid (n -> (n + 1) / 2 while both sizes are odd and the
 * smaller one is at least n_min; spacing doubled, PML width halved, gamma injected), M
 * rediscretised on every level; one z-line then one x-line Jacobi sweep before the
 * coarse-grid correction and the reverse after it; full-weighting restriction, bilinear
 * prolongation; the coarsest level solved exactly by the block factorisation of its M.
 * Each block solve is BiCGStab on A for all K sources in lock step (own scalars per
 * source), right-preconditioned by one V-cycle, stopped when every source meets
 * ||b_k - A x_k|| <= rtol ||b_k|| (by the recurrence).  A^H x = b is solved as
 * A conj(x) = conj(b).  The hierarchy is rebuilt when gamma changes. */
typedef struct {
  int32_t iters;           /* BiCGStab iterations (all sources in lock step) */
  int32_t vcycles;         /* V-cycles applied (two per iteration) */
  int32_t levels;          /* multigrid levels, the coarsest included */
  double rel_res_max;      /* true max_k ||b_k - op(A) x_k|| / ||b_k|| in FP64 (-1 when b and x alias) */
} kf_mg_stats;
/* prec: KF_C64 (complex64 fields, FP32 arithmetic, FP64 inner products) or KF_C128;
 * beta > 0 the shift (0.5 is the usual choice); 0 < inner_rtol < 1 and inner_maxit >= 1
 * for the block solves of KF_PC_MULTIGRID; n_min >= 3.  Defaults before any call:
 * KF_C64, 0.5, 1e-3, 200, 20. */
kf_status kf_set_multigrid(kf_problem *p, int32_t prec, double beta, double inner_rtol, int32_t inner_maxit,
                           int32_t n_min);
/* A x = rhs (adjoint = 0) or A^H x = rhs (1) for all K sources by the multigrid-
 * preconditioned BiCGStab to rtol (c128 rhs, x; they may alias).  KF_ENOCONV (x and stats
 * filled) if maxit iterations do not reach rtol; KF_ESHAPE if the grid has no coarser level.
 * Synchronous. */
kf_status helmholtz_solve_mg(kf_problem *p, int32_t adjoint, const void *rhs, void *x, double rtol, int32_t maxit,
                             kf_mg_stats *st /*[host], may be NULL*/);
/* x = V(b): one V-cycle of the shifted operator for every source from x = 0 (c128 b, x,
 * distinct), in the configured precision.  Asynchronous. */
kf_status kf_mg_vcycle(kf_problem *p, const void *b, void *x);
/* The hierarchy built so far: nlev levels, dims[2 l], dims[2 l + 1] = nx, nz of level l
 * (dims [host][16]). */
kf_status kf_mg_levels(kf_problem *p, int32_t *dims /*[host][16]*/, int32_t *nlev /*[host]*/);

/* ---- the H-block of the preconditioner's middle stage (Section 5) ----
 * The block-triangular preconditioner keeps L in its middle stage,
 *   z_s = L^-1 (y_s + P^* z_lam);
 * Section 5 and the Conclusions note that other approximations of the reduced Hessian
 * H = L + sum_k J_k^* W_k^2 J_k can take its place, L-BFGS among them.  With
 * KF_HBLOCK_LBFGS the middle stage applies the L-BFGS inverse (two-loop recursion over
 * complex vectors, Re(y^H s) as the curvature, L = eps I as the initial matrix) built from
 * up to max_pairs pairs (s, H s): every newton_step that converges adds the pair
 * (ds, H ds) at gamma_n (one more forward and adjoint FP64 block solve of all sources),
 * and kf_hblock_add_pair adds a pair given by the caller (s, y = H s: [Ng] c128, device;
 * KF_EINVAL if Re(y^H s) <= 0).  kf_set_hblock clears the pairs.  KF_HBLOCK_EPS (the
 * default) is L itself. */
typedef enum { KF_HBLOCK_EPS = 0, KF_HBLOCK_LBFGS = 1 } kf_hblock;
kf_status kf_set_hblock(kf_problem *p, int32_t kind, int32_t max_pairs);
kf_status kf_hblock_add_pair(kf_problem *p, const void *s, const void *y);

/* Build the point sources f_k = e_src / h^2 of the problem into f ([K][nz][nx], c128). */
kf_status kf_sources(kf_problem *p, void *f);

/* Sizes of the problem: out[0..5] = nx, nz, K, nrec, Ng, packed length (as int64). */
kf_status kf_sizes(kf_problem *p, int64_t *out /*[host][6]*/);

/* Per-kernel timing with HIP events recorded around every launch of the named kernel
 * family on the problem's stream: enable (1) / disable (0) and reset the counters. */
kf_status kf_profile_enable(kf_problem *p, int32_t on);
/* Read accumulated (launch count, total milliseconds) of a kernel family:
 * "kkt_apply" (the fused kernel and, when it splits the sources into groups, the sum of
 * the groups' parts of the control row; without the receiver term), "stencil", "blu_factor" (the
 * whole FP64 factorisation: chunks, spikes and separator system), "blu_sweep" (a whole
 * block solve), "blu_fwd_c128", "blu_fwd_c64", "blu_bwd_c128", "blu_bwd_c64" (the chunks'
 * forward-sweep and back-substitution launches), "blu_mid", "blu_reduced_rhs",
 * "blu_chain", "blu_correct" (the middle columns, the separators' right-hand sides, the
 * separator system's cyclic-reduction levels, one launch per level, and the interior
 * correction), "precond_stage", "mg_solve" (a whole multigrid-preconditioned block solve), "gs_dot" (the first Gram-Schmidt pass's dot products of
 * each Arnoldi step, with the norm of the new vector), "gs_update" (that pass's fused,
 * normalising update), "orth" (the rest of the orthogonalisation: the occasional second
 * pass, the Hessenberg and solution updates), "reduce".
 * Unknown names give KF_EINVAL. */
kf_status kf_profile_read(kf_problem *p, const char *name, int64_t *launches, double *total_ms);
/* Algorithmic work of the launches of a kernel family recorded since profiling was
 * enabled, as the launchers count it: bytes that must cross HBM for "kkt_apply"
 * (N_u (80 K + 8) + 32 N_g per call), "gs_dot" (the first Gram-Schmidt pass's dot
 * products with |w|^2: nv + 1 packed vectors read) and "gs_update" (its update:
 * nv + 1 vectors read, one written); block bytes plus vector bytes for "blu_chain"
 * (the reduction levels); 0 for families that do not count it. */
kf_status kf_profile_work(kf_problem *p, const char *name, double *work /*[host]*/);
/* Restrict the recording to one kernel family (the names above), so that a timed run
 * carries the events of that family only; NULL or "" records every family again.
 * Counters are kept.  Unknown names give KF_EINVAL. */
kf_status kf_profile_only(kf_problem *p, const char *name);

/* ---- batches: several problems (e.g. frequencies on uneven grids) advanced together ----
 * The frequency sweep of Section 6 treats each frequency as its own Newton step; a batch
 * runs such independent problems together: every factorisation and every batched block
 * solve is one persistent work-list launch over all problems, and the preconditioner +
 * KKT matvec of each FGMRES column can be replayed from a captured hipGraph.  A batch
 * holds up to 8 problems (not owned: destroy the batch before its problems) and orders
 * all their work on its own stream (the problems' streams are set to it while the batch
 * exists; kf_batch_destroy gives each problem back the stream it had before).  With
 * hip_stream = NULL the batch creates a non-blocking stream of its own (the legacy NULL
 * stream cannot be captured); work the caller queued elsewhere must be complete (or
 * ordered by the caller) before a batched call. */
typedef struct kf_batch kf_batch;
kf_status kf_batch_create(kf_problem *const *problems /*[host][n]*/, int32_t n, void *hip_stream, kf_batch **out);
kf_status kf_batch_destroy(kf_batch *b);
/* Factorise every problem that needs it (which: bit 0 FP64 factors, bit 1 complex64 copy). */
kf_status kf_batch_factor(kf_batch *b, int32_t which, double *t_ms /*[host], may be NULL*/);
/* A x = rhs or A^H x = rhs for every source of every problem (prec KF_C128 or KF_C64);
 * rhs[q], x[q] are device fields of problem q ([host] arrays of n pointers). */
kf_status helmholtz_solve_batched(kf_batch *b, int32_t adjoint, int32_t prec, const void *const *rhs,
                                  void *const *x);
/* newton_step (above) for every problem together; per-problem arrays are [host][n] of
 * device pointers (xi_out, gamma_next entries may be NULL) and st is [host][n].  The
 * problems' FGMRES iterations advance in lockstep, each with its own scalars and its own
 * stopping test.  use_graph = 1 replays each Krylov column's preconditioner and matvec
 * for all problems from a captured hipGraph.  opts->fwd_prec must be KF_C128.  Where
 * each problem fills the chip on its own, each launch here lasts as long as its slowest
 * problem's items; newton_step_concurrent (above) overlaps whole problems instead. */
kf_status newton_step_batched(kf_batch *b, const void *const *d_obs, const kf_newton_opts *opts,
                              void *const *xi_out, double *const *gamma_next, int32_t update_in_place,
                              int32_t use_graph, kf_newton_stats *st);

#ifdef __cplusplus
}
#endif
#endif /* KKTFWI_H */
