/*
 * tpf.h -- C ABI of the MI355X (gfx950) two-phase porous-media stage solver.
 *
 * The library implements, on one GPU, the hot path of a fully coupled, fully
 * implicit two-phase (p_w, S_n) Darcy solver discretised with vertex-centred finite
 * volumes (the box method) on structured Q1 quads/hexes:
 *
 *   - create_grid:    upload the scenario, pre-process p_dmin per vertex
 *                     (interface condition, Section 3.3, Eq. pdmin) and the
 *                     Neumann sources;
 *   - residual:       F(u) of the semi-discrete system M(u) u' = F(u) (Section 4),
 *                     built from the storage and SCVF flux sums (Section 3.1,
 *                     Eqs. dsW/dpN) with upwinded mobilities (Section 3.2,
 *                     Eqs. up_krw/up_krn) and the p_dmin saturation rule
 *                     (Eq. hSw, krn_ip, krw_ip);
 *   - assemble_stage: A = M(u0)/h - J(u0), the linearly implicit Euler matrix of
 *                     Section 4 divided by the step, as 2x2-block 27-point (3D) or
 *                     9-point (2D) stencil rows, plus the geometric-multigrid
 *                     hierarchy (Galerkin coarse operators) used as preconditioner;
 *   - solve_stage:    A x = f by BiCGSTAB preconditioned with one GMG V-cycle
 *                     (the linear solver named in Section 1 and Section 5), point-
 *                     or line-block Jacobi smoothing (tpf_grid_desc.smoother);
 *   - limex_step:     one adaptive LIMEX step (Section 4: linearly implicit
 *                     extrapolation, error estimate in the scaled norm Eq. norm_u,
 *                     step-size rule with q = 2);
 *   - ie_step:        one fixed implicit Euler step with Newton's method, the
 *                     scheme Section 5 compares LIMEX with.
 *
 * Conventions
 *   - Device pointers are HIP device addresses owned by the caller (e.g. from a
 *     PyTorch CUDA/ROCm tensor).  The library never allocates device memory: all of
 *     its device state lives in a caller-provided arena of tpf_grid_bytes() bytes.
 *   - State/vector layout: double[2*N], interleaved (p_w [Pa], S_n [-]) per vertex,
 *     vertex index ix + nx*(iy + ny*iz) (x fastest).  Row 2v of a residual or
 *     matrix is the wetting-phase mass balance of vertex v, row 2v+1 the
 *     non-wetting one (kg/s).
 *   - Cell arrays have (nx-1)(ny-1)(nz-1) entries (2D: (nx-1)(ny-1)), x fastest.
 *   - Every call is asynchronous on the given stream unless stated; a grid must be
 *     used from one stream at a time.  Different grids are independent.
 *   - Status: 0 ok, > 0 soft outcome (outputs valid, see stats), < 0 hard error
 *     (outputs untouched); tpf_last_error() gives the message of the calling
 *     thread's last failure.
 */
#ifndef TPF_H
#define TPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tpf_status;
typedef struct tpf_grid tpf_grid; /* opaque; host metadata only */
typedef struct ihipStream_t *tpf_stream; /* hipStream_t */

enum {
  TPF_OK = 0,
  TPF_NOT_CONVERGED = 1,  /* solve hit maxit: x holds the last iterate        */
  TPF_STEP_REJECTED = 2,  /* limex: error > TOL, u and t unchanged, dt reduced */
  TPF_EINVAL = -1,        /* invalid argument / descriptor                     */
  TPF_ENOMEM = -2,        /* arena too small or misaligned                     */
  TPF_EDEVICE = -3,       /* HIP runtime error                                 */
  TPF_EBREAKDOWN = -4,    /* BiCGSTAB breakdown after one restart, or NaN      */
  TPF_ESTATE = -5         /* call out of order (e.g. solve before assemble)    */
};

/* Precision of the multigrid preconditioner (the outer BiCGSTAB, the assembly, the
 * Galerkin products, the coarsest LU and LIMEX are FP64 in every mode):
 *   TPF_FP64     every level FP64;
 *   TPF_MIXED    level matrices, smoother and transfers FP32;
 *   TPF_MIXED16  as TPF_MIXED, but the matrices of the coarse levels (all but the
 *                finest) are stored in FP16 with one FP32 scale per scalar row
 *                (the row's largest magnitude), computed with in FP32. */
enum { TPF_FP64 = 0, TPF_MIXED = 1, TPF_MIXED16 = 2 };

/* Boundary injection patch: a rectangle on one face of the box with a mass rate
 * of one phase per unit face measure into the domain (kg/(m^2 s) in 3D,
 * kg/(m s) in 2D).  This is the Neumann condition of Section 2 (Eqs. BsWn/BpNn)
 * restricted to inflow patches.  lo/hi are bounds in the remaining axes in
 * increasing axis order (2D: only lo[0], hi[0]).  The library integrates the rate
 * exactly over each vertex's dual-box face. */
typedef struct tpf_patch {
  int32_t axis;    /* face normal axis 0,1,2                         */
  int32_t side;    /* 0: coordinate 0; 1: coordinate = extent[axis] */
  int32_t phase;   /* 0 wetting, 1 non-wetting                      */
  int32_t reserved;
  double lo[2], hi[2];
  double rate;
} tpf_patch;

#define TPF_MAX_PATCHES 8

/* Relative-permeability laws (the capillary pressure is Brooks-Corey in both):
 *   TPF_KR_BURDINE  k_rw = S_e^((2+3 lam)/lam), k_rn = (1-S_e)^2 (1 - S_e^((2+lam)/lam))
 *                   (Brooks-Corey-Burdine, the law of Section 5's cases 1-3);
 *   TPF_KR_POLY     k_rw = kr_coef[0] S_e^2, k_rn = kr_coef[1] (1 - S_e)
 *                   (the printed laws of Tables case4 and case5: 0.9 and 0.5). */
enum { TPF_KR_BURDINE = 0, TPF_KR_POLY = 1 };

/* Multigrid smoother (the paper names the multigrid preconditioner, not its parts):
 *   TPF_SMOOTH_POINT  damped 2x2-block Jacobi, x += omega D^{-1} (b - A x);
 *   TPF_SMOOTH_LINE   damped line-block Jacobi along the last axis (y in 2D, z in
 *                     3D: the gravity axis of the layered workloads of Section 5),
 *                     x += omega A_L^{-1} (b - A x), A_L the couplings of A inside each
 *                     vertex line (block tridiagonal, 2x2 blocks), solved exactly by a
 *                     block LU per line factored in FP64 with the hierarchy.  It keeps
 *                     BiCGSTAB + GMG convergent where layers and buoyant transport make
 *                     point smoothing stall.  Needs 12 more level-type values per
 *                     vertex on every level but the coarsest. */
enum { TPF_SMOOTH_POINT = 0, TPF_SMOOTH_LINE = 1 };

/* Scenario: the problem statement of Section 2 (domain, per-element porosity,
 * isotropic permeability and Brooks-Corey parameters, fluids, gravity, Dirichlet
 * and Neumann data) plus the multigrid settings.  Host pointers are read during
 * tpf_create_grid only. */
typedef struct tpf_grid_desc {
  int32_t dim;           /* 2 or 3                                              */
  int32_t n[3];          /* vertices per axis; n[2] = 1 in 2D                   */
  double extent[3];      /* m (extent[2] ignored in 2D: unit depth)             */
  double gravity[3];     /* m/s^2                                               */
  double rho[2];         /* kg/m^3, [wetting, non-wetting]                      */
  double mu[2];          /* Pa s                                                */
  double s_res[2];       /* S_wr, S_nr                                          */
  const double *perm;    /* host, per cell, K [m^2] > 0                          */
  const double *poro;    /* host, per cell, porosity in (0, 1]                  */
  const double *entry_p; /* host, per cell, Brooks-Corey entry pressure >= 0 Pa */
  const double *bc_lambda; /* host, per cell, Brooks-Corey lambda > 0           */
  const uint8_t *dir_mask; /* host, per vertex: bit0 p_w, bit1 S_n Dirichlet    */
  const double *dir_value; /* host, 2 per vertex (p_w, S_n); may be NULL if no mask bit set */
  const tpf_patch *patches; /* host, n_patches entries                          */
  int32_t n_patches;     /* 0..TPF_MAX_PATCHES                                  */
  int32_t levels;        /* multigrid levels >= 1; each coarsening halves the cell count per axis */
  int32_t precision;     /* TPF_FP64, TPF_MIXED or TPF_MIXED16 (see above)      */
  int32_t nu_pre;        /* pre-smoothing sweeps (>= 1)                         */
  int32_t nu_post;       /* post-smoothing sweeps (>= 0)                        */
  int32_t limex_stages;  /* largest LIMEX stage count used with this grid (0: none) */
  double omega;          /* smoother damping in (0, 2)                          */
  int32_t kr_model;      /* TPF_KR_BURDINE or TPF_KR_POLY                       */
  int32_t smoother;      /* TPF_SMOOTH_POINT or TPF_SMOOTH_LINE (see above)     */
  double kr_coef[2];     /* TPF_KR_POLY: a_w, a_n > 0 (ignored otherwise)       */
  const double *vertex_source; /* host, 2 per vertex (w, n), kg/s into the vertex's
                                  control volume (point sources such as case 5's
                                  injection point), or NULL for none           */
} tpf_grid_desc;

typedef struct tpf_solve_stats {
  int32_t iters;         /* BiCGSTAB iterations                                 */
  int32_t restarts;      /* restarts (breakdown or stagnation of the true residual) */
  double rel_res;        /* ||r_k|| / ||f|| of the recursively updated residual */
  double rel_res_true;   /* ||f - A x|| / ||f|| recomputed in FP64 at exit      */
  double fnorm;          /* ||f||_2                                             */
} tpf_solve_stats;

typedef struct tpf_limex_opts {
  int32_t stages;        /* k >= 1 (k = 1 is linearly implicit Euler, no estimate) */
  int32_t maxit;         /* BiCGSTAB iteration cap per stage solve               */
  double tol;            /* TOL of the error estimate                            */
  double safety;         /* rho of the step-size rule                            */
  double dt_max;         /* largest step                                         */
  double rtol;           /* relative residual of every stage solve               */
} tpf_limex_opts;

typedef struct tpf_limex_stats {
  int32_t accepted;      /* 1 accepted, 0 rejected                               */
  int32_t solves;        /* stage solves performed                              */
  int32_t iters_total;   /* BiCGSTAB iterations summed over the solves          */
  int32_t unconverged;   /* failed stage solves (0 or 1: the first one rejects)  */
  double eps;            /* error estimate [[eps]]                               */
  double dt_used;        /* step attempted                                       */
  double dt_next;        /* proposed next step                                   */
} tpf_limex_stats;

typedef struct tpf_newton_opts {
  int32_t max_newton;    /* Newton iterations per step (>= 1)                     */
  int32_t max_halvings;  /* consecutive halvings of a Newton step (>= 0)          */
  int32_t maxit;         /* BiCGSTAB iteration cap per linear solve (>= 1)        */
  int32_t reserved;      /* 0                                                     */
  double atol;           /* absolute defect tolerance, kg (>= 0)                  */
  double rtol;           /* defect tolerance relative to the step's first (>= 0)  */
  double lin_rtol;       /* relative residual of every linear solve (> 0)         */
  double xtol;           /* also converged when the accepted update is below it:
                            max|du_p| <= xtol max|p| and max|du_S| <= xtol
                            (>= 0; 0 turns the criterion off)                    */
} tpf_newton_opts;

typedef struct tpf_newton_stats {
  int32_t converged;     /* 1: converged                                          */
  int32_t newton;        /* Newton iterations (accepted steps of the iteration)   */
  int32_t halvings;      /* step halvings of the backtracking                     */
  int32_t linear_solves; /* BiCGSTAB solves                                       */
  int32_t linear_iters;  /* BiCGSTAB iterations summed over the solves            */
  int32_t criterion;     /* 0: not converged, 1: the defect met atol or rtol,
                            2: the update met xtol                              */
  double defect0;        /* ||G(u_old)|| = tau ||F(u_old)|| (kg)                   */
  double defect;         /* ||G|| at exit                                         */
} tpf_newton_stats;

/* Message of the calling thread's last hard error ("" if none).  The pointer stays
 * valid until the next library call on the same thread. */
const char *tpf_last_error(void);

/* Checks a descriptor on the host only (no HIP call).  TPF_OK or TPF_EINVAL. */
tpf_status tpf_validate(const tpf_grid_desc *desc);

/* Exact arena size in bytes for desc (0 if desc is invalid; see tpf_last_error).
 * Pure host computation. */
size_t tpf_grid_bytes(const tpf_grid_desc *desc);

/* Creates a grid whose device state lives in arena (device memory, at least
 * tpf_grid_bytes(desc) bytes, 256-byte aligned, owned by the caller and kept
 * alive until tpf_destroy_grid).  Uploads the scenario and runs the per-vertex
 * pre-processing (p_dmin and reference medium, Eq. pdmin; Neumann sources) on
 * stream, then synchronises the stream so the host arrays may be freed.  The grid
 * belongs to the device current at this call; every later call on the grid expects
 * that device to be current (the streams the library creates for it are created there).
 * Errors: TPF_EINVAL (descriptor), TPF_ENOMEM (arena), TPF_EDEVICE. */
tpf_status tpf_create_grid(const tpf_grid_desc *desc, void *arena, size_t arena_bytes,
                           tpf_stream stream, tpf_grid **out);

/* Frees the host metadata of g (the caller frees the arena afterwards). */
void tpf_destroy_grid(tpf_grid *g);

/* Writes the Dirichlet values of the descriptor into the masked components of the
 * device state u (double[2N]). */
tpf_status tpf_apply_dirichlet(tpf_grid *g, double *u, tpf_stream stream);

/* f = F(u): the right-hand side of M(u) u' = F(u) (Section 4) -- Neumann sources
 * minus the outward SCVF mass fluxes of both phases, Dirichlet components set to
 * zero.  u, f: device double[2N]; may not alias. */
tpf_status tpf_residual(tpf_grid *g, const double *u, double *f, tpf_stream stream);

/* Stage matrix A = M(u0)/h - J(u0) with J = dF/du exact (upwind and interface
 * branches frozen at u0) and unit rows at Dirichlet components (Section 4, the
 * linearly implicit Euler step divided by tau = h); then the multigrid hierarchy:
 * Galerkin coarse matrices, their FP32 copies in TPF_MIXED, and the inverse of the
 * coarsest matrix from an LU factorisation with partial pivoting.  u0: device
 * double[2N]; h > 0 seconds.  F(u0) is produced by the same kernel: if f0_out is
 * not NULL it receives F(u0) (device double[2N], the right-hand side of the first
 * substep of a stage).  The coarsest factorisation and inverse run on a stream the
 * grid creates for them (default priority), forked from `stream` by an event; the
 * grid's later work on `stream` waits for it where it first needs it (the first
 * coarse solve, tpf_copy_coarse_inverse, the next assembly or rescale), and
 * tpf_destroy_grid waits for it on the host.  While `stream` is being captured the
 * factorisation stays on it. */
tpf_status tpf_assemble_stage(tpf_grid *g, const double *u0, double h, double *f0_out, tpf_stream stream);

/* Moves the assembled stage operator to another step h > 0 without re-assembling:
 * A = M(u0)/h - J(u0) with M and J still those of the last tpf_assemble_stage (the
 * linearly implicit stages of Section 4 freeze both at the step's initial state and
 * differ only in their step H/j).  The flux part of every multigrid level is
 * independent of h and its storage part proportional to 1/h, so each level's storage
 * diagonal is rescaled (the FP32/FP16 copies follow) and the coarsest level is
 * refactored; F(u0) is unchanged.  Equal to a fresh tpf_assemble_stage(u0, h) up to
 * rounding.  Returns TPF_OK, TPF_EINVAL or TPF_ESTATE (nothing assembled). */
tpf_status tpf_rescale_stage(tpf_grid *g, double h, tpf_stream stream);

/* Solves A x = f (A from the last assemble_stage) with right-preconditioned
 * BiCGSTAB, x0 = 0, one V(nu_pre, nu_post) cycle as preconditioner, until
 * ||r|| <= rtol ||f||.  f, x: device double[2N], may not alias.  Synchronises the
 * stream once per iteration to read the residual norm.  stats may be NULL.
 * Returns TPF_OK, TPF_NOT_CONVERGED (x = last iterate), TPF_EBREAKDOWN,
 * TPF_ESTATE (no assembled matrix). */
tpf_status tpf_solve_stage(tpf_grid *g, const double *f, double *x, double rtol, int32_t maxit,
                           tpf_solve_stats *stats, tpf_stream stream);

/* tpf_solve_stage for callers that cannot allocate device memory or bring
 * workspace of their own (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same solve, same kernels and the same result, but the
 * BiCGSTAB work vectors, block partials and device scalars live in a fixed device
 * array inside the library (64 MiB per GPU, held until the process ends) instead of
 * the grid's arena.  The assembled hierarchy and the V-cycle's level vectors stay in
 * the arena.  Grids needing more than the array holds (above about 460,000 vertices,
 * e.g. 65^3 fits, 97^3 does not) get TPF_EINVAL with a message.  Calls nothing that
 * allocates: with tpf_set_coarse_graph on, it replays a graph an earlier
 * tpf_solve_stage or tpf_precondition captured and never captures one itself (until
 * then the coarse levels are stream launches).  Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams or threads) race and must be serialised by the caller.  The
 * array keeps the last call's contents; the solve initialises everything it reads.
 * The grid's device must be current.  Returns as tpf_solve_stage. */
tpf_status tpf_solve_stage_static(tpf_grid *g, const double *f, double *x, double rtol, int32_t maxit,
                                  tpf_solve_stats *stats, tpf_stream stream);

/* One LIMEX step of size *dt from state u at time *t (Section 4): stages
 * j = 1..k take j linearly implicit Euler substeps of *dt/j with M and J frozen
 * at u and F re-evaluated each substep; Aitken-Neville extrapolation; error
 * eps = |||T_kk - T_k,k-1||| / |||T_kk||| in the norm of Eq. norm_u; accept iff
 * eps <= tol; next step min(dt_max, dt (safety tol / eps)^(1/3)).
 * On accept u <- T_kk, *t += *dt; on reject u and *t are unchanged.  Either way
 * *dt <- the proposed next step.  Requires opts->stages <= desc.limex_stages.
 * A stage solve that misses opts->rtol within opts->maxit iterations, or breaks
 * down on finite data, rejects the step at once (the paper gives no rule for a
 * failed linear solve): the remaining stages are skipped, stats->eps = +inf,
 * stats->unconverged = 1, and the next step is min(dt_max, dt / 4).  A
 * non-finite F(u) (non-finite input) is TPF_EBREAKDOWN.
 * Returns TPF_OK, TPF_STEP_REJECTED or an error. */
tpf_status tpf_limex_step(tpf_grid *g, double *u, double *t, double *dt, const tpf_limex_opts *opts,
                          tpf_limex_stats *stats, tpf_stream stream);

/* m = m(u): the storage of both phases in each control volume (kg), the sum over
 * the vertex's sub-control volumes of porosity x density x saturation x volume with
 * the saturation of the interface condition (Section 3.1, Eqs. dsW/dpN; M(u) of
 * Section 4 is dm/du).  u, m: device double[2N] (m interleaved (w, n)); may not
 * alias.  Dirichlet components are not cleared. */
tpf_status tpf_storage(tpf_grid *g, const double *u, double *m, tpf_stream stream);

/* One fixed implicit Euler step of size tau from the state u (device double[2N],
 * in/out), the scheme Section 5 compares LIMEX with: Newton's method on
 * G(u) = m(u) - m(u_old) - tau F(u) = 0 (conservative backward Euler of
 * M(u) u' = F(u)), whose Jacobian is tau times the stage matrix A(u; h = tau) of
 * tpf_assemble_stage.  Every Newton iteration assembles A and F at the iterate, builds
 * the hierarchy and solves A delta = F(u) - (m(u) - m(u_old))/tau (Dirichlet rows 0)
 * with BiCGSTAB + GMG to opts->lin_rtol.  The defect ||G|| (2-norm over the rows
 * without a Dirichlet component, kg) starts at tau ||F(u_old)||; the step converges when
 * it is <= opts->atol or <= opts->rtol times its initial value (the solver settings of
 * Section 5 use 1e-8 and 1e-6), or when the accepted update is negligible
 * (opts->xtol, relative for the pressure, absolute for the saturation: the defect
 * of a step near equilibrium can sit on its FP64 rounding floor above both
 * tolerances, ~1e-7 kg for one-day steps of case 4 at 5e7 Pa).  A trial whose defect
 * does not fall below its base's is
 * halved, at most opts->max_halvings times in a row.  u must satisfy the Dirichlet
 * values.  Leaves the last stage matrix assembled (at the final iterate).
 * Returns TPF_OK (u advanced), TPF_NOT_CONVERGED (no convergence within
 * opts->max_newton iterations, or a linear breakdown: u unchanged), or an error (u
 * unchanged).  Synchronises the stream once per Newton iteration. */
tpf_status tpf_ie_step(tpf_grid *g, double *u, double tau, const tpf_newton_opts *opts, tpf_newton_stats *stats,
                       tpf_stream stream);

/* Makes the pressure of u (device double[2N], in/out) consistent with its saturation.
 * With incompressible phases the pressure column of M(u) u' = F(u) (Section 4)
 * carries no storage: p is an algebraic unknown, and an extrapolated LIMEX state can
 * violate the discrete volume balance by more than one linearised correction with the
 * Jacobian frozen at that state restores; the stages of the next step then differ by
 * an amount that does not vanish with the step (the paper does not discuss this).
 * Newton at fixed saturation on the stage system with a vanishing step h_p > 0:
 * assemble A(u; h_p) and F(u), solve A delta = F(u) (BiCGSTAB + GMG to
 * opts->lin_rtol), p += delta_p with S untouched.  As h_p -> 0 that is the Newton step
 * of F_w/rho_w + F_n/rho_n = 0 (the storages cancel), which holds at the end up to
 * O(h_p).  Stops when max|delta_p| <= max(opts->atol, opts->rtol max|p|) (Pa);
 * opts->max_halvings and opts->xtol are unused.  stats->defect0 / defect: the first and last
 * max|delta_p|.  Leaves A(u; h_p) assembled.  Returns TPF_OK, TPF_NOT_CONVERGED (u
 * unchanged) or an error (u unchanged). */
tpf_status tpf_project_pressure(tpf_grid *g, double *u, double h_p, const tpf_newton_opts *opts,
                                tpf_newton_stats *stats, tpf_stream stream);

/* Selects how the V-cycle issues the levels below the finest (enable != 0: replay one
 * HIP graph captured on the grid's own stream at the first V-cycle; 0: stream
 * launches, the default).  Both issue the same kernels in the same order, so results
 * are identical; the graph saves host and dispatch work per launch on the small,
 * latency-bound levels.  While the TPF_K_COARSE_LEVELS class is being timed
 * (tpf_profile_begin) the stream launches are used.  Returns TPF_OK or TPF_EINVAL. */
tpf_status tpf_set_coarse_graph(tpf_grid *g, int32_t enable);

/* TPF_SMOOTH_LINE: levels with fewer than max_lines vertex lines factor and solve each
 * line with two threads (the two halves of its twisted factorisation, exchanging their
 * edge values), levels with more with one thread per line running both halves in turn
 * (default 32768; 0: one thread per line everywhere).  The solve follows the setting at
 * once, the factorisation from the next assembly or rescale.  Both do the same
 * operations in the same order, so results are identical.  Returns TPF_OK or
 * TPF_EINVAL. */
tpf_status tpf_set_line_pairs(tpf_grid *g, int64_t max_lines);

/* ---- inspection hooks (used by the parity tests and the benchmark) ---------- */

/* Number of multigrid levels and vertices per axis of a level. */
int32_t tpf_levels(const tpf_grid *g);
tpf_status tpf_level_dims(const tpf_grid *g, int32_t level, int32_t n_out[3]);

/* Copies the level's stencil matrix into dst (device): layout
 * [offset][vertex][4] with offset = (dx+1) + 3(dy+1) [+ 9(dz+1)], entries
 * (row w, col p), (row w, col S), (row n, col p), (row n, col S).
 * precision TPF_FP64 -> double; TPF_MIXED -> float, the FP32 copy (TPF_MIXED grids,
 * or the finest level of TPF_MIXED16 grids); TPF_MIXED16 -> float, the stored FP16
 * entries times their row scales (coarse levels of TPF_MIXED16 grids). */
tpf_status tpf_copy_matrix(tpf_grid *g, int32_t level, int32_t precision, void *dst, tpf_stream stream);

/* y = A_level x with the FP64 level matrix; x, y device double[2 N_level]. */
tpf_status tpf_spmv(tpf_grid *g, int32_t level, const double *x, double *y, tpf_stream stream);

/* x = one V-cycle applied to b (the preconditioner of solve_stage).  With
 * TPF_SMOOTH_LINE, TPF_EBREAKDOWN if the line factorisation met a singular pivot. */
tpf_status tpf_precondition(tpf_grid *g, const double *b, double *x, tpf_stream stream);

/* Copies the inverse of the coarsest matrix (row-major, double[nc*nc],
 * nc = 2 N_coarsest) to dst (device). */
tpf_status tpf_copy_coarse_inverse(tpf_grid *g, double *dst, tpf_stream stream);

/* Device buffer with p_dmin per vertex (read-only view into the arena). */
const double *tpf_pdmin_ptr(const tpf_grid *g);

/* ---- kernel timing (HIP events recorded around selected launches) ----------- */
enum {
  TPF_K_ASSEMBLE = 0,   /* fine-level residual + stage-matrix assembly            */
  TPF_K_RAP,            /* Galerkin coarse operator, all levels                   */
  TPF_K_COARSE_LU,      /* dense LU + inverse of the coarsest level               */
  TPF_K_SPMV64,         /* FP64 stencil SpMV on the finest level (all variants)   */
  TPF_K_SMOOTH0,        /* block-Jacobi sweep on the finest level (full sweeps)   */
  TPF_K_SMOOTH0_FIRST,  /* first sweep from a zero guess (diagonal only)          */
  TPF_K_RESID0,         /* level residual on the finest level                     */
  TPF_K_COARSE_LEVELS,  /* every smoother/residual/transfer launch below level 0  */
  TPF_K_TRANSFER0,      /* restriction from and prolongation to the finest level  */
  TPF_K_LINE0,          /* line solve of a TPF_SMOOTH_LINE sweep on the finest level
                           (the sweep's residual is timed as TPF_K_RESID0)         */
  TPF_K_COUNT
};

typedef struct tpf_kernel_time {
  int32_t count;        /* timed launches                                        */
  int32_t reserved;
  double total_ms;      /* summed start-to-end event durations                   */
} tpf_kernel_time;

/* Starts timing each launch of the classes whose bit (1u << class) is set in
 * class_mask (0: every class), up to max_launches launches; later launches are not
 * timed.  A class of single kernel launches gets its pair of HIP events attached to
 * each dispatch (hipExtLaunchKernel: the kernel's own start and end); the classes
 * TPF_K_RAP and TPF_K_COARSE_LU, several launches each, are bracketed by event
 * markers in the stream.  A timed dispatch still costs about 6 us more than an
 * untimed one, so timing only the classes of interest keeps the others
 * unperturbed.  Creates the events; no device memory is allocated. */
tpf_status tpf_profile_begin(tpf_grid *g, int32_t max_launches, uint32_t class_mask);

/* Synchronises the recorded events, writes per-class totals to out[TPF_K_COUNT]
 * and destroys the events. */
tpf_status tpf_profile_end(tpf_grid *g, tpf_kernel_time *out);

#ifdef __cplusplus
}
#endif
#endif /* TPF_H */
