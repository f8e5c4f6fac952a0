/*
 * stokes.h -- C ABI of the MI355X (gfx950) variable-coefficient MAC Stokes
 * solver: GMRES / flexible GMRES preconditioned by the block preconditioners
 * of Cai, Nonaka, Bell, Griffith and Donev, "Efficient Variable-Coefficient
 * Finite-Volume Stokes Solvers" (arXiv:1308.4605), each built from one
 * geometric-multigrid V-cycle for the velocity and one for the pressure.
 *
 * Problem (paper Sec. "Preconditioners", eq. Saddle_sys, discretised as in Sec. "Staggered-grid Discretization"):
 *     M x = b,   M = [[A, G], [-D, 0]],   A = theta rho_f - L_mu,
 * x = (face velocities u, cell pressure p), b = (b_u, b_p) with b_p = -g.
 * D and G are the staggered divergence and gradient, rho_f the mean of the two
 * cells sharing a face, L_mu the stress-form viscous operator
 * div(mu (grad u + grad u^T)) with cell viscosity on the normal stresses and
 * edge (3D) / node (2D) viscosity on the shear stresses.  theta = 0 is steady
 * Stokes flow, theta ~ 1/dt unsteady (Sec. "Preconditioners").  With bulk viscosity gamma
 * (flows with div u = g != 0, Sec. "Preconditioners") the stress gains
 * (gamma - 2/3 mu)(div u) I, added to the normal stresses of each cell.
 *
 * ------------------------------------------------------------------------
 * Array layout (all arrays C-ordered, x fastest; axes 0,1,2 = x,y,z):
 *   cells (p, rho, mu, b_p, gradients w.r.t. cell fields): n[0]*n[1]*n[2]
 *     entries (n[2] = 1 in 2D).
 *   velocity: the d components stored back to back in one buffer.  Component
 *     k lives on faces normal to axis k and has n[a] entries along a != k and
 *     n[k] + w[k] entries along k, w[k] = 1 when axis k has walls (no-slip or
 *     free-slip) and 0 when it is periodic.  Wall faces (index 0 and n[k] on
 *     a wall axis) are not unknowns: inputs may hold anything there (they are
 *     read as 0); outputs hold 0 there.
 *   edge viscosity: families m = 2, 1, 0 (3D) or m = 2 (2D, the grid nodes)
 *     stored back to back.  Family m is parallel to axis m and carries the
 *     viscosity of the shear stress between the two other axes; it has
 *     n[a] + w[a] entries along each a != m and n[m] along m.
 * Every pointer passed to the functions below is a DEVICE pointer except the
 * parameter/stat structs and `hip_stream`, unless stated otherwise.  Inputs
 * are never modified.  All vectors are FP64.
 *
 * Ownership: the caller owns every buffer, including the workspace, which it
 * allocates with at least stokes_workspace_bytes() bytes of device memory
 * (256-byte aligned).  The context owns host metadata and a small pinned host
 * buffer only; the library never allocates device memory.
 *
 * Streams: every call enqueues its kernels on the HIP stream given at
 * creation.  stokes_apply, stokes_precond, stokes_vel_subsolve,
 * stokes_p_subsolve and stokes_grad are asynchronous; stokes_solve,
 * stokes_adjoint_solve and the two *_mg_solve calls read scalars back every
 * iteration and return after the stream has drained.  A context is not thread-safe; two calls on
 * one context must not overlap.
 *
 * Errors: every function returns a status code; validation happens on the
 * host before any launch.  No exception crosses this boundary.
 * ------------------------------------------------------------------------
 */
#ifndef STOKES_MI355X_H
#define STOKES_MI355X_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
  STOKES_OK = 0,
  STOKES_EINVAL = -1,      /* bad sizes/parameters/pointers; nothing launched */
  STOKES_ENOMEM = -2,      /* workspace smaller than stokes_workspace_bytes */
  STOKES_EDEVICE = -3,     /* a HIP runtime call failed */
  STOKES_ENOCONV = -4,     /* max_iter reached; best iterate and stats written */
  STOKES_EBREAKDOWN = -5,  /* Krylov breakdown with an unconverged residual */
  STOKES_ENONFINITE = -6,  /* NaN/Inf in a residual */
  STOKES_EINCOMPAT = -7    /* right-hand side not orthogonal to the null space */
};

/* Boundary conditions (Sec. "Staggered-grid Discretization": a condition at each domain boundary),
   given per axis a in bc[a].  No-slip: u = 0 on the wall, the shear next to
   it one-sided.  Free-slip: zero normal velocity and no tangential momentum
   flux through the wall.  Periodic applies to both ends of an axis; the two
   walls of a wall axis may differ: STOKES_NOSLIP_FREESLIP is no-slip at the
   low end (index 0) and free-slip at the high end (index n), and
   STOKES_FREESLIP_NOSLIP the reverse (e.g. an open channel with a free
   surface on top). */
enum { STOKES_PERIODIC = 0, STOKES_NOSLIP = 1, STOKES_FREESLIP = 2, STOKES_NOSLIP_FREESLIP = 3,
       STOKES_FREESLIP_NOSLIP = 4 };

/* block preconditioners of Sec. "Preconditioners": projection (eq. P1_practical), lower
   triangular (eq. CC_Pre_lower), upper triangular (eq. CC_Pre_upper),
   block diagonal (eq. CC_Pre_diagonal), Uzawa-like (Sec. "Other preconditioners") */
enum { STOKES_P1 = 1, STOKES_P2 = 2, STOKES_P3 = 3, STOKES_P4 = 4, STOKES_P5 = 5 };

/* precision of the preconditioner (multigrid, transfers, coefficients and the
   Schur/projection glue).  The Krylov solver, M, residuals and the solution
   stay FP64.  STOKES_MG_FP32 requires STOKES_FGMRES. */
enum { STOKES_FP64 = 0, STOKES_MG_FP32 = 1 };

/* Krylov method: left-preconditioned GMRES(m) (Sec. "Krylov Solver", Sec. "Results") or flexible
   GMRES(m) (right preconditioning; named in Sec. "Results") */
enum { STOKES_GMRES_LEFT = 0, STOKES_FGMRES = 1 };

/* Scaling of the linear system (Sec. "Rescaling of the Linear System", "Rescaling of the Linear
   System").  UNIFORM: the rescaled system of eq. Stokes_rescaled, velocity
   equations times c and pressure unknowns times c.  DIAGONAL: for a very
   broad range of viscosities the paper rescales velocity and pressure
   separately by diagonal matrices; here the Krylov solver runs on S M' S
   (M' the uniformly rescaled operator) with S = diag(S_u, S_p),
   S_u = diag(A')^{-1/2} on the velocity unknowns and S_p = (2 mu'_cell)^{1/2}
   ((gamma' + 4/3 mu')^{1/2} with bulk viscosity) on the pressure unknowns,
   so that the velocity diagonal is one and the Schur approximation is minus
   the identity.  The preconditioner is the same operator conjugated by S,
   the solution is the same; what changes is the norm in which GMRES
   minimises and the tolerance is measured (stokes_stats.rel_res_true is
   ||S (b' - M' x')|| / ||S b'||).  Needs a positive viscous Schur
   coefficient in every cell (STOKES_EINVAL otherwise). */
enum { STOKES_SCALE_UNIFORM = 0, STOKES_SCALE_DIAGONAL = 1 };

/* edge/node viscosity: arithmetic mean of the neighbouring cells (Sec. "Staggered-grid Discretization"),
   harmonic mean, or caller-supplied values */
enum { STOKES_EDGE_ARITH = 0, STOKES_EDGE_HARMONIC = 1, STOKES_EDGE_GIVEN = 2 };

typedef struct {
  int dim;          /* 2 or 3 */
  int n[3];         /* cells per axis (n[2] ignored in 2D) */
  double h;         /* grid spacing (> 0) */
  int bc[3];        /* STOKES_PERIODIC, STOKES_NOSLIP, STOKES_FREESLIP,
                       STOKES_NOSLIP_FREESLIP or STOKES_FREESLIP_NOSLIP per axis */
  double theta;     /* >= 0 */
  int precond;      /* STOKES_P1..STOKES_P5 */
  int precision;    /* STOKES_FP64 or STOKES_MG_FP32 */
  int krylov;       /* STOKES_GMRES_LEFT or STOKES_FGMRES */
  int restart;      /* GMRES restart length m, 1..32 (the paper uses 10) */
  int nu_pre;       /* Gauss-Seidel sweeps before coarsening (paper: 2) */
  int nu_post;      /* sweeps after prolongation (paper: 2) */
  int nu_coarse;    /* sweeps on the coarsest level (paper: 8 or more) */
  int vcycles;      /* V-cycles per subsolver application (paper: 1) */
  double rescale_c; /* rescaling c of eq. Stokes_rescaled; <= 0: c = h / mu_ref
                       with mu_ref the geometric mean of the positive mu_cell */
  int edge_avg;     /* STOKES_EDGE_* */
  int bulk;         /* 0: incompressible stress form; 1: stress with bulk
                       viscosity (stokes_create then takes gamma_cell) */
  int scaling;      /* STOKES_SCALE_UNIFORM or STOKES_SCALE_DIAGONAL */
  int extended;     /* 1: the Krylov solver's true residuals b - M x in
                       double-double arithmetic (about 106 bits), each entry
                       rounded once to FP64 (Sec. "Rescaling of the Linear System": extended precision in
                       extreme cases); 0: FP64 */
} stokes_params;

typedef struct {
  int iters;            /* Arnoldi steps (applications of P^{-1} M or M P^{-1}) */
  int restarts;         /* restart cycles started */
  int precond_applies;  /* preconditioner applications */
  int scalar_vcycles;   /* precond_applies * vcycles * (d * velocity cycles +
                           pressure cycles): the paper's cost proxy (Sec. "Results") */
  double rel_res_true;  /* ||b' - M' x'|| / ||b'|| of the rescaled system at exit */
  double rel_res_est;   /* last Givens estimate, as a true relative residual */
  double rel_res_unscaled;  /* stokes_solve: ||b - M x|| / ||b|| of the caller's
                               (unscaled) system at exit; stokes_adjoint_solve: the
                               same combination of the velocity and pressure blocks
                               of its residual.  0 when the solve stopped on a
                               breakdown or a non-finite value */
  int history_len;      /* entries written to the stokes_set_history buffer */
  double t_total;       /* wall-clock seconds of the Krylov solve */
  double t_precond;     /* GPU seconds in preconditioner applications (HIP events) */
  double t_krylov;      /* t_total - t_precond: M applies, Arnoldi, host work */
} stokes_stats;

typedef struct stokes_ctx stokes_ctx;

/* Sizes of the ABI arrays for these parameters (host pointers; any may be
   NULL).  Returns STOKES_EINVAL for invalid parameters.  The grid must halve
   exactly until its smallest axis has two cells (Appendix C: coarsening by 2
   down to two cells): the smallest n is a power of two >= 2, every n is
   divisible by min(n)/2, and a periodic axis keeps an even cell count on the
   coarsest level (n divisible by min(n)), which the red-black colouring needs.
   The kernels index face, cell and edge storage with 32-bit integers, so
   3 * prod(n + 1) must stay below 2^31 (about 890^3 cells; a grid that size
   would not fit one GPU's memory with a Krylov basis anyway). */
int stokes_sizes(const stokes_params *p, size_t *nvel, size_t *ncell, size_t *nedge,
                 int *nlevels);

/* Device workspace bytes needed by stokes_create for these parameters; 0 for
   invalid parameters. */
size_t stokes_workspace_bytes(const stokes_params *p);

/* Build the context: face density, rho-weighted coefficients, edge viscosity
   (Sec. "Staggered-grid Discretization"), the rescaling c ~ h/mu0 (Sec. "Rescaling of the Linear System") and the coarse-level
   coefficients (Appendix C), all on the device.
   rho_cell, mu_cell: cell fields (rho > 0, mu >= 0, finite);
   mu_edges: edge viscosity for STOKES_EDGE_GIVEN, else NULL;
   gamma_cell: bulk viscosity per cell (>= 0, finite) when p->bulk = 1, else
     NULL (STOKES_EINVAL otherwise).  With it the stress carries
     (gamma - 2/3 mu)(div u) I (Sec. "Preconditioners"), coarse levels take the mean of the
     fine cells' gamma - 2/3 mu, and the Schur approximation uses
     gamma + 4/3 mu in place of 2 mu (eq. Schur_app_bulk);
   workspace: device buffer of ws_bytes >= stokes_workspace_bytes(p);
   hip_stream: a hipStream_t (NULL = the default stream).
   The coefficient fields are checked for sign and finiteness on the device
   (one synchronisation); rho, mu and gamma are not retained.
   Create also prepares two forms of the velocity V-cycle that compute the
   same map as its kernel-by-kernel form, up to rounding: the coarse levels of
   at most 512 cells (Appendix C's smoothing and coarsest-level relaxations
   from a zero iterate, a fixed linear map of their right-hand side) are run
   once per unit vector and stored as a matrix in the workspace, applied by
   one matrix-vector product per V-cycle; and on a colour-split FP32
   hierarchy the finest-level V-cycle is recorded as a HIP graph (on a
   private stream; nothing runs) and replayed on hip_stream.  The environment
   variables STOKES_TAIL_DENSE=0 and STOKES_VGRAPH=0, read here, turn either
   off for this context (comparisons and tests).  On 3D FP32 levels of at
   least 2^21 cells the velocity residual runs by columns of 8 cells along z
   (bitwise the same result); STOKES_RESIDUAL_COLUMNS=n sets the column
   length for this context (clamped to each level's z extent), and n = 0
   runs it by cells. */
int stokes_create(const stokes_params *p, const double *rho_cell, const double *mu_cell,
                  const double *mu_edges, const double *gamma_cell, void *workspace,
                  size_t ws_bytes, void *hip_stream, stokes_ctx **out);

/* y = M x with the caller's (unscaled) coefficients (Sec. "Preconditioners", eq. Saddle_sys;
   direct evaluation of the stencils at every interior face and cell, Sec. "Krylov Solver"). */
int stokes_apply(stokes_ctx *ctx, const double *xu, const double *xp, double *yu, double *yp);

/* r = b - M x with the caller's coefficients (the residual of the Krylov
   solver's convergence test, Sec. "Krylov Solver"), in FP64 (extended = 0) or in
   double-double arithmetic with each entry rounded once to FP64
   (extended = 1; Sec. "Rescaling of the Linear System", extended precision in extreme cases).  It is
   evaluated on the rescaled system, r_u = (c b_u - c A x_u - G c x_p) / c,
   so the products with c round to FP64 unless c is a power of two.  ru is 0
   on wall faces.  Uses the context's work vectors; asynchronous. */
int stokes_residual(stokes_ctx *ctx, const double *bu, const double *bp, const double *xu,
                    const double *xp, double *ru, double *rp, int extended);

/* Prescribed (non-homogeneous) wall velocities (Sec. "Krylov Solver"): with them the
   operator is affine, M x + c, and the flow solves M x = b - c with the
   homogeneous M used everywhere else.  This computes c = (cu, cp): M applied
   to the field that is zero at the unknowns and carries
     un: normal velocities on the wall faces (velocity layout; only the wall
         entries are read), and
     ut: tangential velocities on the wall edges (edge layout): an edge of
         family m on a wall normal to axis l holds the wall value of velocity
         component 3 - m - l (3D) or of the component parallel to the wall
         (2D nodes); read on no-slip walls only (free-slip walls carry no
         tangential flux).
   cu is 0 on wall faces.  Asynchronous. */
int stokes_boundary_rhs(stokes_ctx *ctx, const double *un, const double *ut, double *cu,
                        double *cp);

/* z = P^{-1} b for the configured preconditioner and precision (Sec. "Preconditioners"), the
   same operator the Krylov solver applies.  Output pressure has zero mean;
   the output velocity components that are singular have zero mean (Sec. "Krylov Solver"
   null-space care).  Component k of the velocity operator is singular when
   theta = 0, axis k is periodic and no wall (at either end of any axis) is
   no-slip. */
int stokes_precond(stokes_ctx *ctx, const double *bu, const double *bp, double *zu, double *zp);

/* The two multigrid subsolvers alone (Sec. "Krylov Solver", Appendix C): e = A~^{-1} r
   (velocity, `vcycles` V-cycles from zero) and e = L~_rho^{-1} r (pressure,
   L_rho = D rho_f^{-1} G; r must have zero mean; e has zero mean). */
int stokes_vel_subsolve(stokes_ctx *ctx, const double *r, double *e);
int stokes_p_subsolve(stokes_ctx *ctx, const double *r, double *e);

/* The same two multigrid solvers run to convergence on their own, the cost
   reference of a split (projection-like) method in the study of V-cycles per
   subsolve (Sec. "The effect of the number of multigrid cycles"): starting from e = 0, each cycle adds one V-cycle
   applied to the current residual, e <- e + V(r - A e), until
   ||r - A e|| <= tol ||r|| or max_cycles cycles.  A is the velocity operator
   theta rho - L_mu (vel) or L_rho (p), unscaled as for the subsolvers; r is
   first projected onto the operator's range (component means for the
   periodic steady velocity, the mean for the pressure), and so is e.
   Residuals, the iterate and the norms are FP64; with STOKES_MG_FP32 the
   V-cycles run in FP32, i.e. as iterative refinement.
   *cycles: V-cycles done; *rel_res: final ||r - A e|| / ||r|| (host
   pointers).  Returns STOKES_OK, STOKES_ENOCONV when max_cycles ran out (e
   holds the last iterate), STOKES_EINVAL for null pointers, tol <= 0 or
   max_cycles < 0.  Synchronous: returns after the stream has drained. */
int stokes_vel_mg_solve(stokes_ctx *ctx, const double *r, double *e, double tol, int max_cycles,
                        int *cycles, double *rel_res);
int stokes_p_mg_solve(stokes_ctx *ctx, const double *r, double *e, double tol, int max_cycles,
                      int *cycles, double *rel_res);

/* Solve M x = b until the true relative residual of the rescaled system
   ||b' - M' x'|| <= tol ||b'|| (Sec. "Krylov Solver" "true residual"), at most max_iter
   Arnoldi steps.  use_x0 != 0 starts from the given x (a restart, Sec. "The effect of restarts"),
   else from 0.  x is the solution of the unscaled system with p of zero mean
   (and zero-mean velocity components when the velocity operator is singular).
   b_p must have zero mean (STOKES_EINCOMPAT otherwise), as must each singular
   velocity component of b_u (see stokes_precond).  stats may be NULL.
   Synchronous. */
int stokes_solve(stokes_ctx *ctx, const double *bu, const double *bp, double *xu, double *xp,
                 double tol, int max_iter, int use_x0, stokes_stats *stats);

/* For callers that cannot allocate device memory (code that runs under HIP
   graph capture, tight serving loops, harnesses that forbid allocation):
   the same solve as stokes_solve, with the same arguments, results and
   status codes, whose Krylov storage -- the restart basis V (restart + 1
   FP64 vectors of nvel + ncell entries), for STOKES_FGMRES the stored
   preconditioned vectors Z (restart vectors in the preconditioner's
   precision), five FP64 work vectors (right-hand side, iterate, residual,
   two temporaries) and the reduction partials -- lives in a static device
   array of the library instead of the context's workspace.  The array holds
   STOKES_STATIC_SCRATCH_BYTES bytes per GPU, from the first call on that GPU
   until the process ends.  The call allocates nothing (no hipMalloc, no
   allocating library routine); the multigrid hierarchy, the coefficients and
   the preconditioner temporaries stay in the context's workspace.
   Returns STOKES_ENOMEM before any launch when the storage above exceeds the
   array (e.g. about 68^3 cells for FP64 FGMRES(10)), STOKES_EDEVICE when the
   array's device address cannot be obtained.  Every call on one GPU shares
   that GPU's array and clears the part it uses when it starts; calls that
   overlap on one GPU (from any contexts, streams or threads) race.
   Synchronous. */
#define STOKES_STATIC_SCRATCH_BYTES (256u << 20)
int stokes_solve_static(stokes_ctx *ctx, const double *bu, const double *bp, double *xu,
                        double *xp, double tol, int max_iter, int use_x0, stokes_stats *stats);

/* Adjoint: with x the forward solution and g = dL/dx = (g_u, g_p), solve
   M^T lambda = g (M = M^T, Sec. "Preconditioners") with the same preconditioner and a fresh
   Krylov space, then contract forward and adjoint strain rates:
     dL/db        = lambda                              (lu, lp),
     dL/dmu_cell  = -2 sum_k (D^k lambda_k)(D^k u_k)  + chain through the
                    derived edge viscosity (EDGE_ARITH/HARMONIC),
     dL/dmu_edge  = -w_e gamma_e(lambda) gamma_e(u),  w_e = 1/2 on no-slip
                    wall edges, 0 on free-slip wall edges, 1 elsewhere
                    (partial derivative),
     dL/drho_cell = -theta sum over the cell's faces of 1/2 lambda_f u_f,
   and with bulk viscosity (p->bulk = 1)
     dL/dgamma_cell = -(D lambda)(D u), with -2/3 of it added to dL/dmu_cell
                      (the coefficient gamma - 2/3 mu).
   dgamma_cell must be NULL for contexts without bulk viscosity.
   g is first projected onto the mean-free space of the solution (the adjoint
   of the zero-mean normalisation of p, and of u when the velocity operator is
   singular), so any g is accepted.  Gradient outputs may be NULL.
   Synchronous. */
int stokes_adjoint_solve(stokes_ctx *ctx, const double *xu, const double *xp, const double *gu,
                         const double *gp, double *lu, double *lp, double *dmu_cell,
                         double *dmu_edge, double *drho_cell, double *dgamma_cell, double tol,
                         int max_iter, stokes_stats *stats);

/* The strain-contraction gradient alone, given forward velocity u and adjoint
   velocity lambda (same formulas as above).  Asynchronous. */
int stokes_grad(stokes_ctx *ctx, const double *xu, const double *lu, double *dmu_cell,
                double *dmu_edge, double *drho_cell, double *dgamma_cell);

/* Residual history of the Krylov solves: buf (HOST memory, cap doubles,
   owned by the caller, kept until replaced or the ctx is destroyed) receives
   after every Arnoldi step of each later stokes_solve / stokes_adjoint_solve
   its rel_res_est, from index 0, while fewer than cap entries are written
   (stokes_stats.history_len counts them).  buf = NULL or cap = 0 turns the
   history off. */
int stokes_set_history(stokes_ctx *ctx, double *buf, int cap);

/* Rescaling factor c in use (Sec. "Rescaling of the Linear System"). */
double stokes_rescale(const stokes_ctx *ctx);

/* Per-kernel timing for the roofline report.  When enabled, every launch of
   the finest-level velocity Gauss-Seidel colour pass is bracketed by HIP
   events on the context stream; stokes_kernel_time returns the accumulated
   milliseconds, the launch count and the algorithmic bytes of those launches
   (each value the pass needs counted once: every velocity component, the
   cell and edge viscosities in full, the pass's own colour half of the
   right-hand side and of the mass coefficient, and the half of the
   component it writes).  Reading the totals synchronises the stream.
   enable: 0 off, 1 per-launch and per-V-cycle events (every V-cycle then runs
   kernel by kernel), 2 per-V-cycle events only (the finest-level V-cycle
   replays its recorded graph as in untimed runs); other values EINVAL.
   Enabling resets the totals. */
int stokes_set_timing(stokes_ctx *ctx, int enable);
int stokes_kernel_time(stokes_ctx *ctx, double *ms_total, long *launches, double *bytes_total);
/* With timing enabled, every V-cycle started from the finest level (in the
   preconditioner, the subsolvers and the *_mg_solve calls) is also bracketed
   by HIP events: pressure = 0 selects the velocity cycles, 1 the pressure
   cycles.  Returns their accumulated milliseconds, their count and their
   algorithmic bytes (each value a kernel of the cycle needs counted once,
   colour passes as above, summed over the levels), for the aggregate V-cycle
   bandwidth.
   Synchronises the stream. */
int stokes_vcycle_time(stokes_ctx *ctx, int pressure, double *ms_total, long *cycles,
                       double *bytes_total);

void stokes_destroy(stokes_ctx *ctx);
const char *stokes_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* STOKES_MI355X_H */
