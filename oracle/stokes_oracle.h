/*
 * stokes_oracle.h -- plain FP64 CPU oracle for the variable-coefficient
 * staggered-grid (MAC) Stokes solver of Cai, Nonaka, Bell, Griffith and Donev,
 * "Efficient Variable-Coefficient Finite-Volume Stokes Solvers" (arXiv:1308.4605).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU product
 * path shares no code, header or table with it.
 *
 * Conventions (same data layout as the product ABI, defined independently):
 *   - axes 0,1,2 = x,y,z; arrays are C-ordered with x fastest;
 *   - d = 2 or 3; for d = 2, n[2] = 1 and there is no z component;
 *   - bc[a] = 0 periodic, 1 no-slip walls at both ends of axis a, 2 free-slip
 *     walls, 3 no-slip low / free-slip high, 4 free-slip low / no-slip high;
 *   - w[a] = 1 when axis a has walls (bc[a] != 0), else 0;
 *   - velocity component k lives on faces normal to axis k; its array has
 *     n[a] entries along a != k and n[k] + w[k] entries along k; wall faces
 *     (index 0 and n[k] on a wall axis) hold 0 and are not unknowns;
 *   - the d velocity arrays are stored back to back in one buffer (x, y, z);
 *   - cell arrays (p, rho, mu) have n[0]*n[1]*n[2] entries;
 *   - edge viscosity: edge family m is parallel to axis m and carries the shear
 *     viscosity for the pair {k,l} = the other two axes; it has n[a] + w[a]
 *     entries along a in {k,l} and n[m] along m.  In 2D only family m = 2 (the
 *     grid nodes) exists.  Families are stored back to back in the order
 *     m = 2, 1, 0 (3D) or m = 2 (2D).
 */
#ifndef STOKES_ORACLE_H
#define STOKES_ORACLE_H
#include <stddef.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ENOCONV = -4,
       ORC_EBREAKDOWN = -5, ORC_ENONFINITE = -6, ORC_EINCOMPAT = -7 };
/* per axis; the last two mix the two walls of one axis: no-slip at the low
   end and free-slip at the high end, or the reverse */
enum { ORC_PERIODIC = 0, ORC_NOSLIP = 1, ORC_FREESLIP = 2, ORC_NOSLIP_FREESLIP = 3,
       ORC_FREESLIP_NOSLIP = 4 };
enum { ORC_P1 = 1, ORC_P2 = 2, ORC_P3 = 3, ORC_P4 = 4, ORC_P5 = 5 };
enum { ORC_GMRES_LEFT = 0, ORC_FGMRES = 1 };
enum { ORC_EDGE_ARITH = 0, ORC_EDGE_HARMONIC = 1, ORC_EDGE_GIVEN = 2 };

typedef struct {
  int dim;
  int n[3];
  double h;
  int bc[3];
  double theta;
  int precond;      /* ORC_P1..ORC_P5 */
  int krylov;       /* ORC_GMRES_LEFT or ORC_FGMRES */
  int restart;      /* GMRES(m) restart length */
  int nu_pre, nu_post, nu_coarse;
  int vcycles;      /* V-cycles per subsolver application */
  double rescale_c; /* <= 0: c = h / geometric mean of mu_cell */
  int edge_avg;     /* ORC_EDGE_* */
  int scaling;      /* ORC_SCALE_UNIFORM: the rescaled system of eq.
                       Stokes_rescaled; ORC_SCALE_DIAGONAL: that system scaled
                       again by diagonal matrices, velocity and pressure
                       separately (Sec. "Rescaling of the Linear System") */
  int extended;     /* 1: the solver's true residuals b - M x in extended
                       precision (__float128), rounded to FP64 */
} orc_params;

enum { ORC_SCALE_UNIFORM = 0, ORC_SCALE_DIAGONAL = 1 };

typedef struct {
  int iters, restarts, precond_applies, scalar_vcycles;
  double rel_res_true, rel_res_est;
} orc_stats;

typedef struct orc_ctx orc_ctx;

/* gamma_cell: bulk viscosity per cell (>= 0), or NULL.  Given, the stress
   is mu (grad u + grad u^T) + (gamma - 2/3 mu)(div u) I (Sec. "Preconditioners", the form
   for div u = g != 0) and the Schur approximation uses gamma + 4/3 mu in place
   of 2 mu (eq. Schur_app_bulk).  NULL: the incompressible stress form. */
int    orc_create(const orc_params *p, const double *rho_cell, const double *mu_cell,
                  const double *mu_edges_given, const double *gamma_cell, orc_ctx **out);
void   orc_destroy(orc_ctx *c);
size_t orc_nvel(const orc_ctx *c);    /* stored velocity entries (all components) */
size_t orc_ncell(const orc_ctx *c);
size_t orc_nedge(const orc_ctx *c);   /* stored edge entries (all families) */
int    orc_nlevels(const orc_ctx *c);
double orc_rescale(const orc_ctx *c);

/* y = M x with the unscaled coefficients. */
int orc_apply(orc_ctx *c, const double *xu, const double *xp, double *yu, double *yp);
/* Boundary terms of the affine operator for prescribed wall velocities
   (Sec. "Krylov Solver"): (cu, cp) = M applied to the field that is zero at the unknowns
   and holds un on the wall faces (normal velocity; interior entries of un
   are ignored) and ut on the wall edges (tangential velocity of the
   component parallel to the wall and normal to the edge; no-slip walls only).
   The flow with those wall velocities solves M x = b - (cu, cp). */
int orc_boundary_rhs(orc_ctx *c, const double *un, const double *ut, double *cu, double *cp);
/* r = b - M x with the caller's (unscaled) coefficients, evaluated in FP64
   (extended = 0) or in __float128 and rounded once to FP64 (extended = 1). */
int orc_residual(orc_ctx *c, const double *bu, const double *bp, const double *xu,
                 const double *xp, double *ru, double *rp, int extended);
/* the diagonal scaling S of the rescaled system's unknowns ([faces | cells],
   nvel + ncell entries; wall faces 1) when scaling = ORC_SCALE_DIAGONAL */
int orc_diag_scaling(orc_ctx *c, double *s);
/* z = P^{-1} b (unscaled system). */
int orc_precond(orc_ctx *c, const double *bu, const double *bp, double *zu, double *zp);
/* velocity subsolver e = A~^{-1} r and pressure subsolver e = L~_rho^{-1} r (unscaled). */
int orc_vel_subsolve(orc_ctx *c, const double *r, double *e);
int orc_p_subsolve(orc_ctx *c, const double *r, double *e);
/* Stand-alone multigrid solves of the same subproblems (unscaled): V-cycles
   e <- e + V(r - A e) from e = 0 until ||r - A e|| <= tol ||r|| or
   max_cycles; *cycles and *rel_res report what was done.  ORC_ENOCONV when
   max_cycles ran out (e holds the last iterate). */
int orc_vel_mg_solve(orc_ctx *c, const double *r, double *e, double tol, int max_cycles,
                     int *cycles, double *rel_res);
int orc_p_mg_solve(orc_ctx *c, const double *r, double *e, double tol, int max_cycles,
                   int *cycles, double *rel_res);
/* one multicolour Gauss-Seidel sweep on level 0 (unscaled operator), in place. */
int orc_vel_sweep(orc_ctx *c, const double *rhs, double *phi);
int orc_p_sweep(orc_ctx *c, const double *rhs, double *phi);
/* The multigrid transfers between level l (fine) and level l + 1 (coarse),
   exposed so that tests can pin them directly (Appendix C):
   face restriction rc = R rf and face prolongation phif += P ec (velocity
   layout of the two levels), cell restriction (mean of the 2^d fine cells)
   and cell prolongation (injection, added).  ORC_EINVAL when l + 1 is not a
   level. */
int orc_restrict_faces(orc_ctx *c, int level, const double *rf, double *rc);
int orc_prolong_add_faces(orc_ctx *c, int level, const double *ec, double *phif);
int orc_restrict_cells(orc_ctx *c, int level, const double *rf, double *rc);
int orc_prolong_add_cells(orc_ctx *c, int level, const double *ec, double *pf);
/* sizes of the velocity and cell arrays of a level */
int orc_level_sizes(orc_ctx *c, int level, size_t *nvel, size_t *ncell);
/* copies of the scaled level coefficients (for tests). which: 0 alpha faces,
   1 beta faces, 2 mu cells, 3 mu edges. */
int orc_level_coef(orc_ctx *c, int level, int which, double *out, size_t cap);
int orc_level_dims(orc_ctx *c, int level, int n_out[3]);
/* Solve M x = b to true relative residual tol. */
int orc_solve(orc_ctx *c, const double *bu, const double *bp, double *xu, double *xp,
              double tol, int max_iter, int use_x0, orc_stats *st);
/* Adjoint: solve M lambda = g, then gradients of L (with dL/dx = g) w.r.t.
   mu_cell (total, through derived edges), mu_edge (partial) and rho_cell. */
int orc_adjoint(orc_ctx *c, const double *xu, const double *xp,
                const double *gu, const double *gp, double *lu, double *lp,
                double *dmu_cell, double *dmu_edge, double *drho_cell,
                double *dgamma_cell, double tol, int max_iter, orc_stats *st);
/* Gradient contraction only (no solve): given forward x and adjoint lambda.
   dgamma_cell (bulk-viscosity contexts only, else NULL) receives
   -(D lambda)(D x) per cell. */
int orc_grad(orc_ctx *c, const double *xu, const double *lu,
             double *dmu_cell, double *dmu_edge, double *drho_cell, double *dgamma_cell);
int orc_threads(void);
/* threads of the OpenMP grid loops from now on (timing of the CPU baseline) */
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
