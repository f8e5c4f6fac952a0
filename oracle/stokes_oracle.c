/*
 * stokes_oracle.c -- plain, slow, obviously correct FP64 CPU oracle for the
 * variable-coefficient MAC Stokes solver of arXiv:1308.4605.
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it; the GPU product path never links or calls it and
 * shares no code with it.
 *
 * What each part follows (sections/equations of the paper):
 *   - saddle-point system M = [[A, G], [-D, 0]], A = theta*rho - L_mu
 *     (Sec. "Preconditioners", eq. Saddle_sys);
 *   - MAC divergence D, gradient G (Sec. "Staggered-grid Discretization"), stress-form viscous operator
 *     L_mu (Sec. "Staggered-grid Discretization", eq. div_stress) with one-sided wall differences and
 *     face density rho_f = mean of the two cells, node/edge viscosity = mean of
 *     the neighbouring cells (Sec. "Staggered-grid Discretization");
 *   - Schur approximation S~^{-1} = -theta L~_rho^{-1} + 2 mu (Sec. "Preconditioners",
 *     eq. Schur_app_varDen_varVis) and preconditioners P1 (eq. P1_practical),
 *     P2 (eq. CC_Pre_lower), P3 (eq. CC_Pre_upper), P4 (eq. CC_Pre_diagonal),
 *     P5 (Sec. "Other preconditioners", the three-step Uzawa-like recipe);
 *   - multigrid V-cycles with multicolour Gauss-Seidel, restriction,
 *     prolongation and coefficient coarsening (Appendix C);
 *   - zero initial guess for subsolvers and null-space handling (Sec. "Krylov Solver");
 *   - rescaling by c ~ h/mu0 (Sec. "Rescaling of the Linear System", eq. Stokes_rescaled);
 *   - GMRES(m) with left preconditioning and FGMRES(m) (Sec. "Krylov Solver" and Sec. "Results"
 *     opening paragraphs; Saad's algorithms).
 * Readings of passages the paper leaves open are listed in the repository's
 * design notes; each is marked "reading" below where it is applied.
 *
 * Precision: FP64 throughout.  Reductions are serial (deterministic).  Grid
 * loops without reductions may run under OpenMP; they write disjoint entries.
 */
#include "stokes_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* grid and level                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
  int d;      /* dimension */
  int n[3];   /* cells per axis (n[2] = 1 for d = 2) */
  int ns[3];  /* 1: walls on this axis (no-slip or free-slip), 0: periodic */
  int fs[3][2]; /* fs[a][0] / fs[a][1]: the low / high wall of axis a is free-slip */
  int sing;   /* bit k: velocity component k is singular (mean removed) */
  double h;   /* grid spacing */
} grid_t;

typedef struct {
  grid_t g;
  size_t foff[3], fcnt[3], nvel; /* velocity component offsets/counts */
  size_t eoff[3], ecnt[3], nedge; /* edge family offsets/counts (by family m) */
  size_t ncell;
  double *alpha; /* theta*rho_f on faces (nvel) */
  double *beta;  /* 1/rho_f on faces (nvel) */
  double *mu_c;  /* cell viscosity (ncell) */
  double *mu_e;  /* edge viscosity (nedge) */
  /* gamma - 2/3 mu per cell: the coefficient of (div u) I in the stress
     when bulk viscosity is included (Sec. "Preconditioners"); NULL = incompressible form */
  double *lam_c;
  /* V-cycle work arrays */
  double *phi_u, *rhs_u, *res_u;
  double *phi_p, *rhs_p, *res_p;
  /* prescribed wall velocities, set only while the boundary terms of the
     affine operator are evaluated: normal values on wall faces (velocity
     layout) and tangential values on wall edges (edge layout); NULL = 0 */
  const double *bd_un, *bd_ut;
} level_t;

struct orc_ctx {
  orc_params p;
  double c;        /* rescale factor (Sec. "Rescaling of the Linear System") */
  int nlev;
  level_t raw;     /* unscaled fine coefficients: used by orc_apply */
  level_t *lev;    /* scaled hierarchy: used by the solver */
  int vel_singular;
  double *given_edges; /* copy of caller edges for ORC_EDGE_GIVEN */
  /* ORC_SCALE_DIAGONAL: the diagonal scaling S of the rescaled unknowns
     ([faces | cells]); NULL otherwise */
  double *sdiag;
};

static void fatal(const char *msg) {
  fprintf(stderr, "stokes_oracle: internal index error: %s\n", msg);
  abort();
}

static inline int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

static inline size_t lin3(const int dm[3], int i0, int i1, int i2) {
  return ((size_t)i2 * (size_t)dm[1] + (size_t)i1) * (size_t)dm[0] + (size_t)i0;
}

/* dims of velocity component k: n[a] cells along a != k, n[k] + walls along k */
static void face_dims(const grid_t *g, int k, int dm[3]) {
  for (int a = 0; a < 3; a++) dm[a] = g->n[a] + ((a == k && a < g->d) ? g->ns[a] : 0);
}

/* dims of edge family m (parallel to axis m): nodes along the other two axes */
static void edge_dims(const grid_t *g, int m, int dm[3]) {
  for (int a = 0; a < 3; a++) dm[a] = g->n[a] + ((a != m && a < g->d) ? g->ns[a] : 0);
}

static void level_layout(level_t *L) {
  const grid_t *g = &L->g;
  size_t off = 0;
  for (int k = 0; k < 3; k++) {
    L->foff[k] = off;
    L->fcnt[k] = 0;
    if (k < g->d) {
      int dm[3];
      face_dims(g, k, dm);
      L->fcnt[k] = (size_t)dm[0] * dm[1] * dm[2];
      off += L->fcnt[k];
    }
  }
  L->nvel = off;
  L->ncell = (size_t)g->n[0] * g->n[1] * g->n[2];
  /* edge families stored in the order m = 2, 1, 0 (3D) or m = 2 (2D) */
  off = 0;
  for (int m = 0; m < 3; m++) { L->eoff[m] = 0; L->ecnt[m] = 0; }
  for (int m = 2; m >= 0; m--) {
    if (g->d == 2 && m != 2) continue;
    int dm[3];
    edge_dims(g, m, dm);
    L->eoff[m] = off;
    L->ecnt[m] = (size_t)dm[0] * dm[1] * dm[2];
    off += L->ecnt[m];
  }
  L->nedge = off;
}

static int is_wall_face(const grid_t *g, int k, const int f[3]) {
  return g->ns[k] && (f[k] == 0 || f[k] == g->n[k]);
}

/* velocity component k at face index f; periodic indices wrap; wall faces
   are not unknowns and read as 0, or as the prescribed normal velocity while
   boundary terms are evaluated. */
static double fget(const level_t *L, const double *u, int k, const int f_in[3]) {
  const grid_t *g = &L->g;
  int f[3] = {f_in[0], f_in[1], f_in[2]};
  int wall = 0;
  for (int a = 0; a < g->d; a++) {
    if (g->ns[a]) {
      if (a == k) {
        if (f[a] < 0 || f[a] > g->n[a]) fatal("face index outside wall range");
        if (f[a] == 0 || f[a] == g->n[a]) wall = 1;
      } else if (f[a] < 0 || f[a] >= g->n[a]) {
        fatal("tangential face index outside no-slip domain");
      }
    } else {
      f[a] = wrapi(f[a], g->n[a]);
    }
  }
  int dm[3];
  face_dims(g, k, dm);
  const size_t q = L->foff[k] + lin3(dm, f[0], f[1], f[2]);
  if (wall) return L->bd_un ? L->bd_un[q] : 0.0;
  return u[q];
}

static size_t fidx(const level_t *L, int k, const int f[3]) {
  int dm[3];
  face_dims(&L->g, k, dm);
  return L->foff[k] + lin3(dm, f[0], f[1], f[2]);
}

/* cell index with periodic wrap */
static size_t cidx(const grid_t *g, const int c_in[3]) {
  int c[3] = {c_in[0], c_in[1], c_in[2]};
  for (int a = 0; a < g->d; a++) {
    if (g->ns[a]) {
      if (c[a] < 0 || c[a] >= g->n[a]) fatal("cell index outside no-slip domain");
    } else {
      c[a] = wrapi(c[a], g->n[a]);
    }
  }
  return lin3(g->n, c[0], c[1], c[2]);
}

/* edge family m at edge index e (nodes along the two axes != m); periodic wrap */
static size_t eidx(const level_t *L, int m, const int e_in[3]) {
  const grid_t *g = &L->g;
  int e[3] = {e_in[0], e_in[1], e_in[2]};
  for (int a = 0; a < g->d; a++) {
    int lim = g->n[a] + ((a != m) ? g->ns[a] : 0);
    if (g->ns[a]) {
      if (e[a] < 0 || e[a] >= lim) fatal("edge index outside domain");
    } else {
      e[a] = wrapi(e[a], g->n[a]);
    }
  }
  int dm[3];
  edge_dims(g, m, dm);
  return L->eoff[m] + lin3(dm, e[0], e[1], e[2]);
}

/* ------------------------------------------------------------------------ */
/* discrete operators (Sec. "Staggered-grid Discretization")                                             */
/* ------------------------------------------------------------------------ */

/* derivative of u_k along axis l at the edge point e (e is a node along k and
   l).  Centred difference of the two faces above/below the edge; at a no-slip
   wall along l the one-sided difference (u_adjacent - 0)/(h/2) is used, the
   wall value of the tangential velocity being 0 (reading of the one-sided wall
   rule of Sec. "Staggered-grid Discretization"). */
static double dkl(const level_t *L, const double *u, int k, int l, const int e[3]) {
  const grid_t *g = &L->g;
  const double h = g->h;
  int f[3] = {e[0], e[1], e[2]};
  if (g->ns[l] && (e[l] == 0 || e[l] == g->n[l])) {
    /* the wall value of u_k at this edge: 0, or the prescribed tangential
       velocity while boundary terms are evaluated */
    const int m = (g->d == 3) ? 3 - k - l : 2;
    const double uw = L->bd_ut ? L->bd_ut[eidx(L, m, e)] : 0.0;
    if (e[l] == 0) return 2.0 * (fget(L, u, k, f) - uw) / h;
    f[l] = g->n[l] - 1;
    return -2.0 * (fget(L, u, k, f) - uw) / h;
  }
  int fb[3] = {e[0], e[1], e[2]};
  fb[l] -= 1;
  return (fget(L, u, k, f) - fget(L, u, k, fb)) / h;
}

/* the edge lies on a free-slip wall of axis a */
static int on_free_slip(const grid_t *g, int a, const int e[3]) {
  return (e[a] == 0 && g->fs[a][0]) || (e[a] == g->n[a] && g->fs[a][1]);
}

/* shear rate gamma_kl = du_k/dx_l + du_l/dx_k at an edge; zero on a free-slip
   wall, where the tangential momentum flux vanishes (Sec. "Staggered-grid Discretization") */
static double shear_rate(const level_t *L, const double *u, int k, int l, const int e[3]) {
  if (on_free_slip(&L->g, k, e) || on_free_slip(&L->g, l, e)) return 0.0;
  return dkl(L, u, k, l, e) + dkl(L, u, l, k, e);
}

/* normal strain rate (D^k u_k) at cell c */
static double normal_rate(const level_t *L, const double *u, int k, const int c[3]) {
  int fr[3] = {c[0], c[1], c[2]};
  fr[k] += 1;
  return (fget(L, u, k, fr) - fget(L, u, k, c)) / L->g.h;
}

static int third_axis(int k, int l) { return 3 - k - l; }

static double div_cell(const level_t *L, const double *u, const int c[3]);

/* (L_mu u)_k at interior face f: divergence of the stress tau = mu (grad u +
   grad u^T), eq. div_stress, with centred staggered differences. */
static double lmu_row(const level_t *L, const double *mu_c, const double *mu_e,
                      const double *u, int k, const int f[3]) {
  const grid_t *g = &L->g;
  const double h = g->h;
  /* normal stress tau_kk = 2 mu_cell D^k u_k at the cells right/left of f */
  int cr[3] = {f[0], f[1], f[2]};
  int cl[3] = {f[0], f[1], f[2]};
  cl[k] -= 1;
  double tr = 2.0 * mu_c[cidx(g, cr)] * normal_rate(L, u, k, cr);
  double tl = 2.0 * mu_c[cidx(g, cl)] * normal_rate(L, u, k, cl);
  /* bulk viscosity: tau_kk gains (gamma - 2/3 mu)(div u) */
  if (L->lam_c) {
    tr += L->lam_c[cidx(g, cr)] * div_cell(L, u, cr);
    tl += L->lam_c[cidx(g, cl)] * div_cell(L, u, cl);
  }
  double s = (tr - tl) / h;
  /* shear stresses tau_kl = mu_edge gamma_kl on the edges above/below f */
  for (int l = 0; l < g->d; l++) {
    if (l == k) continue;
    int m = third_axis(k, l);
    int elo[3] = {f[0], f[1], f[2]};
    int ehi[3] = {f[0], f[1], f[2]};
    ehi[l] += 1;
    if (!g->ns[l]) ehi[l] = wrapi(ehi[l], g->n[l]);
    double thi = mu_e[eidx(L, m, ehi)] * shear_rate(L, u, k, l, ehi);
    double tlo = mu_e[eidx(L, m, elo)] * shear_rate(L, u, k, l, elo);
    s += (thi - tlo) / h;
  }
  return s;
}

/* diagonal of A = alpha - L_mu at face f (Appendix C relaxation needs it). */
static double a_diag(const level_t *L, const double *alpha, const double *mu_c,
                     const double *mu_e, int k, const int f[3]) {
  const grid_t *g = &L->g;
  const double h2 = g->h * g->h;
  int cr[3] = {f[0], f[1], f[2]};
  int cl[3] = {f[0], f[1], f[2]};
  cl[k] -= 1;
  double dg = alpha[fidx(L, k, f)] + 2.0 * (mu_c[cidx(g, cr)] + mu_c[cidx(g, cl)]) / h2;
  if (L->lam_c) dg += (L->lam_c[cidx(g, cr)] + L->lam_c[cidx(g, cl)]) / h2;
  for (int l = 0; l < g->d; l++) {
    if (l == k) continue;
    int m = third_axis(k, l);
    int elo[3] = {f[0], f[1], f[2]};
    int ehi[3] = {f[0], f[1], f[2]};
    ehi[l] += 1;
    if (!g->ns[l]) ehi[l] = wrapi(ehi[l], g->n[l]);
    /* a no-slip wall edge carries the one-sided difference (weight 2), a
       free-slip wall edge no flux (weight 0) */
    double wlo = (g->ns[l] && f[l] == 0) ? (g->fs[l][0] ? 0.0 : 2.0) : 1.0;
    double whi = (g->ns[l] && f[l] + 1 == g->n[l]) ? (g->fs[l][1] ? 0.0 : 2.0) : 1.0;
    dg += (whi * mu_e[eidx(L, m, ehi)] + wlo * mu_e[eidx(L, m, elo)]) / h2;
  }
  return dg;
}

/* (A u)_k at face f */
static double a_row(const level_t *L, const double *alpha, const double *mu_c,
                    const double *mu_e, const double *u, int k, const int f[3]) {
  return alpha[fidx(L, k, f)] * u[fidx(L, k, f)] - lmu_row(L, mu_c, mu_e, u, k, f);
}

/* (D u) at cell c: sum over components of the face difference / h */
static double div_cell(const level_t *L, const double *u, const int c[3]) {
  double s = 0.0;
  for (int k = 0; k < L->g.d; k++) s += normal_rate(L, u, k, c);
  return s;
}

/* (G p)_k at interior face f */
static double grad_face(const level_t *L, const double *p, int k, const int f[3]) {
  int cl[3] = {f[0], f[1], f[2]};
  cl[k] -= 1;
  return (p[cidx(&L->g, f)] - p[cidx(&L->g, cl)]) / L->g.h;
}

/* pressure flux beta G p through face f of normal k; zero on walls (natural
   boundary condition of the pressure equation). */
static double p_flux(const level_t *L, const double *beta, const double *p, int k, const int f[3]) {
  if (is_wall_face(&L->g, k, f)) return 0.0;
  int ff[3] = {f[0], f[1], f[2]};
  if (!L->g.ns[k]) ff[k] = wrapi(ff[k], L->g.n[k]);
  return beta[fidx(L, k, ff)] * grad_face(L, p, k, ff);
}

/* (L_rho p)_c = D (beta G p), L_rho = D rho^{-1} G (Sec. "Preconditioners") */
static double lrho_cell(const level_t *L, const double *beta, const double *p, const int c[3]) {
  double s = 0.0;
  for (int k = 0; k < L->g.d; k++) {
    int fr[3] = {c[0], c[1], c[2]};
    fr[k] += 1;
    s += (p_flux(L, beta, p, k, fr) - p_flux(L, beta, p, k, c)) / L->g.h;
  }
  return s;
}

static double lrho_diag(const level_t *L, const double *beta, const int c[3]) {
  const grid_t *g = &L->g;
  double s = 0.0;
  for (int k = 0; k < g->d; k++) {
    int fr[3] = {c[0], c[1], c[2]};
    fr[k] += 1;
    if (!is_wall_face(g, k, fr)) {
      if (!g->ns[k]) fr[k] = wrapi(fr[k], g->n[k]);
      s -= beta[fidx(L, k, fr)];
    }
    if (!is_wall_face(g, k, c)) s -= beta[fidx(L, k, c)];
  }
  return s / (g->h * g->h);
}

/* face loops: visit every face of component k (walls included) */
#define FOR_FACES(L, k, f)                                          \
  int dm_##f[3];                                                    \
  face_dims(&(L)->g, (k), dm_##f);                                  \
  _Pragma("omp parallel for collapse(2) schedule(static)")          \
  for (int i2_##f = 0; i2_##f < dm_##f[2]; i2_##f++)                \
    for (int i1_##f = 0; i1_##f < dm_##f[1]; i1_##f++)             \
      for (int i0_##f = 0; i0_##f < dm_##f[0]; i0_##f++)

#define FACE_IDX(f) int f[3] = {i0_##f, i1_##f, i2_##f}

/* y = M x on level L with coefficient set (alpha, mu_c, mu_e); xp/yp cells */
static void apply_m(const level_t *L, const double *alpha, const double *mu_c,
                    const double *mu_e, const double *xu, const double *xp,
                    double *yu, double *yp) {
  const grid_t *g = &L->g;
  for (int k = 0; k < g->d; k++) {
    FOR_FACES(L, k, f) {
      FACE_IDX(f);
      size_t q = fidx(L, k, f);
      if (is_wall_face(g, k, f)) { yu[q] = 0.0; continue; }
      yu[q] = a_row(L, alpha, mu_c, mu_e, xu, k, f) + grad_face(L, xp, k, f);
    }
  }
#pragma omp parallel for collapse(2) schedule(static)
  for (int i2 = 0; i2 < g->n[2]; i2++)
    for (int i1 = 0; i1 < g->n[1]; i1++)
      for (int i0 = 0; i0 < g->n[0]; i0++) {
        int c[3] = {i0, i1, i2};
        yp[lin3(g->n, i0, i1, i2)] = -div_cell(L, xu, c);
      }
}

/* ------------------------------------------------------------------------ */
/* extended precision residual (Sec. "Rescaling of the Linear System": in   */
/* extreme cases extended precision arithmetic may be needed in the solver) */
/* ------------------------------------------------------------------------ */

/* The same operator as above, every operation in __float128 (113-bit
   significand) on the FP64 values of u and of the coefficients; only the
   final residual is rounded to FP64. */
typedef __float128 quad;

static quad q_dkl(const level_t *L, const double *u, int k, int l, const int e[3]) {
  const grid_t *g = &L->g;
  const quad h = (quad)g->h;
  int f[3] = {e[0], e[1], e[2]};
  if (g->ns[l] && (e[l] == 0 || e[l] == g->n[l])) {
    const int m = (g->d == 3) ? 3 - k - l : 2;
    const quad uw = L->bd_ut ? (quad)L->bd_ut[eidx(L, m, e)] : (quad)0;
    if (e[l] == 0) return 2 * ((quad)fget(L, u, k, f) - uw) / h;
    f[l] = g->n[l] - 1;
    return -2 * ((quad)fget(L, u, k, f) - uw) / h;
  }
  int fb[3] = {e[0], e[1], e[2]};
  fb[l] -= 1;
  return ((quad)fget(L, u, k, f) - (quad)fget(L, u, k, fb)) / h;
}

static quad q_shear_rate(const level_t *L, const double *u, int k, int l, const int e[3]) {
  if (on_free_slip(&L->g, k, e) || on_free_slip(&L->g, l, e)) return 0;
  return q_dkl(L, u, k, l, e) + q_dkl(L, u, l, k, e);
}

static quad q_normal_rate(const level_t *L, const double *u, int k, const int c[3]) {
  int fr[3] = {c[0], c[1], c[2]};
  fr[k] += 1;
  return ((quad)fget(L, u, k, fr) - (quad)fget(L, u, k, c)) / (quad)L->g.h;
}

static quad q_div_cell(const level_t *L, const double *u, const int c[3]) {
  quad s = 0;
  for (int k = 0; k < L->g.d; k++) s += q_normal_rate(L, u, k, c);
  return s;
}

static quad q_lmu_row(const level_t *L, const double *mu_c, const double *mu_e,
                      const double *u, int k, const int f[3]) {
  const grid_t *g = &L->g;
  const quad h = (quad)g->h;
  int cr[3] = {f[0], f[1], f[2]};
  int cl[3] = {f[0], f[1], f[2]};
  cl[k] -= 1;
  quad tr = 2 * (quad)mu_c[cidx(g, cr)] * q_normal_rate(L, u, k, cr);
  quad tl = 2 * (quad)mu_c[cidx(g, cl)] * q_normal_rate(L, u, k, cl);
  if (L->lam_c) {
    tr += (quad)L->lam_c[cidx(g, cr)] * q_div_cell(L, u, cr);
    tl += (quad)L->lam_c[cidx(g, cl)] * q_div_cell(L, u, cl);
  }
  quad s = (tr - tl) / h;
  for (int l = 0; l < g->d; l++) {
    if (l == k) continue;
    int m = third_axis(k, l);
    int elo[3] = {f[0], f[1], f[2]};
    int ehi[3] = {f[0], f[1], f[2]};
    ehi[l] += 1;
    if (!g->ns[l]) ehi[l] = wrapi(ehi[l], g->n[l]);
    quad thi = (quad)mu_e[eidx(L, m, ehi)] * q_shear_rate(L, u, k, l, ehi);
    quad tlo = (quad)mu_e[eidx(L, m, elo)] * q_shear_rate(L, u, k, l, elo);
    s += (thi - tlo) / h;
  }
  return s;
}

/* r = b - M x on level L (coefficients alpha, mu_c, mu_e, L->lam_c) in
   __float128, rounded once; x, b, r are [faces | cells] */
static void residual_quad(const level_t *L, const double *alpha, const double *mu_c,
                          const double *mu_e, const double *b, const double *x, double *r) {
  const grid_t *g = &L->g;
  const double *xu = x, *xp = x + L->nvel;
  for (int k = 0; k < g->d; k++) {
    FOR_FACES(L, k, f) {
      FACE_IDX(f);
      size_t q = fidx(L, k, f);
      if (is_wall_face(g, k, f)) { r[q] = 0.0; continue; }
      int cl[3] = {f[0], f[1], f[2]};
      cl[k] -= 1;
      const quad au = (quad)alpha[q] * (quad)xu[q] - q_lmu_row(L, mu_c, mu_e, xu, k, f);
      const quad gp = ((quad)xp[cidx(g, f)] - (quad)xp[cidx(g, cl)]) / (quad)g->h;
      r[q] = (double)((quad)b[q] - (au + gp));
    }
  }
#pragma omp parallel for collapse(2) schedule(static)
  for (int i2 = 0; i2 < g->n[2]; i2++)
    for (int i1 = 0; i1 < g->n[1]; i1++)
      for (int i0 = 0; i0 < g->n[0]; i0++) {
        int c[3] = {i0, i1, i2};
        const size_t q = lin3(g->n, i0, i1, i2);
        r[L->nvel + q] = (double)((quad)b[L->nvel + q] + q_div_cell(L, xu, c));
      }
}

/* ------------------------------------------------------------------------ */
/* small vector helpers (serial reductions)                                  */
/* ------------------------------------------------------------------------ */

static double dotv(const double *a, const double *b, size_t n) {
  double s = 0.0;
  for (size_t i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

static void copyv(double *dst, const double *src, size_t n) { memcpy(dst, src, n * sizeof(double)); }
static void zerov(double *a, size_t n) { memset(a, 0, n * sizeof(double)); }

/* remove the mean of each velocity component over its interior faces */
static void remove_vel_means(const level_t *L, double *u) {
  const grid_t *g = &L->g;
  for (int k = 0; k < g->d; k++) {
    if (!((g->sing >> k) & 1)) continue;
    int dm[3];
    face_dims(g, k, dm);
    double s = 0.0;
    size_t cnt = 0;
    for (int i2 = 0; i2 < dm[2]; i2++)
      for (int i1 = 0; i1 < dm[1]; i1++)
        for (int i0 = 0; i0 < dm[0]; i0++) {
          int f[3] = {i0, i1, i2};
          if (is_wall_face(g, k, f)) continue;
          s += u[fidx(L, k, f)];
          cnt++;
        }
    double mean = s / (double)cnt;
    for (int i2 = 0; i2 < dm[2]; i2++)
      for (int i1 = 0; i1 < dm[1]; i1++)
        for (int i0 = 0; i0 < dm[0]; i0++) {
          int f[3] = {i0, i1, i2};
          if (is_wall_face(g, k, f)) continue;
          u[fidx(L, k, f)] -= mean;
        }
  }
}

static void remove_mean(double *p, size_t n) {
  double s = 0.0;
  for (size_t i = 0; i < n; i++) s += p[i];
  double mean = s / (double)n;
  for (size_t i = 0; i < n; i++) p[i] -= mean;
}

/* ------------------------------------------------------------------------ */
/* multigrid (Appendix C)                                                    */
/* ------------------------------------------------------------------------ */

/* one colour of Gauss-Seidel on A phi = rhs for component k:
   phi <- phi + D^{-1} (rhs - A phi) on faces with (i+j+k) % 2 == colour.
   Faces of one colour do not couple, so the in-place update is order-free. */
static void vel_colour_pass(const level_t *L, const double *alpha, const double *mu_c,
                            const double *mu_e, const double *rhs, double *phi,
                            int k, int colour) {
  const grid_t *g = &L->g;
  FOR_FACES(L, k, f) {
    FACE_IDX(f);
    if (((f[0] + f[1] + f[2]) & 1) != colour) continue;
    if (is_wall_face(g, k, f)) continue;
    size_t q = fidx(L, k, f);
    double r = rhs[q] - a_row(L, alpha, mu_c, mu_e, phi, k, f);
    phi[q] += r / a_diag(L, alpha, mu_c, mu_e, k, f);
  }
}

/* one sweep = all 2d colours in the order red-x, black-x, red-y, black-y,
   red-z, black-z (Appendix C; red = even index sum). */
static void vel_sweep(const level_t *L, const double *alpha, const double *mu_c,
                      const double *mu_e, const double *rhs, double *phi) {
  for (int k = 0; k < L->g.d; k++) {
    vel_colour_pass(L, alpha, mu_c, mu_e, rhs, phi, k, 0);
    vel_colour_pass(L, alpha, mu_c, mu_e, rhs, phi, k, 1);
  }
}

static void p_colour_pass(const level_t *L, const double *beta, const double *rhs,
                          double *phi, int colour) {
  const grid_t *g = &L->g;
#pragma omp parallel for collapse(2) schedule(static)
  for (int i2 = 0; i2 < g->n[2]; i2++)
    for (int i1 = 0; i1 < g->n[1]; i1++)
      for (int i0 = 0; i0 < g->n[0]; i0++) {
        if (((i0 + i1 + i2) & 1) != colour) continue;
        int c[3] = {i0, i1, i2};
        size_t q = lin3(g->n, i0, i1, i2);
        double r = rhs[q] - lrho_cell(L, beta, phi, c);
        phi[q] += r / lrho_diag(L, beta, c);
      }
}

static void p_sweep(const level_t *L, const double *beta, const double *rhs, double *phi) {
  p_colour_pass(L, beta, rhs, phi, 0);
  p_colour_pass(L, beta, rhs, phi, 1);
}

static void vel_residual(const level_t *L, const double *rhs, const double *phi, double *res) {
  const grid_t *g = &L->g;
  for (int k = 0; k < g->d; k++) {
    FOR_FACES(L, k, f) {
      FACE_IDX(f);
      size_t q = fidx(L, k, f);
      if (is_wall_face(g, k, f)) { res[q] = 0.0; continue; }
      res[q] = rhs[q] - a_row(L, L->alpha, L->mu_c, L->mu_e, phi, k, f);
    }
  }
}

static void p_residual(const level_t *L, const double *rhs, const double *phi, double *res) {
  const grid_t *g = &L->g;
#pragma omp parallel for collapse(2) schedule(static)
  for (int i2 = 0; i2 < g->n[2]; i2++)
    for (int i1 = 0; i1 < g->n[1]; i1++)
      for (int i0 = 0; i0 < g->n[0]; i0++) {
        int c[3] = {i0, i1, i2};
        size_t q = lin3(g->n, i0, i1, i2);
        res[q] = rhs[q] - lrho_cell(L, L->beta, phi, c);
      }
}

/* face restriction (Appendix C): normal weights 1/4, 1/2, 1/4 at fine faces
   2I-1, 2I, 2I+1 and the mean of the two fine faces along each tangential
   axis.  In 2D this is the printed 6-point stencil (1/8 and 1/4); the 3D
   12-point stencil is its tensor extension (reading). */
static void restrict_faces(const level_t *F, const level_t *C, const double *rf, double *rc) {
  const grid_t *g = &C->g;
  const double wn[3] = {0.25, 0.5, 0.25};
  const double wt = (g->d == 3) ? 0.25 : 0.5;
  for (int k = 0; k < g->d; k++) {
    FOR_FACES(C, k, F_) {
      FACE_IDX(F_);
      size_t q = fidx(C, k, F_);
      if (is_wall_face(g, k, F_)) { rc[q] = 0.0; continue; }
      double s = 0.0;
      for (int a = -1; a <= 1; a++) {
        double t = 0.0;
        for (int o2 = 0; o2 < (g->d == 3 ? 2 : 1); o2++)
          for (int o1 = 0; o1 < 2; o1++) {
            /* tangential offsets o1, o2 map onto the two axes != k */
            int ff[3];
            int tax[2] = {0, 0}, ti = 0;
            for (int b = 0; b < g->d; b++) if (b != k) tax[ti++] = b;
            ff[0] = 2 * F_[0]; ff[1] = 2 * F_[1]; ff[2] = (g->d == 3) ? 2 * F_[2] : 0;
            ff[k] = 2 * F_[k] + a;
            ff[tax[0]] += o1;
            if (g->d == 3) ff[tax[1]] += o2;
            t += fget(F, rf, k, ff);
          }
        s += wn[a + 1] * wt * t;
      }
      rc[q] = s;
    }
  }
}

/* 1D tangential prolongation weights: fine index j -> coarse J = j/2 with
   weight 3/4 and the next coarse neighbour away from j's parent centre with
   weight 1/4 (j even: J-1, j odd: J+1).  At a no-slip wall the missing
   neighbour is the odd reflection -phi(J), consistent with zero tangential
   velocity on the wall; at a free-slip wall the even reflection +phi(J),
   consistent with zero normal derivative (reading). */
static int tang_weights(const grid_t *gc, int a, int j, int idx[2], double w[2]) {
  int J = j / 2;
  int Jn = (j % 2 == 0) ? J - 1 : J + 1;
  idx[0] = J;
  w[0] = 0.75;
  if (gc->ns[a] && (Jn < 0 || Jn >= gc->n[a])) {
    idx[1] = J;
    w[1] = gc->fs[a][Jn < 0 ? 0 : 1] ? 0.25 : -0.25;
  } else {
    idx[1] = gc->ns[a] ? Jn : wrapi(Jn, gc->n[a]);
    w[1] = 0.25;
  }
  return 2;
}

/* phi_f += P e_c for faces (Appendix C): linear along the face normal (fine
   faces on coarse faces copy, the others take the mean of the two coarse
   faces), 3/4-1/4 along each tangential axis; 3D is the tensor product. */
static void prolong_add_faces(const level_t *C, const level_t *F, const double *ec, double *phif) {
  const grid_t *g = &F->g;
  const grid_t *gc = &C->g;
  for (int k = 0; k < g->d; k++) {
    FOR_FACES(F, k, f) {
      FACE_IDX(f);
      if (is_wall_face(g, k, f)) continue;
      int nidx[2];
      double nw[2];
      int nn;
      if (f[k] % 2 == 0) { nidx[0] = f[k] / 2; nw[0] = 1.0; nn = 1; }
      else { nidx[0] = (f[k] - 1) / 2; nidx[1] = (f[k] + 1) / 2; nw[0] = nw[1] = 0.5; nn = 2; }
      int tax[2] = {0, 0}, nt = 0;
      for (int b = 0; b < g->d; b++) if (b != k) tax[nt++] = b;
      int t0i[2], t1i[2] = {0, 0};
      double t0w[2], t1w[2] = {1.0, 0.0};
      tang_weights(gc, tax[0], f[tax[0]], t0i, t0w);
      int n1 = 1;
      if (nt == 2) { tang_weights(gc, tax[1], f[tax[1]], t1i, t1w); n1 = 2; }
      double s = 0.0;
      for (int a = 0; a < nn; a++)
        for (int b0 = 0; b0 < 2; b0++)
          for (int b1 = 0; b1 < n1; b1++) {
            int cf[3] = {0, 0, 0};
            cf[k] = nidx[a];
            cf[tax[0]] = t0i[b0];
            if (nt == 2) cf[tax[1]] = t1i[b1];
            s += nw[a] * t0w[b0] * t1w[b1] * fget(C, ec, k, cf);
          }
      phif[fidx(F, k, f)] += s;
    }
  }
}

/* cell restriction: mean of the 2^d fine cells; prolongation: injection */
static void restrict_cells(const level_t *F, const level_t *C, const double *rf, double *rc) {
  const grid_t *g = &C->g;
  const int d = g->d;
#pragma omp parallel for collapse(2) schedule(static)
  for (int i2 = 0; i2 < g->n[2]; i2++)
    for (int i1 = 0; i1 < g->n[1]; i1++)
      for (int i0 = 0; i0 < g->n[0]; i0++) {
        double s = 0.0;
        for (int o2 = 0; o2 < (d == 3 ? 2 : 1); o2++)
          for (int o1 = 0; o1 < 2; o1++)
            for (int o0 = 0; o0 < 2; o0++)
              s += rf[lin3(F->g.n, 2 * i0 + o0, 2 * i1 + o1, d == 3 ? 2 * i2 + o2 : 0)];
        rc[lin3(g->n, i0, i1, i2)] = s / (double)(1 << d);
      }
}

static void prolong_add_cells(const level_t *C, const level_t *F, const double *ec, double *pf) {
  const grid_t *g = &F->g;
  const int d = g->d;
#pragma omp parallel for collapse(2) schedule(static)
  for (int i2 = 0; i2 < g->n[2]; i2++)
    for (int i1 = 0; i1 < g->n[1]; i1++)
      for (int i0 = 0; i0 < g->n[0]; i0++)
        pf[lin3(g->n, i0, i1, i2)] += ec[lin3(C->g.n, i0 / 2, i1 / 2, d == 3 ? i2 / 2 : 0)];
}

/* velocity V-cycle on level l from a zero initial guess (Appendix C) */
static void vcycle_vel(orc_ctx *X, int l, const double *rhs, double *phi) {
  level_t *L = &X->lev[l];
  zerov(phi, L->nvel);
  if (l == X->nlev - 1) {
    /* coarsest level: many relaxations (the paper asks for 8 or more) */
    double *r = L->res_u;
    copyv(r, rhs, L->nvel);
    if (X->vel_singular) remove_vel_means(L, r);
    for (int s = 0; s < X->p.nu_coarse; s++) vel_sweep(L, L->alpha, L->mu_c, L->mu_e, r, phi);
    if (X->vel_singular) remove_vel_means(L, phi);
    return;
  }
  level_t *C = &X->lev[l + 1];
  for (int s = 0; s < X->p.nu_pre; s++) vel_sweep(L, L->alpha, L->mu_c, L->mu_e, rhs, phi);
  vel_residual(L, rhs, phi, L->res_u);
  restrict_faces(L, C, L->res_u, C->rhs_u);
  vcycle_vel(X, l + 1, C->rhs_u, C->phi_u);
  prolong_add_faces(C, L, C->phi_u, phi);
  for (int s = 0; s < X->p.nu_post; s++) vel_sweep(L, L->alpha, L->mu_c, L->mu_e, rhs, phi);
}

/* pressure (cell-centred Poisson) V-cycle; the operator is always singular
   (periodic or natural boundaries), so the coarsest problem is made
   consistent by removing the mean (Sec. "Krylov Solver" null-space care; reading). */
static void vcycle_p(orc_ctx *X, int l, const double *rhs, double *phi) {
  level_t *L = &X->lev[l];
  zerov(phi, L->ncell);
  if (l == X->nlev - 1) {
    double *r = L->res_p;
    copyv(r, rhs, L->ncell);
    remove_mean(r, L->ncell);
    for (int s = 0; s < X->p.nu_coarse; s++) p_sweep(L, L->beta, r, phi);
    remove_mean(phi, L->ncell);
    return;
  }
  level_t *C = &X->lev[l + 1];
  for (int s = 0; s < X->p.nu_pre; s++) p_sweep(L, L->beta, rhs, phi);
  p_residual(L, rhs, phi, L->res_p);
  restrict_cells(L, C, L->res_p, C->rhs_p);
  vcycle_p(X, l + 1, C->rhs_p, C->phi_p);
  prolong_add_cells(C, L, C->phi_p, phi);
  for (int s = 0; s < X->p.nu_post; s++) p_sweep(L, L->beta, rhs, phi);
}

/* A~^{-1} r on the scaled system: `vcycles` V-cycles from zero (Sec. "Krylov Solver":
   zero initial guess), mean handling for the periodic steady null space. */
static void vel_sub(orc_ctx *X, const double *r_in, double *e) {
  level_t *L = &X->lev[0];
  size_t n = L->nvel;
  double *r = (double *)malloc(n * sizeof(double));
  double *t = (double *)malloc(n * sizeof(double));
  double *de = (double *)malloc(n * sizeof(double));
  copyv(r, r_in, n);
  if (X->vel_singular) remove_vel_means(L, r);
  zerov(e, n);
  for (int v = 0; v < X->p.vcycles; v++) {
    if (v == 0) {
      vcycle_vel(X, 0, r, e);
    } else {
      vel_residual(L, r, e, t);
      vcycle_vel(X, 0, t, de);
      for (size_t i = 0; i < n; i++) e[i] += de[i];
    }
  }
  if (X->vel_singular) remove_vel_means(L, e);
  free(r); free(t); free(de);
}

/* L~_rho^{-1} r on the scaled system */
static void p_sub(orc_ctx *X, const double *r_in, double *e) {
  level_t *L = &X->lev[0];
  size_t n = L->ncell;
  double *r = (double *)malloc(n * sizeof(double));
  double *t = (double *)malloc(n * sizeof(double));
  double *de = (double *)malloc(n * sizeof(double));
  copyv(r, r_in, n);
  remove_mean(r, n);
  zerov(e, n);
  for (int v = 0; v < X->p.vcycles; v++) {
    if (v == 0) {
      vcycle_p(X, 0, r, e);
    } else {
      p_residual(L, r, e, t);
      vcycle_p(X, 0, t, de);
      for (size_t i = 0; i < n; i++) e[i] += de[i];
    }
  }
  remove_mean(e, n);
  free(r); free(t); free(de);
}

/* Stand-alone multigrid on one subproblem of the scaled system (Sec. "The effect of the number of multigrid cycles":
   the velocity and pressure multigrid solvers run to convergence are the
   reference cost of a split, projection-like method).  Starting from e = 0,
   each cycle applies one V-cycle to the current residual and adds the
   correction, e <- e + V(r - A e), until ||r - A e|| <= tol ||r|| or
   max_cycles cycles.  The right-hand side is first projected onto the range
   of a singular operator (component means for the periodic steady velocity,
   the mean for the pressure), and so is the result. */
static int mg_solve(orc_ctx *X, int vel, const double *r_in, double *e, double tol,
                    int max_cycles, int *cycles, double *rel) {
  level_t *L = &X->lev[0];
  const size_t n = vel ? L->nvel : L->ncell;
  double *r = (double *)malloc(n * sizeof(double));
  double *res = (double *)malloc(n * sizeof(double));
  double *de = (double *)malloc(n * sizeof(double));
  if (!r || !res || !de) {
    free(r); free(res); free(de);
    return ORC_ENOMEM;
  }
  copyv(r, r_in, n);
  if (vel) {
    if (X->vel_singular) remove_vel_means(L, r);
  } else {
    remove_mean(r, n);
  }
  const double nr = sqrt(dotv(r, r, n));
  zerov(e, n);
  copyv(res, r, n);
  double q = (nr > 0.0) ? 1.0 : 0.0;
  int c = 0;
  while (q > tol && c < max_cycles) {
    if (vel) vcycle_vel(X, 0, res, de);
    else vcycle_p(X, 0, res, de);
    for (size_t i = 0; i < n; i++) e[i] += de[i];
    c++;
    if (vel) vel_residual(L, r, e, res);
    else p_residual(L, r, e, res);
    q = sqrt(dotv(res, res, n)) / nr;
  }
  if (vel) {
    if (X->vel_singular) remove_vel_means(L, e);
  } else {
    remove_mean(e, n);
  }
  free(r); free(res); free(de);
  *cycles = c;
  *rel = q;
  if (!isfinite(q)) return ORC_ENONFINITE;
  return (q <= tol) ? ORC_OK : ORC_ENOCONV;
}

/* ------------------------------------------------------------------------ */
/* preconditioners (Sec. "Preconditioners")                                                  */
/* ------------------------------------------------------------------------ */

static void div_all(const level_t *L, const double *u, double *out) {
  const grid_t *g = &L->g;
  for (int i2 = 0; i2 < g->n[2]; i2++)
    for (int i1 = 0; i1 < g->n[1]; i1++)
      for (int i0 = 0; i0 < g->n[0]; i0++) {
        int c[3] = {i0, i1, i2};
        out[lin3(g->n, i0, i1, i2)] = div_cell(L, u, c);
      }
}

static void grad_all(const level_t *L, const double *p, double *out) {
  const grid_t *g = &L->g;
  for (int k = 0; k < g->d; k++) {
    FOR_FACES(L, k, f) {
      FACE_IDX(f);
      size_t q = fidx(L, k, f);
      out[q] = is_wall_face(g, k, f) ? 0.0 : grad_face(L, p, k, f);
    }
  }
}

/* viscous part of the Schur complement approximation at cell i: 2 mu
   (eq. Schur_app_varDen_varVis), or gamma + 4/3 mu = 2 mu + (gamma - 2/3 mu)
   with bulk viscosity (eq. Schur_app_bulk) */
static double schur_visc(const level_t *L, size_t i) {
  return 2.0 * L->mu_c[i] + (L->lam_c ? L->lam_c[i] : 0.0);
}

/* x_p = -S~^{-1} c = theta L~_rho^{-1} c - 2 mu c  (eq. Schur_app_varDen_varVis;
   gamma + 4/3 mu in place of 2 mu with bulk viscosity, eq. Schur_app_bulk) */
static void neg_schur(orc_ctx *X, const double *cvec, double *xp) {
  level_t *L = &X->lev[0];
  size_t nc = L->ncell;
  if (X->p.theta != 0.0) {
    double *q = (double *)malloc(nc * sizeof(double));
    p_sub(X, cvec, q);
    for (size_t i = 0; i < nc; i++) xp[i] = X->p.theta * q[i] - schur_visc(L, i) * cvec[i];
    free(q);
  } else {
    for (size_t i = 0; i < nc; i++) xp[i] = -schur_visc(L, i) * cvec[i];
  }
}

/* z = P^{-1} b on the scaled system; b, z are [velocity | pressure] */
static void precond_scaled(orc_ctx *X, const double *b, double *z) {
  level_t *L = &X->lev[0];
  const size_t nv = L->nvel, nc = L->ncell;
  const double *bu = b, *bp = b + nv;
  double *zu = z, *zp = z + nv;
  double *cvec = (double *)malloc(nc * sizeof(double));
  double *tu = (double *)malloc(nv * sizeof(double));
  double *xs = (double *)malloc(nv * sizeof(double));
  switch (X->p.precond) {
  case ORC_P1: {
    /* x* = A~^{-1} b_u; c = -(D x* + b_p); q = L~^{-1} c;
       x_u = x* + rho^{-1} G q; x_p = S~^{-1} c = -theta q + 2 mu c */
    vel_sub(X, bu, xs);
    div_all(L, xs, cvec);
    for (size_t i = 0; i < nc; i++) cvec[i] = -(cvec[i] + bp[i]);
    double *q = (double *)malloc(nc * sizeof(double));
    p_sub(X, cvec, q);
    grad_all(L, q, tu);
    for (size_t i = 0; i < nv; i++) zu[i] = xs[i] + L->beta[i] * tu[i];
    for (size_t i = 0; i < nc; i++) zp[i] = -X->p.theta * q[i] + schur_visc(L, i) * cvec[i];
    free(q);
    break;
  }
  case ORC_P2: {
    /* x_u = A~^{-1} b_u; x_p = -S~^{-1} (D x_u + b_p) */
    vel_sub(X, bu, zu);
    div_all(L, zu, cvec);
    for (size_t i = 0; i < nc; i++) cvec[i] += bp[i];
    neg_schur(X, cvec, zp);
    break;
  }
  case ORC_P3: {
    /* x_p = -S~^{-1} b_p; x_u = A~^{-1} (b_u - G x_p) */
    neg_schur(X, bp, zp);
    grad_all(L, zp, tu);
    for (size_t i = 0; i < nv; i++) tu[i] = bu[i] - tu[i];
    vel_sub(X, tu, zu);
    break;
  }
  case ORC_P4: {
    vel_sub(X, bu, zu);
    neg_schur(X, bp, zp);
    break;
  }
  case ORC_P5: {
    /* x* = A~^{-1} b_u; x_p = -S~^{-1}(D x* + b_p);
       x_u = x* + A~^{-1}(b_u - G x_p - A x*)  (second solve from x*) */
    vel_sub(X, bu, xs);
    div_all(L, xs, cvec);
    for (size_t i = 0; i < nc; i++) cvec[i] += bp[i];
    neg_schur(X, cvec, zp);
    double *gx = (double *)malloc(nv * sizeof(double));
    grad_all(L, zp, gx);
    vel_residual(L, bu, xs, tu); /* b_u - A x* */
    for (size_t i = 0; i < nv; i++) tu[i] -= gx[i];
    vel_sub(X, tu, gx);
    for (size_t i = 0; i < nv; i++) zu[i] = xs[i] + gx[i];
    free(gx);
    break;
  }
  default:
    break;
  }
  /* keep the pressure mean (and the velocity means when the velocity
     operator is singular) at zero (Sec. "Krylov Solver") */
  remove_mean(zp, nc);
  if (X->vel_singular) remove_vel_means(L, zu);
  free(cvec); free(tu); free(xs);
}

static void apply_scaled(orc_ctx *X, const double *x, double *y) {
  level_t *L = &X->lev[0];
  apply_m(L, L->alpha, L->mu_c, L->mu_e, x, x + L->nvel, y, y + L->nvel);
}

static int vel_cycles_per_apply(const orc_ctx *X) {
  return X->p.precond == ORC_P5 ? 2 : 1;
}
static int p_cycles_per_apply(const orc_ctx *X) {
  if (X->p.precond == ORC_P1) return 1;
  return X->p.theta != 0.0 ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* GMRES(m) / FGMRES(m)                                                      */
/* ------------------------------------------------------------------------ */

/* Arnoldi step by modified Gram-Schmidt (Saad's MGS form of the Arnoldi
   process, the Krylov method the paper names in Sec. "Krylov Solver"): for
   i = 0..j in turn, h_i = (w, v_i) on the partly orthogonalised w, then
   w <- w - h_i v_i; the new subdiagonal entry is ||w|| measured on the
   final w.  Fills hcol[0..j]; returns ||w||; w is left orthogonalised. */
static double arnoldi_mgs(double **V, int j, double *w, size_t n, double *hcol) {
  for (int i = 0; i <= j; i++) {
    const double *vi = V[i];
    const double hi = dotv(w, vi, n);
    hcol[i] = hi;
    for (size_t t = 0; t < n; t++) w[t] -= hi * vi[t];
  }
  return sqrt(dotv(w, w, n));
}

/* r-hat = S (b - M' x) on the rescaled system: the true residual, in FP64
   or (extended) in __float128, then scaled by the diagonal scaling S when the
   context has one. */
static void true_residual(orc_ctx *X, const double *b, const double *x, double *r, double *t) {
  level_t *L = &X->lev[0];
  const size_t n = L->nvel + L->ncell;
  if (X->p.extended) {
    residual_quad(L, L->alpha, L->mu_c, L->mu_e, b, x, r);
  } else {
    apply_scaled(X, x, t);
    for (size_t i = 0; i < n; i++) r[i] = b[i] - t[i];
  }
  if (X->sdiag)
    for (size_t i = 0; i < n; i++) r[i] *= X->sdiag[i];
}

/* Solve the scaled system M' x = b by restarted GMRES: left-preconditioned
   (Sec. "Krylov Solver") or flexible (right-preconditioned, Saad).  Stopping (reading):
   the solve ends when the true residual ||b - M x|| <= tol ||b||; each restart
   cycle ends when the Givens residual estimate has dropped by the factor the
   true residual still lacks, or after m steps.
   With the diagonal scaling S the Krylov method runs on M-hat = S M' S for
   x-hat = S^{-1} x, right-hand side S b, with the preconditioner
   P-hat^{-1} = S^{-1} P'^{-1} S^{-1}; the iterate is kept as x = S x-hat. */
static int krylov_solve(orc_ctx *X, const double *b, double *x, double tol, int max_iter,
                        orc_stats *st) {
  level_t *L = &X->lev[0];
  const size_t n = L->nvel + L->ncell;
  const int m = X->p.restart;
  const int flexible = (X->p.krylov == ORC_FGMRES);
  const double *S = X->sdiag;
  orc_stats local;
  if (!st) st = &local;
  memset(st, 0, sizeof(*st));
  int rc = ORC_OK;
  double nb = 0.0;
  for (size_t i = 0; i < n; i++) {
    const double bi = S ? S[i] * b[i] : b[i];
    nb += bi * bi;
  }
  nb = sqrt(nb);
  if (nb == 0.0) {
    zerov(x, n);
    return ORC_OK;
  }
  double **V = (double **)calloc((size_t)m + 1, sizeof(double *));
  double **Z = flexible ? (double **)calloc((size_t)m, sizeof(double *)) : NULL;
  for (int i = 0; i <= m; i++) V[i] = (double *)malloc(n * sizeof(double));
  if (flexible)
    for (int i = 0; i < m; i++) Z[i] = (double *)malloc(n * sizeof(double));
  double *r = (double *)malloc(n * sizeof(double));
  double *w = (double *)malloc(n * sizeof(double));
  double *t = (double *)malloc(n * sizeof(double));
  double *t2 = (double *)malloc(n * sizeof(double));
  double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double)); /* H[i + j*(m+1)] */
  double *cs = (double *)calloc((size_t)m, sizeof(double));
  double *sn = (double *)calloc((size_t)m, sizeof(double));
  double *g = (double *)calloc((size_t)m + 1, sizeof(double));
  double *y = (double *)calloc((size_t)m, sizeof(double));
  int it = 0;
  for (;;) {
    true_residual(X, b, x, r, t);
    double rho = sqrt(dotv(r, r, n));
    st->rel_res_true = rho / nb;
    if (!isfinite(rho)) { rc = ORC_ENONFINITE; break; }
    if (rho <= tol * nb) { rc = ORC_OK; break; }
    if (it >= max_iter) { rc = ORC_ENOCONV; break; }
    st->restarts++;
    double beta;
    if (flexible) {
      beta = rho;
      for (size_t i = 0; i < n; i++) V[0][i] = r[i] / beta;
    } else {
      /* P-hat^{-1} r-hat = S^{-1} P'^{-1} (S^{-1} r-hat) */
      if (S)
        for (size_t i = 0; i < n; i++) r[i] /= S[i];
      precond_scaled(X, r, V[0]);
      if (S)
        for (size_t i = 0; i < n; i++) V[0][i] /= S[i];
      st->precond_applies++;
      beta = sqrt(dotv(V[0], V[0], n));
      if (!isfinite(beta)) { rc = ORC_ENONFINITE; break; }
      if (beta == 0.0) { rc = ORC_EBREAKDOWN; break; }
      for (size_t i = 0; i < n; i++) V[0][i] /= beta;
    }
    const double target = beta * tol * nb / rho;
    memset(H, 0, sizeof(double) * (size_t)(m + 1) * m);
    zerov(g, (size_t)m + 1);
    g[0] = beta;
    int jj = 0;
    for (int j = 0; j < m; j++) {
      if (flexible) {
        /* z = P'^{-1} S^{-1} v is stored; M-hat P-hat^{-1} v = S M' z */
        const double *vin = V[j];
        if (S) {
          for (size_t i = 0; i < n; i++) t2[i] = V[j][i] / S[i];
          vin = t2;
        }
        precond_scaled(X, vin, Z[j]);
        apply_scaled(X, Z[j], w);
        if (S)
          for (size_t i = 0; i < n; i++) w[i] *= S[i];
      } else {
        /* P-hat^{-1} M-hat v = S^{-1} P'^{-1} M' S v */
        const double *vin = V[j];
        if (S) {
          for (size_t i = 0; i < n; i++) t2[i] = S[i] * V[j][i];
          vin = t2;
        }
        apply_scaled(X, vin, t);
        precond_scaled(X, t, w);
        if (S)
          for (size_t i = 0; i < n; i++) w[i] /= S[i];
      }
      st->precond_applies++;
      it++;
      double *hc = H + (size_t)j * (m + 1);
      double hn = arnoldi_mgs(V, j, w, n, hc);
      hc[j + 1] = hn;
      /* previous rotations, then a new one that zeroes H[j+1][j] */
      for (int i = 0; i < j; i++) {
        double a = hc[i], bb = hc[i + 1];
        hc[i] = cs[i] * a + sn[i] * bb;
        hc[i + 1] = -sn[i] * a + cs[i] * bb;
      }
      double den = hypot(hc[j], hc[j + 1]);
      if (den == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
      else { cs[j] = hc[j] / den; sn[j] = hc[j + 1] / den; }
      hc[j] = den;
      hc[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      jj = j + 1;
      double est = fabs(g[j + 1]);
      st->rel_res_est = est / beta * (rho / nb);
      if (!isfinite(est)) break;
      if (hn == 0.0 || est <= target || it >= max_iter) break;
      for (size_t q = 0; q < n; q++) V[j + 1][q] = w[q] / hn;
    }
    /* back substitution H y = g and update x */
    for (int i = jj - 1; i >= 0; i--) {
      double sum = g[i];
      for (int k = i + 1; k < jj; k++) sum -= H[i + (size_t)k * (m + 1)] * y[k];
      double dg = H[i + (size_t)i * (m + 1)];
      y[i] = (dg != 0.0) ? sum / dg : 0.0;
    }
    if (flexible || !S) {
      for (int i = 0; i < jj; i++) {
        const double *vi = flexible ? Z[i] : V[i];
        for (size_t q = 0; q < n; q++) x[q] += y[i] * vi[q];
      }
    } else {
      /* x = S x-hat: x += S (V y) */
      zerov(t, n);
      for (int i = 0; i < jj; i++)
        for (size_t q = 0; q < n; q++) t[q] += y[i] * V[i][q];
      for (size_t q = 0; q < n; q++) x[q] += S[q] * t[q];
    }
  }
  st->iters = it;
  st->scalar_vcycles = st->precond_applies * X->p.vcycles *
                       (L->g.d * vel_cycles_per_apply(X) + p_cycles_per_apply(X));
  for (int i = 0; i <= m; i++) free(V[i]);
  free(V);
  if (flexible) {
    for (int i = 0; i < m; i++) free(Z[i]);
    free(Z);
  }
  free(r); free(w); free(t); free(t2); free(H); free(cs); free(sn); free(g); free(y);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* setup (Sec. "Staggered-grid Discretization" coefficients, Sec. "Rescaling of the Linear System" rescaling, Appendix C coarsening)  */
/* ------------------------------------------------------------------------ */

static int level_alloc(level_t *L, int work, int bulk) {
  level_layout(L);
  if (bulk) {
    L->lam_c = (double *)calloc(L->ncell, sizeof(double));
    if (!L->lam_c) return ORC_ENOMEM;
  }
  L->alpha = (double *)calloc(L->nvel, sizeof(double));
  L->beta = (double *)calloc(L->nvel, sizeof(double));
  L->mu_c = (double *)calloc(L->ncell, sizeof(double));
  L->mu_e = (double *)calloc(L->nedge, sizeof(double));
  if (!L->alpha || !L->beta || !L->mu_c || !L->mu_e) return ORC_ENOMEM;
  if (work) {
    L->phi_u = (double *)calloc(L->nvel, sizeof(double));
    L->rhs_u = (double *)calloc(L->nvel, sizeof(double));
    L->res_u = (double *)calloc(L->nvel, sizeof(double));
    L->phi_p = (double *)calloc(L->ncell, sizeof(double));
    L->rhs_p = (double *)calloc(L->ncell, sizeof(double));
    L->res_p = (double *)calloc(L->ncell, sizeof(double));
    if (!L->phi_u || !L->rhs_u || !L->res_u || !L->phi_p || !L->rhs_p || !L->res_p)
      return ORC_ENOMEM;
  }
  return ORC_OK;
}

static void level_free(level_t *L) {
  free(L->alpha); free(L->beta); free(L->mu_c); free(L->mu_e); free(L->lam_c);
  free(L->phi_u); free(L->rhs_u); free(L->res_u);
  free(L->phi_p); free(L->rhs_p); free(L->res_p);
  memset(L, 0, sizeof(*L));
}

/* fine coefficients: rho_f = mean of the two cells sharing the face
   (alpha = theta rho_f, beta = 1/rho_f); edge mu = arithmetic (or harmonic)
   mean of the existing neighbouring cells (4 in the interior, 2 on a wall,
   1 in a corner: reading for walls), or the caller's values. */
static void fine_coefficients(const orc_ctx *X, level_t *L, const double *rho,
                              const double *mu, const double *edges_given) {
  const grid_t *g = &L->g;
  for (int k = 0; k < g->d; k++) {
    FOR_FACES(L, k, f) {
      FACE_IDX(f);
      size_t q = fidx(L, k, f);
      if (is_wall_face(g, k, f)) { L->alpha[q] = 0.0; L->beta[q] = 0.0; continue; }
      int cl[3] = {f[0], f[1], f[2]};
      cl[k] -= 1;
      double rf = 0.5 * (rho[cidx(g, f)] + rho[cidx(g, cl)]);
      L->alpha[q] = X->p.theta * rf;
      L->beta[q] = 1.0 / rf;
    }
  }
  memcpy(L->mu_c, mu, L->ncell * sizeof(double));
  if (X->p.edge_avg == ORC_EDGE_GIVEN) {
    memcpy(L->mu_e, edges_given, L->nedge * sizeof(double));
    return;
  }
  for (int m = 0; m < 3; m++) {
    if (L->ecnt[m] == 0) continue;
    int k = (m == 0) ? 1 : 0;
    int l = (m == 2) ? 1 : 2;
    int dm[3];
    edge_dims(g, m, dm);
    for (int i2 = 0; i2 < dm[2]; i2++)
      for (int i1 = 0; i1 < dm[1]; i1++)
        for (int i0 = 0; i0 < dm[0]; i0++) {
          int e[3] = {i0, i1, i2};
          double s = 0.0, sinv = 0.0;
          int cnt = 0;
          for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
              int c[3] = {e[0], e[1], e[2]};
              c[k] -= a;
              c[l] -= b;
              if (g->ns[k] && (c[k] < 0 || c[k] >= g->n[k])) continue;
              if (g->ns[l] && (c[l] < 0 || c[l] >= g->n[l])) continue;
              double v = mu[cidx(g, c)];
              s += v;
              sinv += 1.0 / v;
              cnt++;
            }
          double val = (X->p.edge_avg == ORC_EDGE_HARMONIC) ? (double)cnt / sinv : s / (double)cnt;
          L->mu_e[L->eoff[m] + lin3(dm, i0, i1, i2)] = val;
        }
  }
}

/* coarse coefficients (Appendix C): face coefficients = mean of the
   overlaid fine faces; cell mu = mean of the 2^d fine cells; node mu (2D) =
   injection; edge mu (3D) = mean of the two overlaid fine edges.  The
   pressure coefficient beta is coarsened like alpha (reading). */
static void coarsen_coefficients(const level_t *F, level_t *C) {
  const grid_t *g = &C->g;
  const int d = g->d;
  for (int k = 0; k < d; k++) {
    int tax[2] = {0, 0}, nt = 0;
    for (int b = 0; b < d; b++) if (b != k) tax[nt++] = b;
    FOR_FACES(C, k, F_) {
      FACE_IDX(F_);
      size_t q = fidx(C, k, F_);
      if (is_wall_face(g, k, F_)) { C->alpha[q] = 0.0; C->beta[q] = 0.0; continue; }
      double sa = 0.0, sb = 0.0;
      int cnt = 0;
      for (int o1 = 0; o1 < 2; o1++)
        for (int o0 = 0; o0 < (nt == 2 ? 2 : 1); o0++) {
          int ff[3] = {2 * F_[0], 2 * F_[1], d == 3 ? 2 * F_[2] : 0};
          ff[tax[0]] += o1;
          if (nt == 2) ff[tax[1]] += o0;
          size_t fq = fidx(F, k, ff);
          sa += F->alpha[fq];
          sb += F->beta[fq];
          cnt++;
        }
      C->alpha[q] = sa / cnt;
      C->beta[q] = sb / cnt;
    }
  }
  for (int i2 = 0; i2 < g->n[2]; i2++)
    for (int i1 = 0; i1 < g->n[1]; i1++)
      for (int i0 = 0; i0 < g->n[0]; i0++) {
        double s = 0.0;
        for (int o2 = 0; o2 < (d == 3 ? 2 : 1); o2++)
          for (int o1 = 0; o1 < 2; o1++)
            for (int o0 = 0; o0 < 2; o0++)
              s += F->mu_c[lin3(F->g.n, 2 * i0 + o0, 2 * i1 + o1, d == 3 ? 2 * i2 + o2 : 0)];
        C->mu_c[lin3(g->n, i0, i1, i2)] = s / (double)(1 << d);
      }
  /* bulk coefficient: mean of the 2^d fine cells, like the cell viscosity */
  if (C->lam_c)
    for (int i2 = 0; i2 < g->n[2]; i2++)
      for (int i1 = 0; i1 < g->n[1]; i1++)
        for (int i0 = 0; i0 < g->n[0]; i0++) {
          double s = 0.0;
          for (int o2 = 0; o2 < (d == 3 ? 2 : 1); o2++)
            for (int o1 = 0; o1 < 2; o1++)
              for (int o0 = 0; o0 < 2; o0++)
                s += F->lam_c[lin3(F->g.n, 2 * i0 + o0, 2 * i1 + o1, d == 3 ? 2 * i2 + o2 : 0)];
          C->lam_c[lin3(g->n, i0, i1, i2)] = s / (double)(1 << d);
        }
  for (int m = 0; m < 3; m++) {
    if (C->ecnt[m] == 0) continue;
    int dm[3], fdm[3];
    edge_dims(g, m, dm);
    edge_dims(&F->g, m, fdm);
    for (int i2 = 0; i2 < dm[2]; i2++)
      for (int i1 = 0; i1 < dm[1]; i1++)
        for (int i0 = 0; i0 < dm[0]; i0++) {
          int e[3] = {2 * i0, 2 * i1, d == 3 ? 2 * i2 : 0};
          double v;
          if (m < d) {
            int e2[3] = {e[0], e[1], e[2]};
            e2[m] += 1;
            v = 0.5 * (F->mu_e[F->eoff[m] + lin3(fdm, e[0], e[1], e[2])] +
                       F->mu_e[F->eoff[m] + lin3(fdm, e2[0], e2[1], e2[2])]);
          } else {
            v = F->mu_e[F->eoff[m] + lin3(fdm, e[0], e[1], e[2])];
          }
          C->mu_e[C->eoff[m] + lin3(dm, i0, i1, i2)] = v;
        }
  }
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_create(const orc_params *p, const double *rho, const double *mu,
               const double *edges_given, const double *gamma, orc_ctx **out) {
  if (!p || !out || !rho || !mu) return ORC_EINVAL;
  *out = NULL;
  if (p->dim != 2 && p->dim != 3) return ORC_EINVAL;
  if (!(p->h > 0.0) || !(p->theta >= 0.0)) return ORC_EINVAL;
  if (p->precond < ORC_P1 || p->precond > ORC_P5) return ORC_EINVAL;
  if (p->restart < 1 || p->restart > 60 || p->vcycles < 1) return ORC_EINVAL;
  if (p->nu_pre < 0 || p->nu_post < 0 || p->nu_coarse < 1) return ORC_EINVAL;
  if (p->edge_avg == ORC_EDGE_GIVEN && !edges_given) return ORC_EINVAL;
  grid_t g;
  memset(&g, 0, sizeof(g));
  g.d = p->dim;
  g.h = p->h;
  int nmin = 1 << 30;
  for (int a = 0; a < 3; a++) {
    if (a < g.d) {
      if (p->n[a] < 2 || p->bc[a] < ORC_PERIODIC || p->bc[a] > ORC_FREESLIP_NOSLIP)
        return ORC_EINVAL;
      g.n[a] = p->n[a];
      g.ns[a] = (p->bc[a] != ORC_PERIODIC);
      g.fs[a][0] = (p->bc[a] == ORC_FREESLIP || p->bc[a] == ORC_FREESLIP_NOSLIP);
      g.fs[a][1] = (p->bc[a] == ORC_FREESLIP || p->bc[a] == ORC_NOSLIP_FREESLIP);
      if (g.n[a] < nmin) nmin = g.n[a];
    } else {
      g.n[a] = 1;
      g.ns[a] = 0;
      g.fs[a][0] = g.fs[a][1] = 0;
    }
  }
  /* the smallest axis must be a power of two >= 2; every axis must halve
     exactly until the smallest one has two cells (Appendix C) */
  int nlev = 1;
  while ((nmin >> (nlev - 1)) > 2) nlev++;
  if ((nmin >> (nlev - 1)) != 2 || (2 << (nlev - 1)) != nmin) return ORC_EINVAL;
  for (int a = 0; a < g.d; a++) {
    if (g.n[a] % (1 << (nlev - 1)) != 0) return ORC_EINVAL;
    /* multicolour Gauss-Seidel needs an even count around a periodic axis on
       every level (else two neighbours across the wrap share a colour) */
    if (!g.ns[a] && ((g.n[a] >> (nlev - 1)) & 1)) return ORC_EINVAL;
  }

  orc_ctx *X = (orc_ctx *)calloc(1, sizeof(orc_ctx));
  if (!X) return ORC_ENOMEM;
  X->p = *p;
  X->nlev = nlev;
  X->raw.g = g;
  const int bulk = gamma != NULL;
  if (level_alloc(&X->raw, 0, bulk) != ORC_OK) { orc_destroy(X); return ORC_ENOMEM; }
  for (size_t i = 0; i < X->raw.ncell; i++) {
    if (!(rho[i] > 0.0) || !(mu[i] >= 0.0) || !isfinite(rho[i]) || !isfinite(mu[i])) {
      orc_destroy(X);
      return ORC_EINVAL;
    }
    if (bulk && (!(gamma[i] >= 0.0) || !isfinite(gamma[i]))) {
      orc_destroy(X);
      return ORC_EINVAL;
    }
  }
  fine_coefficients(X, &X->raw, rho, mu, edges_given);
  /* stress with bulk viscosity (Sec. "Preconditioners"): the (div u) I coefficient is
     gamma - 2/3 mu per cell */
  if (bulk)
    for (size_t i = 0; i < X->raw.ncell; i++) X->raw.lam_c[i] = gamma[i] - 2.0 / 3.0 * mu[i];
  /* rescale factor c = h / mu_ref, mu_ref = geometric mean of the positive
     cell viscosities (Sec. "Rescaling of the Linear System", reading of "typical magnitude") */
  if (p->rescale_c > 0.0) {
    X->c = p->rescale_c;
  } else {
    double sl = 0.0;
    size_t cnt = 0;
    for (size_t i = 0; i < X->raw.ncell; i++)
      if (mu[i] > 0.0) { sl += log(mu[i]); cnt++; }
    X->c = cnt ? g.h / exp(sl / (double)cnt) : 1.0;
  }
  /* velocity null space at theta = 0: component k is constant-invariant when
     its own axis is periodic and no axis has no-slip walls (free-slip walls
     only fix the normal component) */
  X->vel_singular = 0;
  if (p->theta == 0.0) {
    int noslip = 0;
    for (int a = 0; a < g.d; a++) noslip |= (g.ns[a] && (!g.fs[a][0] || !g.fs[a][1]));
    for (int k = 0; k < g.d; k++)
      if (!g.ns[k] && !noslip) X->vel_singular |= 1 << k;
  }
  g.sing = X->vel_singular;
  X->raw.g.sing = g.sing;

  X->lev = (level_t *)calloc((size_t)nlev, sizeof(level_t));
  if (!X->lev) { orc_destroy(X); return ORC_ENOMEM; }
  for (int l = 0; l < nlev; l++) {
    grid_t gl = g;
    for (int a = 0; a < g.d; a++) gl.n[a] = g.n[a] >> l;
    gl.h = g.h * (double)(1 << l);
    X->lev[l].g = gl;
    if (level_alloc(&X->lev[l], 1, bulk) != ORC_OK) { orc_destroy(X); return ORC_ENOMEM; }
  }
  /* scaled fine level: alpha' = c alpha, mu' = c mu, beta' = beta / c */
  level_t *L0 = &X->lev[0];
  for (size_t i = 0; i < L0->nvel; i++) {
    L0->alpha[i] = X->c * X->raw.alpha[i];
    L0->beta[i] = X->raw.beta[i] / X->c;
  }
  for (size_t i = 0; i < L0->ncell; i++) L0->mu_c[i] = X->c * X->raw.mu_c[i];
  for (size_t i = 0; i < L0->nedge; i++) L0->mu_e[i] = X->c * X->raw.mu_e[i];
  if (bulk)
    for (size_t i = 0; i < L0->ncell; i++) L0->lam_c[i] = X->c * X->raw.lam_c[i];
  for (int l = 1; l < nlev; l++) coarsen_coefficients(&X->lev[l - 1], &X->lev[l]);
  /* diagonal scaling (Sec. "Rescaling of the Linear System": with a very
     broad range of viscosities velocity and pressure are rescaled
     separately by diagonal matrices; the formulation the paper points to is
     not given, reading): S = diag(S_u, S_p) with S_u = diag(A')^{-1/2} on
     the interior faces and S_p = sqrt(2 mu'_cell [+ lam'_cell]), the root of
     the viscous coefficient of the Schur approximation, so that S M' S has a
     unit velocity diagonal and a pressure block whose approximate Schur
     complement is minus the identity.  Wall faces take 1. */
  if (p->scaling == ORC_SCALE_DIAGONAL) {
    const size_t nv = L0->nvel, nc = L0->ncell;
    X->sdiag = (double *)malloc((nv + nc) * sizeof(double));
    if (!X->sdiag) { orc_destroy(X); return ORC_ENOMEM; }
    for (int k = 0; k < g.d; k++) {
      FOR_FACES(L0, k, f) {
        FACE_IDX(f);
        const size_t q = fidx(L0, k, f);
        X->sdiag[q] = is_wall_face(&L0->g, k, f)
                          ? 1.0
                          : 1.0 / sqrt(a_diag(L0, L0->alpha, L0->mu_c, L0->mu_e, k, f));
      }
    }
    for (size_t i = 0; i < nc; i++) {
      const double sig = schur_visc(L0, i);
      if (!(sig > 0.0)) { orc_destroy(X); return ORC_EINVAL; }
      X->sdiag[nv + i] = sqrt(sig);
    }
  } else if (p->scaling != ORC_SCALE_UNIFORM) {
    orc_destroy(X);
    return ORC_EINVAL;
  }
  if (p->extended != 0 && p->extended != 1) { orc_destroy(X); return ORC_EINVAL; }
  *out = X;
  return ORC_OK;
}

void orc_destroy(orc_ctx *X) {
  if (!X) return;
  level_free(&X->raw);
  if (X->lev)
    for (int l = 0; l < X->nlev; l++) level_free(&X->lev[l]);
  free(X->lev);
  free(X->given_edges);
  free(X->sdiag);
  free(X);
}

size_t orc_nvel(const orc_ctx *X) { return X->raw.nvel; }
size_t orc_ncell(const orc_ctx *X) { return X->raw.ncell; }
size_t orc_nedge(const orc_ctx *X) { return X->raw.nedge; }
int orc_nlevels(const orc_ctx *X) { return X->nlev; }
double orc_rescale(const orc_ctx *X) { return X->c; }

int orc_apply(orc_ctx *X, const double *xu, const double *xp, double *yu, double *yp) {
  if (!X || !xu || !xp || !yu || !yp) return ORC_EINVAL;
  apply_m(&X->raw, X->raw.alpha, X->raw.mu_c, X->raw.mu_e, xu, xp, yu, yp);
  return ORC_OK;
}

int orc_residual(orc_ctx *X, const double *bu, const double *bp, const double *xu,
                 const double *xp, double *ru, double *rp, int extended) {
  if (!X || !bu || !bp || !xu || !xp || !ru || !rp) return ORC_EINVAL;
  level_t *L = &X->raw;
  const size_t nv = L->nvel, nc = L->ncell, n = nv + nc;
  double *b = (double *)malloc(n * sizeof(double));
  double *x = (double *)malloc(n * sizeof(double));
  double *r = (double *)malloc(n * sizeof(double));
  if (!b || !x || !r) { free(b); free(x); free(r); return ORC_ENOMEM; }
  memcpy(b, bu, nv * sizeof(double));
  memcpy(b + nv, bp, nc * sizeof(double));
  memcpy(x, xu, nv * sizeof(double));
  memcpy(x + nv, xp, nc * sizeof(double));
  if (extended) {
    residual_quad(L, L->alpha, L->mu_c, L->mu_e, b, x, r);
  } else {
    apply_m(L, L->alpha, L->mu_c, L->mu_e, x, x + nv, r, r + nv);
    for (size_t i = 0; i < n; i++) r[i] = b[i] - r[i];
    for (int k = 0; k < L->g.d; k++) {
      FOR_FACES(L, k, f) {
        FACE_IDX(f);
        if (is_wall_face(&L->g, k, f)) r[fidx(L, k, f)] = 0.0;
      }
    }
  }
  memcpy(ru, r, nv * sizeof(double));
  memcpy(rp, r + nv, nc * sizeof(double));
  free(b); free(x); free(r);
  return ORC_OK;
}

int orc_diag_scaling(orc_ctx *X, double *s) {
  if (!X || !s || !X->sdiag) return ORC_EINVAL;
  memcpy(s, X->sdiag, (X->lev[0].nvel + X->lev[0].ncell) * sizeof(double));
  return ORC_OK;
}

int orc_boundary_rhs(orc_ctx *X, const double *un, const double *ut, double *cu, double *cp) {
  if (!X || !un || !ut || !cu || !cp) return ORC_EINVAL;
  level_t *L = &X->raw;
  double *zu = (double *)calloc(L->nvel, sizeof(double));
  double *zp = (double *)calloc(L->ncell, sizeof(double));
  if (!zu || !zp) { free(zu); free(zp); return ORC_ENOMEM; }
  /* M applied to the field that is zero inside and carries the prescribed
     values on the walls: the boundary terms of the affine operator */
  L->bd_un = un;
  L->bd_ut = ut;
  apply_m(L, L->alpha, L->mu_c, L->mu_e, zu, zp, cu, cp);
  L->bd_un = NULL;
  L->bd_ut = NULL;
  free(zu); free(zp);
  return ORC_OK;
}

int orc_precond(orc_ctx *X, const double *bu, const double *bp, double *zu, double *zp) {
  if (!X || !bu || !bp || !zu || !zp) return ORC_EINVAL;
  const size_t nv = X->raw.nvel, nc = X->raw.ncell;
  double *b = (double *)malloc((nv + nc) * sizeof(double));
  double *z = (double *)malloc((nv + nc) * sizeof(double));
  for (size_t i = 0; i < nv; i++) b[i] = X->c * bu[i];
  memcpy(b + nv, bp, nc * sizeof(double));
  precond_scaled(X, b, z);
  memcpy(zu, z, nv * sizeof(double));
  for (size_t i = 0; i < nc; i++) zp[i] = z[nv + i] / X->c;
  free(b); free(z);
  return ORC_OK;
}

int orc_vel_subsolve(orc_ctx *X, const double *r, double *e) {
  if (!X || !r || !e) return ORC_EINVAL;
  size_t nv = X->raw.nvel;
  double *t = (double *)malloc(nv * sizeof(double));
  for (size_t i = 0; i < nv; i++) t[i] = X->c * r[i];
  vel_sub(X, t, e);
  free(t);
  return ORC_OK;
}

int orc_p_subsolve(orc_ctx *X, const double *r, double *e) {
  if (!X || !r || !e) return ORC_EINVAL;
  p_sub(X, r, e);
  for (size_t i = 0; i < X->raw.ncell; i++) e[i] /= X->c;
  return ORC_OK;
}

int orc_vel_mg_solve(orc_ctx *X, const double *r, double *e, double tol, int max_cycles,
                     int *cycles, double *rel_res) {
  if (!X || !r || !e || !cycles || !rel_res || !(tol > 0.0) || max_cycles < 0) return ORC_EINVAL;
  const size_t nv = X->raw.nvel;
  double *t = (double *)malloc(nv * sizeof(double));
  if (!t) return ORC_ENOMEM;
  for (size_t i = 0; i < nv; i++) t[i] = X->c * r[i];
  const int rc = mg_solve(X, 1, t, e, tol, max_cycles, cycles, rel_res);
  free(t);
  return rc;
}

int orc_p_mg_solve(orc_ctx *X, const double *r, double *e, double tol, int max_cycles,
                   int *cycles, double *rel_res) {
  if (!X || !r || !e || !cycles || !rel_res || !(tol > 0.0) || max_cycles < 0) return ORC_EINVAL;
  const int rc = mg_solve(X, 0, r, e, tol, max_cycles, cycles, rel_res);
  for (size_t i = 0; i < X->raw.ncell; i++) e[i] /= X->c;
  return rc;
}

int orc_vel_sweep(orc_ctx *X, const double *rhs, double *phi) {
  if (!X || !rhs || !phi) return ORC_EINVAL;
  vel_sweep(&X->raw, X->raw.alpha, X->raw.mu_c, X->raw.mu_e, rhs, phi);
  return ORC_OK;
}

int orc_p_sweep(orc_ctx *X, const double *rhs, double *phi) {
  if (!X || !rhs || !phi) return ORC_EINVAL;
  p_sweep(&X->raw, X->raw.beta, rhs, phi);
  return ORC_OK;
}

int orc_level_dims(orc_ctx *X, int level, int n_out[3]) {
  if (!X || level < 0 || level >= X->nlev) return ORC_EINVAL;
  for (int a = 0; a < 3; a++) n_out[a] = X->lev[level].g.n[a];
  return ORC_OK;
}

int orc_level_coef(orc_ctx *X, int level, int which, double *out, size_t cap) {
  if (!X || level < 0 || level >= X->nlev || !out) return ORC_EINVAL;
  level_t *L = &X->lev[level];
  const double *src;
  size_t n;
  switch (which) {
  case 0: src = L->alpha; n = L->nvel; break;
  case 1: src = L->beta; n = L->nvel; break;
  case 2: src = L->mu_c; n = L->ncell; break;
  case 3: src = L->mu_e; n = L->nedge; break;
  case 4: src = L->lam_c; n = L->ncell; if (!src) return ORC_EINVAL; break;
  default: return ORC_EINVAL;
  }
  if (cap < n) return ORC_EINVAL;
  memcpy(out, src, n * sizeof(double));
  return ORC_OK;
}

int orc_level_sizes(orc_ctx *X, int level, size_t *nvel, size_t *ncell) {
  if (!X || level < 0 || level >= X->nlev) return ORC_EINVAL;
  if (nvel) *nvel = X->lev[level].nvel;
  if (ncell) *ncell = X->lev[level].ncell;
  return ORC_OK;
}

int orc_restrict_faces(orc_ctx *X, int level, const double *rf, double *rc) {
  if (!X || !rf || !rc || level < 0 || level + 1 >= X->nlev) return ORC_EINVAL;
  restrict_faces(&X->lev[level], &X->lev[level + 1], rf, rc);
  return ORC_OK;
}

int orc_prolong_add_faces(orc_ctx *X, int level, const double *ec, double *phif) {
  if (!X || !ec || !phif || level < 0 || level + 1 >= X->nlev) return ORC_EINVAL;
  prolong_add_faces(&X->lev[level + 1], &X->lev[level], ec, phif);
  return ORC_OK;
}

int orc_restrict_cells(orc_ctx *X, int level, const double *rf, double *rc) {
  if (!X || !rf || !rc || level < 0 || level + 1 >= X->nlev) return ORC_EINVAL;
  restrict_cells(&X->lev[level], &X->lev[level + 1], rf, rc);
  return ORC_OK;
}

int orc_prolong_add_cells(orc_ctx *X, int level, const double *ec, double *pf) {
  if (!X || !ec || !pf || level < 0 || level + 1 >= X->nlev) return ORC_EINVAL;
  prolong_add_cells(&X->lev[level + 1], &X->lev[level], ec, pf);
  return ORC_OK;
}

/* mean-compatibility of the right-hand side with the null space (Sec. "Krylov Solver") */
static int rhs_compatible(const orc_ctx *X, const double *bu, const double *bp) {
  const level_t *L = &X->raw;
  double s = 0.0, s2 = 0.0;
  for (size_t i = 0; i < L->ncell; i++) { s += bp[i]; s2 += bp[i] * bp[i]; }
  double su2 = 0.0;
  for (size_t i = 0; i < L->nvel; i++) su2 += bu[i] * bu[i];
  double scale = sqrt(s2 + su2) + 1e-300;
  if (fabs(s) > 1e-10 * scale * sqrt((double)L->ncell)) return 0;
  if (X->vel_singular) {
    for (int k = 0; k < L->g.d; k++) {
      if (!((X->vel_singular >> k) & 1)) continue;
      double sk = 0.0;
      for (size_t i = 0; i < L->fcnt[k]; i++) sk += bu[L->foff[k] + i];
      if (fabs(sk) > 1e-10 * scale * sqrt((double)L->fcnt[k])) return 0;
    }
  }
  return 1;
}

int orc_solve(orc_ctx *X, const double *bu, const double *bp, double *xu, double *xp,
              double tol, int max_iter, int use_x0, orc_stats *st) {
  if (!X || !bu || !bp || !xu || !xp || !(tol > 0.0) || max_iter < 0) return ORC_EINVAL;
  if (!rhs_compatible(X, bu, bp)) return ORC_EINCOMPAT;
  const size_t nv = X->raw.nvel, nc = X->raw.ncell, n = nv + nc;
  double *b = (double *)malloc(n * sizeof(double));
  double *x = (double *)malloc(n * sizeof(double));
  /* rescaled system (eq. Stokes_rescaled): [c A, G; -D, 0][x_u; c x_p] = [c b_u; b_p] */
  for (size_t i = 0; i < nv; i++) b[i] = X->c * bu[i];
  memcpy(b + nv, bp, nc * sizeof(double));
  if (use_x0) {
    memcpy(x, xu, nv * sizeof(double));
    for (size_t i = 0; i < nc; i++) x[nv + i] = X->c * xp[i];
  } else {
    zerov(x, n);
  }
  int rc = krylov_solve(X, b, x, tol, max_iter, st);
  memcpy(xu, x, nv * sizeof(double));
  for (size_t i = 0; i < nc; i++) xp[i] = x[nv + i] / X->c;
  remove_mean(xp, nc);
  if (X->vel_singular) remove_vel_means(&X->raw, xu);
  free(b); free(x);
  return rc;
}

/* Gradient of L(x(mu, rho)) given the forward solution x and the adjoint
   lambda (M lambda = dL/dx; M is symmetric, Sec. "Preconditioners").  With the symmetric form
   -L_mu = B^T W B (B: cell normal rates and edge shear rates; W: 2 mu_cell and
   w_e mu_edge with w_e = 1/2 on no-slip wall edges, 1 elsewhere):
     dL/dmu_cell = -2 sum_k (D^k lambda_k)(D^k x_k),
     dL/dmu_edge = -w_e gamma_e(lambda) gamma_e(x),
     dL/drho_cell = -theta sum_{faces of the cell} 1/2 lambda_f x_f.
   With bulk viscosity W also holds lam = gamma - 2/3 mu on the cell
   divergences, so dL/dlam = -(D lambda)(D x) per cell; it is dL/dgamma, and
   -2/3 of it is added to dL/dmu_cell.
   When the edges are derived from cells the chain through the averaging is
   added to dL/dmu_cell. */
int orc_grad(orc_ctx *X, const double *xu, const double *lu, double *dmu_cell,
             double *dmu_edge, double *drho, double *dgamma) {
  if (!X || !xu || !lu) return ORC_EINVAL;
  if (dgamma && !X->raw.lam_c) return ORC_EINVAL;
  const level_t *L = &X->raw;
  const grid_t *g = &L->g;
  double *de = (double *)calloc(L->nedge, sizeof(double));
  double *dc = (double *)calloc(L->ncell, sizeof(double));
  for (int i2 = 0; i2 < g->n[2]; i2++)
    for (int i1 = 0; i1 < g->n[1]; i1++)
      for (int i0 = 0; i0 < g->n[0]; i0++) {
        int c[3] = {i0, i1, i2};
        double s = 0.0;
        for (int k = 0; k < g->d; k++) s += normal_rate(L, lu, k, c) * normal_rate(L, xu, k, c);
        dc[lin3(g->n, i0, i1, i2)] = -2.0 * s;
        if (L->lam_c) {
          const double dlam = -div_cell(L, lu, c) * div_cell(L, xu, c);
          dc[lin3(g->n, i0, i1, i2)] -= 2.0 / 3.0 * dlam;
          if (dgamma) dgamma[lin3(g->n, i0, i1, i2)] = dlam;
        }
      }
  for (int m = 0; m < 3; m++) {
    if (L->ecnt[m] == 0) continue;
    int k = (m == 0) ? 1 : 0;
    int l = (m == 2) ? 1 : 2;
    int dm[3];
    edge_dims(g, m, dm);
    for (int i2 = 0; i2 < dm[2]; i2++)
      for (int i1 = 0; i1 < dm[1]; i1++)
        for (int i0 = 0; i0 < dm[0]; i0++) {
          int e[3] = {i0, i1, i2};
          int on_wall = (g->ns[k] && (e[k] == 0 || e[k] == g->n[k])) ||
                        (g->ns[l] && (e[l] == 0 || e[l] == g->n[l]));
          double w = on_wall ? 0.5 : 1.0;
          de[L->eoff[m] + lin3(dm, i0, i1, i2)] =
              -w * shear_rate(L, lu, k, l, e) * shear_rate(L, xu, k, l, e);
        }
  }
  if (drho) {
    for (size_t i = 0; i < L->ncell; i++) drho[i] = 0.0;
    for (int k = 0; k < g->d; k++) {
      int dm[3];
      face_dims(g, k, dm);
      for (int i2 = 0; i2 < dm[2]; i2++)
        for (int i1 = 0; i1 < dm[1]; i1++)
          for (int i0 = 0; i0 < dm[0]; i0++) {
            int f[3] = {i0, i1, i2};
            if (is_wall_face(g, k, f)) continue;
            size_t q = fidx(L, k, f);
            double v = -X->p.theta * 0.5 * lu[q] * xu[q];
            int cl[3] = {f[0], f[1], f[2]};
            cl[k] -= 1;
            drho[cidx(g, f)] += v;
            drho[cidx(g, cl)] += v;
          }
    }
  }
  if (dmu_edge) memcpy(dmu_edge, de, L->nedge * sizeof(double));
  if (dmu_cell) {
    memcpy(dmu_cell, dc, L->ncell * sizeof(double));
    if (X->p.edge_avg != ORC_EDGE_GIVEN) {
      /* chain rule through the cell -> edge averaging */
      for (int m = 0; m < 3; m++) {
        if (L->ecnt[m] == 0) continue;
        int k = (m == 0) ? 1 : 0;
        int l = (m == 2) ? 1 : 2;
        int dm[3];
        edge_dims(g, m, dm);
        for (int i2 = 0; i2 < dm[2]; i2++)
          for (int i1 = 0; i1 < dm[1]; i1++)
            for (int i0 = 0; i0 < dm[0]; i0++) {
              int e[3] = {i0, i1, i2};
              size_t eq = L->eoff[m] + lin3(dm, i0, i1, i2);
              int cells[4][3], cnt = 0;
              for (int a = 0; a < 2; a++)
                for (int b = 0; b < 2; b++) {
                  int c[3] = {e[0], e[1], e[2]};
                  c[k] -= a;
                  c[l] -= b;
                  if (g->ns[k] && (c[k] < 0 || c[k] >= g->n[k])) continue;
                  if (g->ns[l] && (c[l] < 0 || c[l] >= g->n[l])) continue;
                  memcpy(cells[cnt++], c, sizeof(c));
                }
              for (int t = 0; t < cnt; t++) {
                size_t cq = cidx(g, cells[t]);
                double dmu_de;
                if (X->p.edge_avg == ORC_EDGE_HARMONIC) {
                  double me = L->mu_e[eq], mc = L->mu_c[cq];
                  dmu_de = me * me / ((double)cnt * mc * mc);
                } else {
                  dmu_de = 1.0 / (double)cnt;
                }
                dmu_cell[cq] += de[eq] * dmu_de;
              }
            }
      }
    }
  }
  free(de);
  free(dc);
  return ORC_OK;
}

int orc_adjoint(orc_ctx *X, const double *xu, const double *xp, const double *gu,
                const double *gp, double *lu, double *lp, double *dmu_cell,
                double *dmu_edge, double *drho, double *dgamma, double tol, int max_iter,
                orc_stats *st) {
  (void)xp;
  if (!X || !xu || !gu || !gp || !lu || !lp || !(tol > 0.0)) return ORC_EINVAL;
  if (dgamma && !X->raw.lam_c) return ORC_EINVAL;
  const size_t nv = X->raw.nvel, nc = X->raw.ncell, n = nv + nc;
  double *b = (double *)malloc(n * sizeof(double));
  double *x = (double *)calloc(n, sizeof(double));
  /* with M' = diag(c,1) M diag(1,1/c) symmetric,
     lambda = diag(c,1) M'^{-1} (g_u, g_p / c); g is first projected onto the
     mean-free space of the solution (adjoint of the zero-mean normalisation) */
  memcpy(b, gu, nv * sizeof(double));
  for (size_t i = 0; i < nc; i++) b[nv + i] = gp[i] / X->c;
  remove_mean(b + nv, nc);
  if (X->vel_singular) remove_vel_means(&X->raw, b);
  int rc = krylov_solve(X, b, x, tol, max_iter, st);
  for (size_t i = 0; i < nv; i++) lu[i] = X->c * x[i];
  memcpy(lp, x + nv, nc * sizeof(double));
  remove_mean(lp, nc);
  if (X->vel_singular) remove_vel_means(&X->raw, lu);
  free(b); free(x);
  int rg = orc_grad(X, xu, lu, dmu_cell, dmu_edge, drho, dgamma);
  return rc != ORC_OK ? rc : rg;
}
