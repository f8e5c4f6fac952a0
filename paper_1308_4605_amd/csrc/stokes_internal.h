// stokes_internal.h -- device geometry descriptor and kernel launch wrappers
// shared by the HIP kernels (stokes_kernels.hip) and the host driver
// (stokes_api.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace stk {

typedef long long i64;

// Geometry of one multigrid level on the staggered (MAC) grid.
//   cells: n[0] x n[1] x n[2] (n[2] = 1 in 2D), x fastest;
//   velocity component k: dims fd[k] = n + ns[k] e_k, offset foff[k] in the
//     concatenated velocity buffer;
//   edge family m (parallel to axis m): dims ed[m] = n + ns on the other axes,
//     offset eoff[m] in the concatenated edge buffer.
struct Geo {
  int d;
  int n[3];
  int ns[3];  // walls on this axis (no-slip or free-slip)
  int fs[3];  // free-slip ends of this axis: bit 0 low end, bit 1 high end
  int sing;   // bit k: velocity component k has a constant null space
  double h, ih;  // spacing and its reciprocal
  i64 ncell, nvel, nedge;
  i64 foff[3];
  int fd[3][3];
  i64 fcnt[3];
  i64 eoff[3];
  int ed[3][3];
  i64 ecnt[3];
  int xcd;  // stencil kernels: one band of rows per XCD
  // velocity storage order along x: 0 natural; 1 split by the parity of the
  // x index (even positions of a row first, then odd), so that the faces of
  // one Gauss-Seidel colour lie contiguously in every row
  int split;
  // velocity residual (3D, FP32 arrays): 0 one thread per cell; > 0 one
  // thread per column of this many cells along z, carrying the values two
  // planes share (FP64 residuals run by cells whatever its value)
  int col;
};

// bc[a]: STOKES_PERIODIC, STOKES_NOSLIP or STOKES_FREESLIP per axis
Geo make_geo(int d, const int n[3], const int bc[3], double h);

// ---- launch wrappers (all asynchronous on stream s) ----------------------

// velocity arrays between storage orders: out (order of gout) = in (order of
// gin), same grid; with sums (per-component sums from launch_vel_sums), the
// mean of each singular component is subtracted on the way
template <typename T>
void launch_vel_permute(const Geo &gin, const Geo &gout, const T *in, T *out, const double *sums,
                        hipStream_t s);

// coefficient setup (scaled by c): faces alpha = c*theta*rho_f, beta =
// (1/rho_f)/c; cells mu_c = c*mu; edges = c * mean/harmonic/given.
void launch_setup_faces(const Geo &g, const double *rho, double theta, double c, double *alpha,
                        double *beta, hipStream_t s);
void launch_setup_cells(const Geo &g, const double *mu, double c, double *muc, hipStream_t s);
void launch_setup_edges(const Geo &g, const double *mu, const double *given, int mode, double c,
                        double *mue, hipStream_t s);
void launch_coarsen(const Geo &gf, const Geo &gc, const double *af, const double *bf,
                    const double *mcf, const double *mef, double *ac, double *bc, double *mcc,
                    double *mec, hipStream_t s);
void launch_check_coefs(const double *rho, const double *mu, i64 n, int *flag, hipStream_t s);
// bulk viscosity: lam = c (gamma - 2/3 mu) and sig = c mu + lam / 2 per cell
void launch_setup_bulk(const double *gamma, const double *mu, double c, i64 n, double *lam,
                       double *sig, hipStream_t s);

// element-wise
template <typename TO, typename TI>
void launch_cast(const TI *in, TO *out, i64 n, hipStream_t s);
template <typename T>
void launch_fill(T *a, T v, i64 n, hipStream_t s);
// out = scale * in on a velocity buffer with wall faces forced to 0
void launch_pack_vel(const Geo &g, const double *in, double scale, double *out, hipStream_t s);
void launch_scale(const double *in, double scale, double *out, i64 n, hipStream_t s);
template <typename T>
void launch_axpy(T a, const T *x, T *y, i64 n, hipStream_t s);  // y += a x

// saddle operator on the fine level in FP64:
//   y_u = alpha u - L_mu u + G p, y_p = -D u            (b == nullptr)
//   y = b - M x                                         (b != nullptr)
// lam (may be null): bulk coefficient per cell, gamma - 2/3 mu (scaled)
template <typename TI>
void launch_apply_m(const Geo &g, const double *alpha, const double *muc, const double *mue,
                    const double *lam, const TI *xu, const TI *xp, const double *bu,
                    const double *bp, double *yu, double *yp, hipStream_t s);
// boundary terms of prescribed wall velocities: M applied to the wall-data
// field xu (normal values on wall faces, zero inside) with tangential wall
// values gw (edge layout) in the no-slip ghosts
// r = b - M x like launch_apply_m (FP64 input), every operation in
// double-double arithmetic and each entry rounded once to FP64
void launch_residual_dd(const Geo &g, const double *alpha, const double *muc, const double *mue,
                        const double *lam, const double *xu, const double *xp, const double *bu,
                        const double *bp, double *ru, double *rp, hipStream_t s);
// sd = the diagonal scaling of the unknowns [faces | cells]: 1/sqrt(diag A)
// on interior faces (1 on wall faces), sqrt(2 mu_cell + lam) on cells (*bad
// set to 1 where that is not positive); zero: an all-zero velocity array
void launch_diag_scaling(const Geo &g, const double *alpha, const double *muc, const double *mue,
                         const double *lam, const double *zero, double *sd, int *bad,
                         hipStream_t s);
// y = x * sd (inv = 0) or x / sd (inv = 1); y may equal x
void launch_mul_scaling(const double *x, const double *sd, int inv, i64 n, double *y,
                        hipStream_t s);
void launch_apply_m_walls(const Geo &g, const double *alpha, const double *muc,
                          const double *mue, const double *lam, const double *xu,
                          const double *xp, const double *gw, double *yu, double *yp,
                          hipStream_t s);
void launch_pack_walls(const Geo &g, const double *in, double scale, double *out, hipStream_t s);

// multigrid level kernels, T = float or double
// (lam: bulk coefficient per cell or null, as for launch_apply_m)
// first != 0: a pass of the first sweep from a zero iterate whose memory has
// not been cleared (allowed when gs_first_ok(g), i.e. every extent even so
// that the colouring holds across periodic wraps; the sweep writes every
// value, the velocity wall faces included, before any pass reads it)
bool gs_first_ok(const Geo &g);
template <typename T>
void launch_vel_gs(const Geo &g, int k, int colour, int first, const T *alpha, const T *muc,
                   const T *mue, const T *lam, const T *rhs, T *phi, hipStream_t s);
template <typename T>  // res = rhs - A phi - G p
void launch_vel_residual(const Geo &g, const T *alpha, const T *muc, const T *mue, const T *lam,
                         const T *rhs, const T *phi, const T *p, T *res, hipStream_t s);
template <typename T>
void launch_face_restrict(const Geo &gf, const Geo &gc, const T *rf, T *rc, hipStream_t s);
template <typename T>
void launch_face_prolong_add(const Geo &gc, const Geo &gf, const T *ec, T *phif, hipStream_t s);
template <typename T>  // first: as for launch_vel_gs
void launch_p_gs(const Geo &g, int colour, int first, const T *beta, const T *rhs, T *phi,
                 hipStream_t s);
template <typename T>
void launch_p_residual(const Geo &g, const T *beta, const T *rhs, const T *phi, T *res,
                       hipStream_t s);
template <typename T>
void launch_cell_restrict(const Geo &gf, const Geo &gc, const T *rf, T *rc, hipStream_t s);
template <typename T>
void launch_cell_prolong_add(const Geo &gc, const Geo &gf, const T *ec, T *pf, hipStream_t s);

// coarse tail of a V-cycle (levels l0..nlev-1) in one workgroup
constexpr int kTailMax = 8;
constexpr int kTailBlock = 1024;
constexpr i64 kTailCells = 512;  // largest level run inside the tail
template <typename T>
struct TailLevels {
  int nl;        // number of levels in the tail (the last is the coarsest)
  int singular;  // velocity: bit k set = remove component k's mean at the coarsest level
  int nu_pre, nu_post, nu_coarse;
  Geo g[kTailMax];
  const T *a[kTailMax], *b[kTailMax], *mc[kTailMax], *me[kTailMax];  // alpha, beta, mu_c, mu_e
  const T *lam[kTailMax];  // bulk coefficient per cell (null: none)
  T *phi[kTailMax], *rhs[kTailMax], *res[kTailMax];
  // levels lds0..nl-1 live in dynamic LDS: byte offsets of
  // {alpha or beta, mu_c, mu_e, phi, rhs, res, lam}; lds_bytes in total
  int lds0;
  unsigned lds_bytes;
  unsigned off[kTailMax][7];
  // vec0: the first level's phi, rhs and res live in LDS too (at off[0][3..5];
  // its coefficients stay in global memory); set for the column launches
  int vec0;
};
constexpr unsigned kTailLds = 60 * 1024;  // dynamic LDS budget of a tail launch
// fills lds0 / off / lds_bytes for the velocity (vel) or pressure tail;
// vec0: also place the first level's vectors in LDS (reserved first).
// Returns false when vec0 is asked for and not every level's vectors fit.
template <typename T>
bool tail_plan_lds(TailLevels<T> &L, bool vel, bool vec0 = false);
template <typename T>
void launch_tail_vel(const TailLevels<T> &L, hipStream_t s);
// The velocity tail from a zero iterate is a fixed linear map B of its
// right-hand side (nv = the first tail level's velocity count).  Column
// launch: workgroup j runs the tail on the unit vector e_j with all vectors
// in LDS (L planned with vec0) and stores the result as column j of the
// row-major nv x nv matrix B.  Apply: phi = B rhs, one wave per row, FP64
// accumulation.
template <typename T>
void launch_tail_vel_columns(const TailLevels<T> &L, T *B, int nv, hipStream_t s);
template <typename T>
void launch_tail_matvec(const T *B, int nv, const T *rhs, T *phi, hipStream_t s);
template <typename T>
void launch_tail_p(const TailLevels<T> &L, hipStream_t s);

// preconditioner glue (level 0, precision T)
template <typename T>  // out = sgn * (D u + bp)   (bp may be null)
void launch_div(const Geo &g, const T *u, const T *bp, T sgn, T *out, hipStream_t s);
template <typename T>  // out = b mu (sgn (D u + bp)): the divergence and a cellwise scaling
void launch_div_scaled(const Geo &g, const T *u, const T *bp, T sgn, const T *mu, T b, T *out,
                       hipStream_t s);
template <typename T>  // zu = xs + beta * G q
void launch_proj_update(const Geo &g, const T *xs, const T *beta, const T *q, T *zu, hipStream_t s);
template <typename T>  // out = bu - G p
void launch_grad_sub(const Geo &g, const T *bu, const T *p, T *out, hipStream_t s);
template <typename T>  // out = a*q + b*mu*c  (q may be null)
void launch_schur_combine(const T *q, const T *c, const T *mu, T a, T b, T *out, i64 n,
                          hipStream_t s);

// means (deterministic two-stage reductions; result stays on the device)
template <typename T>
void launch_sum(const T *a, i64 n, double *partials, double *out, hipStream_t s);
template <typename T>
void launch_sub_mean(T *a, i64 n, const double *sum, hipStream_t s);

// sums[k] = sum of velocity component k (any storage order)
template <typename T>
void launch_vel_sums(const Geo &g, const T *in, double *partials, double *sums, hipStream_t s);
// out = in minus each velocity component's mean (all axes periodic: every
// face is an unknown); out may alias in
template <typename T>
void launch_vel_remove_means(const Geo &g, const T *in, T *out, double *partials, double *sums,
                             hipStream_t s);

// Krylov (FP64)
constexpr int kRedBlocks = 2048;
// Arnoldi passes (classical Gram-Schmidt, the second pass lagged into the
// basis transform; see launch_dcgs_update):
//   h[i] = (w, v_i), i < nv
//   (with_norm: h[nv] = (w, w))
void launch_cgs_dots(const double *w, const double *const *v, int nv, i64 n, double *partials,
                     double *h, hipStream_t s, bool with_norm = false);
//   the explicit second pass when the lagged one would remove half or more
//   of a vector: out = (w - sum_i (h1_i + h2_i) v_i) * inv_nu (nv = 0: plain
//   scale), also cast to out32 when out32 != nullptr; nrm2 = (out, out) when
//   nrm2 != nullptr.  out may alias w.
void launch_cgs_next(const double *w, const double *const *v, const double *h1, const double *h2,
                     int nv, double inv_nu, i64 n, double *out, float *out32, double *partials,
                     double *nrm2, hipStream_t s);
// Arnoldi step with lagged reorthogonalisation (second pass of the
// two-pass form): the stored v[0..j] are once-orthogonalised vectors whose
// orthonormal basis is V = v T (T upper triangular, row-major, row stride
// ld, on the device); dots = {(w, v_l), l <= j; (w, w)} from
// launch_cgs_dots.  Writes vnext = (w - v T d) / nu with d = T^T dots (also
// as FP32 to out32 when given), coef_out = {d_0..d_j, nu} and
// red = {(vnext, v_l), l <= j; (vnext, vnext)}.  T (row-major, row stride
// ld) is read from the host array tm_host into the kernel arguments while
// j < 12, else from the device copy tm_dev, which must then hold it.
void launch_dcgs_update(const double *w, const double *const *v, int j, const double *dots,
                        const double *tm_host, const double *tm_dev, int ld, i64 n,
                        double *vnext, float *out32, double *coef_out, double *partials,
                        double *red, hipStream_t s);
// x += sum_i y_i z_i with z in precision TZ (y: host array, passed by value)
template <typename TZ>
void launch_update_x(double *x, const TZ *const *z, const double *y, int nz, i64 n,
                     hipStream_t s);
// out2 = {sum of log(mu) over mu > 0, count of mu > 0}
void launch_logsum(const double *mu, i64 n, double *partials, double *out2, hipStream_t s);
// nrm2 = (a, a)
void launch_norm2(const double *a, i64 n, double *partials, double *nrm2, hipStream_t s);

// gradient contraction (unscaled forward u and adjoint lambda)
// bulk != 0: also the bulk-coefficient terms (dgamma may be null)
void launch_grad_cells(const Geo &g, const double *u, const double *lam, double theta, int bulk,
                       double *dmu_cell, double *drho, double *dgamma, hipStream_t s);
void launch_grad_edges(const Geo &g, const double *u, const double *lam, double *dmu_edge,
                       hipStream_t s);
void launch_grad_chain(const Geo &g, const double *dmu_edge, const double *mue_raw,
                       const double *muc_raw, int mode, double *dmu_cell, hipStream_t s);

}  // namespace stk
