// stokes_kernels.hip -- gfx950 kernels of the variable-coefficient MAC Stokes
// solver (arXiv:1308.4605).  Every kernel is bandwidth bound: low-order
// stencils, transfers, pointwise glue and reductions.  No matrix cores: no
// step is a dense contraction.
//
// Conventions: cell-indexed launches cover the cells of a level; a thread at
// cell (i0,i1,i2) handles the face of component k whose index is the same
// triple (the face on the low side of the cell along k).  That visits every
// face with index < n[k] along k; the high wall faces (index n[k] on a wall
// axis) are written only with 0 (by the first smoothing sweep from an
// uncleared iterate), and the low wall faces (index 0) are skipped except
// for that same zero write.  All internal velocity vectors therefore hold 0
// on every wall face, which lets the stencils read wall values without
// branches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "stokes_internal.h"

namespace stk {

constexpr int kBlock = 256;

static inline unsigned blocks_for(i64 n) {
  i64 b = (n + kBlock - 1) / kBlock;
  return (unsigned)(b < 1 ? 1 : b);
}
static inline dim3 box_blocks(const Geo &g, int W) {
  if (g.xcd && (g.n[1] & 7) == 0)
    return dim3(8u * blocks_for((i64)(g.n[1] >> 3) * W), (unsigned)g.n[2]);
  return dim3(blocks_for((i64)g.n[1] * W), (unsigned)g.n[2]);
}

Geo make_geo(int d, const int n[3], const int bc[3], double h) {
  Geo g;
  g.d = d;
  g.h = h;
  g.ih = 1.0 / h;
  for (int a = 0; a < 3; a++) {
    g.n[a] = (a < d) ? n[a] : 1;
    g.ns[a] = (a < d) ? (bc[a] != 0) : 0;
    // free-slip ends: bit 0 the low end, bit 1 the high end
    const int b = (a < d) ? bc[a] : 0;
    g.fs[a] = (b == 2) ? 3 : (b == 3) ? 2 : (b == 4) ? 1 : 0;
  }
  g.sing = 0;
  g.ncell = (i64)g.n[0] * g.n[1] * g.n[2];
  g.xcd = 1;
  g.split = 0;
  g.col = 0;
  i64 off = 0;
  for (int k = 0; k < 3; k++) {
    for (int a = 0; a < 3; a++) g.fd[k][a] = g.n[a] + ((a == k && k < d) ? g.ns[a] : 0);
    g.foff[k] = off;
    g.fcnt[k] = (k < d) ? (i64)g.fd[k][0] * g.fd[k][1] * g.fd[k][2] : 0;
    off += g.fcnt[k];
  }
  g.nvel = off;
  off = 0;
  for (int m = 0; m < 3; m++) {
    for (int a = 0; a < 3; a++) g.ed[m][a] = g.n[a] + ((a != m && a < d) ? g.ns[a] : 0);
    g.eoff[m] = 0;
    g.ecnt[m] = 0;
  }
  for (int m = 2; m >= 0; m--) {  // storage order m = 2, 1, 0 (2D: m = 2)
    if (d == 2 && m != 2) continue;
    g.eoff[m] = off;
    g.ecnt[m] = (i64)g.ed[m][0] * g.ed[m][1] * g.ed[m][2];
    off += g.ecnt[m];
  }
  g.nedge = off;
  return g;
}

// ------------------------------------------------------------------------
// index helpers
// ------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Index arithmetic is 32-bit: stokes_create rejects grids whose face, cell
// or edge storage exceeds 2^31 - 1 entries.
// position of x index i in a velocity row of length L (Geo::split)
__device__ __forceinline__ int xpos(const Geo &g, int L, int i) {
  return g.split ? ((i & 1) ? ((L + 1) >> 1) + (i >> 1) : (i >> 1)) : i;
}
// x index handled by thread w of a row of n0 cells.  On split levels the
// row is cut into groups of G = min(64, largest power of two dividing n0)
// threads; the first half of a group takes the group's even cells and the
// second half its odd ones.  A wave's load from a split velocity array is
// then two contiguous runs, and its load from a natural-order cell or edge
// array covers the same cache lines as with the identity mapping.
__device__ __forceinline__ int split_x(const Geo &g, int w) {
  if (!g.split) return w;
  const int n0 = g.n[0];
  const int G = min(64, n0 & -n0);
  if (G < 2) return w;
  const int j = w & (G - 1), half = G >> 1;
  return (w - j) + ((j < half) ? 2 * j : 2 * (j - half) + 1);
}
__device__ __forceinline__ int fidx(const Geo &g, int k, int i0, int i1, int i2) {
  const int L = g.fd[k][0];
  return (int)g.foff[k] + (i2 * g.fd[k][1] + i1) * L + xpos(g, L, i0);
}
__device__ __forceinline__ int fidx3(const Geo &g, int k, const int i[3]) {
  return fidx(g, k, i[0], i[1], i[2]);
}
__device__ __forceinline__ int cidx3(const Geo &g, const int i[3]) {
  return (i[2] * g.n[1] + i[1]) * g.n[0] + i[0];
}
__device__ __forceinline__ int eidx3(const Geo &g, int m, const int i[3]) {
  return (int)g.eoff[m] + (i[2] * g.ed[m][1] + i[1]) * g.ed[m][0] + i[0];
}
__device__ __forceinline__ void cell_of(const Geo &g, i64 t, int i[3]) {
  const unsigned u = (unsigned)t;
  const unsigned q = u / (unsigned)g.n[0];
  i[0] = (int)(u - q * (unsigned)g.n[0]);
  i[2] = (int)(q / (unsigned)g.n[1]);
  i[1] = (int)(q - (unsigned)i[2] * (unsigned)g.n[1]);
}
// +1 / -1 neighbour along a periodic axis (index stays in range otherwise)
__device__ __forceinline__ int up1(const Geo &g, int a, int i) {
  int j = i + 1;
  return (!g.ns[a] && j == g.n[a]) ? 0 : j;
}
__device__ __forceinline__ int dn1(const Geo &g, int a, int i) {
  int j = i - 1;
  return (j < 0) ? j + g.n[a] : j;
}

// Thread -> (w, y, z) over an index box of n2 planes x n1 rows x W, on a
// grid of box_blocks() = (gx, n2) workgroups with z = blockIdx.y.  With
// g.xcd set and n1 % 8 == 0, workgroup x-index b takes band b % 8 of n1/8
// rows of its plane.  The hardware deals workgroups to the 8 XCDs in turn
// (gx is a multiple of 8), so each XCD streams its own band plane by plane
// and the y and z neighbours a stencil reads were fetched into that XCD's
// L2 shortly before.
__device__ __forceinline__ bool box_thread(const Geo &g, int W, int &w, int &y, int &z) {
  z = (int)blockIdx.y;
  unsigned u, y0 = 0;
  if (g.xcd && (g.n[1] & 7) == 0) {
    const unsigned band = (unsigned)g.n[1] >> 3;
    u = (blockIdx.x >> 3) * blockDim.x + threadIdx.x;
    if (u >= band * (unsigned)W) return false;
    y0 = (blockIdx.x & 7u) * band;
  } else {
    u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= (unsigned)g.n[1] * (unsigned)W) return false;
  }
  const unsigned r = u / (unsigned)W;
  y = (int)(y0 + r);
  w = (int)(u - r * (unsigned)W);
  return true;
}

// ------------------------------------------------------------------------
// A = alpha - L_mu at one face (paper Sec. "Staggered-grid Discretization", eq. div_stress).  Returns
// (A u)_f and the diagonal of A at f.  Tangential no-slip walls use the ghost
// value -u_f, which equals the one-sided wall difference (u_f - 0)/(h/2).

// Arithmetic of one row of A at face (k, i) from loaded values: u_f, its
// neighbours along k (ukp, ukm) and, per tangential axis l, the u_k values
// above/below (ua[l], ub[l], wall ghosts applied), the u_l values beside the
// upper and lower edge on the right/left cell (ulh_r, ulh_l, ull_r, ull_l),
// the edge viscosities (mhi, mlo), the cell viscosities right/left of f
// (mr, ml), alpha at f and, with a bulk coefficient, lam right/left (lr, ll).
template <typename T, int DIM>
__device__ __forceinline__ void a_row_core(const Geo &g, int k, const int i[3], T uf, T ukp,
                                           T ukm, const T (&ua)[3], const T (&ub)[3],
                                           const T (&ulh_r)[3], const T (&ulh_l)[3],
                                           const T (&ull_r)[3], const T (&ull_l)[3],
                                           const T (&mhi)[3], const T (&mlo)[3], T mr, T ml,
                                           T al, bool bulk, T lr, T ll, T &Au, T &diag) {
  const T ih = (T)g.ih;
  const T ih2 = ih * ih;
  const T tr = (T)2 * mr * ((ukp - uf) * ih);
  const T tl = (T)2 * ml * ((uf - ukm) * ih);
  T s = (tr - tl) * ih;
  T dg = al + (T)2 * (mr + ml) * ih2;
  // h * divergence of the cells right (r) and left (l) of f
  T hdr = ukp - uf, hdl = uf - ukm;
#pragma unroll
  for (int l = 0; l < DIM; l++) {
    if (l == k) continue;
    const bool top = g.ns[l] && (i[l] + 1 == g.n[l]);
    const bool bot = g.ns[l] && (i[l] == 0);
    const T ghi = (ua[l] - uf) * ih + (ulh_r[l] - ulh_l[l]) * ih;
    const T glo = (uf - ub[l]) * ih + (ull_r[l] - ull_l[l]) * ih;
    s += (mhi[l] * ghi - mlo[l] * glo) * ih;
    // wall edge: one-sided difference (no-slip, weight 2) or no flux (free-slip)
    const T wt = (g.fs[l] & 2) ? (T)0 : (T)2, wb = (g.fs[l] & 1) ? (T)0 : (T)2;
    dg += ((top ? wt : (T)1) * mhi[l] + (bot ? wb : (T)1) * mlo[l]) * ih2;
    hdr += ulh_r[l] - ull_r[l];
    hdl += ulh_l[l] - ull_l[l];
  }
  if (bulk) {
    s += (lr * hdr - ll * hdl) * ih2;
    dg += (lr + ll) * ih2;
  }
  Au = al * uf - s;
  diag = dg;
}

// Core of the row: the caller supplies u_f, its two neighbours along the
// normal axis k (ukp, ukm) and, for each tangential axis l, the u_k values
// above/below (ua[l], ub[l]) with the wall ghost already applied; u_l values
// and the coefficients are read from the component arrays comp[l].
// lam (may be null): gamma - 2/3 mu per cell; the normal stresses of the two
// cells beside f then gain lam (div u) (bulk viscosity, Sec. "Preconditioners").  The u_l
// values the shear terms load are exactly the cells' tangential faces, so the
// cell divergences cost no extra velocity loads.
// Z != 0 (first sweep from a zero iterate): the components l > k have not
// been written yet and are read as zero.
template <typename T, int DIM, int Z = 0>
__device__ __forceinline__ void a_row_nb(const Geo &g, int k, const int i[3], T uf, T ukp, T ukm,
                                         const T (&ua)[3], const T (&ub)[3],
                                         const T *const *comp, const T *__restrict__ alpha,
                                         const T *__restrict__ muc, const T *__restrict__ mue,
                                         const T *__restrict__ lam, T &Au, T &diag) {
  const i64 fq = fidx3(g, k, i);
  int t[3] = {i[0], i[1], i[2]};
  const int km = dn1(g, k, i[k]);
  t[k] = km;
  const T mr = muc[cidx3(g, i)];
  const T ml = muc[cidx3(g, t)];
  t[k] = i[k];
  const T al = alpha ? alpha[fq] : (T)0;  // no alpha array: theta = 0
  T ulh_r[3] = {0, 0, 0}, ulh_l[3] = {0, 0, 0}, ull_r[3] = {0, 0, 0}, ull_l[3] = {0, 0, 0};
  T mhi[3] = {0, 0, 0}, mlo[3] = {0, 0, 0};
#pragma unroll
  for (int l = 0; l < DIM; l++) {
    if (l == k) continue;
    const int m = 3 - k - l;
    const int lp = up1(g, l, i[l]);
    const T *__restrict__ ul = comp[l];
    const int f0 = g.fd[l][0], f1 = g.fd[l][1];
    const bool lz = Z && l > k;
    t[l] = lp;
    mhi[l] = mue[eidx3(g, m, t)];
    // u_l on the two faces beside the upper edge (cells i[k] and i[k]-1 along k)
    ulh_r[l] = lz ? (T)0 : ul[(t[2] * f1 + t[1]) * f0 + xpos(g, f0, t[0])];
    t[k] = km;
    ulh_l[l] = lz ? (T)0 : ul[(t[2] * f1 + t[1]) * f0 + xpos(g, f0, t[0])];
    t[k] = i[k];
    t[l] = i[l];
    mlo[l] = mue[eidx3(g, m, t)];
    ull_r[l] = lz ? (T)0 : ul[(t[2] * f1 + t[1]) * f0 + xpos(g, f0, t[0])];
    t[k] = km;
    ull_l[l] = lz ? (T)0 : ul[(t[2] * f1 + t[1]) * f0 + xpos(g, f0, t[0])];
    t[k] = i[k];
  }
  T lr = 0, ll = 0;
  if (lam) {
    t[k] = km;
    lr = lam[cidx3(g, i)];
    ll = lam[cidx3(g, t)];
    t[k] = i[k];
  }
  a_row_core<T, DIM>(g, k, i, uf, ukp, ukm, ua, ub, ulh_r, ulh_l, ull_r, ull_l, mhi, mlo, mr, ml,
                     al, lam != nullptr, lr, ll, Au, diag);
}

// A = alpha - L_mu at one face (paper Sec. "Staggered-grid Discretization", eq. div_stress), all values
// from the concatenated velocity buffer u.  Returns (A u)_f and the diagonal
// of A at f.  Tangential no-slip walls use the ghost value -u_f, which equals
// the one-sided wall difference (u_f - 0)/(h/2).
// Z (first Gauss-Seidel sweep from a zero iterate, where memory has not been
// cleared): bit 0 reads u_f as zero, bit 1 the other-colour neighbours of
// component k as zero, and any nonzero Z reads the high wall face of
// component k and the components after k as zero.  The values are those the
// cleared iterate would hold, so the arithmetic is unchanged.
template <typename T, int DIM, int Z = 0>
__device__ __forceinline__ void a_row(const Geo &g, int k, const int i[3], const T *__restrict__ u,
                                      const T *__restrict__ alpha, const T *__restrict__ muc,
                                      const T *__restrict__ mue, const T *__restrict__ lam,
                                      T &Au, T &diag) {
  const i64 fq = fidx3(g, k, i);
  const T uf = (Z & 1) ? (T)0 : u[fq];
  int t[3] = {i[0], i[1], i[2]};
  t[k] = up1(g, k, i[k]);
  const bool kz = (Z & 2) || (Z && g.ns[k] && i[k] + 1 == g.n[k]);
  const T ukp = kz ? (T)0 : u[fidx3(g, k, t)];
  t[k] = dn1(g, k, i[k]);
  const T ukm = (Z & 2) ? (T)0 : u[fidx3(g, k, t)];
  t[k] = i[k];
  T ua[3] = {0, 0, 0}, ub[3] = {0, 0, 0};
#pragma unroll
  for (int l = 0; l < DIM; l++) {
    if (l == k) continue;
    const bool top = g.ns[l] && (i[l] + 1 == g.n[l]);
    const bool bot = g.ns[l] && (i[l] == 0);
    // loads are unconditional (from an in-range index) so that all of them
    // issue before the first wait; the wall ghost -u_f is selected afterwards
    t[l] = top ? i[l] : up1(g, l, i[l]);  // component k has no face at index n[l] along l
    const T va = (Z & 2) ? (T)0 : u[fidx3(g, k, t)];
    t[l] = dn1(g, l, i[l]);
    const T vb = (Z & 2) ? (T)0 : u[fidx3(g, k, t)];
    t[l] = i[l];
    // no-slip: odd ghost (zero wall value); free-slip: even ghost (no shear)
    ua[l] = top ? ((g.fs[l] & 2) ? uf : -uf) : va;
    ub[l] = bot ? ((g.fs[l] & 1) ? uf : -uf) : vb;
  }
  const T *comp[3] = {u + g.foff[0], u + g.foff[1], u + g.foff[2]};
  a_row_nb<T, DIM, Z>(g, k, i, uf, ukp, ukm, ua, ub, comp, alpha, muc, mue, lam, Au, diag);
}

__device__ __forceinline__ bool low_wall(const Geo &g, int k, const int i[3]) {
  return g.ns[k] && i[k] == 0;
}

// ------------------------------------------------------------------------
// coefficient setup (Sec. "Staggered-grid Discretization" averages, Sec. "Rescaling of the Linear System" rescaling)
// ------------------------------------------------------------------------

__global__ void k_setup_faces(Geo g, const double *__restrict__ rho, double theta, double c,
                              double *__restrict__ alpha, double *__restrict__ beta) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.ncell) return;
  int i[3];
  cell_of(g, t, i);
  for (int k = 0; k < g.d; k++) {
    const i64 q = fidx3(g, k, i);
    if (low_wall(g, k, i)) {
      alpha[q] = 0.0;
      beta[q] = 0.0;
      continue;
    }
    int l[3] = {i[0], i[1], i[2]};
    l[k] = dn1(g, k, i[k]);
    const double rf = 0.5 * (rho[cidx3(g, i)] + rho[cidx3(g, l)]);
    alpha[q] = c * (theta * rf);
    beta[q] = (1.0 / rf) / c;
  }
}

__global__ void k_scale_copy(const double *__restrict__ in, double c, double *__restrict__ out,
                             i64 n) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = c * in[t];
}

// edge family m: mean (arithmetic, harmonic) of the existing neighbouring
// cells; 4 inside, 2 on a wall, 1 in a corner
__global__ void k_setup_edges(Geo g, int m, const double *__restrict__ mu,
                              const double *__restrict__ given, int mode, double c,
                              double *__restrict__ mue) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.ecnt[m]) return;
  int e[3];
  {
    i64 q = t / g.ed[m][0];
    e[0] = (int)(t - q * g.ed[m][0]);
    e[2] = (int)(q / g.ed[m][1]);
    e[1] = (int)(q - (i64)e[2] * g.ed[m][1]);
  }
  const i64 out = g.eoff[m] + t;
  if (mode == 2) {
    mue[out] = c * given[out];
    return;
  }
  const int k = (m == 0) ? 1 : 0;
  const int l = (m == 2) ? 1 : 2;
  double s = 0.0, sinv = 0.0;
  int cnt = 0;
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++) {
      int cc[3] = {e[0], e[1], e[2]};
      cc[k] -= a;
      cc[l] -= b;
      if (g.ns[k] && (cc[k] < 0 || cc[k] >= g.n[k])) continue;
      if (g.ns[l] && (cc[l] < 0 || cc[l] >= g.n[l])) continue;
      if (cc[k] < 0) cc[k] += g.n[k];
      if (cc[k] >= g.n[k]) cc[k] -= g.n[k];
      if (cc[l] < 0) cc[l] += g.n[l];
      if (cc[l] >= g.n[l]) cc[l] -= g.n[l];
      const double v = mu[cidx3(g, cc)];
      s += v;
      sinv += 1.0 / v;
      cnt++;
    }
  const double val = (mode == 1) ? (double)cnt / sinv : s / (double)cnt;
  mue[out] = c * val;
}

// coarse coefficients (Appendix C): faces = mean of overlaid fine faces,
// cells = mean of 2^d fine cells, edges = mean of the two overlaid fine edges
// (3D) or injection (2D nodes)
__global__ void k_coarsen_faces_cells(Geo gf, Geo gc, const double *__restrict__ af,
                                      const double *__restrict__ bf,
                                      const double *__restrict__ mcf, double *__restrict__ ac,
                                      double *__restrict__ bc, double *__restrict__ mcc) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= gc.ncell) return;
  int I[3];
  cell_of(gc, t, I);
  const int d = gc.d;
  for (int k = 0; k < d; k++) {
    const i64 q = fidx3(gc, k, I);
    if (low_wall(gc, k, I)) {
      ac[q] = 0.0;
      bc[q] = 0.0;
      continue;
    }
    int tax[2] = {0, 0}, nt = 0;
    for (int b = 0; b < d; b++)
      if (b != k) tax[nt++] = b;
    double sa = 0.0, sb = 0.0;
    int cnt = 0;
    for (int o1 = 0; o1 < 2; o1++)
      for (int o0 = 0; o0 < (nt == 2 ? 2 : 1); o0++) {
        int f[3] = {2 * I[0], 2 * I[1], d == 3 ? 2 * I[2] : 0};
        f[tax[0]] += o1;
        if (nt == 2) f[tax[1]] += o0;
        const i64 fq = fidx3(gf, k, f);
        sa += af[fq];
        sb += bf[fq];
        cnt++;
      }
    ac[q] = sa / cnt;
    bc[q] = sb / cnt;
  }
  double s = 0.0;
  for (int o2 = 0; o2 < (d == 3 ? 2 : 1); o2++)
    for (int o1 = 0; o1 < 2; o1++)
      for (int o0 = 0; o0 < 2; o0++) {
        int f[3] = {2 * I[0] + o0, 2 * I[1] + o1, d == 3 ? 2 * I[2] + o2 : 0};
        s += mcf[cidx3(gf, f)];
      }
  mcc[t] = s / (double)(1 << d);
}

__global__ void k_coarsen_edges(Geo gf, Geo gc, int m, const double *__restrict__ mef,
                                double *__restrict__ mec) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= gc.ecnt[m]) return;
  int E[3];
  {
    i64 q = t / gc.ed[m][0];
    E[0] = (int)(t - q * gc.ed[m][0]);
    E[2] = (int)(q / gc.ed[m][1]);
    E[1] = (int)(q - (i64)E[2] * gc.ed[m][1]);
  }
  int e[3] = {2 * E[0], 2 * E[1], gc.d == 3 ? 2 * E[2] : 0};
  double v;
  if (m < gc.d) {
    int e2[3] = {e[0], e[1], e[2]};
    e2[m] += 1;
    v = 0.5 * (mef[eidx3(gf, m, e)] + mef[eidx3(gf, m, e2)]);
  } else {
    v = mef[eidx3(gf, m, e)];
  }
  mec[gc.eoff[m] + t] = v;
}

__global__ void k_check_coefs(const double *__restrict__ rho, const double *__restrict__ mu,
                              i64 n, int *flag) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double r = rho[t], m = mu[t];
  const bool ok = (r > 0.0) && (m >= 0.0) && isfinite(r) && isfinite(m);
  if (!ok) atomicOr(flag, 1);
}

// bulk coefficient of the stress, lam = c (gamma - 2/3 mu) per cell (Sec. "Preconditioners");
// sig = c mu + lam / 2 = c (gamma + 4/3 mu) / 2 is what the Schur
// approximation multiplies by 2 (eq. Schur_app_bulk)
__global__ void k_setup_bulk(const double *__restrict__ gamma, const double *__restrict__ mu,
                             double c, i64 n, double *__restrict__ lam, double *__restrict__ sig) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double m = mu[t];
  const double l = c * (gamma[t] - 2.0 / 3.0 * m);
  lam[t] = l;
  sig[t] = c * m + 0.5 * l;
}
void launch_setup_bulk(const double *gamma, const double *mu, double c, i64 n, double *lam,
                       double *sig, hipStream_t s) {
  hipLaunchKernelGGL(k_setup_bulk, dim3(blocks_for(n)), dim3(kBlock), 0, s, gamma, mu, c, n, lam,
                     sig);
}

void launch_setup_faces(const Geo &g, const double *rho, double theta, double c, double *alpha,
                        double *beta, hipStream_t s) {
  hipLaunchKernelGGL(k_setup_faces, dim3(blocks_for(g.ncell)), dim3(kBlock), 0, s, g, rho, theta,
                     c, alpha, beta);
}
void launch_setup_cells(const Geo &g, const double *mu, double c, double *muc, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(blocks_for(g.ncell)), dim3(kBlock), 0, s, mu, c, muc,
                     g.ncell);
}
void launch_setup_edges(const Geo &g, const double *mu, const double *given, int mode, double c,
                        double *mue, hipStream_t s) {
  for (int m = 0; m < 3; m++) {
    if (g.ecnt[m] == 0) continue;
    hipLaunchKernelGGL(k_setup_edges, dim3(blocks_for(g.ecnt[m])), dim3(kBlock), 0, s, g, m, mu,
                       given, mode, c, mue);
  }
}
void launch_coarsen(const Geo &gf, const Geo &gc, const double *af, const double *bf,
                    const double *mcf, const double *mef, double *ac, double *bc, double *mcc,
                    double *mec, hipStream_t s) {
  hipLaunchKernelGGL(k_coarsen_faces_cells, dim3(blocks_for(gc.ncell)), dim3(kBlock), 0, s, gf,
                     gc, af, bf, mcf, ac, bc, mcc);
  for (int m = 0; m < 3; m++) {
    if (gc.ecnt[m] == 0) continue;
    hipLaunchKernelGGL(k_coarsen_edges, dim3(blocks_for(gc.ecnt[m])), dim3(kBlock), 0, s, gf, gc,
                       m, mef, mec);
  }
}
void launch_check_coefs(const double *rho, const double *mu, i64 n, int *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_coefs, dim3(blocks_for(n)), dim3(kBlock), 0, s, rho, mu, n, flag);
}

// ------------------------------------------------------------------------
// element-wise helpers
// ------------------------------------------------------------------------

template <typename TO, typename TI>
__global__ void k_cast(const TI *__restrict__ in, TO *__restrict__ out, i64 n) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = (TO)in[t];
}
template <typename TO, typename TI>
void launch_cast(const TI *in, TO *out, i64 n, hipStream_t s) {
  hipLaunchKernelGGL((k_cast<TO, TI>), dim3(blocks_for(n)), dim3(kBlock), 0, s, in, out, n);
}
template void launch_cast<float, double>(const double *, float *, i64, hipStream_t);
template void launch_cast<double, float>(const float *, double *, i64, hipStream_t);
template void launch_cast<double, double>(const double *, double *, i64, hipStream_t);
template void launch_cast<float, float>(const float *, float *, i64, hipStream_t);

template <typename T>
__global__ void k_fill(T *__restrict__ a, T v, i64 n) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) a[t] = v;
}
template <typename T>
void launch_fill(T *a, T v, i64 n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, v, n);
}
template void launch_fill<float>(float *, float, i64, hipStream_t);
template void launch_fill<double>(double *, double, i64, hipStream_t);
template void launch_fill<int>(int *, int, i64, hipStream_t);

__global__ void k_pack_vel(Geo g, const double *__restrict__ in, double scale,
                           double *__restrict__ out) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.nvel) return;
  int k = 0;
  while (k + 1 < g.d && t >= g.foff[k + 1]) k++;
  const i64 r = t - g.foff[k];
  // index along axis k
  i64 stride = 1;
  for (int a = 0; a < k; a++) stride *= g.fd[k][a];
  const int ik = (int)((r / stride) % g.fd[k][k]);
  const bool wall = g.ns[k] && (ik == 0 || ik == g.n[k]);
  out[t] = wall ? 0.0 : scale * in[t];
}
void launch_pack_vel(const Geo &g, const double *in, double scale, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_vel, dim3(blocks_for(g.nvel)), dim3(kBlock), 0, s, g, in, scale, out);
}
void launch_scale(const double *in, double scale, double *out, i64 n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(blocks_for(n)), dim3(kBlock), 0, s, in, scale, out, n);
}

template <typename T>
__global__ void k_axpy(T a, const T *__restrict__ x, T *__restrict__ y, i64 n) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] += a * x[t];
}
template <typename T>
void launch_axpy(T a, const T *x, T *y, i64 n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, x, y, n);
}
template void launch_axpy<float>(float, const float *, float *, i64, hipStream_t);
template void launch_axpy<double>(double, const double *, double *, i64, hipStream_t);

// ------------------------------------------------------------------------
// double-double arithmetic for the extended-precision residual (paper Sec.
// "Rescaling of the Linear System": extended precision arithmetic in extreme
// cases).  A value is hi + lo with |lo| <= ulp(hi) / 2, about 106 bits of
// significand.  The building blocks are the error-free transformations of
// Knuth (two_sum: a + b = s + e exactly) and of the fused multiply-add
// (two_prod: a * b = p + e exactly); sums and products renormalise with
// fast_two_sum (Dekker).  Written from those definitions.  The identities
// hold only for separately rounded operations, so no multiply-add in these
// functions may be contracted into a fused one (the pragma below; the
// compiler otherwise fuses p = a * b with the following p + lo).
// ------------------------------------------------------------------------

struct dd {
  double hi, lo;
  dd() = default;
  __device__ constexpr dd(double h) : hi(h), lo(0.0) {}
  __device__ constexpr dd(double h, double l) : hi(h), lo(l) {}
};

__device__ __forceinline__ dd dd_two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  return dd(s, (a - (s - bb)) + (b - bb));
}
__device__ __forceinline__ dd dd_fast_two_sum(double a, double b) {  // needs |a| >= |b|
#pragma clang fp contract(off)
  const double s = a + b;
  return dd(s, b - (s - a));
}
__device__ __forceinline__ dd dd_two_prod(double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  return dd(p, fma(a, b, -p));
}
__device__ __forceinline__ dd operator+(const dd &a, const dd &b) {
#pragma clang fp contract(off)
  dd s = dd_two_sum(a.hi, b.hi);
  const dd t = dd_two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = dd_fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return dd_fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd operator-(const dd &a) { return dd(-a.hi, -a.lo); }
__device__ __forceinline__ dd operator-(const dd &a, const dd &b) { return a + (-b); }
__device__ __forceinline__ dd operator*(const dd &a, const dd &b) {
#pragma clang fp contract(off)
  dd p = dd_two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return dd_fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ double to_double(double a) { return a; }
__device__ __forceinline__ double to_double(const dd &a) {
#pragma clang fp contract(off)
  return a.hi + a.lo;
}
// 1/h in the row arithmetic: the FP64 reciprocal, or with R = dd the
// reciprocal to about 106 bits (ih_lo = (1 - h ih) / h from the host)
__device__ __forceinline__ void make_ih(double ih, double, double &out) { out = ih; }
__device__ __forceinline__ void make_ih(double ih, double ih_lo, dd &out) { out = dd(ih, ih_lo); }

// ------------------------------------------------------------------------
// saddle operator (FP64 or double-double arithmetic, input in TI)
// ------------------------------------------------------------------------

// One row of A at face (k, i) in FP64 from loaded values (the names of
// a_row_core).  GW: prescribed tangential wall velocities (gwhi, gwlo at the
// upper/lower edge, edge layout) replace the zero wall value of the no-slip
// ghost, 2 gw - u_f, and a free-slip wall's flux is zero (boundary terms only).
template <typename R, int DIM, bool GW>
__device__ __forceinline__ R a_row_mixed_core(
    const Geo &g, int k, const int i[3], R ih, R uf, R ukp, R ukm, const R (&va)[3],
    const R (&vb)[3], const R (&ulh_r)[3], const R (&ulh_l)[3], const R (&ull_r)[3],
    const R (&ull_l)[3], const R (&mhi)[3], const R (&mlo)[3], const R (&gwhi)[3],
    const R (&gwlo)[3], R mr, R ml, R al, bool bulk, R lr, R ll) {
  const R tr = R(2.0) * mr * ((ukp - uf) * ih);
  const R tl = R(2.0) * ml * ((uf - ukm) * ih);
  R s = (tr - tl) * ih;
  R hdr = ukp - uf, hdl = uf - ukm;  // h * divergence of cells r and l
#pragma unroll
  for (int l = 0; l < DIM; l++) {
    if (l == k) continue;
    const bool top = g.ns[l] && (i[l] + 1 == g.n[l]);
    const bool bot = g.ns[l] && (i[l] == 0);
    // wall ghosts: even (free-slip end) or odd (no-slip end)
    const bool fs_hi = g.fs[l] & 2, fs_lo = g.fs[l] & 1;
    R ua = top ? (fs_hi ? uf : -uf) : va[l];
    R ub = bot ? (fs_lo ? uf : -uf) : vb[l];
    if (GW) {
      if (top && !fs_hi) ua = R(2.0) * gwhi[l] - uf;
      if (bot && !fs_lo) ub = R(2.0) * gwlo[l] - uf;
    }
    R ghi = (ua - uf) * ih + (ulh_r[l] - ulh_l[l]) * ih;
    R glo = (uf - ub) * ih + (ull_r[l] - ull_l[l]) * ih;
    // with prescribed normal velocities on a free-slip wall the cross
    // derivative along the wall need not vanish; the whole flux does
    if (GW) {
      if (top && fs_hi) ghi = R(0.0);
      if (bot && fs_lo) glo = R(0.0);
    }
    s = s + (mhi[l] * ghi - mlo[l] * glo) * ih;
    hdr = hdr + (ulh_r[l] - ull_r[l]);
    hdl = hdl + (ulh_l[l] - ull_l[l]);
  }
  if (bulk) s = s + (lr * hdr - ll * hdl) * (ih * ih);  // lam (div u) on the normal stresses
  return al * uf - s;
}

// y = M x (or y = b - M x) at cell i: the velocity rows of the low faces of
// all components, the pressure gradient, and the divergence row of the cell.
// The rows share most of their velocity values, which are loaded once per
// cell (per component c at i, at i +- e_a and at i + e_c - e_k), as are the
// cell and edge coefficients.
// R = double: FP64 arithmetic; R = dd: every value and operation in
// double-double and the result rounded once (the extended-precision
// residual, with ih_lo the low part of 1/h).
template <typename TI, int DIM, bool GW, typename R = double>
__global__ void k_apply_m(Geo g, const double *__restrict__ alpha, const double *__restrict__ muc,
                          const double *__restrict__ mue, const double *__restrict__ lam,
                          const TI *__restrict__ xu,
                          const TI *__restrict__ xp, const double *__restrict__ bu,
                          const double *__restrict__ bp, const double *__restrict__ gw,
                          double *__restrict__ yu, double *__restrict__ yp, double ih_lo) {
  int i[3];
  if (!box_thread(g, g.n[0], i[0], i[1], i[2])) return;
  const i64 t = cidx3(g, i);
  R ih;
  make_ih(g.ih, ih_lo, ih);
  int ip[3] = {0, 0, 0}, im[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; a++) {
    ip[a] = up1(g, a, i[a]);
    im[a] = dn1(g, a, i[a]);
  }
  // V[c][0] at i, V[c][1 + 2a] at i + e_a, V[c][2 + 2a] at i - e_a; X[c][k]
  // at i + e_c - e_k.  Component c has no face at index n[a] along a wall
  // axis a != c: that load is clamped to i (the wall ghost replaces it).
  R V[DIM][1 + 2 * DIM], X[DIM][DIM];
#pragma unroll
  for (int c = 0; c < DIM; c++) {
    int q[3] = {i[0], i[1], i[2]};
    V[c][0] = R((double)xu[fidx3(g, c, q)]);
#pragma unroll
    for (int a = 0; a < DIM; a++) {
      const bool top = a != c && g.ns[a] && (i[a] + 1 == g.n[a]);
      q[a] = top ? i[a] : ip[a];
      V[c][1 + 2 * a] = R((double)xu[fidx3(g, c, q)]);
      q[a] = im[a];
      V[c][2 + 2 * a] = R((double)xu[fidx3(g, c, q)]);
      q[a] = i[a];
    }
#pragma unroll
    for (int k = 0; k < DIM; k++) {
      X[c][k] = R(0.0);
      if (k == c) continue;
      q[c] = ip[c];
      q[k] = im[k];
      X[c][k] = R((double)xu[fidx3(g, c, q)]);
      q[c] = i[c];
      q[k] = i[k];
    }
  }
  // cell values at i and at i - e_k
  R mc[1 + DIM], lc[1 + DIM], pc[1 + DIM];
  mc[0] = R(muc[t]);
  lc[0] = R(lam ? lam[t] : 0.0);
  pc[0] = R((double)xp[t]);
#pragma unroll
  for (int k = 0; k < DIM; k++) {
    int q[3] = {i[0], i[1], i[2]};
    q[k] = im[k];
    const i64 cq = cidx3(g, q);
    mc[1 + k] = R(muc[cq]);
    lc[1 + k] = R(lam ? lam[cq] : 0.0);
    pc[1 + k] = R((double)xp[cq]);
  }
  // edge family m at i (E0) and at i + e_a for the axes a != m (E1), and the
  // prescribed wall velocities at the same edges
  R E0[3] = {R(0.0), R(0.0), R(0.0)};
  R E1[3][3] = {{R(0.0), R(0.0), R(0.0)}, {R(0.0), R(0.0), R(0.0)}, {R(0.0), R(0.0), R(0.0)}};
  R G0[3] = {R(0.0), R(0.0), R(0.0)};
  R G1[3][3] = {{R(0.0), R(0.0), R(0.0)}, {R(0.0), R(0.0), R(0.0)}, {R(0.0), R(0.0), R(0.0)}};
#pragma unroll
  for (int m = (DIM == 3 ? 0 : 2); m < 3; m++) {
    const int e0 = eidx3(g, m, i);
    E0[m] = R(mue[e0]);
    if (GW) G0[m] = R(gw[e0]);
#pragma unroll
    for (int a = 0; a < DIM; a++) {
      if (a == m) continue;
      int q[3] = {i[0], i[1], i[2]};
      q[a] = ip[a];
      const int e1 = eidx3(g, m, q);
      E1[m][a] = R(mue[e1]);
      if (GW) G1[m][a] = R(gw[e1]);
    }
  }
  R div = R(0.0);
#pragma unroll
  for (int k = 0; k < DIM; k++) {
    // the face above along k: index i[k] + 1 (the wall face on a wall axis,
    // wrapped on a periodic one)
    div = div + (V[k][1 + 2 * k] - V[k][0]) * ih;
    if (low_wall(g, k, i)) continue;
    R va[3] = {R(0.0), R(0.0), R(0.0)}, vb[3] = {R(0.0), R(0.0), R(0.0)};
    R ulh_r[3] = {R(0.0), R(0.0), R(0.0)}, ulh_l[3] = {R(0.0), R(0.0), R(0.0)};
    R ull_r[3] = {R(0.0), R(0.0), R(0.0)}, ull_l[3] = {R(0.0), R(0.0), R(0.0)};
    R mhi[3] = {R(0.0), R(0.0), R(0.0)}, mlo[3] = {R(0.0), R(0.0), R(0.0)};
    R gwhi[3] = {R(0.0), R(0.0), R(0.0)}, gwlo[3] = {R(0.0), R(0.0), R(0.0)};
#pragma unroll
    for (int l = 0; l < DIM; l++) {
      if (l == k) continue;
      const int m = 3 - k - l;
      va[l] = V[k][1 + 2 * l];
      vb[l] = V[k][2 + 2 * l];
      ulh_r[l] = V[l][1 + 2 * l];
      ulh_l[l] = X[l][k];
      ull_r[l] = V[l][0];
      ull_l[l] = V[l][2 + 2 * k];
      mhi[l] = E1[m][l];
      mlo[l] = E0[m];
      gwhi[l] = G1[m][l];
      gwlo[l] = G0[m];
    }
    const i64 q = fidx3(g, k, i);
    const R al = R(alpha ? alpha[q] : 0.0);  // no alpha array: theta = 0
    const R Au = a_row_mixed_core<R, DIM, GW>(
        g, k, i, ih, V[k][0], V[k][1 + 2 * k], V[k][2 + 2 * k], va, vb, ulh_r, ulh_l, ull_r,
        ull_l, mhi, mlo, gwhi, gwlo, mc[0], mc[1 + k], al, lam != nullptr, lc[0], lc[1 + k]);
    const R gp = (pc[0] - pc[1 + k]) * ih;
    const R y = Au + gp;
    yu[q] = to_double(bu ? R(bu[q]) - y : y);
  }
  yp[t] = to_double(bp ? R(bp[t]) + div : -div);
}

template <typename TI>
void launch_apply_m(const Geo &g, const double *alpha, const double *muc, const double *mue,
                    const double *lam, const TI *xu, const TI *xp, const double *bu,
                    const double *bp, double *yu, double *yp, hipStream_t s) {
  if (g.d == 3)
    hipLaunchKernelGGL((k_apply_m<TI, 3, false>), box_blocks(g, g.n[0]), dim3(kBlock), 0, s, g,
                       alpha, muc, mue, lam, xu, xp, bu, bp, nullptr, yu, yp, 0.0);
  else
    hipLaunchKernelGGL((k_apply_m<TI, 2, false>), box_blocks(g, g.n[0]), dim3(kBlock), 0, s, g,
                       alpha, muc, mue, lam, xu, xp, bu, bp, nullptr, yu, yp, 0.0);
}
template void launch_apply_m<double>(const Geo &, const double *, const double *, const double *,
                                     const double *, const double *, const double *,
                                     const double *, const double *, double *, double *,
                                     hipStream_t);
template void launch_apply_m<float>(const Geo &, const double *, const double *, const double *,
                                    const double *, const float *, const float *, const double *,
                                    const double *, double *, double *, hipStream_t);

void launch_apply_m_walls(const Geo &g, const double *alpha, const double *muc,
                          const double *mue, const double *lam, const double *xu,
                          const double *xp, const double *gw, double *yu, double *yp,
                          hipStream_t s) {
  if (g.d == 3)
    hipLaunchKernelGGL((k_apply_m<double, 3, true>), box_blocks(g, g.n[0]), dim3(kBlock), 0, s,
                       g, alpha, muc, mue, lam, xu, xp, nullptr, nullptr, gw, yu, yp, 0.0);
  else
    hipLaunchKernelGGL((k_apply_m<double, 2, true>), box_blocks(g, g.n[0]), dim3(kBlock), 0, s,
                       g, alpha, muc, mue, lam, xu, xp, nullptr, nullptr, gw, yu, yp, 0.0);
}

void launch_residual_dd(const Geo &g, const double *alpha, const double *muc, const double *mue,
                        const double *lam, const double *xu, const double *xp, const double *bu,
                        const double *bp, double *ru, double *rp, hipStream_t s) {
  // low part of 1/h: the FMA remainder 1 - h ih is exact
  const double ih_lo = std::fma(-g.h, g.ih, 1.0) / g.h;
  if (g.d == 3)
    hipLaunchKernelGGL((k_apply_m<double, 3, false, dd>), box_blocks(g, g.n[0]), dim3(kBlock), 0,
                       s, g, alpha, muc, mue, lam, xu, xp, bu, bp, nullptr, ru, rp, ih_lo);
  else
    hipLaunchKernelGGL((k_apply_m<double, 2, false, dd>), box_blocks(g, g.n[0]), dim3(kBlock), 0,
                       s, g, alpha, muc, mue, lam, xu, xp, bu, bp, nullptr, ru, rp, ih_lo);
}

// Diagonal scaling of the rescaled unknowns: 1 / sqrt(diag A) at the interior
// velocity faces (1 on wall faces), sqrt(2 mu_cell + lam) at the cells.
template <int DIM>
__global__ void k_diag_scaling_faces(Geo g, int k, const double *__restrict__ alpha,
                                     const double *__restrict__ muc,
                                     const double *__restrict__ mue,
                                     const double *__restrict__ lam,
                                     const double *__restrict__ zero, double *__restrict__ sd) {
  int i[3];
  if (!box_thread(g, g.n[0], i[0], i[1], i[2])) return;
  const i64 q = fidx3(g, k, i);
  if (low_wall(g, k, i)) {
    sd[q] = 1.0;
    if (i[k] == 0) {  // the high wall face of the same line
      int t[3] = {i[0], i[1], i[2]};
      t[k] = g.n[k];
      sd[fidx3(g, k, t)] = 1.0;
    }
    return;
  }
  double Au, dg;
  a_row<double, DIM>(g, k, i, zero, alpha, muc, mue, lam, Au, dg);
  sd[q] = 1.0 / sqrt(dg);
}

__global__ void k_diag_scaling_cells(const double *__restrict__ muc, const double *__restrict__ lam,
                                     i64 n, double *__restrict__ sd, int *__restrict__ bad) {
  const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double sig = 2.0 * muc[t] + (lam ? lam[t] : 0.0);
  if (!(sig > 0.0)) *bad = 1;
  sd[t] = sig > 0.0 ? sqrt(sig) : 1.0;
}

void launch_diag_scaling(const Geo &g, const double *alpha, const double *muc, const double *mue,
                         const double *lam, const double *zero, double *sd, int *bad,
                         hipStream_t s) {
  for (int k = 0; k < g.d; k++) {
    if (g.d == 3)
      hipLaunchKernelGGL((k_diag_scaling_faces<3>), box_blocks(g, g.n[0]), dim3(kBlock), 0, s, g,
                         k, alpha, muc, mue, lam, zero, sd);
    else
      hipLaunchKernelGGL((k_diag_scaling_faces<2>), box_blocks(g, g.n[0]), dim3(kBlock), 0, s, g,
                         k, alpha, muc, mue, lam, zero, sd);
  }
  hipLaunchKernelGGL(k_diag_scaling_cells, dim3((unsigned)((g.ncell + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, muc, lam, g.ncell, sd + g.nvel, bad);
}

// y = x * s (inv = 0) or y = x / s (inv = 1), elementwise; y may equal x
__global__ void k_mul_scaling(const double *x, const double *__restrict__ sd, int inv, i64 n,
                              double *y) {
  const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  y[t] = inv ? x[t] / sd[t] : x[t] * sd[t];
}

void launch_mul_scaling(const double *x, const double *sd, int inv, i64 n, double *y,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_mul_scaling, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, x, sd, inv, n, y);
}

// out = scale * in on the wall faces, 0 elsewhere (the wall-data field)
__global__ void k_pack_walls(Geo g, const double *__restrict__ in, double scale,
                             double *__restrict__ out) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.nvel) return;
  int k = 0;
  while (k + 1 < g.d && t >= g.foff[k + 1]) k++;
  const i64 r = t - g.foff[k];
  i64 stride = 1;
  for (int a = 0; a < k; a++) stride *= g.fd[k][a];
  const int ik = (int)((r / stride) % g.fd[k][k]);
  const bool wall = g.ns[k] && (ik == 0 || ik == g.n[k]);
  out[t] = wall ? scale * in[t] : 0.0;
}
void launch_pack_walls(const Geo &g, const double *in, double scale, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_walls, dim3(blocks_for(g.nvel)), dim3(kBlock), 0, s, g, in, scale,
                     out);
}

// out = in with the velocity storage order of gout (in has that of gin);
// with sums, the mean of each singular component (gin.sing) is subtracted.
// Thread p of a row of L faces moves the pair of x positions 2p, 2p+1: in
// natural order the pair is adjacent, in split order it sits at p and
// (L+1)/2 + p, so every load and store of a wave is contiguous.
template <typename T>
struct Pair;
template <>
struct Pair<float> {
  typedef float2 V;
};
template <>
struct Pair<double> {
  typedef double2 V;
};
__host__ __device__ inline i64 permute_pairs(const Geo &g, int k) {
  return (i64)g.fd[k][1] * g.fd[k][2] * ((g.fd[k][0] + 1) >> 1);
}
template <typename T>
__global__ void k_vel_permute(Geo gin, Geo gout, const T *__restrict__ in, T *__restrict__ out,
                              const double *__restrict__ sums, int in_al, int out_al) {
  typedef typename Pair<T>::V V;
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  int k = 0;
  for (; k < gin.d; k++) {
    const i64 np = permute_pairs(gin, k);
    if (t < np) break;
    t -= np;
  }
  if (k == gin.d) return;
  const unsigned L = (unsigned)gin.fd[k][0], ne = (L + 1) >> 1;
  const unsigned row = (unsigned)t / ne;
  const unsigned p = (unsigned)t - row * ne;
  const i64 base = gin.foff[k] + (i64)row * L;
  const bool two = 2 * p + 1 < L;
  const T mean =
      (sums && ((gin.sing >> k) & 1)) ? (T)(sums[k] / (double)gin.fcnt[k]) : (T)0;
  T a, b = (T)0;
  if (gin.split) {
    a = in[base + p];
    if (two) b = in[base + ne + p];
  } else if (in_al && two && !(base & 1)) {
    const V v = *reinterpret_cast<const V *>(in + base + 2 * p);
    a = v.x;
    b = v.y;
  } else {
    a = in[base + 2 * p];
    if (two) b = in[base + 2 * p + 1];
  }
  a -= mean;
  b -= mean;
  if (gout.split) {
    out[base + p] = a;
    if (two) out[base + ne + p] = b;
  } else if (out_al && two && !(base & 1)) {
    V v;
    v.x = a;
    v.y = b;
    *reinterpret_cast<V *>(out + base + 2 * p) = v;
  } else {
    out[base + 2 * p] = a;
    if (two) out[base + 2 * p + 1] = b;
  }
}
// FP32 rows whose length is a multiple of 4: thread q of a row moves the
// natural positions 4q..4q+3 (one float4) to the split positions 2q, 2q+1
// and (L/2) + 2q, (L/2) + 2q + 1 (two float2), or back.
__host__ __device__ inline i64 permute_quads(const Geo &g, int k) {
  return (i64)g.fd[k][1] * g.fd[k][2] * (g.fd[k][0] >> 2);
}
__global__ void k_vel_permute4(Geo gin, Geo gout, const float *__restrict__ in,
                               float *__restrict__ out, const double *__restrict__ sums) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  int k = 0;
  for (; k < gin.d; k++) {
    const i64 nq = permute_quads(gin, k);
    if (t < nq) break;
    t -= nq;
  }
  if (k == gin.d) return;
  const unsigned L = (unsigned)gin.fd[k][0], nq = L >> 2, ne = L >> 1;
  const unsigned row = (unsigned)t / nq;
  const unsigned q = (unsigned)t - row * nq;
  const i64 base = gin.foff[k] + (i64)row * L;
  const float mean =
      (sums && ((gin.sing >> k) & 1)) ? (float)(sums[k] / (double)gin.fcnt[k]) : 0.0f;
  float x0, x1, x2, x3;  // natural positions 4q .. 4q+3
  if (gin.split) {
    const float2 e = *reinterpret_cast<const float2 *>(in + base + 2 * q);
    const float2 o = *reinterpret_cast<const float2 *>(in + base + ne + 2 * q);
    x0 = e.x;
    x2 = e.y;
    x1 = o.x;
    x3 = o.y;
  } else {
    const float4 v = *reinterpret_cast<const float4 *>(in + base + 4 * q);
    x0 = v.x;
    x1 = v.y;
    x2 = v.z;
    x3 = v.w;
  }
  x0 -= mean;
  x1 -= mean;
  x2 -= mean;
  x3 -= mean;
  if (gout.split) {
    *reinterpret_cast<float2 *>(out + base + 2 * q) = make_float2(x0, x2);
    *reinterpret_cast<float2 *>(out + base + ne + 2 * q) = make_float2(x1, x3);
  } else {
    *reinterpret_cast<float4 *>(out + base + 4 * q) = make_float4(x0, x1, x2, x3);
  }
}

template <typename T>
void launch_vel_permute(const Geo &gin, const Geo &gout, const T *in, T *out, const double *sums,
                        hipStream_t s) {
  if (sizeof(T) == 4 && ((uintptr_t)in % 16) == 0 && ((uintptr_t)out % 16) == 0) {
    bool quads = true;
    i64 nq = 0;
    for (int k = 0; k < gin.d; k++) {
      quads = quads && (gin.fd[k][0] % 4 == 0) && (gin.foff[k] % 4 == 0);
      nq += permute_quads(gin, k);
    }
    if (quads) {
      hipLaunchKernelGGL(k_vel_permute4, dim3(blocks_for(nq)), dim3(kBlock), 0, s, gin, gout,
                         (const float *)in, (float *)out, sums);
      return;
    }
  }
  i64 np = 0;
  for (int k = 0; k < gin.d; k++) np += permute_pairs(gin, k);
  // pair loads and stores need the buffer itself aligned to a pair
  const int in_al = ((uintptr_t)in % (2 * sizeof(T))) == 0;
  const int out_al = ((uintptr_t)out % (2 * sizeof(T))) == 0;
  hipLaunchKernelGGL(k_vel_permute<T>, dim3(blocks_for(np)), dim3(kBlock), 0, s, gin, gout, in,
                     out, sums, in_al, out_al);
}
template void launch_vel_permute<float>(const Geo &, const Geo &, const float *, float *,
                                        const double *, hipStream_t);
template void launch_vel_permute<double>(const Geo &, const Geo &, const double *, double *,
                                         const double *, hipStream_t);

// ------------------------------------------------------------------------
// velocity multigrid (Appendix C)
// ------------------------------------------------------------------------

// one colour of multicolour Gauss-Seidel for component K: faces with
// (i0 + i1 + i2) % 2 == colour.  Thread t covers one face of that colour:
// i0 = 2 * (t mod n0/2) + parity.  Same-colour faces do not couple, so the
// in-place update is race-free.
// colour mapping shared by the Gauss-Seidel kernels: thread t -> (tx, row)
// with tx < ceil(n0/2); i0 = 2 tx + parity (odd n0 occurs only on no-slip x
// axes at the coarsest level; periodic axes are even on every level)
__device__ __forceinline__ bool colour_cell(const Geo &g, i64 t, int colour, int i[3]) {
  const unsigned hx = (unsigned)(g.n[0] + 1) >> 1;
  const i64 rows = (i64)g.n[1] * g.n[2];
  if (t >= (i64)hx * rows) return false;
  const unsigned u = (unsigned)t;
  const unsigned q = u / hx;
  const int tx = (int)(u - q * hx);
  i[2] = (int)(q / (unsigned)g.n[1]);
  i[1] = (int)(q - (unsigned)i[2] * (unsigned)g.n[1]);
  i[0] = 2 * tx + ((i[1] + i[2] + colour) & 1);
  return i[0] < g.n[0];
}
__host__ __device__ __forceinline__ i64 colour_threads(const Geo &g) {
  return (i64)((g.n[0] + 1) >> 1) * g.n[1] * g.n[2];
}

// Gauss-Seidel update of one velocity face (component k, cell index i).
// Z != 0: a pass of the first sweep from a zero iterate whose memory has not
// been cleared (Z = 3 colour 0, Z = 1 colour 1; the loads a_row skips for
// that Z are the values not yet written in that sweep).
template <typename T, int DIM, int Z = 0>
__device__ __forceinline__ void gs_point(const Geo &g, int k, const int i[3],
                                         const T *__restrict__ alpha, const T *__restrict__ muc,
                                         const T *__restrict__ mue, const T *__restrict__ lam,
                                         const T *__restrict__ rhs, T *__restrict__ phi) {
  const i64 fq = fidx3(g, k, i);
  if (low_wall(g, k, i)) {
    if (Z) phi[fq] = (T)0;  // wall faces hold zero; the first sweep writes them
    return;
  }
  T Au, dg;
  a_row<T, DIM, Z>(g, k, i, phi, alpha, muc, mue, lam, Au, dg);
  if (Z) {
    phi[fq] = (T)0 + (rhs[fq] - Au) / dg;
    if (g.ns[k] && i[k] + 1 == g.n[k]) {
      int t[3] = {i[0], i[1], i[2]};
      t[k] = g.n[k];
      phi[fidx3(g, k, t)] = (T)0;
    }
  } else {
    phi[fq] += (rhs[fq] - Au) / dg;
  }
}

// one face of one colour of the velocity Gauss-Seidel sweep
template <typename T, int DIM>
__device__ __forceinline__ void vel_gs_elem(const Geo &g, int k, int colour, i64 t,
                                            const T *__restrict__ alpha, const T *__restrict__ muc,
                                            const T *__restrict__ mue, const T *__restrict__ lam,
                                            const T *__restrict__ rhs, T *__restrict__ phi) {
  int i[3];
  if (!colour_cell(g, t, colour, i)) return;
  gs_point<T, DIM>(g, k, i, alpha, muc, mue, lam, rhs, phi);
}

template <typename T, int DIM, int K, int Z>
__global__ void k_vel_gs(Geo g, int colour, const T *__restrict__ alpha,
                         const T *__restrict__ muc, const T *__restrict__ mue,
                         const T *__restrict__ lam, const T *__restrict__ rhs,
                         T *__restrict__ phi) {
  int tx, i[3];
  if (!box_thread(g, (g.n[0] + 1) >> 1, tx, i[1], i[2])) return;
  i[0] = 2 * tx + ((i[1] + i[2] + colour) & 1);
  if (i[0] < g.n[0]) gs_point<T, DIM, Z>(g, K, i, alpha, muc, mue, lam, rhs, phi);
}

bool gs_first_ok(const Geo &g) {
  // the colouring must hold across periodic wraps: every extent even
  for (int a = 0; a < g.d; a++)
    if (g.n[a] & 1) return false;
  return true;
}

template <typename T>
void launch_vel_gs(const Geo &g, int k, int colour, int first, const T *alpha, const T *muc,
                   const T *mue, const T *lam, const T *rhs, T *phi, hipStream_t s) {
  const dim3 nb = box_blocks(g, (g.n[0] + 1) >> 1);
  const int z = first ? (colour == 0 ? 3 : 1) : 0;
#define GS_CASE(D, KK, ZZ)                                                                     \
  hipLaunchKernelGGL((k_vel_gs<T, D, KK, ZZ>), nb, dim3(kBlock), 0, s, g, colour, alpha, muc, \
                     mue, lam, rhs, phi)
#define GS_Z(D, KK)           \
  if (z == 0) GS_CASE(D, KK, 0); \
  else if (z == 1) GS_CASE(D, KK, 1); \
  else GS_CASE(D, KK, 3)
  if (g.d == 3) {
    if (k == 0) { GS_Z(3, 0); }
    else if (k == 1) { GS_Z(3, 1); }
    else { GS_Z(3, 2); }
  } else {
    if (k == 0) { GS_Z(2, 0); }
    else { GS_Z(2, 1); }
  }
#undef GS_Z
#undef GS_CASE
}

// The velocity rows of all components at cell i from their loaded values:
// V[c][0] = u_c at i, V[c][1 + 2a] at i + e_a, V[c][2 + 2a] at i - e_a
// (wall clamps applied), X[c][k] = u_c at i + e_c - e_k, mc / lc = mu / lam
// at i and at i - e_k, E0[m] = edge family m at i and E1[m][a] at i + e_a,
// rh / alr = rhs and alpha of the rows, pg = the pressure gradients, fq = the
// rows' face indices; each row runs the arithmetic of a_row_core, as the
// smoother does, and res = rh - A u (- pg) is stored at the low faces of i
// that are not wall faces.
template <typename T, int DIM, bool HL, bool HP>
__device__ __forceinline__ void vel_residual_rows(
    const Geo &g, const int i[3], const T (&V)[DIM][1 + 2 * DIM], const T (&X)[DIM][DIM],
    const T (&mc)[1 + DIM], const T (&lc)[1 + DIM], const T (&E0)[3], const T (&E1)[3][3],
    const T (&rh)[DIM], const T (&alr)[DIM], const T (&pg)[DIM], const int (&fq)[DIM],
    T *__restrict__ res) {
#pragma unroll
  for (int k = 0; k < DIM; k++) {
    if (low_wall(g, k, i)) continue;
    const T uf = V[k][0];
    T ua[3] = {0, 0, 0}, ub[3] = {0, 0, 0};
    T ulh_r[3] = {0, 0, 0}, ulh_l[3] = {0, 0, 0}, ull_r[3] = {0, 0, 0}, ull_l[3] = {0, 0, 0};
    T mhi[3] = {0, 0, 0}, mlo[3] = {0, 0, 0};
#pragma unroll
    for (int l = 0; l < DIM; l++) {
      if (l == k) continue;
      const int m = 3 - k - l;
      const bool top = g.ns[l] && (i[l] + 1 == g.n[l]);
      const bool bot = g.ns[l] && (i[l] == 0);
      // no-slip: odd ghost (zero wall value); free-slip: even ghost (no shear)
      ua[l] = top ? ((g.fs[l] & 2) ? uf : -uf) : V[k][1 + 2 * l];
      ub[l] = bot ? ((g.fs[l] & 1) ? uf : -uf) : V[k][2 + 2 * l];
      ulh_r[l] = V[l][1 + 2 * l];
      ulh_l[l] = X[l][k];
      ull_r[l] = V[l][0];
      ull_l[l] = V[l][2 + 2 * k];
      mhi[l] = E1[m][l];
      mlo[l] = E0[m];
    }
    T Au, dg;
    a_row_core<T, DIM>(g, k, i, uf, V[k][1 + 2 * k], V[k][2 + 2 * k], ua, ub, ulh_r, ulh_l, ull_r,
                       ull_l, mhi, mlo, mc[0], mc[1 + k], alr[k], HL, lc[0], lc[1 + k], Au,
                       dg);
    T r = rh[k] - Au;
    if (HP) r -= pg[k];
    res[fq[k]] = r;
  }
}

// res = rhs - A phi - G p (p may be null) at the low faces of cell i, all
// components.  The rows share most of their velocity values, so those are
// loaded once: per component c the value at i, at i +- e_a for every axis a,
// and at i + e_c - e_k for k != c (27 loads in 3D instead of 45), and the
// cell and edge viscosities around i likewise.  HA, HL, HP: alpha, the
// bulk coefficient and p are given (compile-time, so that no load sits in
// a branch and every load issues before the first row is evaluated).
template <typename T, int DIM, bool HA, bool HL, bool HP>
__device__ __forceinline__ void vel_residual_at(const Geo &g, const int i[3], i64 t,
                                                const T *__restrict__ alpha,
                                                const T *__restrict__ muc,
                                                const T *__restrict__ mue,
                                                const T *__restrict__ lam,
                                                const T *__restrict__ rhs,
                                                const T *__restrict__ phi,
                                                const T *__restrict__ p, T *__restrict__ res) {
  int ip[3] = {0, 0, 0}, im[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; a++) {
    ip[a] = up1(g, a, i[a]);
    im[a] = dn1(g, a, i[a]);
  }
  // Component c has no face at index n[a] along a wall axis a != c: that
  // load is clamped to i (the wall ghost replaces it).
  T V[DIM][1 + 2 * DIM], X[DIM][DIM];
#pragma unroll
  for (int c = 0; c < DIM; c++) {
    int q[3] = {i[0], i[1], i[2]};
    V[c][0] = phi[fidx3(g, c, q)];
#pragma unroll
    for (int a = 0; a < DIM; a++) {
      const bool top = a != c && g.ns[a] && (i[a] + 1 == g.n[a]);
      q[a] = top ? i[a] : ip[a];
      V[c][1 + 2 * a] = phi[fidx3(g, c, q)];
      q[a] = im[a];
      V[c][2 + 2 * a] = phi[fidx3(g, c, q)];
      q[a] = i[a];
    }
#pragma unroll
    for (int k = 0; k < DIM; k++) {
      X[c][k] = (T)0;
      if (k == c) continue;
      q[c] = ip[c];
      q[k] = im[k];
      X[c][k] = phi[fidx3(g, c, q)];
      q[c] = i[c];
      q[k] = i[k];
    }
  }
  // cell viscosity (and bulk coefficient) at i and at i - e_k
  T mc[1 + DIM], lc[1 + DIM];
  mc[0] = muc[t];
  lc[0] = HL ? lam[t] : (T)0;
#pragma unroll
  for (int k = 0; k < DIM; k++) {
    int q[3] = {i[0], i[1], i[2]};
    q[k] = im[k];
    const i64 cq = cidx3(g, q);
    mc[1 + k] = muc[cq];
    lc[1 + k] = HL ? lam[cq] : (T)0;
  }
  // edge family m at i (E0) and at i + e_a for the axes a != m (E1)
  T E0[3] = {0, 0, 0}, E1[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int m = (DIM == 3 ? 0 : 2); m < 3; m++) {
    E0[m] = mue[eidx3(g, m, i)];
#pragma unroll
    for (int a = 0; a < DIM; a++) {
      if (a == m) continue;
      int q[3] = {i[0], i[1], i[2]};
      q[a] = ip[a];
      E1[m][a] = mue[eidx3(g, m, q)];
    }
  }
  // the right-hand side and alpha of the d rows (and the pressures), loaded
  // with the rest before the first row is evaluated and stored
  T rh[DIM], alr[DIM], pg[DIM];
  int fq[DIM];
#pragma unroll
  for (int k = 0; k < DIM; k++) {
    fq[k] = fidx3(g, k, i);
    rh[k] = rhs[fq[k]];
    alr[k] = HA ? alpha[fq[k]] : (T)0;  // no alpha array: theta = 0
    pg[k] = (T)0;
    if (HP) {
      int l[3] = {i[0], i[1], i[2]};
      l[k] = im[k];
      pg[k] = (p[t] - p[cidx3(g, l)]) * (T)g.ih;
    }
  }
  vel_residual_rows<T, DIM, HL, HP>(g, i, V, X, mc, lc, E0, E1, rh, alr, pg, fq, res);
}

// Loads at (x, y, z) of a face, cell or edge array.  PER (every axis
// periodic): every array has the cells' extents, so the in-plane part of the
// index is written once for all of them and shared by the compiler.
template <bool PER, typename T>
__device__ __forceinline__ T face_at(const Geo &g, const T *__restrict__ u, int c, int x, int y,
                                     int z) {
  if (PER) return u[(int)g.foff[c] + (z * g.n[1] + y) * g.n[0] + xpos(g, g.n[0], x)];
  const int q[3] = {x, y, z};
  return u[fidx3(g, c, q)];
}
template <bool PER, typename T>
__device__ __forceinline__ T cell_at(const Geo &g, const T *__restrict__ u, int x, int y, int z) {
  const int q[3] = {x, y, z};
  return u[cidx3(g, q)];
}
template <bool PER, typename T>
__device__ __forceinline__ T edge_at(const Geo &g, const T *__restrict__ u, int m, int x, int y,
                                     int z) {
  if (PER) return u[(int)g.eoff[m] + (z * g.n[1] + y) * g.n[0] + x];
  const int q[3] = {x, y, z};
  return u[eidx3(g, m, q)];
}

// The 3D residual by columns: a thread takes the cells (x, y, z0 .. z0+nz-1)
// and carries from one plane to the next what the two share: u_c at z and
// z - 1, the diagonal values u_0(i + e_0 - e_2) and u_1(i + e_1 - e_2) (the
// x and y neighbours one plane down), u_2 at i - e_0 and i - e_1 (the
// diagonal values i + e_2 - e_k one plane up), mu and lam at z - 1, the
// edges of families 0 and 1 at z, and p at z - 1.  A cell then loads 30 values
// instead of 43; each value and each row is the one vel_residual_at forms, so
// the result is bitwise the same.
template <typename T, bool HA, bool HL, bool HP, bool PER>
__global__ void k_vel_residual_col(Geo g, int nz, const T *__restrict__ alpha,
                                   const T *__restrict__ muc, const T *__restrict__ mue,
                                   const T *__restrict__ lam, const T *__restrict__ rhs,
                                   const T *__restrict__ phi, const T *__restrict__ p,
                                   T *__restrict__ res) {
  int w, i[3], zb;
  if (!box_thread(g, g.n[0], w, i[1], zb)) return;
  i[0] = split_x(g, w);
  const int x = i[0], y = i[1];
  const int z0 = zb * nz, z1 = min(z0 + nz, g.n[2]);
  const int xp = up1(g, 0, x), xm = dn1(g, 0, x), yp = up1(g, 1, y), ym = dn1(g, 1, y);
  // upper neighbours of the components without a face at n along a wall axis
  const int xpc = (!PER && g.ns[0] && x + 1 == g.n[0]) ? x : xp;  // components 1, 2 along x
  const int ypc = (!PER && g.ns[1] && y + 1 == g.n[1]) ? y : yp;  // components 0, 2 along y
  const T ih = (T)g.ih;
  // carried values, primed for z0
  const int zm0 = dn1(g, 2, z0);
  T cu[3], cum[3];
#pragma unroll
  for (int c = 0; c < 3; c++) {
    cu[c] = face_at<PER>(g, phi, c, x, y, z0);
    cum[c] = face_at<PER>(g, phi, c, x, y, zm0);
  }
  T cx02 = face_at<PER>(g, phi, 0, xp, y, zm0), cx12 = face_at<PER>(g, phi, 1, x, yp, zm0);
  T cv22 = face_at<PER>(g, phi, 2, xm, y, z0), cv24 = face_at<PER>(g, phi, 2, x, ym, z0);
  T cmz = cell_at<PER>(g, muc, x, y, zm0), clz = HL ? cell_at<PER>(g, lam, x, y, zm0) : (T)0;
  T ce0 = edge_at<PER>(g, mue, 0, x, y, z0), ce1 = edge_at<PER>(g, mue, 1, x, y, z0);
  T cpz = HP ? cell_at<PER>(g, p, x, y, zm0) : (T)0;
  for (int z = z0; z < z1; z++) {
    i[2] = z;
    const int zp = up1(g, 2, z);
    const int zpc = (!PER && g.ns[2] && z + 1 == g.n[2]) ? z : zp;  // components 0, 1 along z
    T V[3][7], X[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    V[0][1] = face_at<PER>(g, phi, 0, xp, y, z);
    V[0][2] = face_at<PER>(g, phi, 0, xm, y, z);
    V[0][3] = face_at<PER>(g, phi, 0, x, ypc, z);
    V[0][4] = face_at<PER>(g, phi, 0, x, ym, z);
    V[0][5] = face_at<PER>(g, phi, 0, x, y, zpc);
    V[1][1] = face_at<PER>(g, phi, 1, xpc, y, z);
    V[1][2] = face_at<PER>(g, phi, 1, xm, y, z);
    V[1][3] = face_at<PER>(g, phi, 1, x, yp, z);
    V[1][4] = face_at<PER>(g, phi, 1, x, ym, z);
    V[1][5] = face_at<PER>(g, phi, 1, x, y, zpc);
    V[2][1] = face_at<PER>(g, phi, 2, xpc, y, z);
    V[2][3] = face_at<PER>(g, phi, 2, x, ypc, z);
    V[2][5] = face_at<PER>(g, phi, 2, x, y, zp);
    X[0][1] = face_at<PER>(g, phi, 0, xp, ym, z);
    X[1][0] = face_at<PER>(g, phi, 1, xm, yp, z);
    X[2][0] = face_at<PER>(g, phi, 2, xm, y, zp);
    X[2][1] = face_at<PER>(g, phi, 2, x, ym, zp);
    T mc[4], lc[4] = {0, 0, 0, 0};
    mc[0] = cell_at<PER>(g, muc, x, y, z);
    mc[1] = cell_at<PER>(g, muc, xm, y, z);
    mc[2] = cell_at<PER>(g, muc, x, ym, z);
    if (HL) {
      lc[0] = cell_at<PER>(g, lam, x, y, z);
      lc[1] = cell_at<PER>(g, lam, xm, y, z);
      lc[2] = cell_at<PER>(g, lam, x, ym, z);
    }
    T E0[3], E1[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    E0[2] = edge_at<PER>(g, mue, 2, x, y, z);
    E1[0][1] = edge_at<PER>(g, mue, 0, x, yp, z);
    E1[0][2] = edge_at<PER>(g, mue, 0, x, y, zp);
    E1[1][0] = edge_at<PER>(g, mue, 1, xp, y, z);
    E1[1][2] = edge_at<PER>(g, mue, 1, x, y, zp);
    E1[2][0] = edge_at<PER>(g, mue, 2, xp, y, z);
    E1[2][1] = edge_at<PER>(g, mue, 2, x, yp, z);
    T rh[3], alr[3], pg[3] = {0, 0, 0};
    int fq[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
      fq[k] = PER ? (int)g.foff[k] + (z * g.n[1] + y) * g.n[0] + xpos(g, g.n[0], x)
                  : fidx3(g, k, i);
      rh[k] = rhs[fq[k]];
      alr[k] = HA ? alpha[fq[k]] : (T)0;
    }
    T pc0 = (T)0;
    if (HP) {
      pc0 = cell_at<PER>(g, p, x, y, z);
      pg[0] = (pc0 - cell_at<PER>(g, p, xm, y, z)) * ih;
      pg[1] = (pc0 - cell_at<PER>(g, p, x, ym, z)) * ih;
      pg[2] = (pc0 - cpz) * ih;
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
      V[c][0] = cu[c];
      V[c][6] = cum[c];
    }
    X[0][2] = cx02;
    X[1][2] = cx12;
    V[2][2] = cv22;
    V[2][4] = cv24;
    mc[3] = cmz;
    lc[3] = clz;
    E0[0] = ce0;
    E0[1] = ce1;
    vel_residual_rows<T, 3, HL, HP>(g, i, V, X, mc, lc, E0, E1, rh, alr, pg, fq, res);
    // what plane z + 1 shares with this one (the last plane's values go unused)
#pragma unroll
    for (int c = 0; c < 3; c++) {
      cum[c] = V[c][0];
      cu[c] = V[c][5];
    }
    cx02 = V[0][1];
    cx12 = V[1][3];
    cv22 = X[2][0];
    cv24 = X[2][1];
    cmz = mc[0];
    clz = lc[0];
    ce0 = E1[0][2];
    ce1 = E1[1][2];
    cpz = pc0;
  }
}

// The same residual one row at a time through a_row (fewer registers: the
// form the single-workgroup coarse tail uses).
template <typename T, int DIM>
__device__ __forceinline__ void vel_residual_rows_at(const Geo &g, const int i[3], i64 t,
                                                     const T *__restrict__ alpha,
                                                     const T *__restrict__ muc,
                                                     const T *__restrict__ mue,
                                                     const T *__restrict__ lam,
                                                     const T *__restrict__ rhs,
                                                     const T *__restrict__ phi,
                                                     const T *__restrict__ p,
                                                     T *__restrict__ res) {
#pragma unroll
  for (int k = 0; k < DIM; k++) {
    if (low_wall(g, k, i)) continue;
    T Au, dg;
    a_row<T, DIM>(g, k, i, phi, alpha, muc, mue, lam, Au, dg);
    const i64 fq = fidx3(g, k, i);
    T r = rhs[fq] - Au;
    if (p) {
      int l[3] = {i[0], i[1], i[2]};
      l[k] = dn1(g, k, i[k]);
      r -= (p[t] - p[cidx3(g, l)]) * (T)g.ih;
    }
    res[fq] = r;
  }
}

template <typename T, int DIM>
__device__ __forceinline__ void vel_residual_elem(const Geo &g, i64 t, const T *__restrict__ alpha,
                                                  const T *__restrict__ muc,
                                                  const T *__restrict__ mue,
                                                  const T *__restrict__ lam,
                                                  const T *__restrict__ rhs,
                                                  const T *__restrict__ phi,
                                                  const T *__restrict__ p, T *__restrict__ res) {
  if (t >= g.ncell) return;
  int i[3];
  cell_of(g, t, i);
  vel_residual_rows_at<T, DIM>(g, i, t, alpha, muc, mue, lam, rhs, phi, p, res);
}

template <typename T, int DIM, bool HA, bool HL, bool HP>
__global__ void k_vel_residual(Geo g, const T *__restrict__ alpha, const T *__restrict__ muc,
                               const T *__restrict__ mue, const T *__restrict__ lam,
                               const T *__restrict__ rhs, const T *__restrict__ phi,
                               const T *__restrict__ p, T *__restrict__ res) {
  int w, i[3];
  if (!box_thread(g, g.n[0], w, i[1], i[2])) return;
  i[0] = split_x(g, w);
  vel_residual_at<T, DIM, HA, HL, HP>(g, i, cidx3(g, i), alpha, muc, mue, lam, rhs, phi, p, res);
}

template <typename T, int DIM, bool HA, bool HL>
static void launch_vel_residual_hp(const Geo &g, const T *alpha, const T *muc, const T *mue,
                                   const T *lam, const T *rhs, const T *phi, const T *p, T *res,
                                   hipStream_t s) {
  // by columns in FP32 only: the FP64 column kernel exceeds the register file
  if constexpr (DIM == 3 && sizeof(T) == 4) {
    if (g.col > 0) {
      dim3 nb = box_blocks(g, g.n[0]);
      nb.y = (unsigned)((g.n[2] + g.col - 1) / g.col);
      const bool per = !g.ns[0] && !g.ns[1] && !g.ns[2];
#define COL_CASE(HPV, PERV)                                                                     \
  hipLaunchKernelGGL((k_vel_residual_col<T, HA, HL, HPV, PERV>), nb, dim3(kBlock), 0, s, g, g.col, \
                     alpha, muc, mue, lam, rhs, phi, p, res)
      if (p) {
        if (per) COL_CASE(true, true);
        else COL_CASE(true, false);
      } else {
        if (per) COL_CASE(false, true);
        else COL_CASE(false, false);
      }
#undef COL_CASE
      return;
    }
  }
  if (p)
    hipLaunchKernelGGL((k_vel_residual<T, DIM, HA, HL, true>), box_blocks(g, g.n[0]),
                       dim3(kBlock), 0, s, g, alpha, muc, mue, lam, rhs, phi, p, res);
  else
    hipLaunchKernelGGL((k_vel_residual<T, DIM, HA, HL, false>), box_blocks(g, g.n[0]),
                       dim3(kBlock), 0, s, g, alpha, muc, mue, lam, rhs, phi, p, res);
}

template <typename T, int DIM>
static void launch_vel_residual_d(const Geo &g, const T *alpha, const T *muc, const T *mue,
                                  const T *lam, const T *rhs, const T *phi, const T *p, T *res,
                                  hipStream_t s) {
  if (alpha && lam)
    launch_vel_residual_hp<T, DIM, true, true>(g, alpha, muc, mue, lam, rhs, phi, p, res, s);
  else if (alpha)
    launch_vel_residual_hp<T, DIM, true, false>(g, alpha, muc, mue, lam, rhs, phi, p, res, s);
  else if (lam)
    launch_vel_residual_hp<T, DIM, false, true>(g, alpha, muc, mue, lam, rhs, phi, p, res, s);
  else
    launch_vel_residual_hp<T, DIM, false, false>(g, alpha, muc, mue, lam, rhs, phi, p, res, s);
}

template <typename T>
void launch_vel_residual(const Geo &g, const T *alpha, const T *muc, const T *mue, const T *lam,
                         const T *rhs, const T *phi, const T *p, T *res, hipStream_t s) {
  if (g.d == 3)
    launch_vel_residual_d<T, 3>(g, alpha, muc, mue, lam, rhs, phi, p, res, s);
  else
    launch_vel_residual_d<T, 2>(g, alpha, muc, mue, lam, rhs, phi, p, res, s);
}

// face restriction (Appendix C): normal weights 1/4, 1/2, 1/4 at fine faces
// 2I-1, 2I, 2I+1 times the mean over the 2^(d-1) fine faces along the
// tangential axes (2D: the printed 6-point stencil; 3D: 12 points)
template <typename T, int DIM>
__device__ __forceinline__ void face_restrict_elem(const Geo &gf, const Geo &gc, i64 t,
                                                   const T *__restrict__ rf, T *__restrict__ rc) {
  if (t >= gc.ncell) return;
  int I[3];
  cell_of(gc, t, I);
  const T wn[3] = {(T)0.25, (T)0.5, (T)0.25};
  const T wt = (DIM == 3) ? (T)0.25 : (T)0.5;
#pragma unroll
  for (int k = 0; k < DIM; k++) {
    if (low_wall(gc, k, I)) continue;
    int tax[2] = {0, 0}, nt = 0;
    for (int b = 0; b < DIM; b++)
      if (b != k) tax[nt++] = b;
    T s = 0;
    for (int a = -1; a <= 1; a++) {
      T acc = 0;
      for (int o2 = 0; o2 < (DIM == 3 ? 2 : 1); o2++)
        for (int o1 = 0; o1 < 2; o1++) {
          int f[3] = {2 * I[0], 2 * I[1], DIM == 3 ? 2 * I[2] : 0};
          int fk = 2 * I[k] + a;
          if (!gf.ns[k]) {
            if (fk < 0) fk += gf.n[k];
            if (fk >= gf.n[k]) fk -= gf.n[k];
          }
          f[k] = fk;
          f[tax[0]] += o1;
          if (DIM == 3) f[tax[1]] += o2;
          acc += rf[fidx3(gf, k, f)];
        }
      s += wn[a + 1] * wt * acc;
    }
    rc[fidx3(gc, k, I)] = s;
  }
}

template <typename T, int DIM>
__global__ void k_face_restrict(Geo gf, Geo gc, const T *__restrict__ rf, T *__restrict__ rc) {
  face_restrict_elem<T, DIM>(gf, gc, (i64)blockIdx.x * blockDim.x + threadIdx.x, rf, rc);
}

template <typename T>
void launch_face_restrict(const Geo &gf, const Geo &gc, const T *rf, T *rc, hipStream_t s) {
  if (gc.d == 3)
    hipLaunchKernelGGL((k_face_restrict<T, 3>), dim3(blocks_for(gc.ncell)), dim3(kBlock), 0, s, gf,
                       gc, rf, rc);
  else
    hipLaunchKernelGGL((k_face_restrict<T, 2>), dim3(blocks_for(gc.ncell)), dim3(kBlock), 0, s, gf,
                       gc, rf, rc);
}

// tangential prolongation weights (Appendix C): 3/4 on the parent coarse
// face, 1/4 on the next one away from the parent's centre; at a no-slip wall
// the missing neighbour is the odd reflection -phi(J), at a free-slip wall
// the even one
__device__ __forceinline__ void tang_w(const Geo &gc, int a, int j, int idx[2], double w[2]) {
  const int J = j >> 1;
  const int Jn = (j & 1) ? J + 1 : J - 1;
  idx[0] = J;
  w[0] = 0.75;
  if (gc.ns[a] && (Jn < 0 || Jn >= gc.n[a])) {
    idx[1] = J;
    const int end = (Jn < 0) ? 1 : 2;  // low or high end of axis a
    w[1] = (gc.fs[a] & end) ? 0.25 : -0.25;
  } else {
    int jj = Jn;
    if (!gc.ns[a]) {
      if (jj < 0) jj += gc.n[a];
      if (jj >= gc.n[a]) jj -= gc.n[a];
    }
    idx[1] = jj;
    w[1] = 0.25;
  }
}

// Fixed taps, unconditional loads: two along the normal (weights 1 and 0 on
// an even fine index, 1/2 and 1/2 on an odd one) times two per tangential
// axis (3/4 and +-1/4, the odd wall reflection giving -1/4 on J itself).
template <typename T, int DIM>
__device__ __forceinline__ void face_prolong_at(const Geo &gc, const Geo &gf, const int f[3],
                                                const T *__restrict__ ec, T *__restrict__ phif) {
#pragma unroll
  for (int k = 0; k < DIM; k++) {
    if (low_wall(gf, k, f)) continue;
    const int fk = f[k];
    int nidx[2];
    nidx[0] = fk >> 1;
    nidx[1] = (fk + 1) >> 1;
    if (!gc.ns[k] && nidx[1] == gc.n[k]) nidx[1] = 0;
    const T nw[2] = {(fk & 1) ? (T)0.5 : (T)1, (fk & 1) ? (T)0.5 : (T)0};
    const int ta = (k == 0) ? 1 : 0;
    const int tb = (k == 2) ? 1 : 2;
    int t0i[2], t1i[2] = {0, 0};
    double t0w[2], t1w[2] = {1.0, 0.0};
    tang_w(gc, ta, f[ta], t0i, t0w);
    if (DIM == 3) tang_w(gc, tb, f[tb], t1i, t1w);
    T s = 0;
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b0 = 0; b0 < 2; b0++)
#pragma unroll
        for (int b1 = 0; b1 < (DIM == 3 ? 2 : 1); b1++) {
          int cf[3] = {0, 0, 0};
          cf[k] = nidx[a];
          cf[ta] = t0i[b0];
          if (DIM == 3) cf[tb] = t1i[b1];
          s += nw[a] * (T)t0w[b0] * (T)t1w[b1] * ec[fidx3(gc, k, cf)];
        }
    phif[fidx3(gf, k, f)] += s;
  }
}

template <typename T, int DIM>
__device__ __forceinline__ void face_prolong_elem(const Geo &gc, const Geo &gf, i64 t,
                                                  const T *__restrict__ ec, T *__restrict__ phif) {
  if (t >= gf.ncell) return;
  int f[3];
  cell_of(gf, t, f);
  face_prolong_at<T, DIM>(gc, gf, f, ec, phif);
}

// Coarse index J of a tangential tap: periodic axes wrap; on a wall axis an
// index past the end is clamped (that value is replaced by the wall ghost).
__device__ __forceinline__ int tap_index(const Geo &gc, int a, int J) {
  if (!gc.ns[a]) return (J < 0) ? J + gc.n[a] : (J >= gc.n[a]) ? J - gc.n[a] : J;
  return (J < 0) ? 0 : (J >= gc.n[a]) ? gc.n[a] - 1 : J;
}

// Prolongation by coarse cell.  The thread of coarse cell C adds the
// correction to the low faces of its 2^d fine cells.  For component k those
// faces use the 2 (normal) x 3 x 3 (tangential offsets -1, 0, +1) coarse
// values around C, loaded once.  At a wall end the tap past the wall is
// (+1 free-slip, -1 no-slip) times the tap at C, so every fine face takes
// weight 3/4 at offset 0 and 1/4 on its own side, with the same products and
// order of operations as face_prolong_at (the sign moves through the
// products exactly).
template <typename T, int DIM>
__global__ void k_face_prolong_add(Geo gc, Geo gf, const T *__restrict__ ec,
                                   T *__restrict__ phif) {
  int C[3];
  if (!box_thread(gc, gc.n[0], C[0], C[1], C[2])) return;
  constexpr int NB = (DIM == 3) ? 3 : 1;
  constexpr int NF = (DIM == 3) ? 8 : 4;
  // Loads (coarse taps and the fine values the thread updates) before the
  // stores: a store to phif would otherwise order every later load of phif
  // after it.  FP32: all components' loads first; FP64 (twice the
  // registers): component by component.
  constexpr bool kHoist = sizeof(T) == 4;
  T cv[DIM][2][3][NB];
  T old[DIM][NF];
  auto load = [&](int k) {
    const int ta = (k == 0) ? 1 : 0;
    const int tb = (k == 2) ? 1 : 2;
    int cf[3] = {0, 0, 0};
#pragma unroll
    for (int n = 0; n < 2; n++) {
      cf[k] = C[k] + n;
      if (!gc.ns[k] && cf[k] == gc.n[k]) cf[k] = 0;
#pragma unroll
      for (int s0 = 0; s0 < 3; s0++) {
        cf[ta] = tap_index(gc, ta, C[ta] + s0 - 1);
#pragma unroll
        for (int s1 = 0; s1 < NB; s1++) {
          if (DIM == 3) cf[tb] = tap_index(gc, tb, C[tb] + s1 - 1);
          cv[k][n][s0][s1] = ec[fidx3(gc, k, cf)];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NF; q++) {
      int f[3] = {2 * C[0] + (q & 1), 2 * C[1] + ((q >> 1) & 1),
                  (DIM == 3) ? 2 * C[2] + ((q >> 2) & 1) : 0};
      old[k][q] = low_wall(gf, k, f) ? (T)0 : phif[fidx3(gf, k, f)];
    }
  };
  if (kHoist) {
#pragma unroll
    for (int k = 0; k < DIM; k++) load(k);
  }
#pragma unroll
  for (int k = 0; k < DIM; k++) {
    if (!kHoist) load(k);
    const int ta = (k == 0) ? 1 : 0;
    const int tb = (k == 2) ? 1 : 2;
    // wall ghosts, axis ta then tb (a corner takes both signs)
    if (gc.ns[ta]) {
      const T slo = (gc.fs[ta] & 1) ? (T)1 : (T)-1, shi = (gc.fs[ta] & 2) ? (T)1 : (T)-1;
      const bool lo = C[ta] == 0, hi = C[ta] + 1 == gc.n[ta];
#pragma unroll
      for (int n = 0; n < 2; n++)
#pragma unroll
        for (int s1 = 0; s1 < NB; s1++) {
          if (lo) cv[k][n][0][s1] = slo * cv[k][n][1][s1];
          if (hi) cv[k][n][2][s1] = shi * cv[k][n][1][s1];
        }
    }
    if (DIM == 3 && gc.ns[tb]) {
      const T slo = (gc.fs[tb] & 1) ? (T)1 : (T)-1, shi = (gc.fs[tb] & 2) ? (T)1 : (T)-1;
      const bool lo = C[tb] == 0, hi = C[tb] + 1 == gc.n[tb];
#pragma unroll
      for (int n = 0; n < 2; n++)
#pragma unroll
        for (int s0 = 0; s0 < 3; s0++) {
          if (lo) cv[k][n][s0][0] = slo * cv[k][n][s0][1];
          if (hi) cv[k][n][s0][NB - 1] = shi * cv[k][n][s0][1];
        }
    }
#pragma unroll
    for (int o2 = 0; o2 < (DIM == 3 ? 2 : 1); o2++)
#pragma unroll
      for (int o1 = 0; o1 < 2; o1++)
#pragma unroll
        for (int o0 = 0; o0 < 2; o0++) {
          const int o[3] = {o0, o1, o2};
          int f[3] = {2 * C[0] + o0, 2 * C[1] + o1, (DIM == 3) ? 2 * C[2] + o2 : 0};
          if (low_wall(gf, k, f)) continue;
          const int ok = o[k];
          const T nw[2] = {ok ? (T)0.5 : (T)1, ok ? (T)0.5 : (T)0};
          const int ns[2] = {0, ok};                  // normal slots of the two taps
          const int s0i[2] = {1, o[ta] ? 2 : 0};      // tangential slots along ta
          const int s1i[2] = {(DIM == 3) ? 1 : 0, o[tb] ? 2 : 0};
          const double w0[2] = {0.75, 0.25};
          const double w1[2] = {(DIM == 3) ? 0.75 : 1.0, (DIM == 3) ? 0.25 : 0.0};
          T sum = 0;
#pragma unroll
          for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b0 = 0; b0 < 2; b0++)
#pragma unroll
              for (int b1 = 0; b1 < (DIM == 3 ? 2 : 1); b1++)
                sum += nw[a] * (T)w0[b0] * (T)w1[b1] * cv[k][ns[a]][s0i[b0]][s1i[b1]];
          phif[fidx3(gf, k, f)] = old[k][o0 + 2 * o1 + 4 * o2] + sum;
        }
  }
}

template <typename T>
void launch_face_prolong_add(const Geo &gc, const Geo &gf, const T *ec, T *phif, hipStream_t s) {
  if (gf.d == 3)
    hipLaunchKernelGGL((k_face_prolong_add<T, 3>), box_blocks(gc, gc.n[0]), dim3(kBlock), 0, s,
                       gc, gf, ec, phif);
  else
    hipLaunchKernelGGL((k_face_prolong_add<T, 2>), box_blocks(gc, gc.n[0]), dim3(kBlock), 0, s,
                       gc, gf, ec, phif);
}

// ------------------------------------------------------------------------
// pressure multigrid: L_rho = D beta G with zero flux through walls
// ------------------------------------------------------------------------

// Z (first red-black sweep from a zero iterate whose memory has not been
// cleared): bit 0 reads the cell itself as zero, bit 1 its neighbours (the
// other colour) as zero.
template <typename T, int DIM, int Z = 0>
__device__ __forceinline__ void p_row(const Geo &g, const int i[3], const T *__restrict__ beta,
                                      const T *__restrict__ p, T &Lp, T &diag) {
  const T ih = (T)g.ih;
  const T pc = (Z & 1) ? (T)0 : p[cidx3(g, i)];
  T s = 0, dg = 0;
#pragma unroll
  for (int k = 0; k < DIM; k++) {
    // flux through the high face (index i+1) and the low face (index i); a
    // wall face carries none.  Loads use in-range indices unconditionally and
    // the wall cases are selected afterwards.
    const bool wr = g.ns[k] && (i[k] + 1 == g.n[k]);
    const bool wl = g.ns[k] && (i[k] == 0);
    int f[3] = {i[0], i[1], i[2]}, c[3] = {i[0], i[1], i[2]};
    f[k] = wr ? i[k] : up1(g, k, i[k]);
    c[k] = f[k];
    const T br = beta[fidx3(g, k, f)];
    const T pr = (Z & 2) ? (T)0 : p[cidx3(g, c)];
    c[k] = dn1(g, k, i[k]);
    const T bl = beta[fidx3(g, k, i)];
    const T pl = (Z & 2) ? (T)0 : p[cidx3(g, c)];
    const T fr = wr ? (T)0 : br * ((pr - pc) * ih);
    const T fl = wl ? (T)0 : bl * ((pc - pl) * ih);
    dg -= (wr ? (T)0 : br) + (wl ? (T)0 : bl);
    s += (fr - fl) * ih;
  }
  Lp = s;
  diag = dg * (ih * ih);
}

template <typename T, int DIM, int Z = 0>
__device__ __forceinline__ void p_gs_elem(const Geo &g, int colour, i64 t,
                                          const T *__restrict__ beta, const T *__restrict__ rhs,
                                          T *__restrict__ phi) {
  int i[3];
  if (!colour_cell(g, t, colour, i)) return;
  T Lp, dg;
  p_row<T, DIM, Z>(g, i, beta, phi, Lp, dg);
  const i64 c = cidx3(g, i);
  if (Z)
    phi[c] = (T)0 + (rhs[c] - Lp) / dg;
  else
    phi[c] += (rhs[c] - Lp) / dg;
}

template <typename T, int DIM, int Z>
__global__ void k_p_gs(Geo g, int colour, const T *__restrict__ beta, const T *__restrict__ rhs,
                       T *__restrict__ phi) {
  p_gs_elem<T, DIM, Z>(g, colour, (i64)blockIdx.x * blockDim.x + threadIdx.x, beta, rhs, phi);
}

template <typename T>
void launch_p_gs(const Geo &g, int colour, int first, const T *beta, const T *rhs, T *phi,
                 hipStream_t s) {
  const unsigned nb = blocks_for(colour_threads(g));
  const int z = first ? (colour == 0 ? 3 : 1) : 0;
#define PGS(D, ZZ) \
  hipLaunchKernelGGL((k_p_gs<T, D, ZZ>), dim3(nb), dim3(kBlock), 0, s, g, colour, beta, rhs, phi)
  if (g.d == 3) {
    if (z == 0) PGS(3, 0);
    else if (z == 1) PGS(3, 1);
    else PGS(3, 3);
  } else {
    if (z == 0) PGS(2, 0);
    else if (z == 1) PGS(2, 1);
    else PGS(2, 3);
  }
#undef PGS
}

template <typename T, int DIM>
__device__ __forceinline__ void p_residual_elem(const Geo &g, i64 t, const T *__restrict__ beta,
                                                const T *__restrict__ rhs,
                                                const T *__restrict__ phi, T *__restrict__ res) {
  if (t >= g.ncell) return;
  int i[3];
  cell_of(g, t, i);
  T Lp, dg;
  p_row<T, DIM>(g, i, beta, phi, Lp, dg);
  res[t] = rhs[t] - Lp;
}

template <typename T, int DIM>
__global__ void k_p_residual(Geo g, const T *__restrict__ beta, const T *__restrict__ rhs,
                             const T *__restrict__ phi, T *__restrict__ res) {
  p_residual_elem<T, DIM>(g, (i64)blockIdx.x * blockDim.x + threadIdx.x, beta, rhs, phi, res);
}

template <typename T>
void launch_p_residual(const Geo &g, const T *beta, const T *rhs, const T *phi, T *res,
                       hipStream_t s) {
  if (g.d == 3)
    hipLaunchKernelGGL((k_p_residual<T, 3>), dim3(blocks_for(g.ncell)), dim3(kBlock), 0, s, g, beta,
                       rhs, phi, res);
  else
    hipLaunchKernelGGL((k_p_residual<T, 2>), dim3(blocks_for(g.ncell)), dim3(kBlock), 0, s, g, beta,
                       rhs, phi, res);
}

template <typename T>
__device__ __forceinline__ void cell_restrict_elem(const Geo &gf, const Geo &gc, i64 t,
                                                   const T *__restrict__ rf, T *__restrict__ rc) {
  if (t >= gc.ncell) return;
  int I[3];
  cell_of(gc, t, I);
  const int d = gc.d;
  T s = 0;
  for (int o2 = 0; o2 < (d == 3 ? 2 : 1); o2++)
    for (int o1 = 0; o1 < 2; o1++)
      for (int o0 = 0; o0 < 2; o0++) {
        int f[3] = {2 * I[0] + o0, 2 * I[1] + o1, d == 3 ? 2 * I[2] + o2 : 0};
        s += rf[cidx3(gf, f)];
      }
  rc[t] = s / (T)(1 << d);
}

template <typename T>
__global__ void k_cell_restrict(Geo gf, Geo gc, const T *__restrict__ rf, T *__restrict__ rc) {
  cell_restrict_elem<T>(gf, gc, (i64)blockIdx.x * blockDim.x + threadIdx.x, rf, rc);
}

template <typename T>
void launch_cell_restrict(const Geo &gf, const Geo &gc, const T *rf, T *rc, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_restrict<T>, dim3(blocks_for(gc.ncell)), dim3(kBlock), 0, s, gf, gc,
                     rf, rc);
}

template <typename T>
__device__ __forceinline__ void cell_prolong_elem(const Geo &gc, const Geo &gf, i64 t,
                                                  const T *__restrict__ ec, T *__restrict__ pf) {
  if (t >= gf.ncell) return;
  int f[3];
  cell_of(gf, t, f);
  int I[3] = {f[0] >> 1, f[1] >> 1, gf.d == 3 ? f[2] >> 1 : 0};
  pf[t] += ec[cidx3(gc, I)];
}

template <typename T>
__global__ void k_cell_prolong_add(Geo gc, Geo gf, const T *__restrict__ ec, T *__restrict__ pf) {
  cell_prolong_elem<T>(gc, gf, (i64)blockIdx.x * blockDim.x + threadIdx.x, ec, pf);
}

template <typename T>
void launch_cell_prolong_add(const Geo &gc, const Geo &gf, const T *ec, T *pf, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_prolong_add<T>, dim3(blocks_for(gf.ncell)), dim3(kBlock), 0, s, gc, gf,
                     ec, pf);
}

// ------------------------------------------------------------------------
// Coarse tail of a V-cycle in one workgroup.  On the coarse levels every
// kernel above is launch-latency bound (a few thousand unknowns each); one
// 1024-thread workgroup runs all of them back to back, separated by block
// barriers, with the same element functions (same arithmetic) and the same
// order of operations as the host-sequenced cycle.  Mean removals use a
// block reduction instead of the two-stage grid reduction.
// ------------------------------------------------------------------------

__device__ double tail_block_sum(double v) {
  __shared__ double sh[kTailBlock / 64];
  __shared__ double total;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) r += sh[w];
    total = r;
  }
  __syncthreads();
  const double r = total;
  __syncthreads();
  return r;
}

// dst = src minus its mean over [0, n) (dst may alias src)
template <typename T>
__device__ void tail_sub_mean(const T *src, T *dst, i64 n) {
  double acc = 0.0;
  for (i64 t = threadIdx.x; t < n; t += blockDim.x) acc += (double)src[t];
  const T mean = (T)(tail_block_sum(acc) / (double)n);
  for (i64 t = threadIdx.x; t < n; t += blockDim.x) dst[t] = src[t] - mean;
  __syncthreads();
}

template <typename T>
__device__ void tail_copy(const T *src, T *dst, i64 n) {
  for (i64 t = threadIdx.x; t < n; t += blockDim.x) dst[t] = src[t];
  __syncthreads();
}

template <typename T>
__device__ void tail_zero(T *dst, i64 n) {
  for (i64 t = threadIdx.x; t < n; t += blockDim.x) dst[t] = (T)0;
  __syncthreads();
}

template <typename T, int DIM>
__device__ void tail_vel_smooth(const Geo &g, const T *alpha, const T *muc, const T *mue,
                                const T *lam, const T *rhs, T *phi, int sweeps) {
  const i64 nt = colour_threads(g);
  for (int s = 0; s < sweeps; s++)
    for (int k = 0; k < DIM; k++)
      for (int colour = 0; colour < 2; colour++) {
        for (i64 t = threadIdx.x; t < nt; t += blockDim.x)
          vel_gs_elem<T, DIM>(g, k, colour, t, alpha, muc, mue, lam, rhs, phi);
        __syncthreads();
      }
}

// Per-level pointers of a tail launch.  Levels lds0.. (the smallest ones)
// are staged in LDS: their coefficients are copied there at the start and
// their iterates, right-hand sides and residuals live there, so their
// phases wait on LDS instead of L2 latency.  The element functions address
// both through generic pointers.
template <typename T>
struct TailPtrs {
  const T *a[kTailMax], *b[kTailMax], *mc[kTailMax], *me[kTailMax], *lam[kTailMax];
  T *phi[kTailMax], *rhs[kTailMax], *res[kTailMax];
};

template <typename T>
__device__ void tail_stage(const TailLevels<T> &L, unsigned char *lds, TailPtrs<T> &P, bool vel) {
  if (threadIdx.x == 0) {
    for (int l = 0; l < L.nl; l++) {
      const bool in = l >= L.lds0;
      P.a[l] = (in && L.a[l]) ? (const T *)(lds + L.off[l][0]) : L.a[l];
      P.b[l] = in ? (const T *)(lds + L.off[l][0]) : L.b[l];
      P.mc[l] = in ? (const T *)(lds + L.off[l][1]) : L.mc[l];
      P.me[l] = in ? (const T *)(lds + L.off[l][2]) : L.me[l];
      P.lam[l] = (in && L.lam[l]) ? (const T *)(lds + L.off[l][6]) : L.lam[l];
      const bool vin = in || (l == 0 && L.vec0);
      P.phi[l] = vin ? (T *)(lds + L.off[l][3]) : L.phi[l];
      P.rhs[l] = vin ? (T *)(lds + L.off[l][4]) : L.rhs[l];
      P.res[l] = vin ? (T *)(lds + L.off[l][5]) : L.res[l];
    }
  }
  for (int l = L.lds0; l < L.nl; l++) {
    const Geo &g = L.g[l];
    if (vel) {
      T *a = (T *)(lds + L.off[l][0]), *mc = (T *)(lds + L.off[l][1]), *me = (T *)(lds + L.off[l][2]);
      if (L.a[l])
        for (i64 t = threadIdx.x; t < g.nvel; t += blockDim.x) a[t] = L.a[l][t];
      for (i64 t = threadIdx.x; t < g.ncell; t += blockDim.x) mc[t] = L.mc[l][t];
      for (i64 t = threadIdx.x; t < g.nedge; t += blockDim.x) me[t] = L.me[l][t];
      if (L.lam[l]) {
        T *lm = (T *)(lds + L.off[l][6]);
        for (i64 t = threadIdx.x; t < g.ncell; t += blockDim.x) lm[t] = L.lam[l][t];
      }
    } else {
      T *b = (T *)(lds + L.off[l][0]);
      for (i64 t = threadIdx.x; t < g.nvel; t += blockDim.x) b[t] = L.b[l][t];
    }
  }
  __syncthreads();
}

// the velocity tail cycle on staged levels (ends with a barrier)
template <typename T, int DIM>
__device__ __forceinline__ void tail_vel_run(const TailLevels<T> &L, const TailPtrs<T> &P) {
  const int nl = L.nl;
  for (int l = 0; l < nl - 1; l++) {
    const Geo &g = L.g[l];
    tail_zero<T>(P.phi[l], g.nvel);
    tail_vel_smooth<T, DIM>(g, P.a[l], P.mc[l], P.me[l], P.lam[l], P.rhs[l], P.phi[l],
                            L.nu_pre);
    for (i64 t = threadIdx.x; t < g.ncell; t += blockDim.x)
      vel_residual_elem<T, DIM>(g, t, P.a[l], P.mc[l], P.me[l], P.lam[l], P.rhs[l], P.phi[l],
                                (const T *)nullptr, P.res[l]);
    __syncthreads();
    for (i64 t = threadIdx.x; t < L.g[l + 1].ncell; t += blockDim.x)
      face_restrict_elem<T, DIM>(g, L.g[l + 1], t, P.res[l], P.rhs[l + 1]);
    __syncthreads();
  }
  {
    const int l = nl - 1;
    const Geo &g = L.g[l];
    tail_zero<T>(P.phi[l], g.nvel);
    for (int k = 0; k < g.d; k++) {
      if ((L.singular >> k) & 1)
        tail_sub_mean<T>(P.rhs[l] + g.foff[k], P.res[l] + g.foff[k], g.fcnt[k]);
      else
        tail_copy<T>(P.rhs[l] + g.foff[k], P.res[l] + g.foff[k], g.fcnt[k]);
    }
    tail_vel_smooth<T, DIM>(g, P.a[l], P.mc[l], P.me[l], P.lam[l], P.res[l], P.phi[l],
                            L.nu_coarse);
    for (int k = 0; k < g.d; k++)
      if ((L.singular >> k) & 1)
        tail_sub_mean<T>(P.phi[l] + g.foff[k], P.phi[l] + g.foff[k], g.fcnt[k]);
  }
  for (int l = nl - 2; l >= 0; l--) {
    const Geo &g = L.g[l];
    for (i64 t = threadIdx.x; t < g.ncell; t += blockDim.x)
      face_prolong_elem<T, DIM>(L.g[l + 1], g, t, P.phi[l + 1], P.phi[l]);
    __syncthreads();
    tail_vel_smooth<T, DIM>(g, P.a[l], P.mc[l], P.me[l], P.lam[l], P.rhs[l], P.phi[l],
                            L.nu_post);
  }
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kTailBlock) k_tail_vel(TailLevels<T> L) {
  extern __shared__ __align__(16) unsigned char tail_lds[];
  __shared__ TailPtrs<T> P;
  tail_stage<T>(L, tail_lds, P, true);
  tail_vel_run<T, DIM>(L, P);
}

// column blockIdx.x of the tail's matrix: the tail on the unit vector
template <typename T, int DIM>
__global__ void __launch_bounds__(kTailBlock) k_tail_vel_columns(TailLevels<T> L,
                                                                 T *__restrict__ B, int nv) {
  extern __shared__ __align__(16) unsigned char tail_lds[];
  __shared__ TailPtrs<T> P;
  tail_stage<T>(L, tail_lds, P, true);
  const int j = (int)blockIdx.x;
  for (int t = threadIdx.x; t < nv; t += blockDim.x) P.rhs[0][t] = (t == j) ? (T)1 : (T)0;
  __syncthreads();
  tail_vel_run<T, DIM>(L, P);
  for (int t = threadIdx.x; t < nv; t += blockDim.x) B[(i64)t * nv + j] = P.phi[0][t];
}

// phi = B rhs: wave w of the launch takes row w
template <typename T>
__global__ void k_tail_matvec(const T *__restrict__ B, int nv, const T *__restrict__ rhs,
                              T *__restrict__ phi) {
  const int row = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = (int)(threadIdx.x & 63);
  if (row >= nv) return;  // the whole wave
  const T *__restrict__ b = B + (i64)row * nv;
  double acc = 0.0;
  for (int c = lane; c < nv; c += 64) acc += (double)b[c] * (double)rhs[c];
  acc = wave_sum(acc);
  if (lane == 0) phi[row] = (T)acc;
}

template <typename T, int DIM>
__device__ void tail_p_smooth(const Geo &g, const T *beta, const T *rhs, T *phi, int sweeps) {
  const i64 nt = colour_threads(g);
  for (int s = 0; s < sweeps; s++)
    for (int colour = 0; colour < 2; colour++) {
      for (i64 t = threadIdx.x; t < nt; t += blockDim.x)
        p_gs_elem<T, DIM>(g, colour, t, beta, rhs, phi);
      __syncthreads();
    }
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kTailBlock) k_tail_p(TailLevels<T> L) {
  extern __shared__ __align__(16) unsigned char tail_lds[];
  __shared__ TailPtrs<T> P;
  tail_stage<T>(L, tail_lds, P, false);
  const int nl = L.nl;
  for (int l = 0; l < nl - 1; l++) {
    const Geo &g = L.g[l];
    tail_zero<T>(P.phi[l], g.ncell);
    tail_p_smooth<T, DIM>(g, P.b[l], P.rhs[l], P.phi[l], L.nu_pre);
    for (i64 t = threadIdx.x; t < g.ncell; t += blockDim.x)
      p_residual_elem<T, DIM>(g, t, P.b[l], P.rhs[l], P.phi[l], P.res[l]);
    __syncthreads();
    for (i64 t = threadIdx.x; t < L.g[l + 1].ncell; t += blockDim.x)
      cell_restrict_elem<T>(g, L.g[l + 1], t, P.res[l], P.rhs[l + 1]);
    __syncthreads();
  }
  {
    const int l = nl - 1;
    const Geo &g = L.g[l];
    tail_zero<T>(P.phi[l], g.ncell);
    tail_sub_mean<T>(P.rhs[l], P.res[l], g.ncell);
    tail_p_smooth<T, DIM>(g, P.b[l], P.res[l], P.phi[l], L.nu_coarse);
    tail_sub_mean<T>(P.phi[l], P.phi[l], g.ncell);
  }
  for (int l = nl - 2; l >= 0; l--) {
    const Geo &g = L.g[l];
    for (i64 t = threadIdx.x; t < g.ncell; t += blockDim.x)
      cell_prolong_elem<T>(L.g[l + 1], g, t, P.phi[l + 1], P.phi[l]);
    __syncthreads();
    tail_p_smooth<T, DIM>(g, P.b[l], P.rhs[l], P.phi[l], L.nu_post);
  }
}

template <typename T>
bool tail_plan_lds(TailLevels<T> &L, bool vel, bool vec0) {
  auto up = [](unsigned x) { return (x + 15u) & ~15u; };
  L.lds0 = L.nl;
  L.lds_bytes = 0;
  L.vec0 = vec0 ? 1 : 0;
  for (int l = 0; l < kTailMax; l++)
    for (int q = 0; q < 7; q++) L.off[l][q] = 0;
  unsigned total = 0;
  if (vec0) {
    const unsigned v = up((unsigned)(vel ? L.g[0].nvel : L.g[0].ncell) * sizeof(T));
    for (int q = 3; q < 6; q++) {
      L.off[0][q] = total;
      total += v;
    }
    if (total > kTailLds) return false;
  }
  // from the coarsest level up; the first tail level keeps the caller's
  // buffers in global memory
  for (int l = L.nl - 1; l >= 1; l--) {
    const Geo &g = L.g[l];
    const unsigned nv = (unsigned)g.nvel * sizeof(T), nc = (unsigned)g.ncell * sizeof(T);
    const unsigned ne = (unsigned)g.nedge * sizeof(T);
    const unsigned sz[7] = {up(nv), vel ? up(nc) : 0u, vel ? up(ne) : 0u,
                            up(vel ? nv : nc), up(vel ? nv : nc), up(vel ? nv : nc),
                            (vel && L.lam[l]) ? up(nc) : 0u};
    unsigned need = 0;
    for (int q = 0; q < 7; q++) need += sz[q];
    if (total + need > kTailLds) break;
    unsigned o = total;
    for (int q = 0; q < 7; q++) {
      L.off[l][q] = o;
      o += sz[q];
    }
    total += need;
    L.lds0 = l;
  }
  L.lds_bytes = total;
  return !vec0 || L.lds0 <= 1;
}
template bool tail_plan_lds<float>(TailLevels<float> &, bool, bool);
template bool tail_plan_lds<double>(TailLevels<double> &, bool, bool);

template <typename T>
void launch_tail_vel(const TailLevels<T> &L, hipStream_t s) {
  if (L.g[0].d == 3)
    hipLaunchKernelGGL((k_tail_vel<T, 3>), dim3(1), dim3(kTailBlock), L.lds_bytes, s, L);
  else
    hipLaunchKernelGGL((k_tail_vel<T, 2>), dim3(1), dim3(kTailBlock), L.lds_bytes, s, L);
}
template <typename T>
void launch_tail_p(const TailLevels<T> &L, hipStream_t s) {
  if (L.g[0].d == 3)
    hipLaunchKernelGGL((k_tail_p<T, 3>), dim3(1), dim3(kTailBlock), L.lds_bytes, s, L);
  else
    hipLaunchKernelGGL((k_tail_p<T, 2>), dim3(1), dim3(kTailBlock), L.lds_bytes, s, L);
}
template <typename T>
void launch_tail_vel_columns(const TailLevels<T> &L, T *B, int nv, hipStream_t s) {
  if (L.g[0].d == 3)
    hipLaunchKernelGGL((k_tail_vel_columns<T, 3>), dim3(nv), dim3(kTailBlock), L.lds_bytes, s, L,
                       B, nv);
  else
    hipLaunchKernelGGL((k_tail_vel_columns<T, 2>), dim3(nv), dim3(kTailBlock), L.lds_bytes, s, L,
                       B, nv);
}
template <typename T>
void launch_tail_matvec(const T *B, int nv, const T *rhs, T *phi, hipStream_t s) {
  const unsigned nb = (unsigned)((nv + 3) / 4);  // four waves (rows) per workgroup
  hipLaunchKernelGGL(k_tail_matvec<T>, dim3(nb), dim3(256), 0, s, B, nv, rhs, phi);
}
template void launch_tail_vel_columns<float>(const TailLevels<float> &, float *, int, hipStream_t);
template void launch_tail_vel_columns<double>(const TailLevels<double> &, double *, int,
                                              hipStream_t);
template void launch_tail_matvec<float>(const float *, int, const float *, float *, hipStream_t);
template void launch_tail_matvec<double>(const double *, int, const double *, double *,
                                         hipStream_t);
template void launch_tail_vel<float>(const TailLevels<float> &, hipStream_t);
template void launch_tail_vel<double>(const TailLevels<double> &, hipStream_t);
template void launch_tail_p<float>(const TailLevels<float> &, hipStream_t);
template void launch_tail_p<double>(const TailLevels<double> &, hipStream_t);

// ------------------------------------------------------------------------
// preconditioner glue (Sec. "Preconditioners": P1..P5 compositions)
// ------------------------------------------------------------------------

template <typename T, int DIM>
__global__ void k_div(Geo g, const T *__restrict__ u, const T *__restrict__ bp, T sgn,
                      const T *__restrict__ mu, T b, T *__restrict__ out) {
  int i[3];
  if (!box_thread(g, g.n[0], i[0], i[1], i[2])) return;
  const i64 t = cidx3(g, i);
  T s = 0;
#pragma unroll
  for (int k = 0; k < DIM; k++) {
    int r[3] = {i[0], i[1], i[2]};
    r[k] = up1(g, k, i[k]);
    s += (u[fidx3(g, k, r)] - u[fidx3(g, k, i)]) * (T)g.ih;
  }
  if (bp) s += bp[t];
  const T c = sgn * s;
  out[t] = mu ? b * mu[t] * c : c;
}

template <typename T>
void launch_div(const Geo &g, const T *u, const T *bp, T sgn, T *out, hipStream_t s) {
  launch_div_scaled<T>(g, u, bp, sgn, nullptr, (T)0, out, s);
}

template <typename T>
void launch_div_scaled(const Geo &g, const T *u, const T *bp, T sgn, const T *mu, T b, T *out,
                       hipStream_t s) {
  if (g.d == 3)
    hipLaunchKernelGGL((k_div<T, 3>), box_blocks(g, g.n[0]), dim3(kBlock), 0, s, g, u, bp, sgn,
                       mu, b, out);
  else
    hipLaunchKernelGGL((k_div<T, 2>), box_blocks(g, g.n[0]), dim3(kBlock), 0, s, g, u, bp, sgn,
                       mu, b, out);
}

// mode 0: zu = xs + beta * G q ; mode 1: out = bu - G q
template <typename T, int DIM>
__global__ void k_grad_combine(Geo g, int mode, const T *__restrict__ base,
                               const T *__restrict__ beta, const T *__restrict__ q,
                               T *__restrict__ out) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.ncell) return;
  int i[3];
  cell_of(g, t, i);
  const T qc = q[t];
#pragma unroll
  for (int k = 0; k < DIM; k++) {
    if (low_wall(g, k, i)) continue;
    int l[3] = {i[0], i[1], i[2]};
    l[k] = dn1(g, k, i[k]);
    const i64 fq = fidx3(g, k, i);
    const T gq = (qc - q[cidx3(g, l)]) * (T)g.ih;
    out[fq] = (mode == 0) ? base[fq] + beta[fq] * gq : base[fq] - gq;
  }
}

template <typename T>
void launch_proj_update(const Geo &g, const T *xs, const T *beta, const T *q, T *zu,
                        hipStream_t s) {
  if (g.d == 3)
    hipLaunchKernelGGL((k_grad_combine<T, 3>), dim3(blocks_for(g.ncell)), dim3(kBlock), 0, s, g, 0,
                       xs, beta, q, zu);
  else
    hipLaunchKernelGGL((k_grad_combine<T, 2>), dim3(blocks_for(g.ncell)), dim3(kBlock), 0, s, g, 0,
                       xs, beta, q, zu);
}
template <typename T>
void launch_grad_sub(const Geo &g, const T *bu, const T *p, T *out, hipStream_t s) {
  if (g.d == 3)
    hipLaunchKernelGGL((k_grad_combine<T, 3>), dim3(blocks_for(g.ncell)), dim3(kBlock), 0, s, g, 1,
                       bu, (const T *)nullptr, p, out);
  else
    hipLaunchKernelGGL((k_grad_combine<T, 2>), dim3(blocks_for(g.ncell)), dim3(kBlock), 0, s, g, 1,
                       bu, (const T *)nullptr, p, out);
}

template <typename T>
__global__ void k_schur_combine(const T *__restrict__ q, const T *__restrict__ c,
                                const T *__restrict__ mu, T a, T b, T *__restrict__ out, i64 n) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const T v = b * mu[t] * c[t];
  out[t] = q ? a * q[t] + v : v;
}
template <typename T>
void launch_schur_combine(const T *q, const T *c, const T *mu, T a, T b, T *out, i64 n,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_schur_combine<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, q, c, mu, a, b,
                     out, n);
}

// ------------------------------------------------------------------------
// reductions: fixed grid, fixed tree -> bitwise reproducible
// ------------------------------------------------------------------------

__device__ __forceinline__ double warp_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// block-wide sum; result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = warp_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; w++) r += sh[w];
  }
  __syncthreads();
  return r;
}

template <typename T>
__global__ void k_sum_partial(const T *__restrict__ a, i64 n, double *__restrict__ partials) {
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x)
    acc += (double)a[t];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// out[j] = sum_b partials[b * stride + j] for j < nout, fixed order
// out[j] = sum over the blocks of partials[b * stride + j], j < nout <=
// kFinishMax: every thread adds its blocks b = t, t + blockDim, ... for all
// outputs (independent loads, no barrier between the outputs), each wave
// adds its lanes, and thread j adds the waves' sums of output j (a fixed
// order: the result does not depend on timing)
constexpr int kFinishBlock = 1024;
constexpr int kFinishMax = 34;
__global__ void __launch_bounds__(kFinishBlock)
    k_finish(const double *__restrict__ partials, int nblocks, int stride, int nout,
             double *__restrict__ out) {
  __shared__ double sh[kFinishMax][kFinishBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = 0; j < nout; j++) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) acc += partials[(i64)b * stride + j];
    acc = wave_sum(acc);
    if (lane == 0) sh[j][wid] = acc;
  }
  __syncthreads();
  if ((int)threadIdx.x < nout) {
    double r = 0.0;
    for (int w = 0; w < nw; w++) r += sh[threadIdx.x][w];
    out[threadIdx.x] = r;
  }
}

static int red_blocks(i64 n) {
  i64 b = (n + kBlock - 1) / kBlock;
  if (b > kRedBlocks) b = kRedBlocks;
  return (int)(b < 1 ? 1 : b);
}

template <typename T>
void launch_sum(const T *a, i64 n, double *partials, double *out, hipStream_t s) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_sum_partial<T>, dim3(nb), dim3(kBlock), 0, s, a, n, partials);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, s, partials, nb, 1, 1, out);
}

template <typename T>
__global__ void k_sub_mean(T *__restrict__ a, i64 n, const double *__restrict__ sum) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) a[t] -= (T)(sum[0] / (double)n);
}
template <typename T>
void launch_sub_mean(T *a, i64 n, const double *sum, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_mean<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, n, sum);
}

// Per-component sums of a velocity vector (used only when every axis is
// periodic): blockIdx.y is the component, each block reduces a contiguous
// stretch of it with four independent accumulators per thread.
template <typename T>
__global__ void k_vel_sums_partial(Geo g, const T *__restrict__ u, double *__restrict__ partials) {
  __shared__ double sh[kBlock / 64];
  const int k = blockIdx.y;
  const T *__restrict__ c = u + g.foff[k];
  const i64 n = g.fcnt[k];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (sizeof(T) == 4 && ((uintptr_t)c % 16) == 0) {
    // FP32: one float4 per thread and iteration, the remainder below
    const float4 *__restrict__ c4 = (const float4 *)c;
    const i64 n4 = n >> 2;
    for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < n4;
         t += (i64)gridDim.x * blockDim.x) {
      const float4 v = c4[t];
      acc[0] += (double)v.x;
      acc[1] += (double)v.y;
      acc[2] += (double)v.z;
      acc[3] += (double)v.w;
    }
    if (blockIdx.x == 0 && (i64)threadIdx.x < n - 4 * n4)
      acc[0] += (double)c[4 * n4 + threadIdx.x];
  } else {
    const i64 stride = (i64)gridDim.x * blockDim.x * 4;
    for (i64 t0 = (i64)blockIdx.x * blockDim.x * 4 + threadIdx.x; t0 < n; t0 += stride) {
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const i64 t = t0 + (i64)j * blockDim.x;
        if (t < n) acc[j] += (double)c[t];
      }
    }
  }
  double r = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  r = wave_sum(r);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double q = 0.0;
    for (int w = 0; w < kBlock / 64; w++) q += sh[w];
    partials[(i64)blockIdx.x * 3 + k] = q;
  }
}

// out = in - (component mean); out may alias in; blockIdx.y is the component
template <typename T>
__global__ void k_vel_sub_means(Geo g, const T *__restrict__ in, T *__restrict__ out,
                                const double *__restrict__ sums) {
  const int k = blockIdx.y;
  const i64 n = g.fcnt[k];
  // components without a constant null space are copied unchanged
  const T mean = ((g.sing >> k) & 1) ? (T)(sums[k] / (double)n) : (T)0;
  const T *__restrict__ a = in + g.foff[k];
  T *__restrict__ o = out + g.foff[k];
  const i64 t0 = (i64)blockIdx.x * blockDim.x * 4 + threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const i64 t = t0 + (i64)j * blockDim.x;
    if (t < n) o[t] = a[t] - mean;
  }
}

template <typename T>
void launch_vel_sums(const Geo &g, const T *in, double *partials, double *sums, hipStream_t s) {
  i64 nmax = 0;
  for (int k = 0; k < g.d; k++) nmax = g.fcnt[k] > nmax ? g.fcnt[k] : nmax;
  const i64 nbx = (nmax + 4 * kBlock - 1) / (4 * kBlock);
  const int nr = (int)(nbx < kRedBlocks ? (nbx < 1 ? 1 : nbx) : kRedBlocks);
  hipLaunchKernelGGL(k_vel_sums_partial<T>, dim3(nr, g.d), dim3(kBlock), 0, s, g, in, partials);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, s, partials, nr, 3, g.d, sums);
}
template void launch_vel_sums<float>(const Geo &, const float *, double *, double *, hipStream_t);
template void launch_vel_sums<double>(const Geo &, const double *, double *, double *,
                                      hipStream_t);

template <typename T>
void launch_vel_remove_means(const Geo &g, const T *in, T *out, double *partials, double *sums,
                             hipStream_t s) {
  i64 nmax = 0;
  for (int k = 0; k < g.d; k++) nmax = g.fcnt[k] > nmax ? g.fcnt[k] : nmax;
  const i64 nbx = (nmax + 4 * kBlock - 1) / (4 * kBlock);
  launch_vel_sums<T>(g, in, partials, sums, s);
  hipLaunchKernelGGL(k_vel_sub_means<T>, dim3((unsigned)(nbx < 1 ? 1 : nbx), g.d), dim3(kBlock),
                     0, s, g, in, out, sums);
}
template void launch_vel_remove_means<float>(const Geo &, const float *, float *, double *,
                                             double *, hipStream_t);
template void launch_vel_remove_means<double>(const Geo &, const double *, double *, double *,
                                              double *, hipStream_t);

struct PtrPack {
  const void *p[34];
};

struct CoefPack {
  double c[34];
};


// ---- Arnoldi: classical Gram-Schmidt, second pass lagged -----------------
// Streaming passes over [w, v_0..v_j] with double2 loads, a fixed grid and
// per-block partial sums (bitwise reproducible):
//   R (k_cgs_dots): V^T w and (w, w)
//   U (k_dcgs_update): the projections on the orthonormal basis V T, the next
//      stored vector (and its FP32 copy, the next flexible preconditioner
//      input) and its dots with the stored vectors
//   k_cgs_next: the explicit second pass applied to a stored vector when the
//      lagged one would remove half or more of it (and a plain scale); it
//      runs one double2 per thread when there is no norm to reduce

constexpr int kArnBlock = 256;
constexpr int kArnGrid = 2048;


// reduce over the block: acc[0..nv) go to partials[blockIdx.x*stride + i] and,
// when with_extra, acc[MAXV] goes to slot nv (constant register indices only)
template <int MAXV>
__device__ __forceinline__ void block_store(double (&acc)[MAXV + 1], int nv, bool with_extra,
                                            int stride, double *__restrict__ partials) {
  __shared__ double sh[kArnBlock / 64][MAXV + 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i <= MAXV; i++) {
    if (i < nv || (i == MAXV && with_extra)) {
      const double r = wave_sum(acc[i]);
      if (lane == 0) sh[wid][i] = r;
    }
  }
  __syncthreads();
  const int cnt = nv + (with_extra ? 1 : 0);
  if (threadIdx.x < cnt) {
    const int src = ((int)threadIdx.x < nv) ? (int)threadIdx.x : MAXV;
    double r = 0.0;
    for (int wv = 0; wv < kArnBlock / 64; wv++) r += sh[wv][src];
    partials[(i64)blockIdx.x * stride + threadIdx.x] = r;
  }
}

// with_norm: slot nv also receives (w, w)
template <int MAXV>
__global__ void __launch_bounds__(kArnBlock) k_cgs_dots(const double *__restrict__ w, PtrPack v,
                                                        int nv, i64 n, int stride, int with_norm,
                                                        double *__restrict__ partials) {
  double acc[MAXV + 1];
#pragma unroll
  for (int i = 0; i <= MAXV; i++) acc[i] = 0.0;
  const i64 n2 = n >> 1;
  const double2 *__restrict__ w2 = (const double2 *)w;
  for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < n2; t += (i64)gridDim.x * blockDim.x) {
    const double2 a = w2[t];
#pragma unroll
    for (int i = 0; i < MAXV; i++) {
      if (i < nv) {
        const double2 b = ((const double2 *)v.p[i])[t];
        acc[i] += a.x * b.x + a.y * b.y;
      }
    }
    if (with_norm) acc[MAXV] += a.x * a.x + a.y * a.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const double a = w[n - 1];
    for (int i = 0; i < nv; i++) acc[i] += a * ((const double *)v.p[i])[n - 1];
    if (with_norm) acc[MAXV] += a * a;
  }
  block_store<MAXV>(acc, nv, with_norm != 0, stride, partials);
}

// out may equal w (the norm-forming call runs in place): each element is
// read and written by the same thread, and neither pointer is restrict.
template <int MAXV>
__global__ void __launch_bounds__(kArnBlock) k_cgs_next(const double *w, PtrPack v,
                                                        const double *__restrict__ h1,
                                                        const double *__restrict__ h2, int nv,
                                                        double inv_nu, i64 n, double *out,
                                                        float *__restrict__ out32,
                                                        double *__restrict__ partials) {
  double hh[MAXV];
#pragma unroll
  for (int i = 0; i < MAXV; i++) hh[i] = (i < nv) ? h1[i] + h2[i] : 0.0;
  double acc[MAXV + 1];
#pragma unroll
  for (int i = 0; i <= MAXV; i++) acc[i] = 0.0;
  const i64 n2 = n >> 1;
  const double2 *w2 = (const double2 *)w;
  double2 *o2 = (double2 *)out;
  float2 *__restrict__ f2 = (float2 *)out32;
  for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < n2; t += (i64)gridDim.x * blockDim.x) {
    double2 a = w2[t];
#pragma unroll
    for (int i = 0; i < MAXV; i++) {
      if (i < nv) {
        const double2 b = ((const double2 *)v.p[i])[t];
        a.x -= hh[i] * b.x;
        a.y -= hh[i] * b.y;
      }
    }
    a.x *= inv_nu;
    a.y *= inv_nu;
    o2[t] = a;
    if (out32) f2[t] = make_float2((float)a.x, (float)a.y);
    acc[MAXV] += a.x * a.x + a.y * a.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double a = w[n - 1];
    for (int i = 0; i < nv; i++) a -= hh[i] * ((const double *)v.p[i])[n - 1];
    a *= inv_nu;
    out[n - 1] = a;
    if (out32) out32[n - 1] = (float)a;
    acc[MAXV] += a * a;
  }
  if (partials) block_store<MAXV>(acc, 0, true, 1, partials);
}

// ---- Arnoldi with lagged reorthogonalisation (two passes per step) -------
// The stored basis vectors vt_0..vt_j are the once-orthogonalised ones; the
// orthonormal basis is V = Vt T with T upper triangular (the second
// Gram-Schmidt pass of each vector, applied to coefficients instead of
// being written back).  T is row-major with row stride ld.  Given
// dots = {(w, vt_l) for l <= j, (w, w)} (the first pass), this pass forms
//   d = T^T (Vt^T w)          the projections of w on the orthonormal basis,
//   nu^2 = (w, w) - |d|^2     (clamped: nu only scales the new vector),
//   vt_{j+1} = (w - Vt (T d)) / nu, also as FP32 when out32 is given,
// and reduces (vt_{j+1}, vt_l) for l <= j and (vt_{j+1}, vt_{j+1}), from
// which the next step finds the new column of T.  Block 0 stores d and nu
// in coef_out[0..j+1].
// T travels as a kernel argument (column-packed upper triangle) when it has
// at most kTriDim rows, else through device memory (tm, row stride ld).
constexpr int kTriDim = 12;
struct TriPack {
  double t[kTriDim * (kTriDim + 1) / 2];
};

template <int MAXV>
__global__ void __launch_bounds__(kArnBlock) k_dcgs_update(const double *__restrict__ w, PtrPack v,
                                                           int j, const double *__restrict__ dots,
                                                           TriPack tp,
                                                           const double *__restrict__ tm, int ld,
                                                           i64 n, double *__restrict__ vnext,
                                                           float *__restrict__ out32,
                                                           double *__restrict__ coef_out,
                                                           double *__restrict__ partials) {
  // T(l, i), l <= i, read straight from the argument (no reference to tp
  // is taken, which would give it a private copy in every lane)
#define TRI(l, i) \
  (tm ? tm[(l) * ld + (i)] : ((i) < kTriDim ? tp.t[(i) * ((i) + 1) / 2 + (l)] : 0.0))
  // coefficients (the same few values in every thread), over compile-time
  // register indices
  double d[MAXV], g[MAXV];
  double dd2 = 0.0;
#pragma unroll
  for (int i = 0; i < MAXV; i++) {
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < MAXV; l++)
      if (l <= i && i <= j) acc += TRI(l, i) * dots[l];
    d[i] = (i <= j) ? acc : 0.0;
    dd2 += d[i] * d[i];
  }
  // g = T d (T is upper triangular)
#pragma unroll
  for (int l = 0; l < MAXV; l++) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < MAXV; i++)
      if (i >= l && i <= j) acc += TRI(l, i) * d[i];
    g[l] = (l <= j) ? acc : 0.0;
  }
#undef TRI
  const double q = dots[j + 1];
  const double nu2 = q - dd2;
  const double floor2 = q * 0x1p-60;
  const double nu = (nu2 > floor2) ? sqrt(nu2) : (q > 0.0 ? sqrt(floor2) : 1.0);
  const double inu = 1.0 / nu;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int i = 0; i <= j && i < MAXV; i++) coef_out[i] = d[i];
    coef_out[j + 1] = nu;
  }
  double acc[MAXV + 1];
#pragma unroll
  for (int i = 0; i <= MAXV; i++) acc[i] = 0.0;
  const i64 n2 = n >> 1;
  const double2 *__restrict__ w2 = (const double2 *)w;
  double2 *__restrict__ vn2 = (double2 *)vnext;
  float2 *__restrict__ f2 = (float2 *)out32;
  for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < n2; t += (i64)gridDim.x * blockDim.x) {
    double2 wp = w2[t];
    double2 b[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; i++) {
      if (i <= j) {
        b[i] = ((const double2 *)v.p[i])[t];
        wp.x -= g[i] * b[i].x;
        wp.y -= g[i] * b[i].y;
      }
    }
    wp.x *= inu;
    wp.y *= inu;
    vn2[t] = wp;
    if (out32) f2[t] = make_float2((float)wp.x, (float)wp.y);
#pragma unroll
    for (int i = 0; i < MAXV; i++)
      if (i <= j) acc[i] += b[i].x * wp.x + b[i].y * wp.y;
    acc[MAXV] += wp.x * wp.x + wp.y * wp.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const i64 e = n - 1;
    double wp = w[e];
    for (int i = 0; i <= j && i < MAXV; i++) wp -= g[i] * ((const double *)v.p[i])[e];
    wp *= inu;
    vnext[e] = wp;
    if (out32) out32[e] = (float)wp;
#pragma unroll
    for (int i = 0; i < MAXV; i++)
      if (i <= j) acc[i] += ((const double *)v.p[i])[e] * wp;
    acc[MAXV] += wp * wp;
  }
  // slots 0..j: (vt_{j+1}, vt_l); slot j + 1: (vt_{j+1}, vt_{j+1})
  block_store<MAXV>(acc, j + 1, true, j + 2, partials);
}

static int arn_blocks(i64 n) {
  i64 b = ((n >> 1) + kArnBlock - 1) / kArnBlock;
  if (b > kArnGrid) b = kArnGrid;
  return (int)(b < 1 ? 1 : b);
}

#define ARN_DISPATCH(KERN, nv, ...)                                                          \
  do {                                                                                       \
    if ((nv) <= 12)                                                                          \
      hipLaunchKernelGGL(KERN<12>, dim3(nb), dim3(kArnBlock), 0, s, __VA_ARGS__);            \
    else                                                                                     \
      hipLaunchKernelGGL(KERN<33>, dim3(nb), dim3(kArnBlock), 0, s, __VA_ARGS__);            \
  } while (0)

void launch_cgs_dots(const double *w, const double *const *v, int nv, i64 n, double *partials,
                     double *h, hipStream_t s, bool with_norm) {
  PtrPack pk;
  for (int j = 0; j < nv; j++) pk.p[j] = v[j];
  const int nb = arn_blocks(n);
  const int nout = nv + (with_norm ? 1 : 0);
  ARN_DISPATCH(k_cgs_dots, nv, w, pk, nv, n, nout, with_norm ? 1 : 0, partials);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, s, partials, nb, nout, nout, h);
}

void launch_cgs_next(const double *w, const double *const *v, const double *h1, const double *h2,
                     int nv, double inv_nu, i64 n, double *out, float *out32, double *partials,
                     double *nrm2, hipStream_t s) {
  PtrPack pk;
  for (int j = 0; j < nv; j++) pk.p[j] = v[j];
  // Without the norm there is nothing to reduce: one double2 per thread
  // (the grid-stride loop then runs once), which streams faster than the
  // fixed reduction grid.  With the norm the fixed grid keeps the partial
  // sums, and so the result, independent of the launch.
  const i64 pairs = std::max<i64>(1, ((n >> 1) + kArnBlock - 1) / kArnBlock);
  const int nb = nrm2 ? arn_blocks(n) : (int)std::min<i64>(pairs, 0x7fffffff);
  ARN_DISPATCH(k_cgs_next, nv, w, pk, h1, h2, nv, inv_nu, n, out, out32,
               nrm2 ? partials : nullptr);
  if (nrm2)
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, s, partials, nb, 1, 1, nrm2);
}
void launch_dcgs_update(const double *w, const double *const *v, int j, const double *dots,
                        const double *tm_host, const double *tm_dev, int ld, i64 n,
                        double *vnext, float *out32, double *coef_out, double *partials,
                        double *red, hipStream_t s) {
  PtrPack pk;
  for (int i = 0; i <= j; i++) pk.p[i] = v[i];
  TriPack tp;
  for (int i = 0; i < kTriDim * (kTriDim + 1) / 2; i++) tp.t[i] = 0.0;
  const double *tm = nullptr;
  if (j + 1 <= kTriDim) {
    for (int i = 0; i <= j; i++)
      for (int l = 0; l <= i; l++) tp.t[i * (i + 1) / 2 + l] = tm_host[l * ld + i];
  } else {
    tm = tm_dev;
  }
  const int nb = arn_blocks(n);
  ARN_DISPATCH(k_dcgs_update, j + 1, w, pk, j, dots, tp, tm, ld, n, vnext, out32, coef_out,
               partials);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, s, partials, nb, j + 2, j + 2, red);
}
#undef ARN_DISPATCH


template <typename TZ>
__global__ void k_update_x(double *__restrict__ x, PtrPack z, CoefPack y, int nz, i64 n) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double acc = x[t];
  for (int j = 0; j < nz; j++) acc += y.c[j] * (double)((const TZ *)z.p[j])[t];
  x[t] = acc;
}

template <typename TZ>
void launch_update_x(double *x, const TZ *const *z, const double *y, int nz, i64 n,
                     hipStream_t s) {
  PtrPack pk;
  CoefPack cy;
  for (int j = 0; j < nz; j++) {
    pk.p[j] = z[j];
    cy.c[j] = y[j];
  }
  hipLaunchKernelGGL(k_update_x<TZ>, dim3(blocks_for(n)), dim3(kBlock), 0, s, x, pk, cy, nz, n);
}
template void launch_update_x<double>(double *, const double *const *, const double *, int, i64,
                                      hipStream_t);
template void launch_update_x<float>(double *, const float *const *, const double *, int, i64,
                                     hipStream_t);

__global__ void k_norm2_partial(const double *__restrict__ a, i64 n, double *__restrict__ partials) {
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x)
    acc += a[t] * a[t];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}
void launch_norm2(const double *a, i64 n, double *partials, double *nrm2, hipStream_t s) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_norm2_partial, dim3(nb), dim3(kBlock), 0, s, a, n, partials);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, s, partials, nb, 1, 1, nrm2);
}


// sum of log(mu) over mu > 0 and the count of such cells (rescaling, Sec. "Rescaling of the Linear System")
__global__ void k_logsum_partial(const double *__restrict__ mu, i64 n, double *__restrict__ partials) {
  __shared__ double sh[kBlock / 64];
  double acc = 0.0, cnt = 0.0;
  for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) {
    const double v = mu[t];
    if (v > 0.0) {
      acc += log(v);
      cnt += 1.0;
    }
  }
  const double r0 = block_sum(acc, sh);
  const double r1 = block_sum(cnt, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = r0;
    partials[2 * blockIdx.x + 1] = r1;
  }
}
void launch_logsum(const double *mu, i64 n, double *partials, double *out2, hipStream_t s) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_logsum_partial, dim3(nb), dim3(kBlock), 0, s, mu, n, partials);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishBlock), 0, s, partials, nb, 2, 2, out2);
}

// ------------------------------------------------------------------------
// gradient contraction (adjoint): strain rates of u and lambda
// ------------------------------------------------------------------------

// derivative of component k along axis l at an edge point e (node along k, l)
// with the one-sided no-slip wall rule
__device__ __forceinline__ double dkl(const Geo &g, const double *__restrict__ u, int k, int l,
                                      const int e[3]) {
  int f[3] = {e[0], e[1], e[2]};
  const double h = g.h;
  if (g.ns[l] && e[l] == 0) return 2.0 * u[fidx3(g, k, f)] / h;
  if (g.ns[l] && e[l] == g.n[l]) {
    f[l] = g.n[l] - 1;
    return -2.0 * u[fidx3(g, k, f)] / h;
  }
  int fb[3] = {e[0], e[1], e[2]};
  fb[l] = dn1(g, l, e[l]);
  return (u[fidx3(g, k, f)] - u[fidx3(g, k, fb)]) / h;
}

// bulk != 0: the stress carries (gamma - 2/3 mu)(div u) I, whose coefficient
// has derivative dgam = -(D lambda)(D u) per cell; -2/3 of it joins dmu.
__global__ void k_grad_cells(Geo g, const double *__restrict__ u, const double *__restrict__ lam,
                             double theta, int bulk, double *__restrict__ dmu,
                             double *__restrict__ drho, double *__restrict__ dgam) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.ncell) return;
  int i[3];
  cell_of(g, t, i);
  double s = 0.0, r = 0.0, divu = 0.0, divl = 0.0;
  for (int k = 0; k < g.d; k++) {
    int hi[3] = {i[0], i[1], i[2]};
    hi[k] = up1(g, k, i[k]);
    const i64 ql = fidx3(g, k, i), qh = fidx3(g, k, hi);
    const double du = (u[qh] - u[ql]) / g.h;
    const double dl = (lam[qh] - lam[ql]) / g.h;
    s += dl * du;
    divu += du;
    divl += dl;
    // density: both faces of the cell along k (wall faces hold 0)
    r += lam[ql] * u[ql] + lam[qh] * u[qh];
  }
  const double dg = -divl * divu;
  if (dmu) dmu[t] = bulk ? -2.0 * s - 2.0 / 3.0 * dg : -2.0 * s;
  if (drho) drho[t] = -theta * 0.5 * r;
  if (dgam) dgam[t] = dg;
}

__global__ void k_grad_edges(Geo g, int m, const double *__restrict__ u,
                             const double *__restrict__ lam, double *__restrict__ dme) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.ecnt[m]) return;
  int e[3];
  {
    i64 q = t / g.ed[m][0];
    e[0] = (int)(t - q * g.ed[m][0]);
    e[2] = (int)(q / g.ed[m][1]);
    e[1] = (int)(q - (i64)e[2] * g.ed[m][1]);
  }
  const int k = (m == 0) ? 1 : 0;
  const int l = (m == 2) ? 1 : 2;
  const bool wall = (g.ns[k] && (e[k] == 0 || e[k] == g.n[k])) ||
                    (g.ns[l] && (e[l] == 0 || e[l] == g.n[l]));
  // no shear stress (and no dependence on mu_edge) on a free-slip wall
  const bool free = ((g.fs[k] & 1) && e[k] == 0) || ((g.fs[k] & 2) && e[k] == g.n[k]) ||
                    ((g.fs[l] & 1) && e[l] == 0) || ((g.fs[l] & 2) && e[l] == g.n[l]);
  const double gu = dkl(g, u, k, l, e) + dkl(g, u, l, k, e);
  const double gl = dkl(g, lam, k, l, e) + dkl(g, lam, l, k, e);
  dme[g.eoff[m] + t] = free ? 0.0 : -(wall ? 0.5 : 1.0) * gl * gu;
}

// dmu_cell += sum over the cell's edges of dmu_edge * d mu_edge / d mu_cell
__global__ void k_grad_chain(Geo g, const double *__restrict__ dme, const double *__restrict__ mue,
                             const double *__restrict__ muc, int mode, double *__restrict__ dmu) {
  i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.ncell) return;
  int i[3];
  cell_of(g, t, i);
  double acc = 0.0;
  for (int m = 0; m < 3; m++) {
    if (g.ecnt[m] == 0) continue;
    const int k = (m == 0) ? 1 : 0;
    const int l = (m == 2) ? 1 : 2;
    for (int a = 0; a < 2; a++)
      for (int b = 0; b < 2; b++) {
        int e[3] = {i[0], i[1], i[2]};
        e[k] += a;
        e[l] += b;
        if (!g.ns[k] && e[k] == g.n[k]) e[k] = 0;
        if (!g.ns[l] && e[l] == g.n[l]) e[l] = 0;
        // number of cells adjacent to this edge
        int ck = (g.ns[k] && (e[k] == 0 || e[k] == g.n[k])) ? 1 : 2;
        int cl = (g.ns[l] && (e[l] == 0 || e[l] == g.n[l])) ? 1 : 2;
        const int cnt = ck * cl;
        const i64 q = eidx3(g, m, e);
        double w;
        if (mode == 1) {
          const double me = mue[q], mc = muc[t];
          w = me * me / ((double)cnt * mc * mc);
        } else {
          w = 1.0 / (double)cnt;
        }
        acc += dme[q] * w;
      }
  }
  dmu[t] += acc;
}

void launch_grad_cells(const Geo &g, const double *u, const double *lam, double theta, int bulk,
                       double *dmu_cell, double *drho, double *dgamma, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_cells, dim3(blocks_for(g.ncell)), dim3(kBlock), 0, s, g, u, lam, theta,
                     bulk, dmu_cell, drho, dgamma);
}
void launch_grad_edges(const Geo &g, const double *u, const double *lam, double *dmu_edge,
                       hipStream_t s) {
  for (int m = 0; m < 3; m++) {
    if (g.ecnt[m] == 0) continue;
    hipLaunchKernelGGL(k_grad_edges, dim3(blocks_for(g.ecnt[m])), dim3(kBlock), 0, s, g, m, u, lam,
                       dmu_edge);
  }
}
void launch_grad_chain(const Geo &g, const double *dmu_edge, const double *mue_raw,
                       const double *muc_raw, int mode, double *dmu_cell, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_chain, dim3(blocks_for(g.ncell)), dim3(kBlock), 0, s, g, dmu_edge,
                     mue_raw, muc_raw, mode, dmu_cell);
}

// ------------------------------------------------------------------------
// explicit instantiations
// ------------------------------------------------------------------------
#define INST(T)                                                                                  \
  template void launch_vel_gs<T>(const Geo &, int, int, int, const T *, const T *, const T *,    \
                                 const T *, const T *, T *, hipStream_t);                        \
  template void launch_vel_residual<T>(const Geo &, const T *, const T *, const T *, const T *,  \
                                       const T *, const T *, const T *, T *, hipStream_t);       \
  template void launch_face_restrict<T>(const Geo &, const Geo &, const T *, T *, hipStream_t);  \
  template void launch_face_prolong_add<T>(const Geo &, const Geo &, const T *, T *,             \
                                           hipStream_t);                                         \
  template void launch_p_gs<T>(const Geo &, int, int, const T *, const T *, T *, hipStream_t);   \
  template void launch_p_residual<T>(const Geo &, const T *, const T *, const T *, T *,          \
                                     hipStream_t);                                               \
  template void launch_cell_restrict<T>(const Geo &, const Geo &, const T *, T *, hipStream_t);  \
  template void launch_cell_prolong_add<T>(const Geo &, const Geo &, const T *, T *,             \
                                           hipStream_t);                                         \
  template void launch_div<T>(const Geo &, const T *, const T *, T, T *, hipStream_t);           \
  template void launch_div_scaled<T>(const Geo &, const T *, const T *, T, const T *, T, T *,    \
                                     hipStream_t);                                               \
  template void launch_proj_update<T>(const Geo &, const T *, const T *, const T *, T *,         \
                                      hipStream_t);                                              \
  template void launch_grad_sub<T>(const Geo &, const T *, const T *, T *, hipStream_t);         \
  template void launch_schur_combine<T>(const T *, const T *, const T *, T, T, T *, i64,         \
                                        hipStream_t);                                            \
  template void launch_sum<T>(const T *, i64, double *, double *, hipStream_t);                  \
  template void launch_sub_mean<T>(T *, i64, const double *, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace stk
