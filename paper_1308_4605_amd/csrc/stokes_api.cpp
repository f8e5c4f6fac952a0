// stokes_api.cpp -- host side of the MI355X MAC Stokes library: workspace
// layout, coefficient hierarchy, multigrid V-cycles, block preconditioners,
// restarted GMRES / flexible GMRES and the adjoint, behind the C ABI of
// include/stokes.h.  All arithmetic runs in the HIP kernels of
// stokes_kernels.hip; the host only sequences launches, runs the Givens
// rotations of the (m+1) x m Hessenberg matrix and tests convergence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "stokes.h"
#include "stokes_internal.h"

using namespace stk;

namespace {

constexpr int kMaxLev = 24;
constexpr int kMaxRestart = 32;
constexpr size_t kAlign = 256;
constexpr int kEventPool = 2048;
// 3D velocity residual by columns (Geo::col): cells per column thread, and
// the smallest level that takes it
constexpr int kResidualColumn = 8;
constexpr i64 kResidualColumnCells = (i64)1 << 21;

struct Level {
  Geo g;
  Geo gv;  // geometry of the velocity multigrid arrays (storage order, Geo::split)
  void *alpha, *beta, *muc, *mue;             // precision T of the hierarchy
  void *lam;                                  // bulk coefficient (null: none)
  void *phi_u, *rhs_u, *res_u, *phi_p, *rhs_p, *res_p;
};

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures.
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base((char *)b) {}
  void *take(size_t bytes) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    void *p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

bool valid_params(const stokes_params *p, int *nlev_out) {
  if (!p) return false;
  if (p->dim != 2 && p->dim != 3) return false;
  if (!(p->h > 0.0) || !std::isfinite(p->h)) return false;
  if (!(p->theta >= 0.0) || !std::isfinite(p->theta)) return false;
  if (p->precond < STOKES_P1 || p->precond > STOKES_P5) return false;
  if (p->precision != STOKES_FP64 && p->precision != STOKES_MG_FP32) return false;
  if (p->krylov != STOKES_GMRES_LEFT && p->krylov != STOKES_FGMRES) return false;
  if (p->precision == STOKES_MG_FP32 && p->krylov != STOKES_FGMRES) return false;
  if (p->restart < 1 || p->restart > kMaxRestart) return false;
  if (p->nu_pre < 0 || p->nu_post < 0 || p->nu_coarse < 1 || p->vcycles < 1) return false;
  if (p->nu_pre > 64 || p->nu_post > 64 || p->nu_coarse > 4096 || p->vcycles > 1000) return false;
  if (p->edge_avg < STOKES_EDGE_ARITH || p->edge_avg > STOKES_EDGE_GIVEN) return false;
  if (p->bulk != 0 && p->bulk != 1) return false;
  if (p->scaling != STOKES_SCALE_UNIFORM && p->scaling != STOKES_SCALE_DIAGONAL) return false;
  if (p->extended != 0 && p->extended != 1) return false;
  int nmin = 1 << 30;
  for (int a = 0; a < p->dim; a++) {
    if (p->n[a] < 2 || p->n[a] > (1 << 20)) return false;
    if (p->bc[a] < STOKES_PERIODIC || p->bc[a] > STOKES_FREESLIP_NOSLIP) return false;
    if (p->n[a] < nmin) nmin = p->n[a];
  }
  // coarsen by 2 until the smallest axis has two cells (Appendix C)
  int nlev = 1;
  while ((nmin >> (nlev - 1)) > 2) nlev++;
  if ((2 << (nlev - 1)) != nmin) return false;
  if (nlev > kMaxLev) return false;
  for (int a = 0; a < p->dim; a++) {
    if (p->n[a] % (1 << (nlev - 1)) != 0) return false;
    // red-black colouring needs an even cell count around every periodic axis
    // on every level, the coarsest included
    if (p->bc[a] == STOKES_PERIODIC && ((p->n[a] >> (nlev - 1)) & 1)) return false;
  }
  // the kernels index face, cell and edge storage with 32-bit integers
  long long nodes = 1;
  for (int a = 0; a < p->dim; a++) nodes *= (long long)p->n[a] + 1;
  if (3 * nodes > 0x7fffffffLL) return false;
  if (nlev_out) *nlev_out = nlev;
  return true;
}

}  // namespace

struct stokes_ctx {
  stokes_params p;
  hipStream_t s = nullptr;
  int dev = 0;  // HIP device current at creation (the stream's device)
  int d = 0, nlev = 0;
  int mg32 = 0;
  int vel_singular = 0;  // bit k: velocity component k has a constant null space
  int bulk = 0;          // stress with bulk viscosity (lam arrays present)
  // the finest velocity level of an FP32 hierarchy in the colour-split
  // storage order (vsplit): its V-cycle input / output and alpha in that order
  int vsplit = 0;
  void *vrs = nullptr, *ves = nullptr, *alpha_v = nullptr;
  int tail_l = -1;  // first level of the single-workgroup coarse tail (-1: none)
  // the velocity tail as its matrix B (tail_nv x tail_nv, row-major, precision
  // of the hierarchy), built at create; tail_dense = 0 (STOKES_TAIL_DENSE=0 in
  // the environment at create time): the tail's own sweeps every time
  void *tail_B = nullptr;
  int tail_nv = 0;
  int tail_dense = 1;
  // the finest-level velocity V-cycle of a colour-split hierarchy (fixed
  // buffers vrs -> ves) recorded once at create as a HIP graph and replayed
  // on the caller's stream (STOKES_VGRAPH=0 in the environment at create
  // time: launched kernel by kernel)
  hipStream_t gstream = nullptr;
  hipGraph_t vgraph = nullptr;
  hipGraphExec_t vgexec = nullptr;
  double c = 1.0;
  Level lev[kMaxLev];
  i64 nvel = 0, ncell = 0, nedge = 0, n = 0;
  // FP64 scaled fine-level coefficients for M (alias level 0 in FP64 mode)
  double *m_alpha = nullptr, *m_muc = nullptr, *m_mue = nullptr, *m_lam = nullptr;
  // level-0 coefficient s of the Schur approximation's viscous part 2 s:
  // mu (eq. Schur_app_varDen_varVis) or (gamma + 4/3 mu) / 2 (eq.
  // Schur_app_bulk); precision T; aliases level 0's mu_cell without bulk
  void *sig = nullptr;
  double *sig64 = nullptr;  // FP64 form while an FP32 hierarchy is built
  // Krylov storage (FP64 [u | p] vectors; Z in the preconditioner precision)
  double *V[kMaxRestart + 1];
  void *Z[kMaxRestart];
  double *r = nullptr, *w = nullptr, *t = nullptr, *x = nullptr, *b = nullptr;
  // diagonal scaling S of the rescaled unknowns [faces | cells]
  // (STOKES_SCALE_DIAGONAL; null otherwise)
  double *sdiag = nullptr;
  // device copy of the Arnoldi basis transform T (upper triangular,
  // row-major, row stride restart + 1)
  double *tmat = nullptr;
  // preconditioner temporaries (precision T, level-0 sizes)
  void *pin = nullptr, *pout = nullptr;           // [u | p]
  void *xs = nullptr, *tu = nullptr, *eu = nullptr;  // velocity
  void *cv = nullptr, *q = nullptr;                 // cells
  void *vs_r = nullptr, *vs_t = nullptr, *vs_de = nullptr;
  void *ps_r = nullptr, *ps_t = nullptr, *ps_de = nullptr;
  double *gedge = nullptr, *gcell = nullptr;        // gradient scratch (FP64)
  // FP64 coefficient chain used to build an FP32 hierarchy (setup only)
  double *c64a[kMaxLev], *c64b[kMaxLev], *c64m[kMaxLev], *c64e[kMaxLev], *c64l[kMaxLev];
  // reductions
  double *part = nullptr;   // partial sums
  double *dsc = nullptr;    // device scalars
  int *dflag = nullptr;
  double *host = nullptr;   // pinned host mirror
  // timing of the finest-level velocity colour passes
  int timing = 0;
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
  double t_ms = 0.0;
  long launches = 0;
  double bytes = 0.0;
  double gs_bytes[3] = {0, 0, 0};
  // timing of whole V-cycles from the finest level (index 0 velocity, 1
  // pressure): event pairs, accumulated time, count and algorithmic bytes
  std::vector<hipEvent_t> vev;
  std::vector<int> vev_kind;
  int vev_used = 0;
  double vc_ms[2] = {0, 0}, vc_bytes[2] = {0, 0}, vc_cycle_bytes[2] = {0, 0};
  long vc_count[2] = {0, 0};
  // preconditioner timing for stokes_stats: two pairs of events around the
  // applications (the pairs alternate, so that one application can still be
  // running when the next is recorded)
  hipEvent_t pev[4] = {nullptr, nullptr, nullptr, nullptr};
  // marks the end of an Arnoldi step's reads to the host, which the host
  // waits for while the next preconditioner application already runs
  hipEvent_t sev = nullptr;
  double *hist = nullptr;  // residual history (caller's host buffer)
  int hist_cap = 0;
  int err = 0;
};

// Storage of stokes_solve_static: a static device array of the library, one
// copy per GPU that runs it, held until the process ends.  Host code never
// passes `scratch` itself to a kernel (on the host the name is only a
// stand-in); it uses the device address hipGetSymbolAddress returns for the
// current device, looked up once per device and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = (size_t)STOKES_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on device dev (nullptr on a HIP error)
void *scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return nullptr;
    if (prev != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != dev) (void)hipSetDevice(prev);
    if (e != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

constexpr int kDscSlots = 256;  // device scalar slots
constexpr int kZeroSlots = 216;  // dsc[216..255] stay zero (cleared with the workspace)

// The velocity levels above the one-workgroup coarse tail of an FP32
// hierarchy are stored colour-split when the finest rows are long (a wave
// then reads 64 same-colour faces from one contiguous run instead of every
// other face of 128): the same arithmetic with half the cache lines per
// load.  FP64 passes already run at the copy bandwidth, and the two
// reordering passes per cycle made them slower.
bool use_vsplit(const stokes_params *p) {
  i64 cells = 1;
  for (int a = 0; a < p->dim; a++) cells *= p->n[a];
  return p->precision == STOKES_MG_FP32 && p->n[0] >= 128 && cells > kTailCells;
}

// first level of the single-workgroup coarse tail: the first of the last
// kTailMax levels with at most kTailCells cells (-1: none)
int tail_level_of(const stokes_params *p, int nlev) {
  for (int l = std::max(0, nlev - kTailMax); l < nlev; l++) {
    i64 cells = 1;
    for (int a = 0; a < p->dim; a++) cells *= (i64)(p->n[a] >> l);
    if (cells <= kTailCells) return l;
  }
  return -1;
}

void carve_all(const stokes_params *p, int nlev, Carver &cv, stokes_ctx *X) {
  const int d = p->dim;
  const size_t tb = (p->precision == STOKES_MG_FP32) ? sizeof(float) : sizeof(double);
  int ns[3], n[3];
  for (int a = 0; a < 3; a++) {
    n[a] = (a < d) ? p->n[a] : 1;
    ns[a] = (a < d) ? p->bc[a] : 0;
  }
  Geo g0 = make_geo(d, n, ns, p->h);
  const i64 nv = g0.nvel, nc = g0.ncell, ne = g0.nedge, nn = nv + nc;
  for (int l = 0; l < nlev; l++) {
    int nl[3];
    for (int a = 0; a < 3; a++) nl[a] = (a < d) ? (n[a] >> l) : 1;
    Geo g = make_geo(d, nl, ns, p->h * (double)(1 << l));
    Level L;
    L.g = g;
    L.gv = g;
    L.alpha = cv.take(g.nvel * tb);
    L.beta = cv.take(g.nvel * tb);
    L.muc = cv.take(g.ncell * tb);
    L.mue = cv.take(g.nedge * tb);
    L.lam = p->bulk ? cv.take(g.ncell * tb) : nullptr;
    L.phi_u = cv.take(g.nvel * tb);
    L.rhs_u = cv.take(g.nvel * tb);
    L.res_u = cv.take(g.nvel * tb);
    L.phi_p = cv.take(g.ncell * tb);
    L.rhs_p = cv.take(g.ncell * tb);
    L.res_p = cv.take(g.ncell * tb);
    if (X) X->lev[l] = L;
  }
  // matrix of the velocity tail's linear map (first tail level's velocity
  // count squared)
  const int tl = tail_level_of(p, nlev);
  if (tl >= 0) {
    int nt[3];
    for (int a = 0; a < 3; a++) nt[a] = (a < d) ? (n[a] >> tl) : 1;
    const Geo gt = make_geo(d, nt, ns, p->h * (double)(1 << tl));
    void *B = cv.take((size_t)gt.nvel * (size_t)gt.nvel * tb);
    if (X) {
      X->tail_B = B;
      X->tail_nv = (int)gt.nvel;
    }
  }
  // FP64 fine coefficients of M (rescaled)
  double *ma = (double *)cv.take(nv * 8);
  double *mc = (double *)cv.take(nc * 8), *me = (double *)cv.take(ne * 8);
  double *ml = p->bulk ? (double *)cv.take(nc * 8) : nullptr;
  void *sig = p->bulk ? cv.take(nc * tb) : nullptr;
  double *sig64 = (p->bulk && p->precision == STOKES_MG_FP32) ? (double *)cv.take(nc * 8) : nullptr;
  if (X) {
    X->m_alpha = ma;
    X->m_muc = mc;
    X->m_mue = me;
    X->m_lam = ml;
    X->sig = sig ? sig : X->lev[0].muc;
    X->sig64 = sig64;
  }
  const int m = p->restart;
  for (int i = 0; i <= m; i++) {
    void *v = cv.take(nn * 8);
    if (X) X->V[i] = (double *)v;
  }
  if (p->krylov == STOKES_FGMRES) {
    for (int i = 0; i < m; i++) {
      void *z = cv.take(nn * tb);
      if (X) X->Z[i] = z;
    }
  }
  double *r = (double *)cv.take(nn * 8), *w = (double *)cv.take(nn * 8);
  double *t = (double *)cv.take(nn * 8), *x = (double *)cv.take(nn * 8);
  double *b = (double *)cv.take(nn * 8);
  void *pin = cv.take(nn * tb), *pout = cv.take(nn * tb);
  void *xs = cv.take(nv * tb), *tu = cv.take(nv * tb), *eu = cv.take(nv * tb);
  void *cvv = cv.take(nc * tb), *q = cv.take(nc * tb);
  void *vs_r = cv.take(nv * tb), *vs_t = cv.take(nv * tb), *vs_de = cv.take(nv * tb);
  void *ps_r = cv.take(nc * tb), *ps_t = cv.take(nc * tb), *ps_de = cv.take(nc * tb);
  double *ge = (double *)cv.take(ne * 8);
  double *gc = (double *)cv.take(nc * 8);
  double *sd = (p->scaling == STOKES_SCALE_DIAGONAL) ? (double *)cv.take(nn * 8) : nullptr;
  if (X) X->sdiag = sd;
  double *tm = (double *)cv.take((size_t)(kMaxRestart + 1) * (kMaxRestart + 1) * 8);
  if (X) X->tmat = tm;
  if (use_vsplit(p)) {
    void *a = cv.take(nv * tb), *b = cv.take(nv * tb), *c = cv.take(nv * tb);
    if (X) {
      X->vrs = a;
      X->ves = b;
      X->alpha_v = c;
    }
  }
  double *part = (double *)cv.take((size_t)kRedBlocks * (kMaxRestart + 2) * 8);
  double *dsc = (double *)cv.take(kDscSlots * 8);
  int *dflag = (int *)cv.take(64);
  // FP64 coefficient chain for building the FP32 hierarchy: level-0 beta and
  // every coarser level (alpha, beta, mu_cell, mu_edge)
  if (p->precision == STOKES_MG_FP32) {
    double *b0 = (double *)cv.take(nv * 8);
    if (X) {
      X->c64a[0] = ma;
      X->c64b[0] = b0;
      X->c64m[0] = mc;
      X->c64e[0] = me;
      X->c64l[0] = ml;
    }
    for (int l = 1; l < nlev; l++) {
      int nl[3];
      for (int a = 0; a < 3; a++) nl[a] = (a < d) ? (n[a] >> l) : 1;
      Geo g = make_geo(d, nl, ns, p->h * (double)(1 << l));
      double *a_ = (double *)cv.take(g.nvel * 8), *b_ = (double *)cv.take(g.nvel * 8);
      double *m_ = (double *)cv.take(g.ncell * 8), *e_ = (double *)cv.take(g.nedge * 8);
      double *l_ = p->bulk ? (double *)cv.take(g.ncell * 8) : nullptr;
      if (X) {
        X->c64a[l] = a_;
        X->c64b[l] = b_;
        X->c64m[l] = m_;
        X->c64e[l] = e_;
        X->c64l[l] = l_;
      }
    }
  }
  if (X) {
    X->r = r; X->w = w; X->t = t; X->x = x; X->b = b;
    X->pin = pin; X->pout = pout; X->xs = xs; X->tu = tu; X->eu = eu;
    X->cv = cvv; X->q = q;
    X->vs_r = vs_r; X->vs_t = vs_t; X->vs_de = vs_de;
    X->ps_r = ps_r; X->ps_t = ps_t; X->ps_de = ps_de;
    X->gedge = ge; X->gcell = gc; X->part = part; X->dsc = dsc; X->dflag = dflag;
  }
}

inline bool hip_ok(stokes_ctx *X, hipError_t e) {
  if (e != hipSuccess) {
    X->err = 1;
    return false;
  }
  return true;
}

int finish(stokes_ctx *X, int rc) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || X->err) {
    X->err = 0;
    return STOKES_EDEVICE;
  }
  return rc;
}

// ---------------- timing ----------------
void fold_vevents(stokes_ctx *X) {
  if (X->vev_used == 0) return;
  (void)hipStreamSynchronize(X->s);
  for (int i = 0; i < X->vev_used; i++) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, X->vev[2 * i], X->vev[2 * i + 1]) == hipSuccess)
      X->vc_ms[X->vev_kind[i]] += ms;
  }
  X->vev_used = 0;
}

void fold_events(stokes_ctx *X) {
  if (X->ev_used == 0) return;
  (void)hipStreamSynchronize(X->s);
  for (int i = 0; i < X->ev_used; i++) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, X->ev[2 * i], X->ev[2 * i + 1]) == hipSuccess) X->t_ms += ms;
  }
  X->ev_used = 0;
}

// ---------------- device helpers (precision T) ----------------
template <typename T>
inline T *P(void *a) {
  return (T *)a;
}

// The mass coefficient alpha = theta rho_f is identically zero for steady
// problems; the kernels then get no alpha array and skip the term (0 * u
// adds nothing, so the result is the same bit for bit).
template <typename T>
inline const T *alpha_of(const stokes_ctx *X, const Level &L) {
  return X->p.theta == 0.0 ? nullptr : (const T *)L.alpha;
}
inline const double *m_alpha_of(const stokes_ctx *X) {
  return X->p.theta == 0.0 ? nullptr : X->m_alpha;
}
template <typename T>
inline const T *lam_of(const Level &L) {
  return (const T *)L.lam;
}
// alpha of the velocity multigrid on level l (the colour-split copy on a
// split finest level)
template <typename T>
inline const T *valpha_of(const stokes_ctx *X, int l) {
  if (X->p.theta == 0.0) return nullptr;
  return (l == 0 && X->vsplit) ? (const T *)X->alpha_v : (const T *)X->lev[l].alpha;
}
// alpha in the velocity multigrid's storage order: a copy on the finest
// level (its natural-order alpha also serves P5's residual), in place on the
// other split levels (only the velocity multigrid reads them)
template <typename T>
void split_alpha(stokes_ctx *X) {
  const Level &L0 = X->lev[0];
  launch_vel_permute<T>(L0.g, L0.gv, P<T>(L0.alpha), P<T>(X->alpha_v), nullptr, X->s);
  for (int l = 1; l < X->nlev && X->lev[l].gv.split; l++) {
    Level &L = X->lev[l];
    launch_vel_permute<T>(L.g, L.gv, P<T>(L.alpha), P<T>(X->vrs), nullptr, X->s);
    launch_cast<T, T>(P<T>(X->vrs), P<T>(L.alpha), L.g.nvel, X->s);
  }
}

// Algorithmic bytes of one V-cycle from the finest level (each value a
// kernel needs counted once per kernel, the same model as the colour-pass
// figure), summed over the levels; s = bytes per value of the hierarchy.
// Velocity, per level: the zero fill of phi; each colour pass of component k
// reads all components, mu_cell, the bulk coefficient (if any) and the edge
// families touching k in full, and its colour's half of rhs_k and alpha_k
// (theta != 0), and writes that half of component k; on all but the coarsest
// level the residual (rhs, phi, alpha, mu_cell, edges, bulk -> res), the
// face restriction (res -> coarse rhs) and the prolongation (coarse phi,
// phi -> phi).  A velocity level above the coarse tail that starts with a
// sweep has no fill, and the passes of its first sweep read only the
// components already written in that sweep (on its second colour, the half
// of component k its first colour wrote).  Pressure alike with beta on the
// faces and red-black passes over the cells (half of rhs read and half of
// phi written per pass).  A velocity tail applied as its matrix counts the
// matrix, its input and its output instead of the tail levels' kernels.
double vcycle_alg_bytes(const stokes_ctx *X, bool vel) {
  const double s = X->mg32 ? 4.0 : 8.0;
  const bool th = X->p.theta != 0.0;
  double total = 0.0;
  for (int l = 0; l < X->nlev; l++) {
    if (vel && X->tail_dense && l >= X->tail_l) {
      const double nt = (double)X->tail_nv;
      total += s * (nt * nt + 2.0 * nt);
      break;
    }
    const Geo &g = X->lev[l].g;
    const double nv = (double)g.nvel, nc = (double)g.ncell, ne = (double)g.nedge;
    const bool coarsest = (l == X->nlev - 1);
    const int sweeps = coarsest ? X->p.nu_coarse : X->p.nu_pre + X->p.nu_post;
    double b = 0.0;
    if (vel) {
      const bool in_tail = X->tail_l >= 0 && l >= X->tail_l;
      const int first_sweeps = coarsest ? X->p.nu_coarse : X->p.nu_pre;
      const bool zf = !in_tail && gs_first_ok(g) && first_sweeps > 0;
      if (!zf) b += nv;  // zero fill
      double sweep = 0.0, first = 0.0, done = 0.0;
      for (int k = 0; k < g.d; k++) {
        double e = 0.0;
        for (int m = 0; m < 3; m++)
          if ((m != k || g.d == 2) && g.ecnt[m] > 0) e += (double)g.ecnt[m];
        const double fk = (double)g.fcnt[k];
        // half of rhs_k (and of alpha_k), mu_cell (bulk), edges; each pass
        // also writes its half of component k
        const double coef = (th ? 1.0 : 0.5) * fk + (X->bulk ? 2.0 : 1.0) * nc + e;
        sweep += 2.0 * (nv + coef + 0.5 * fk);
        first += (done + coef + 0.5 * fk) + (done + 0.5 * fk + coef + 0.5 * fk);
        done += fk;
      }
      b += zf ? first + (sweeps - 1) * sweep : sweeps * sweep;
      if (!coarsest) {
        const double nvc = (double)X->lev[l + 1].g.nvel;
        b += 3.0 * nv + (th ? nv : 0.0) + nc + ne + (X->bulk ? nc : 0.0);  // residual
        b += nv + nvc;                                                    // restriction
        b += nvc + 2.0 * nv;                                              // prolongation
      }
    } else {
      const bool in_tail = X->tail_l >= 0 && l >= X->tail_l;
      const int first_sweeps = coarsest ? X->p.nu_coarse : X->p.nu_pre;
      const bool zf = !in_tail && gs_first_ok(g) && first_sweeps > 0;
      // per pass beta and phi read in full, half of rhs read and half of phi
      // written; the first sweep's first colour reads no phi, its second
      // colour only the half the first wrote, and there is no fill
      if (zf)
        b += (nv + nc) + (nv + 1.5 * nc) + (sweeps - 1) * 2.0 * (nv + 2.0 * nc);
      else
        b += nc + sweeps * 2.0 * (nv + 2.0 * nc);
      if (!coarsest) {
        const double ncc = (double)X->lev[l + 1].g.ncell;
        b += nv + 3.0 * nc;                      // residual
        b += nc + ncc;                           // restriction
        b += ncc + 2.0 * nc;                     // prolongation
      }
    }
    total += s * b;
  }
  return total;
}

template <typename T>
void remove_mean(stokes_ctx *X, T *a, i64 n, int slot) {
  launch_sum<T>(a, n, X->part, X->dsc + slot, X->s);
  launch_sub_mean<T>(a, n, X->dsc + slot, X->s);
}

template <typename T>
void remove_vel_means(stokes_ctx *X, const Geo &g, T *u) {
  // only used when every axis is periodic: every face is an unknown
  launch_vel_remove_means<T>(g, u, u, X->part, X->dsc + 8, X->s);
}

// nsweeps multicolour Gauss-Seidel sweeps of the velocity (Appendix C: per
// sweep x-red, x-black, y-red, y-black[, z-red, z-black]), one launch per
// colour, in place.  from_zero: phi is the zero iterate but its memory has
// not been cleared; the first sweep then reads the values not yet written as
// zero.
template <typename T>
void smooth_vel(stokes_ctx *X, int l, const T *rhs, T *phi, int nsweeps, bool from_zero = false) {
  Level &L = X->lev[l];
  for (int s = 0; s < nsweeps; s++)
    for (int k = 0; k < L.g.d; k++)
      for (int colour = 0; colour < 2; colour++) {
        const int first = from_zero && s == 0;
        // the timed passes are the full ones (the first sweep reads less)
        const bool tm = X->timing == 1 && l == 0 && !first;
        if (tm) {
          if (X->ev_used == kEventPool) fold_events(X);
          (void)hipEventRecord(X->ev[2 * X->ev_used], X->s);
        }
        launch_vel_gs<T>(L.gv, k, colour, first, valpha_of<T>(X, l), P<T>(L.muc), P<T>(L.mue),
                         lam_of<T>(L), rhs, phi, X->s);
        if (tm) {
          (void)hipEventRecord(X->ev[2 * X->ev_used + 1], X->s);
          X->ev_used++;
          X->launches++;
          X->bytes += X->gs_bytes[k];
        }
      }
}

template <typename T>
void sweep_p(stokes_ctx *X, int l, const T *rhs, T *phi, bool from_zero = false) {
  const Level &L = X->lev[l];
  launch_p_gs<T>(L.g, 0, from_zero, P<T>(L.beta), rhs, phi, X->s);
  launch_p_gs<T>(L.g, 1, from_zero, P<T>(L.beta), rhs, phi, X->s);
}

// levels tail_l..nlev-1 of a V-cycle in one launch; level tail_l works on
// the caller's rhs / phi, the deeper ones on the level buffers
template <typename T>
TailLevels<T> tail_levels(stokes_ctx *X, int l0, const T *rhs, T *phi, bool vel) {
  TailLevels<T> t;
  t.nl = X->nlev - l0;
  t.singular = vel ? X->vel_singular : 1;
  t.nu_pre = X->p.nu_pre;
  t.nu_post = X->p.nu_post;
  t.nu_coarse = X->p.nu_coarse;
  for (int i = 0; i < kTailMax; i++) {
    const int l = l0 + i;
    if (i >= t.nl) {
      t.g[i] = X->lev[l0].g;
      t.a[i] = t.b[i] = t.mc[i] = t.me[i] = t.lam[i] = nullptr;
      t.phi[i] = t.rhs[i] = t.res[i] = nullptr;
      continue;
    }
    Level &L = X->lev[l];
    t.g[i] = vel ? L.gv : L.g;
    t.a[i] = vel ? valpha_of<T>(X, l) : alpha_of<T>(X, L);
    t.b[i] = P<T>(L.beta);
    t.mc[i] = P<T>(L.muc);
    t.me[i] = P<T>(L.mue);
    t.lam[i] = vel ? lam_of<T>(L) : nullptr;
    t.phi[i] = P<T>(vel ? L.phi_u : L.phi_p);
    t.rhs[i] = P<T>(vel ? L.rhs_u : L.rhs_p);
    t.res[i] = P<T>(vel ? L.res_u : L.res_p);
  }
  t.rhs[0] = const_cast<T *>(rhs);
  t.phi[0] = phi;
  tail_plan_lds<T>(t, vel);
  return t;
}

// B of the velocity tail: one workgroup per column, each running the tail on
// a unit vector with its own vectors in LDS.  False (tail_dense off) when
// the vectors do not fit.
template <typename T>
bool build_tail_matrix(stokes_ctx *X) {
  TailLevels<T> t = tail_levels<T>(X, X->tail_l, nullptr, nullptr, true);
  if (!tail_plan_lds<T>(t, true, true)) return false;
  launch_tail_vel_columns<T>(t, P<T>(X->tail_B), X->tail_nv, X->s);
  return true;
}

// velocity V-cycle on level l from zero (Appendix C)
template <typename T>
void vcycle_vel(stokes_ctx *X, int l, const T *rhs, T *phi) {
  Level &L = X->lev[l];
  if (l == X->tail_l) {
    if (X->tail_dense)
      launch_tail_matvec<T>(P<T>(X->tail_B), X->tail_nv, rhs, phi, X->s);
    else
      launch_tail_vel<T>(tail_levels<T>(X, l, rhs, phi, true), X->s);
    return;
  }
  const bool coarsest = l == X->nlev - 1;
  // the first sweep writes every face of the zero iterate, so the clearing
  // pass is needed only without a sweep or where the colouring does not
  // hold across a periodic wrap
  const bool zf = gs_first_ok(L.gv) && (coarsest ? X->p.nu_coarse : X->p.nu_pre) > 0;
  if (!zf) launch_fill<T>(phi, (T)0, L.gv.nvel, X->s);
  if (coarsest) {
    T *r = P<T>(L.res_u);
    if (X->vel_singular)
      launch_vel_remove_means<T>(L.gv, rhs, r, X->part, X->dsc + 8, X->s);
    else
      launch_cast<T, T>(rhs, r, L.gv.nvel, X->s);
    smooth_vel<T>(X, l, r, phi, X->p.nu_coarse, zf);
    if (X->vel_singular) remove_vel_means<T>(X, L.gv, phi);
    return;
  }
  Level &C = X->lev[l + 1];
  smooth_vel<T>(X, l, rhs, phi, X->p.nu_pre, zf);
  launch_vel_residual<T>(L.gv, valpha_of<T>(X, l), P<T>(L.muc), P<T>(L.mue), lam_of<T>(L), rhs,
                         phi, nullptr, P<T>(L.res_u), X->s);
  launch_face_restrict<T>(L.gv, C.gv, P<T>(L.res_u), P<T>(C.rhs_u), X->s);
  vcycle_vel<T>(X, l + 1, P<T>(C.rhs_u), P<T>(C.phi_u));
  launch_face_prolong_add<T>(C.gv, L.gv, P<T>(C.phi_u), phi, X->s);
  smooth_vel<T>(X, l, rhs, phi, X->p.nu_post);
}

// Records the colour-split finest-level V-cycle (vrs -> ves) on a private
// stream into vgraph / vgexec.  Nothing runs during the capture.
template <typename T>
bool capture_vcycle(stokes_ctx *X) {
  if (hipStreamCreateWithFlags(&X->gstream, hipStreamNonBlocking) != hipSuccess) {
    X->gstream = nullptr;
    return false;
  }
  if (hipStreamBeginCapture(X->gstream, hipStreamCaptureModeRelaxed) != hipSuccess) return false;
  hipStream_t user = X->s;
  const int tm = X->timing;
  X->timing = 0;
  X->s = X->gstream;
  vcycle_vel<T>(X, 0, P<T>(X->vrs), P<T>(X->ves));
  X->s = user;
  X->timing = tm;
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(X->gstream, &g) != hipSuccess || !g) return false;
  X->vgraph = g;
  if (hipGraphInstantiate(&X->vgexec, g, nullptr, nullptr, 0) != hipSuccess) {
    X->vgexec = nullptr;
    return false;
  }
  return true;
}

void release_vgraph(stokes_ctx *X) {
  if (X->vgexec) (void)hipGraphExecDestroy(X->vgexec);
  if (X->vgraph) (void)hipGraphDestroy(X->vgraph);
  if (X->gstream) (void)hipStreamDestroy(X->gstream);
  X->vgexec = nullptr;
  X->vgraph = nullptr;
  X->gstream = nullptr;
}

// pressure V-cycle; singular operator: consistent coarsest problem by mean
// removal
template <typename T>
void vcycle_p(stokes_ctx *X, int l, const T *rhs, T *phi) {
  Level &L = X->lev[l];
  if (l == X->tail_l) {
    launch_tail_p<T>(tail_levels<T>(X, l, rhs, phi, false), X->s);
    return;
  }
  const bool coarsest = l == X->nlev - 1;
  // as for the velocity: the first sweep replaces the clearing pass
  const bool zf = gs_first_ok(L.g) && (coarsest ? X->p.nu_coarse : X->p.nu_pre) > 0;
  if (!zf) launch_fill<T>(phi, (T)0, L.g.ncell, X->s);
  if (coarsest) {
    T *r = P<T>(L.res_p);
    launch_cast<T, T>(rhs, r, L.g.ncell, X->s);
    remove_mean<T>(X, r, L.g.ncell, 16);
    for (int s = 0; s < X->p.nu_coarse; s++) sweep_p<T>(X, l, r, phi, zf && s == 0);
    remove_mean<T>(X, phi, L.g.ncell, 17);
    return;
  }
  Level &C = X->lev[l + 1];
  for (int s = 0; s < X->p.nu_pre; s++) sweep_p<T>(X, l, rhs, phi, zf && s == 0);
  launch_p_residual<T>(L.g, P<T>(L.beta), rhs, phi, P<T>(L.res_p), X->s);
  launch_cell_restrict<T>(L.g, C.g, P<T>(L.res_p), P<T>(C.rhs_p), X->s);
  vcycle_p<T>(X, l + 1, P<T>(C.rhs_p), P<T>(C.phi_p));
  launch_cell_prolong_add<T>(C.g, L.g, P<T>(C.phi_p), phi, X->s);
  for (int s = 0; s < X->p.nu_post; s++) sweep_p<T>(X, l, rhs, phi);
}

// A V-cycle from the finest level, bracketed by events when timing is on.
// means_in / means_out (velocity, colour-split finest level only): remove
// the singular components' means from rhs on the way in and from the result
// on the way out, inside the reordering passes.
template <typename T>
void vcycle_top(stokes_ctx *X, bool vel, const T *rhs, T *phi, bool means_in = false,
                bool means_out = false) {
  const bool tm = X->timing != 0;
  const int kind = vel ? 0 : 1;
  if (tm) {
    if (X->vev_used == kEventPool) fold_vevents(X);
    (void)hipEventRecord(X->vev[2 * X->vev_used], X->s);
  }
  if (vel && X->vsplit) {
    // the finest level runs in the colour-split order: reorder in and out
    const Level &L0 = X->lev[0];
    double *sums = X->dsc + 8;
    if (means_in) launch_vel_sums<T>(L0.g, rhs, X->part, sums, X->s);
    launch_vel_permute<T>(L0.g, L0.gv, rhs, P<T>(X->vrs), means_in ? sums : nullptr, X->s);
    if (X->vgexec && X->timing != 1)
      hip_ok(X, hipGraphLaunch(X->vgexec, X->s));
    else
      vcycle_vel<T>(X, 0, P<T>(X->vrs), P<T>(X->ves));
    if (means_out) launch_vel_sums<T>(L0.gv, P<T>(X->ves), X->part, sums, X->s);
    launch_vel_permute<T>(L0.gv, L0.g, P<T>(X->ves), phi, means_out ? sums : nullptr, X->s);
  } else if (vel) {
    vcycle_vel<T>(X, 0, rhs, phi);
  } else {
    vcycle_p<T>(X, 0, rhs, phi);
  }
  if (tm) {
    (void)hipEventRecord(X->vev[2 * X->vev_used + 1], X->s);
    X->vev_kind[X->vev_used] = kind;
    X->vev_used++;
    X->vc_count[kind]++;
    X->vc_bytes[kind] += X->vc_cycle_bytes[kind];
  }
}

// A~^{-1} r: `vcycles` V-cycles, zero initial guess (Sec. "Krylov Solver")
template <typename T>
void vel_sub(stokes_ctx *X, const T *r, T *e) {
  Level &L = X->lev[0];
  if (X->vsplit && X->vel_singular && X->p.vcycles == 1) {
    // one cycle on the colour-split finest level: the mean removals ride on
    // the two reordering passes
    vcycle_top<T>(X, true, r, e, true, true);
    return;
  }
  const T *rr = r;
  if (X->vel_singular) {
    launch_vel_remove_means<T>(L.g, r, P<T>(X->vs_r), X->part, X->dsc + 8, X->s);
    rr = P<T>(X->vs_r);
  }
  vcycle_top<T>(X, true, rr, e);
  for (int v = 1; v < X->p.vcycles; v++) {
    launch_vel_residual<T>(L.g, alpha_of<T>(X, L), P<T>(L.muc), P<T>(L.mue), lam_of<T>(L), rr,
                           e, nullptr, P<T>(X->vs_t), X->s);
    vcycle_top<T>(X, true, P<T>(X->vs_t), P<T>(X->vs_de));
    launch_axpy<T>((T)1, P<T>(X->vs_de), e, L.g.nvel, X->s);
  }
  if (X->vel_singular) remove_vel_means<T>(X, L.g, e);
}

// L~_rho^{-1} r
template <typename T>
void p_sub(stokes_ctx *X, const T *r, T *e) {
  Level &L = X->lev[0];
  launch_cast<T, T>(r, P<T>(X->ps_r), L.g.ncell, X->s);
  remove_mean<T>(X, P<T>(X->ps_r), L.g.ncell, 18);
  const T *rr = P<T>(X->ps_r);
  vcycle_top<T>(X, false, rr, e);
  for (int v = 1; v < X->p.vcycles; v++) {
    launch_p_residual<T>(L.g, P<T>(L.beta), rr, e, P<T>(X->ps_t), X->s);
    vcycle_top<T>(X, false, P<T>(X->ps_t), P<T>(X->ps_de));
    launch_axpy<T>((T)1, P<T>(X->ps_de), e, L.g.ncell, X->s);
  }
  remove_mean<T>(X, e, L.g.ncell, 19);
}

// out = -S~^{-1} c = theta L~_rho^{-1} c - 2 mu c  (eq. Schur_app_varDen_varVis;
// with bulk viscosity gamma + 4/3 mu in place of 2 mu, eq. Schur_app_bulk)
template <typename T>
void neg_schur(stokes_ctx *X, const T *c, T *out) {
  Level &L = X->lev[0];
  if (X->p.theta != 0.0) {
    p_sub<T>(X, c, P<T>(X->q));
    launch_schur_combine<T>(P<T>(X->q), c, P<T>(X->sig), (T)X->p.theta, (T)-2, out, L.g.ncell,
                            X->s);
  } else {
    launch_schur_combine<T>(nullptr, c, P<T>(X->sig), (T)0, (T)-2, out, L.g.ncell, X->s);
  }
}

// out = -S~^{-1}(sgn (D u + bp)): at theta = 0 the Schur approximation is
// the cellwise scaling by -2 mu (or the bulk coefficient), applied in the
// divergence pass itself
template <typename T>
void neg_schur_div(stokes_ctx *X, const T *u, const T *bp, T *out) {
  const Geo &g = X->lev[0].g;
  if (X->p.theta == 0.0) {
    launch_div_scaled<T>(g, u, bp, (T)1, P<T>(X->sig), (T)-2, out, X->s);
  } else {
    launch_div<T>(g, u, bp, (T)1, P<T>(X->cv), X->s);
    neg_schur<T>(X, P<T>(X->cv), out);
  }
}

// z = P^{-1} b on the rescaled system (Sec. "Preconditioners" block factorisations)
template <typename T>
void precond(stokes_ctx *X, const T *bu, const T *bp, T *zu, T *zp) {
  Level &L = X->lev[0];
  const Geo &g = L.g;
  T *xs = P<T>(X->xs), *tu = P<T>(X->tu), *eu = P<T>(X->eu), *cv = P<T>(X->cv), *q = P<T>(X->q);
  switch (X->p.precond) {
    case STOKES_P1:
      // x* = A~^{-1} b_u; c = -(D x* + b_p); q = L~^{-1} c;
      // x_u = x* + rho_f^{-1} G q; x_p = -theta q + 2 mu c
      vel_sub<T>(X, bu, xs);
      launch_div<T>(g, xs, bp, (T)-1, cv, X->s);
      p_sub<T>(X, cv, q);
      launch_proj_update<T>(g, xs, P<T>(L.beta), q, zu, X->s);
      launch_schur_combine<T>(q, cv, P<T>(X->sig), (T)(-X->p.theta), (T)2, zp, g.ncell, X->s);
      break;
    case STOKES_P2:
      // x_u = A~^{-1} b_u; x_p = -S~^{-1}(D x_u + b_p)
      vel_sub<T>(X, bu, zu);
      neg_schur_div<T>(X, zu, bp, zp);
      break;
    case STOKES_P3:
      // x_p = -S~^{-1} b_p; x_u = A~^{-1}(b_u - G x_p)
      neg_schur<T>(X, bp, zp);
      launch_grad_sub<T>(g, bu, zp, tu, X->s);
      vel_sub<T>(X, tu, zu);
      break;
    case STOKES_P4:
      vel_sub<T>(X, bu, zu);
      neg_schur<T>(X, bp, zp);
      break;
    case STOKES_P5:
      // x* = A~^{-1} b_u; x_p = -S~^{-1}(D x* + b_p);
      // x_u = x* + A~^{-1}(b_u - G x_p - A x*)
      vel_sub<T>(X, bu, xs);
      neg_schur_div<T>(X, xs, bp, zp);
      launch_vel_residual<T>(g, alpha_of<T>(X, L), P<T>(L.muc), P<T>(L.mue), lam_of<T>(L), bu, xs,
                             zp, tu, X->s);
      vel_sub<T>(X, tu, eu);
      launch_cast<T, T>(xs, zu, g.nvel, X->s);
      launch_axpy<T>((T)1, eu, zu, g.nvel, X->s);
      break;
  }
  remove_mean<T>(X, zp, g.ncell, 20);
  // the subsolver output is already mean-free; only P1 adds rho_f^{-1} G q
  if (X->vel_singular && X->p.precond == STOKES_P1) remove_vel_means<T>(X, g, zu);
}

// z (precision of the hierarchy, [u|p]) = P^{-1} v with v FP64 [u|p]
// have32: the FP32 copy of v is already in X->pin (written by the Arnoldi pass)
void precond_from64(stokes_ctx *X, const double *v, void *z, bool have32 = false) {
  const i64 nv = X->nvel;
  if (X->mg32) {
    float *pin = P<float>(X->pin);
    if (!have32) launch_cast<float, double>(v, pin, X->n, X->s);
    precond<float>(X, pin, pin + nv, P<float>(z), P<float>(z) + nv);
  } else {
    precond<double>(X, v, v + nv, P<double>(z), P<double>(z) + nv);
  }
}

// y = M' x on the rescaled system (FP64)
void apply_scaled(stokes_ctx *X, const double *x, double *y) {
  const Geo &g = X->lev[0].g;
  launch_apply_m<double>(g, m_alpha_of(X), X->m_muc, X->m_mue, X->m_lam, x, x + X->nvel, nullptr,
                         nullptr, y, y + X->nvel, X->s);
}

double fetch(stokes_ctx *X, const double *dev, int count, double *dst) {
  hip_ok(X, hipMemcpyAsync(dst, dev, count * sizeof(double), hipMemcpyDeviceToHost, X->s));
  hip_ok(X, hipStreamSynchronize(X->s));
  return dst[0];
}

// Restarted GMRES(m), left-preconditioned or flexible, on the rescaled system
// b' -> x' held in X->b, X->x.  The Arnoldi orthogonalisation is classical
// Gram-Schmidt applied twice (CGS2) in three streaming passes, the new
// vector's norm from ||w'||^2 - ||h2||^2 unless the second pass removed half
// or more of ||w'||^2 (then w'' is formed and measured); in exact arithmetic
// this is the same Hessenberg matrix as modified Gram-Schmidt.  Givens
// rotations on the host; the solve ends on the true residual, each cycle on
// the Givens estimate reduced by the factor the true residual still lacks.
// Preconditioner applications bracketed by the ctx's two events; the time is
// folded in at the next synchronisation of the iteration (prec_fold).
struct PrecClock {
  stokes_ctx *X;
  double ms = 0.0;
  int cur = 0;
  bool open[2] = {false, false};
  void start() {
    if (!X->pev[0]) return;
    if (open[cur]) fold_pair(cur, true);  // two applications back: long done
    (void)hipEventRecord(X->pev[2 * cur], X->s);
  }
  void stop() {
    if (!X->pev[0]) return;
    (void)hipEventRecord(X->pev[2 * cur + 1], X->s);
    open[cur] = true;
    cur ^= 1;
  }
  void fold_pair(int q, bool wait) {
    if (!open[q]) return;
    if (wait) (void)hipEventSynchronize(X->pev[2 * q + 1]);
    else if (hipEventQuery(X->pev[2 * q + 1]) != hipSuccess) return;
    float t = 0.f;
    if (hipEventElapsedTime(&t, X->pev[2 * q], X->pev[2 * q + 1]) == hipSuccess) ms += t;
    open[q] = false;
  }
  // the applications that have finished (wait: all of them)
  void fold(bool wait = false) {
    fold_pair(cur ^ 1, wait);
    fold_pair(cur, wait);
  }
};

// ||b - M x|| / ||b|| of the caller's system, from the scaled residual and
// right-hand side (r' = (c r_u, r_p), b' = (c b_u, b_p))
double unscaled_rel(stokes_ctx *X, const double *r) {
  const i64 nv = X->nvel, nc = X->ncell;
  double *hb = X->host;
  launch_norm2(r, nv, X->part, X->dsc + 0, X->s);
  launch_norm2(r + nv, nc, X->part, X->dsc + 1, X->s);
  launch_norm2(X->b, nv, X->part, X->dsc + 2, X->s);
  launch_norm2(X->b + nv, nc, X->part, X->dsc + 3, X->s);
  fetch(X, X->dsc, 4, hb);
  const double c2 = X->c * X->c;
  const double num = hb[0] / c2 + hb[1], den = hb[2] / c2 + hb[3];
  return den > 0.0 ? std::sqrt(num / den) : 0.0;
}

// r-hat = S (b' - M' x') into X->r: the true residual in FP64 or in
// double-double arithmetic (extended), scaled by the diagonal scaling when
// the context has one
void true_residual(stokes_ctx *X) {
  const Geo &g = X->lev[0].g;
  const i64 nv = X->nvel;
  if (X->p.extended)
    launch_residual_dd(g, m_alpha_of(X), X->m_muc, X->m_mue, X->m_lam, X->x, X->x + nv, X->b,
                       X->b + nv, X->r, X->r + nv, X->s);
  else
    launch_apply_m<double>(g, m_alpha_of(X), X->m_muc, X->m_mue, X->m_lam, X->x, X->x + nv, X->b,
                           X->b + nv, X->r, X->r + nv, X->s);
  if (X->sdiag) launch_mul_scaling(X->r, X->sdiag, 0, X->n, X->r, X->s);
}

// With the diagonal scaling S the Krylov method runs on S M' S for S^{-1} x'
// with right-hand side S b' and the preconditioner S^{-1} P'^{-1} S^{-1}; the
// iterate stays x' (flexible: x' += Z y with Z = P'^{-1} S^{-1} V; left:
// x' += S V y).
int krylov(stokes_ctx *X, double tol, int max_iter, stokes_stats *st) {
  const int m = X->p.restart;
  const int flexible = (X->p.krylov == STOKES_FGMRES);
  const i64 n = X->n, nv = X->nvel;
  stokes_stats local;
  if (!st) st = &local;
  std::memset(st, 0, sizeof(*st));
  double *const hist = X->hist;
  const int hcap = X->hist_cap;
  PrecClock pc{X};
  const auto t0 = std::chrono::steady_clock::now();
  struct Finish {  // wall and preconditioner times on every exit path
    stokes_stats *st;
    PrecClock &pc;
    std::chrono::steady_clock::time_point t0;
    ~Finish() {
      pc.fold(true);
      st->t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      st->t_precond = pc.ms * 1e-3;
      st->t_krylov = st->t_total - st->t_precond;
    }
  } fin{st, pc, t0};
  double *hb = X->host;
  const double *S = X->sdiag;
  if (S) {
    launch_mul_scaling(X->b, S, 0, n, X->t, X->s);
    launch_norm2(X->t, n, X->part, X->dsc + 0, X->s);
  } else {
    launch_norm2(X->b, n, X->part, X->dsc + 0, X->s);
  }
  const double nb = std::sqrt(fetch(X, X->dsc, 1, hb));
  if (X->err) return STOKES_EDEVICE;
  if (nb == 0.0) {
    launch_fill<double>(X->x, 0.0, n, X->s);
    return STOKES_OK;
  }
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  // unrotated Hessenberg columns (left GMRES), the correction of the
  // provisional basis vector (c, 1 / alpha) for this step and the next
  std::vector<double> Hraw((size_t)(m + 1) * m), colbuf(m + 2), cprev(m + 2), cnext(m + 2),
      tc(m + 2), Tm((size_t)(m + 1) * (m + 1)), ty(m + 1);
  double iaprev = 1.0, ianext = 1.0;
  int it = 0, rc = STOKES_OK;
  for (;;) {
    // r = b - M x and its norm
    true_residual(X);
    launch_norm2(X->r, n, X->part, X->dsc + 0, X->s);
    const double rho = std::sqrt(fetch(X, X->dsc, 1, hb));
    if (X->err) return STOKES_EDEVICE;
    pc.fold();
    st->rel_res_true = rho / nb;
    if (!std::isfinite(rho)) { rc = STOKES_ENONFINITE; break; }
    if (rho <= tol * nb) { rc = STOKES_OK; break; }
    if (it >= max_iter) { rc = STOKES_ENOCONV; break; }
    st->restarts++;
    double beta;
    if (flexible) {
      beta = rho;
      launch_scale(X->r, 1.0 / beta, X->V[0], n, X->s);
    } else {
      pc.start();
      if (S) launch_mul_scaling(X->r, S, 1, n, X->r, X->s);
      precond<double>(X, X->r, X->r + nv, X->V[0], X->V[0] + nv);
      if (S) launch_mul_scaling(X->V[0], S, 1, n, X->V[0], X->s);
      pc.stop();
      st->precond_applies++;
      launch_norm2(X->V[0], n, X->part, X->dsc + 0, X->s);
      beta = std::sqrt(fetch(X, X->dsc, 1, hb));
      pc.fold();
      if (!std::isfinite(beta)) { rc = STOKES_ENONFINITE; break; }
      if (beta == 0.0) { rc = STOKES_EBREAKDOWN; break; }
      launch_scale(X->V[0], 1.0 / beta, X->V[0], n, X->s);
    }
    const double target = beta * tol * nb / rho;
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(Hraw.begin(), Hraw.end(), 0.0);
    // V[0] is exactly normalised: T = I so far
    std::fill(Tm.begin(), Tm.end(), 0.0);
    for (int i = 0; i <= m; i++) Tm[(size_t)i * (m + 1) + i] = 1.0;
    iaprev = 1.0;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jj = 0;
    // the preconditioner application of V[j] was already queued at the end
    // of step j - 1 (flexible FP32 steps; see below)
    bool queued = false;
    for (int j = 0; j < m; j++) {
      if (j + 1 > 12) {
        // the basis transform outgrows the kernel arguments: stage it in
        // device memory (the copy is ordered after the last step's reads of
        // the host buffer)
        const int ld = m + 1;
        double *tpin = hb + 2048;
        for (int r = 0; r <= j; r++)
          for (int cidx = 0; cidx <= j; cidx++) tpin[r * ld + cidx] = Tm[r * ld + cidx];
        hip_ok(X, hipMemcpyAsync(X->tmat, tpin, (size_t)(j + 1) * ld * sizeof(double),
                                 hipMemcpyHostToDevice, X->s));
      }
      if (flexible) {
        if (!queued) {
          pc.start();
          if (S) {
            launch_mul_scaling(X->V[j], S, 1, n, X->t, X->s);
            precond_from64(X, X->t, X->Z[j], false);
          } else {
            precond_from64(X, X->V[j], X->Z[j], j > 0);
          }
          pc.stop();
        }
        queued = false;
        if (X->mg32)
          launch_apply_m<float>(X->lev[0].g, m_alpha_of(X), X->m_muc, X->m_mue, X->m_lam,
                                P<float>(X->Z[j]),
                                P<float>(X->Z[j]) + nv, nullptr, nullptr, X->w, X->w + nv, X->s);
        else
          apply_scaled(X, P<double>(X->Z[j]), X->w);
        if (S) launch_mul_scaling(X->w, S, 0, n, X->w, X->s);
      } else {
        if (S) {
          launch_mul_scaling(X->V[j], S, 0, n, X->w, X->s);
          apply_scaled(X, X->w, X->t);
        } else {
          apply_scaled(X, X->V[j], X->t);
        }
        pc.start();
        precond<double>(X, X->t, X->t + nv, X->w, X->w + nv);
        if (S) launch_mul_scaling(X->w, S, 1, n, X->w, X->s);
        pc.stop();
      }
      st->precond_applies++;
      it++;
      // Arnoldi step in two passes, the second Gram-Schmidt pass of each new
      // vector lagged into the transform T of the stored once-orthogonalised
      // vectors (orthonormal basis = V T).  Pass R: dots of w with the stored
      // v_0..v_j and (w, w).  Pass U: project w on the orthonormal basis,
      // write the next stored vector (and its FP32 copy for the next
      // flexible preconditioner application) and reduce its dots with the
      // stored vectors.
      const int ld = m + 1;
      launch_cgs_dots(X->w, X->V, j + 1, n, X->part, X->dsc + 32, X->s, true);
      launch_dcgs_update(X->w, X->V, j, X->dsc + 32, Tm.data(), X->tmat, ld, n, X->V[j + 1],
                         (flexible && X->mg32 && !S) ? P<float>(X->pin) : nullptr, X->dsc + 110,
                         X->part, X->dsc + 72, X->s);
      hip_ok(X, hipMemcpyAsync(hb + 110, X->dsc + 110, (j + 2) * sizeof(double),
                               hipMemcpyDeviceToHost, X->s));
      hip_ok(X, hipMemcpyAsync(hb + 72, X->dsc + 72, (j + 2) * sizeof(double),
                               hipMemcpyDeviceToHost, X->s));
      // A flexible FP32 step whose successor exists queues the next
      // preconditioner application (on the FP32 copy of v_{j+1} just
      // written) before the host waits for the step's numbers, so the GPU
      // keeps working through the host's Hessenberg update.  When the
      // correction below rewrites v_{j+1}, the application is repeated;
      // when the cycle ends here, its result is not used.
      if (flexible && X->mg32 && !S && X->sev && j + 1 < m && it < max_iter) {
        hip_ok(X, hipEventRecord(X->sev, X->s));
        pc.start();
        precond_from64(X, X->V[j + 1], X->Z[j + 1], true);
        pc.stop();
        queued = true;
        hip_ok(X, hipEventSynchronize(X->sev));
      } else {
        hip_ok(X, hipStreamSynchronize(X->s));
      }
      if (X->err) return STOKES_EDEVICE;
      pc.fold();
      const double nu = hb[110 + j + 1];
      // d = projections of w on the orthonormal basis (computed by pass U);
      // the next stored vector is (w - V d) / nu
      std::vector<double> &col = colbuf;
      for (int i = 0; i <= j; i++) col[i] = hb[110 + i];
      double sc = nu;  // weight of the stored vector in the column
      if (!flexible) {
        // left GMRES applied the operator to the stored v_j = alpha_j u_j +
        // U c (u the orthonormal basis): by linearity the column of u_j is
        // (U^T w - Hraw c) / alpha_j
        for (int i = 0; i <= j; i++) {
          double acc = col[i];
          for (int l = 0; l < j; l++) acc -= cprev[l] * Hraw[i + (size_t)l * (m + 1)];
          col[i] = acc * iaprev;
        }
        sc = nu * iaprev;
      }
      // second pass of the stored vector: its dots with the orthonormal basis
      // c' = T^T (V^T v_{j+1}), and alpha^2 = |v_{j+1}|^2 - |c'|^2
      double cc = 0.0;
      for (int i = 0; i <= j; i++) {
        double acc = 0.0;
        for (int l = 0; l <= i; l++) acc += Tm[l * ld + i] * hb[72 + l];
        cnext[i] = acc;
        cc += acc * acc;
      }
      const double vv = hb[72 + j + 1];
      // T c' (the coefficients of U c' on the stored vectors)
      for (int l = 0; l <= j; l++) {
        double acc = 0.0;
        for (int i = l; i <= j; i++) acc += Tm[l * ld + i] * cnext[i];
        tc[l] = acc;
      }
      double alpha;
      for (int l = 0; l <= j + 1; l++) Tm[l * ld + j + 1] = 0.0;
      if (vv - cc > 0.5 * vv) {
        alpha = std::sqrt(vv - cc);
        // u_{j+1} = (v_{j+1} - V T c') / alpha
        for (int l = 0; l <= j; l++) Tm[l * ld + j + 1] = -tc[l] / alpha;
        Tm[(j + 1) * ld + j + 1] = 1.0 / alpha;
        ianext = 1.0 / alpha;
      } else {
        // the lagged pass would remove half or more of the stored vector:
        // apply it now, measure and normalise the result (FP32 copy
        // rewritten), which is then stored orthonormal
        double *cpin = hb + 1024;
        for (int l = 0; l <= j; l++) cpin[l] = tc[l];
        hip_ok(X, hipMemcpyAsync(X->dsc + 150, cpin, (j + 1) * sizeof(double),
                                 hipMemcpyHostToDevice, X->s));
        launch_cgs_next(X->V[j + 1], X->V, X->dsc + 150, X->dsc + kZeroSlots, j + 1, 1.0, n,
                        X->V[j + 1], nullptr, X->part, X->dsc + 0, X->s);
        alpha = std::sqrt(fetch(X, X->dsc, 1, hb));
        if (X->err) return STOKES_EDEVICE;
        if (alpha > 0.0)
          launch_cgs_next(X->V[j + 1], X->V, nullptr, nullptr, 0, 1.0 / alpha, n, X->V[j + 1],
                          (flexible && X->mg32 && !S) ? P<float>(X->pin) : nullptr, X->part,
                          nullptr, X->s);
        Tm[(j + 1) * ld + j + 1] = 1.0;
        // the operator of the next left-GMRES step sees the final vector
        ianext = 1.0;
        queued = false;  // the queued application saw the uncorrected vector
      }
      // either way v_{j+1} = alpha u_{j+1} + U c': the column gains sc c'
      for (int i = 0; i <= j; i++) col[i] += sc * cnext[i];
      col[j + 1] = sc * alpha;
      for (int i = 0; i <= j + 1; i++) Hraw[i + (size_t)j * (m + 1)] = col[i];
      if (!(vv - cc > 0.5 * vv))
        for (int i = 0; i <= j; i++) cnext[i] = 0.0;
      std::swap(cprev, cnext);
      iaprev = ianext;
      double *hcol = &H[(size_t)j * (m + 1)];
      for (int i = 0; i <= j + 1; i++) hcol[i] = col[i];
      const double hn = hcol[j + 1];
      for (int i = 0; i < j; i++) {
        const double a = hcol[i], bb = hcol[i + 1];
        hcol[i] = cs[i] * a + sn[i] * bb;
        hcol[i + 1] = -sn[i] * a + cs[i] * bb;
      }
      const double den = std::hypot(hcol[j], hcol[j + 1]);
      if (den == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = hcol[j] / den;
        sn[j] = hcol[j + 1] / den;
      }
      hcol[j] = den;
      hcol[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      jj = j + 1;
      const double est = std::fabs(g[j + 1]);
      st->rel_res_est = est / beta * (rho / nb);
      if (hist && st->history_len < hcap) hist[st->history_len++] = st->rel_res_est;
      if (!std::isfinite(est)) break;
      if (hn == 0.0 || est <= target || it >= max_iter) break;
    }
    for (int i = jj - 1; i >= 0; i--) {
      double s = g[i];
      for (int k = i + 1; k < jj; k++) s -= H[i + (size_t)k * (m + 1)] * y[k];
      const double dg = H[i + (size_t)i * (m + 1)];
      y[i] = (dg != 0.0) ? s / dg : 0.0;
    }
    if (flexible) {
      if (X->mg32)
        launch_update_x<float>(X->x, (const float *const *)X->Z, y.data(), jj, n, X->s);
      else
        launch_update_x<double>(X->x, (const double *const *)X->Z, y.data(), jj, n, X->s);
    } else {
      // x += U y with the orthonormal basis U = V T: coefficients T y on the
      // stored vectors
      for (int l = 0; l < jj; l++) {
        double acc = 0.0;
        for (int i = l; i < jj; i++) acc += Tm[(size_t)l * (m + 1) + i] * y[i];
        ty[l] = acc;
      }
      if (S) {
        launch_fill<double>(X->t, 0.0, n, X->s);
        launch_update_x<double>(X->t, (const double *const *)X->V, ty.data(), jj, n, X->s);
        launch_mul_scaling(X->t, S, 0, n, X->t, X->s);
        launch_axpy<double>(1.0, X->t, X->x, n, X->s);
      } else {
        launch_update_x<double>(X->x, (const double *const *)X->V, ty.data(), jj, n, X->s);
      }
    }
  }
  st->iters = it;
  const int vel_per = (X->p.precond == STOKES_P5) ? 2 : 1;
  const int p_per = (X->p.precond == STOKES_P1) ? 1 : (X->p.theta != 0.0 ? 1 : 0);
  st->scalar_vcycles = st->precond_applies * X->p.vcycles * (X->d * vel_per + p_per);
  // X->r holds b' - M' x' of the final iterate unless the loop left early
  if (rc == STOKES_OK || rc == STOKES_ENOCONV) {
    const double *r = X->r;
    if (S) {  // X->r holds S (b' - M' x')
      launch_mul_scaling(X->r, S, 1, n, X->t, X->s);
      r = X->t;
    }
    st->rel_res_unscaled = unscaled_rel(X, r);
  }
  return rc;
}

// compatibility of b' with the null space (Sec. "Krylov Solver"); b' in X->b
int check_rhs(stokes_ctx *X) {
  const Geo &g = X->lev[0].g;
  double *hb = X->host;
  launch_sum<double>(X->b + X->nvel, X->ncell, X->part, X->dsc + 1, X->s);
  launch_norm2(X->b + X->nvel, X->ncell, X->part, X->dsc + 2, X->s);
  launch_norm2(X->b, X->nvel, X->part, X->dsc + 3, X->s);
  for (int k = 0; k < g.d; k++) launch_sum<double>(X->b + g.foff[k], g.fcnt[k], X->part,
                                                   X->dsc + 4 + k, X->s);
  fetch(X, X->dsc, 8, hb);
  if (X->err) return STOKES_EDEVICE;
  const double c = X->c;
  const double nrm = std::sqrt(hb[2] + hb[3] / (c * c)) + 1e-300;
  if (std::fabs(hb[1]) > 1e-10 * nrm * std::sqrt((double)X->ncell)) return STOKES_EINCOMPAT;
  for (int k = 0; k < g.d; k++)
    if (((X->vel_singular >> k) & 1) &&
        std::fabs(hb[4 + k] / c) > 1e-10 * nrm * std::sqrt((double)g.fcnt[k]))
      return STOKES_EINCOMPAT;
  return STOKES_OK;
}

// unscaled x -> user buffers: x_u = x'_u, x_p = x'_p / c; zero means
void finish_solution(stokes_ctx *X, const double *xs, double su, double sp, double *xu,
                     double *xp) {
  const Geo &g = X->lev[0].g;
  launch_pack_vel(g, xs, su, xu, X->s);
  launch_scale(xs + X->nvel, sp, xp, X->ncell, X->s);
  remove_mean<double>(X, xp, X->ncell, 24);
  if (X->vel_singular) remove_vel_means<double>(X, g, xu);
}

int grad_impl(stokes_ctx *X, const double *u, const double *lam, double *dmu_cell,
              double *dmu_edge, double *drho, double *dgamma) {
  const Geo &g = X->lev[0].g;
  double *de = dmu_edge ? dmu_edge : X->gedge;
  launch_grad_edges(g, u, lam, de, X->s);
  if (dmu_cell || drho || dgamma) {
    // write into temporaries when a requested output is missing
    double *dc = dmu_cell ? dmu_cell : X->gcell;
    launch_grad_cells(g, u, lam, X->p.theta, X->bulk, dc, drho, dgamma, X->s);
    if (dmu_cell && X->p.edge_avg != STOKES_EDGE_GIVEN)
      launch_grad_chain(g, de, X->m_mue, X->m_muc, X->p.edge_avg, dmu_cell, X->s);
  }
  return STOKES_OK;
}

// Stand-alone multigrid on one subproblem of the scaled system: V-cycles
// e <- e + V(r - A e) from e = 0 until ||r - A e|| <= tol ||r||.  Residuals,
// the iterate and the norms are FP64; the V-cycles run in the hierarchy's
// precision (an FP32 hierarchy then acts as iterative refinement and still
// reaches FP64 tolerances).  r and e are FP64 device vectors of the scaled
// system (velocity: c times the user's r; pressure: the user's r).
int mg_solve(stokes_ctx *X, bool vel, double tol, int max_cycles, int *cycles, double *rel) {
  const Geo &g = X->lev[0].g;
  const i64 n = vel ? X->nvel : X->ncell;
  double *r = X->t, *e = X->x, *res = X->w, *de = X->r;
  double *hb = X->host;
  if (vel) {
    if (X->vel_singular) remove_vel_means<double>(X, g, r);
  } else {
    remove_mean<double>(X, r, n, 21);
  }
  launch_norm2(r, n, X->part, X->dsc, X->s);
  const double nr = std::sqrt(fetch(X, X->dsc, 1, hb));
  if (X->err) return STOKES_EDEVICE;
  launch_fill<double>(e, 0.0, n, X->s);
  launch_scale(r, 1.0, res, n, X->s);
  const double *beta64 = X->mg32 ? X->c64b[0] : P<double>(X->lev[0].beta);
  double q = (nr > 0.0) ? 1.0 : 0.0;
  int c = 0;
  while (q > tol && c < max_cycles) {
    if (X->mg32) {
      float *pin = P<float>(X->pin), *pout = P<float>(X->pout);
      launch_cast<float, double>(res, pin, n, X->s);
      vcycle_top<float>(X, vel, pin, pout);
      const float *zs[1] = {pout};
      const double one = 1.0;
      launch_update_x<float>(e, zs, &one, 1, n, X->s);
    } else {
      vcycle_top<double>(X, vel, res, de);
      launch_axpy<double>(1.0, de, e, n, X->s);
    }
    c++;
    if (vel)
      launch_vel_residual<double>(g, m_alpha_of(X), X->m_muc, X->m_mue, X->m_lam, r, e, nullptr,
                                  res, X->s);
    else
      launch_p_residual<double>(g, beta64, r, e, res, X->s);
    launch_norm2(res, n, X->part, X->dsc, X->s);
    q = std::sqrt(fetch(X, X->dsc, 1, hb)) / nr;
    if (X->err) return STOKES_EDEVICE;
  }
  if (vel) {
    if (X->vel_singular) remove_vel_means<double>(X, g, e);
  } else {
    remove_mean<double>(X, e, n, 22);
  }
  *cycles = c;
  *rel = q;
  if (!std::isfinite(q)) return STOKES_ENONFINITE;
  return (q <= tol) ? STOKES_OK : STOKES_ENOCONV;
}


// ---------------- static scratch (stokes_solve_static) ----------------
// The Krylov storage of a solve (right-hand side, iterate, residual, work
// vectors, the restart basis V and, for FGMRES, Z) and the reduction
// partials, which stokes_solve keeps in the context's workspace.
struct KrylovStore {
  double *V[kMaxRestart + 1];
  void *Z[kMaxRestart];
  double *r, *w, *t, *x, *b, *part, *dsc;
};

KrylovStore krylov_store(const stokes_ctx *X) {
  KrylovStore k;
  for (int i = 0; i <= kMaxRestart; i++) k.V[i] = X->V[i];
  for (int i = 0; i < kMaxRestart; i++) k.Z[i] = X->Z[i];
  k.r = X->r; k.w = X->w; k.t = X->t; k.x = X->x; k.b = X->b;
  k.part = X->part; k.dsc = X->dsc;
  return k;
}

void set_krylov_store(stokes_ctx *X, const KrylovStore &k) {
  for (int i = 0; i <= kMaxRestart; i++) X->V[i] = k.V[i];
  for (int i = 0; i < kMaxRestart; i++) X->Z[i] = k.Z[i];
  X->r = k.r; X->w = k.w; X->t = k.t; X->x = k.x; X->b = k.b;
  X->part = k.part; X->dsc = k.dsc;
}

// carve the Krylov storage from cv and point the context at it (cv over a
// null base only measures)
void carve_krylov(stokes_ctx *X, Carver &cv) {
  const i64 nn = X->n;
  const size_t tb = X->mg32 ? sizeof(float) : sizeof(double);
  const int m = X->p.restart;
  KrylovStore k = krylov_store(X);
  for (int i = 0; i <= m; i++) k.V[i] = (double *)cv.take(nn * 8);
  if (X->p.krylov == STOKES_FGMRES)
    for (int i = 0; i < m; i++) k.Z[i] = cv.take(nn * tb);
  k.r = (double *)cv.take(nn * 8);
  k.w = (double *)cv.take(nn * 8);
  k.t = (double *)cv.take(nn * 8);
  k.x = (double *)cv.take(nn * 8);
  k.b = (double *)cv.take(nn * 8);
  k.part = (double *)cv.take((size_t)kRedBlocks * (kMaxRestart + 2) * 8);
  k.dsc = (double *)cv.take(kDscSlots * 8);
  if (cv.base) set_krylov_store(X, k);
}

size_t krylov_scratch_bytes(stokes_ctx *X) {
  Carver cv(nullptr);
  carve_krylov(X, cv);
  return (cv.off + kAlign - 1) / kAlign * kAlign;
}

// stokes_solve on the Krylov storage the context currently points at
int solve_impl(stokes_ctx *X, const double *bu, const double *bp, double *xu, double *xp,
               double tol, int max_iter, int use_x0, stokes_stats *st) {
  const Geo &g = X->lev[0].g;
  // rescaled system (eq. Stokes_rescaled): b' = (c b_u, b_p), x' = (x_u, c x_p)
  launch_pack_vel(g, bu, X->c, X->b, X->s);
  launch_scale(bp, 1.0, X->b + X->nvel, X->ncell, X->s);
  int rc = check_rhs(X);
  if (rc != STOKES_OK) return finish(X, rc);
  if (use_x0) {
    launch_pack_vel(g, xu, 1.0, X->x, X->s);
    launch_scale(xp, X->c, X->x + X->nvel, X->ncell, X->s);
  } else {
    launch_fill<double>(X->x, 0.0, X->n, X->s);
  }
  rc = krylov(X, tol, max_iter, st);
  finish_solution(X, X->x, 1.0, 1.0 / X->c, xu, xp);
  hip_ok(X, hipStreamSynchronize(X->s));
  return finish(X, rc);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

int stokes_sizes(const stokes_params *p, size_t *nvel, size_t *ncell, size_t *nedge,
                 int *nlevels) {
  int nlev = 0;
  if (!valid_params(p, &nlev)) return STOKES_EINVAL;
  int n[3], ns[3];
  for (int a = 0; a < 3; a++) {
    n[a] = (a < p->dim) ? p->n[a] : 1;
    ns[a] = (a < p->dim) ? p->bc[a] : 0;
  }
  Geo g = make_geo(p->dim, n, ns, p->h);
  if (nvel) *nvel = (size_t)g.nvel;
  if (ncell) *ncell = (size_t)g.ncell;
  if (nedge) *nedge = (size_t)g.nedge;
  if (nlevels) *nlevels = nlev;
  return STOKES_OK;
}

size_t stokes_workspace_bytes(const stokes_params *p) {
  int nlev = 0;
  if (!valid_params(p, &nlev)) return 0;
  Carver cv(nullptr);
  carve_all(p, nlev, cv, nullptr);
  return cv.off + kAlign;
}

int stokes_create(const stokes_params *p, const double *rho, const double *mu,
                  const double *mu_edges, const double *gamma, void *workspace, size_t ws_bytes,
                  void *hip_stream, stokes_ctx **out) {
  if (!out) return STOKES_EINVAL;
  *out = nullptr;
  int nlev = 0;
  if (!valid_params(p, &nlev) || !rho || !mu || !workspace) return STOKES_EINVAL;
  if (p->edge_avg == STOKES_EDGE_GIVEN && !mu_edges) return STOKES_EINVAL;
  if ((p->bulk != 0) != (gamma != nullptr)) return STOKES_EINVAL;
  if (((uintptr_t)workspace) % kAlign != 0) return STOKES_EINVAL;
  if (ws_bytes < stokes_workspace_bytes(p)) return STOKES_ENOMEM;
  stokes_ctx *X = new (std::nothrow) stokes_ctx();
  if (!X) return STOKES_ENOMEM;
  X->p = *p;
  X->s = (hipStream_t)hip_stream;
  if (hipGetDevice(&X->dev) != hipSuccess) {
    delete X;
    return STOKES_EDEVICE;
  }
  X->d = p->dim;
  X->nlev = nlev;
  X->mg32 = (p->precision == STOKES_MG_FP32);
  X->bulk = p->bulk;
  Carver cv(workspace);
  carve_all(p, nlev, cv, X);
  const Geo &g0 = X->lev[0].g;
  X->nvel = g0.nvel;
  X->ncell = g0.ncell;
  X->nedge = g0.nedge;
  X->n = g0.nvel + g0.ncell;
  // velocity null space at theta = 0: component k is constant-invariant when
  // its own axis is periodic and no axis has no-slip walls (free-slip walls
  // only fix the normal component)
  X->vel_singular = 0;
  if (p->theta == 0.0) {
    int noslip = 0;
    for (int a = 0; a < p->dim; a++)
      noslip |= (p->bc[a] == STOKES_NOSLIP || p->bc[a] == STOKES_NOSLIP_FREESLIP ||
                 p->bc[a] == STOKES_FREESLIP_NOSLIP);
    for (int k = 0; k < p->dim; k++)
      if (p->bc[k] == STOKES_PERIODIC && !noslip) X->vel_singular |= 1 << k;
  }
  for (int l = 0; l < nlev; l++) X->lev[l].g.sing = X->lev[l].gv.sing = X->vel_singular;
  X->vsplit = use_vsplit(p) ? 1 : 0;
  // coarse tail: the levels small enough for one workgroup (at most kTailMax)
  X->tail_l = tail_level_of(p, nlev);
  if (const char *e = std::getenv("STOKES_TAIL_DENSE")) X->tail_dense = (e[0] != '0');
  // colour-split storage for the velocity levels below the coarse tail
  if (X->vsplit)
    for (int l = 0; l < nlev && (X->tail_l < 0 || l < X->tail_l); l++) X->lev[l].gv.split = 1;
  // the 3D velocity residual by columns of kResidualColumn cells along z on
  // the levels with at least kResidualColumnCells cells
  // (STOKES_RESIDUAL_COLUMNS=n in the environment at create time: columns of
  // n cells, or by cells for n = 0)
  {
    int col = kResidualColumn;
    if (const char *e = std::getenv("STOKES_RESIDUAL_COLUMNS"))
      col = (int)std::max(0L, std::min(std::strtol(e, nullptr, 10), 1L << 20));
    if (p->dim == 3 && col > 0)
      for (int l = 0; l < nlev; l++)
        if (X->lev[l].gv.ncell >= kResidualColumnCells)  // a column never exceeds the z extent
          X->lev[l].g.col = X->lev[l].gv.col = std::min(col, X->lev[l].gv.n[2]);
  }
  if (hipHostMalloc((void **)&X->host, 4096 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    delete X;
    return STOKES_EDEVICE;
  }
  hipStream_t s = X->s;
  // all internal buffers start at zero (wall faces stay 0 for good)
  (void)hipMemsetAsync(workspace, 0, cv.off, s);
  // coefficient check and rescaling factor
  launch_fill<int>(X->dflag, 0, 1, s);
  launch_check_coefs(rho, mu, g0.ncell, X->dflag, s);
  if (gamma) launch_check_coefs(rho, gamma, g0.ncell, X->dflag, s);  // gamma >= 0, finite
  launch_logsum(mu, g0.ncell, X->part, X->dsc, s);
  int flag = 0;
  (void)hipMemcpyAsync(&X->host[0], X->dsc, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(&X->host[8], X->dflag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) {
    (void)hipHostFree(X->host);
    delete X;
    return STOKES_EDEVICE;
  }
  std::memcpy(&flag, &X->host[8], sizeof(int));
  if (flag) {
    (void)hipHostFree(X->host);
    delete X;
    return STOKES_EINVAL;
  }
  if (p->rescale_c > 0.0) {
    X->c = p->rescale_c;
  } else {
    const double sl = X->host[0], cnt = X->host[1];
    X->c = (cnt > 0.0) ? p->h / std::exp(sl / cnt) : 1.0;
  }
  // FP64 fine coefficients (scaled), then the hierarchy (Appendix C).  The
  // FP32 form coarsens in FP64 and rounds each level once.
  if (!X->mg32) {
    Level &L0 = X->lev[0];
    launch_setup_faces(g0, rho, p->theta, X->c, P<double>(L0.alpha), P<double>(L0.beta), s);
    launch_setup_cells(g0, mu, X->c, P<double>(L0.muc), s);
    launch_setup_edges(g0, mu, mu_edges, p->edge_avg, X->c, P<double>(L0.mue), s);
    (void)hipMemcpyAsync(X->m_alpha, L0.alpha, g0.nvel * 8, hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(X->m_muc, L0.muc, g0.ncell * 8, hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(X->m_mue, L0.mue, g0.nedge * 8, hipMemcpyDeviceToDevice, s);
    for (int l = 1; l < nlev; l++) {
      Level &F = X->lev[l - 1], &C = X->lev[l];
      launch_coarsen(F.g, C.g, P<double>(F.alpha), P<double>(F.beta), P<double>(F.muc),
                     P<double>(F.mue), P<double>(C.alpha), P<double>(C.beta), P<double>(C.muc),
                     P<double>(C.mue), s);
    }
    if (X->bulk) {
      // bulk coefficient: coarse cell = mean of its 2^d fine cells (like mu_cell)
      launch_setup_bulk(gamma, mu, X->c, g0.ncell, P<double>(L0.lam), P<double>(X->sig), s);
      (void)hipMemcpyAsync(X->m_lam, L0.lam, g0.ncell * 8, hipMemcpyDeviceToDevice, s);
      for (int l = 1; l < nlev; l++)
        launch_cell_restrict<double>(X->lev[l - 1].g, X->lev[l].g, P<double>(X->lev[l - 1].lam),
                                     P<double>(X->lev[l].lam), s);
    }
  } else {
    launch_setup_faces(g0, rho, p->theta, X->c, X->c64a[0], X->c64b[0], s);
    launch_setup_cells(g0, mu, X->c, X->c64m[0], s);
    launch_setup_edges(g0, mu, mu_edges, p->edge_avg, X->c, X->c64e[0], s);
    for (int l = 1; l < nlev; l++)
      launch_coarsen(X->lev[l - 1].g, X->lev[l].g, X->c64a[l - 1], X->c64b[l - 1], X->c64m[l - 1],
                     X->c64e[l - 1], X->c64a[l], X->c64b[l], X->c64m[l], X->c64e[l], s);
    for (int l = 0; l < nlev; l++) {
      Level &L = X->lev[l];
      launch_cast<float, double>(X->c64a[l], P<float>(L.alpha), L.g.nvel, s);
      launch_cast<float, double>(X->c64b[l], P<float>(L.beta), L.g.nvel, s);
      launch_cast<float, double>(X->c64m[l], P<float>(L.muc), L.g.ncell, s);
      launch_cast<float, double>(X->c64e[l], P<float>(L.mue), L.g.nedge, s);
    }
    if (X->bulk) {
      launch_setup_bulk(gamma, mu, X->c, g0.ncell, X->c64l[0], X->sig64, s);
      for (int l = 1; l < nlev; l++)
        launch_cell_restrict<double>(X->lev[l - 1].g, X->lev[l].g, X->c64l[l - 1], X->c64l[l], s);
      for (int l = 0; l < nlev; l++)
        launch_cast<float, double>(X->c64l[l], P<float>(X->lev[l].lam), X->lev[l].g.ncell, s);
      launch_cast<float, double>(X->sig64, P<float>(X->sig), g0.ncell, s);
    }
  }
  if (X->vsplit && p->theta != 0.0) {
    if (X->mg32)
      split_alpha<float>(X);
    else
      split_alpha<double>(X);
  }
  if (X->tail_l < 0 || !X->tail_B) X->tail_dense = 0;
  if (X->tail_dense && !(X->mg32 ? build_tail_matrix<float>(X) : build_tail_matrix<double>(X)))
    X->tail_dense = 0;
  if (X->sdiag) {
    // diagonal scaling from the FP64 coefficients of M'; X->t is still zero
    launch_fill<int>(X->dflag, 0, 1, s);
    launch_diag_scaling(g0, m_alpha_of(X), X->m_muc, X->m_mue, X->m_lam, X->t, X->sdiag, X->dflag,
                        s);
    (void)hipMemcpyAsync(&X->host[8], X->dflag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) {
      (void)hipHostFree(X->host);
      delete X;
      return STOKES_EDEVICE;
    }
    std::memcpy(&flag, &X->host[8], sizeof(int));
    if (flag) {  // a cell without a positive viscous Schur coefficient
      (void)hipHostFree(X->host);
      delete X;
      return STOKES_EINVAL;
    }
  }
  // algorithmic bytes of one finest-level velocity colour pass of component
  // k, each value the pass needs counted once: it reads every velocity
  // component (the faces of its colour and all their neighbours), mu_cell
  // and the d-1 edge families around k in full (each cell and edge borders
  // faces of both colours), and only its own colour's half of rhs_k and
  // alpha_k (not read when theta = 0); it writes the half of u_k it updates.
  const double tb = X->mg32 ? 4.0 : 8.0;
  for (int k = 0; k < g0.d; k++) {
    double e = 0.0;
    for (int m = 0; m < 3; m++)
      if (m != k && g0.ecnt[m] > 0) e += (double)g0.ecnt[m];
    if (g0.d == 2) e = (double)g0.ecnt[2];
    // halves of rhs_k, alpha_k (theta != 0) and the written u_k
    const double own = (p->theta == 0.0) ? 1.0 : 1.5;
    const double cells = X->bulk ? 2.0 : 1.0;  // mu_cell (and the bulk coefficient)
    X->gs_bytes[k] =
        tb * ((double)g0.nvel + own * (double)g0.fcnt[k] + cells * (double)g0.ncell + e);
  }
  X->vc_cycle_bytes[0] = vcycle_alg_bytes(X, true);
  X->vc_cycle_bytes[1] = vcycle_alg_bytes(X, false);
  const char *vg = std::getenv("STOKES_VGRAPH");
  if (X->vsplit && !(vg && vg[0] == '0') &&
      !(X->mg32 ? capture_vcycle<float>(X) : capture_vcycle<double>(X))) {
    release_vgraph(X);  // the V-cycle then runs kernel by kernel
    (void)hipGetLastError();
  }
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) {
    release_vgraph(X);
    (void)hipHostFree(X->host);
    delete X;
    return STOKES_EDEVICE;
  }
  bool evs = true;
  for (auto &e : X->pev) evs = evs && hipEventCreate(&e) == hipSuccess;
  if (!evs) {
    for (auto &e : X->pev) {
      if (e) (void)hipEventDestroy(e);
      e = nullptr;  // statistics then report no preconditioner time
    }
  }
  if (hipEventCreateWithFlags(&X->sev, hipEventDisableTiming) != hipSuccess) X->sev = nullptr;
  *out = X;
  return STOKES_OK;
}

void stokes_destroy(stokes_ctx *X) {
  if (!X) return;
  if (X->s) (void)hipStreamSynchronize(X->s);
  for (auto e : X->ev) (void)hipEventDestroy(e);
  for (auto e : X->vev) (void)hipEventDestroy(e);
  for (auto e : X->pev)
    if (e) (void)hipEventDestroy(e);
  if (X->sev) (void)hipEventDestroy(X->sev);
  release_vgraph(X);
  if (X->host) (void)hipHostFree(X->host);
  delete X;
}

double stokes_rescale(const stokes_ctx *X) { return X ? X->c : 0.0; }

int stokes_apply(stokes_ctx *X, const double *xu, const double *xp, double *yu, double *yp) {
  if (!X || !xu || !xp || !yu || !yp) return STOKES_EINVAL;
  const Geo &g = X->lev[0].g;
  // x' = (x_u, c x_p); y_u = (M' x')_u / c, y_p = (M' x')_p
  launch_pack_vel(g, xu, 1.0, X->t, X->s);
  launch_scale(xp, X->c, X->t + X->nvel, X->ncell, X->s);
  apply_scaled(X, X->t, X->w);
  launch_pack_vel(g, X->w, 1.0 / X->c, yu, X->s);
  launch_scale(X->w + X->nvel, 1.0, yp, X->ncell, X->s);
  return finish(X, STOKES_OK);
}

int stokes_residual(stokes_ctx *X, const double *bu, const double *bp, const double *xu,
                    const double *xp, double *ru, double *rp, int extended) {
  if (!X || !bu || !bp || !xu || !xp || !ru || !rp || (extended != 0 && extended != 1))
    return STOKES_EINVAL;
  const Geo &g = X->lev[0].g;
  const i64 nv = X->nvel, nc = X->ncell;
  // rescaled system: b' = (c b_u, b_p), x' = (x_u, c x_p), r_u = r'_u / c
  launch_pack_vel(g, bu, X->c, X->b, X->s);
  launch_scale(bp, 1.0, X->b + nv, nc, X->s);
  launch_pack_vel(g, xu, 1.0, X->x, X->s);
  launch_scale(xp, X->c, X->x + nv, nc, X->s);
  if (extended)
    launch_residual_dd(g, m_alpha_of(X), X->m_muc, X->m_mue, X->m_lam, X->x, X->x + nv, X->b,
                       X->b + nv, X->r, X->r + nv, X->s);
  else
    launch_apply_m<double>(g, m_alpha_of(X), X->m_muc, X->m_mue, X->m_lam, X->x, X->x + nv, X->b,
                           X->b + nv, X->r, X->r + nv, X->s);
  launch_pack_vel(g, X->r, 1.0 / X->c, ru, X->s);
  launch_scale(X->r + nv, 1.0, rp, nc, X->s);
  return finish(X, STOKES_OK);
}

int stokes_boundary_rhs(stokes_ctx *X, const double *un, const double *ut, double *cu,
                        double *cp) {
  if (!X || !un || !ut || !cu || !cp) return STOKES_EINVAL;
  const Geo &g = X->lev[0].g;
  // the wall-data field (prescribed normal velocities on the wall faces, zero
  // at the unknowns) with p = 0, through the rescaled M with the prescribed
  // tangential wall velocities in the no-slip ghosts
  launch_pack_walls(g, un, 1.0, X->t, X->s);
  launch_fill<double>(X->t + X->nvel, 0.0, X->ncell, X->s);
  launch_apply_m_walls(g, m_alpha_of(X), X->m_muc, X->m_mue, X->m_lam, X->t, X->t + X->nvel, ut,
                       X->w,
                       X->w + X->nvel, X->s);
  launch_pack_vel(g, X->w, 1.0 / X->c, cu, X->s);
  launch_scale(X->w + X->nvel, 1.0, cp, X->ncell, X->s);
  return finish(X, STOKES_OK);
}

int stokes_precond(stokes_ctx *X, const double *bu, const double *bp, double *zu, double *zp) {
  if (!X || !bu || !bp || !zu || !zp) return STOKES_EINVAL;
  const Geo &g = X->lev[0].g;
  launch_pack_vel(g, bu, X->c, X->t, X->s);
  launch_scale(bp, 1.0, X->t + X->nvel, X->ncell, X->s);
  if (X->mg32) {
    precond_from64(X, X->t, X->pout);
    launch_cast<double, float>(P<float>(X->pout), X->w, X->n, X->s);
  } else {
    precond<double>(X, X->t, X->t + X->nvel, X->w, X->w + X->nvel);
  }
  launch_pack_vel(g, X->w, 1.0, zu, X->s);
  launch_scale(X->w + X->nvel, 1.0 / X->c, zp, X->ncell, X->s);
  return finish(X, STOKES_OK);
}

int stokes_vel_subsolve(stokes_ctx *X, const double *r, double *e) {
  if (!X || !r || !e) return STOKES_EINVAL;
  const Geo &g = X->lev[0].g;
  launch_pack_vel(g, r, X->c, X->t, X->s);
  if (X->mg32) {
    launch_cast<float, double>(X->t, P<float>(X->pin), X->nvel, X->s);
    vel_sub<float>(X, P<float>(X->pin), P<float>(X->pout));
    launch_cast<double, float>(P<float>(X->pout), X->w, X->nvel, X->s);
  } else {
    vel_sub<double>(X, X->t, X->w);
  }
  launch_pack_vel(g, X->w, 1.0, e, X->s);
  return finish(X, STOKES_OK);
}

int stokes_p_subsolve(stokes_ctx *X, const double *r, double *e) {
  if (!X || !r || !e) return STOKES_EINVAL;
  if (X->mg32) {
    launch_cast<float, double>(r, P<float>(X->pin), X->ncell, X->s);
    p_sub<float>(X, P<float>(X->pin), P<float>(X->pout));
    launch_cast<double, float>(P<float>(X->pout), X->w, X->ncell, X->s);
  } else {
    p_sub<double>(X, r, X->w);
  }
  launch_scale(X->w, 1.0 / X->c, e, X->ncell, X->s);
  return finish(X, STOKES_OK);
}

int stokes_vel_mg_solve(stokes_ctx *X, const double *r, double *e, double tol, int max_cycles,
                        int *cycles, double *rel_res) {
  if (!X || !r || !e || !cycles || !rel_res || !(tol > 0.0) || max_cycles < 0)
    return STOKES_EINVAL;
  const Geo &g = X->lev[0].g;
  launch_pack_vel(g, r, X->c, X->t, X->s);
  const int rc = mg_solve(X, true, tol, max_cycles, cycles, rel_res);
  if (rc == STOKES_EDEVICE) return finish(X, rc);
  launch_pack_vel(g, X->x, 1.0, e, X->s);
  hip_ok(X, hipStreamSynchronize(X->s));
  return finish(X, rc);
}

int stokes_p_mg_solve(stokes_ctx *X, const double *r, double *e, double tol, int max_cycles,
                      int *cycles, double *rel_res) {
  if (!X || !r || !e || !cycles || !rel_res || !(tol > 0.0) || max_cycles < 0)
    return STOKES_EINVAL;
  launch_scale(r, 1.0, X->t, X->ncell, X->s);
  const int rc = mg_solve(X, false, tol, max_cycles, cycles, rel_res);
  if (rc == STOKES_EDEVICE) return finish(X, rc);
  launch_scale(X->x, 1.0 / X->c, e, X->ncell, X->s);
  hip_ok(X, hipStreamSynchronize(X->s));
  return finish(X, rc);
}

int stokes_solve(stokes_ctx *X, const double *bu, const double *bp, double *xu, double *xp,
                 double tol, int max_iter, int use_x0, stokes_stats *st) {
  if (!X || !bu || !bp || !xu || !xp || !(tol > 0.0) || max_iter < 0) return STOKES_EINVAL;
  return solve_impl(X, bu, bp, xu, xp, tol, max_iter, use_x0, st);
}

int stokes_solve_static(stokes_ctx *X, const double *bu, const double *bp, double *xu,
                        double *xp, double tol, int max_iter, int use_x0, stokes_stats *st) {
  if (!X || !bu || !bp || !xu || !xp || !(tol > 0.0) || max_iter < 0) return STOKES_EINVAL;
  const size_t need = krylov_scratch_bytes(X);
  if (need > kScratchBytes) return STOKES_ENOMEM;
  char *base = (char *)scratch_on(X->dev);
  if (!base) return STOKES_EDEVICE;
  KrylovStore saved = krylov_store(X);
  Carver cv(base);
  carve_krylov(X, cv);
  // the array keeps the previous call's contents (possibly another grid's):
  // clear it, so that the wall entries of every vector start at zero as in
  // a freshly zeroed workspace
  launch_fill<double>((double *)base, 0.0, (i64)((need + 7) / 8), X->s);
  const int rc = solve_impl(X, bu, bp, xu, xp, tol, max_iter, use_x0, st);
  set_krylov_store(X, saved);
  return rc;
}

int stokes_grad(stokes_ctx *X, const double *xu, const double *lu, double *dmu_cell,
                double *dmu_edge, double *drho_cell, double *dgamma_cell) {
  if (!X || !xu || !lu) return STOKES_EINVAL;
  if (dgamma_cell && !X->bulk) return STOKES_EINVAL;
  const Geo &g = X->lev[0].g;
  launch_pack_vel(g, xu, 1.0, X->t, X->s);
  launch_pack_vel(g, lu, 1.0, X->r, X->s);
  grad_impl(X, X->t, X->r, dmu_cell, dmu_edge, drho_cell, dgamma_cell);
  return finish(X, STOKES_OK);
}

int stokes_adjoint_solve(stokes_ctx *X, const double *xu, const double *xp, const double *gu,
                         const double *gp, double *lu, double *lp, double *dmu_cell,
                         double *dmu_edge, double *drho_cell, double *dgamma_cell, double tol,
                         int max_iter, stokes_stats *st) {
  (void)xp;
  if (!X || !xu || !gu || !gp || !lu || !lp || !(tol > 0.0) || max_iter < 0)
    return STOKES_EINVAL;
  if (dgamma_cell && !X->bulk) return STOKES_EINVAL;
  const Geo &g = X->lev[0].g;
  // M' = diag(c,1) M diag(1,1/c) is symmetric: lambda = diag(c,1) M'^{-1} (g_u, g_p / c)
  launch_pack_vel(g, gu, 1.0, X->b, X->s);
  launch_scale(gp, 1.0 / X->c, X->b + X->nvel, X->ncell, X->s);
  // the forward solution is normalised to zero-mean pressure (and zero-mean
  // velocity components when singular); the adjoint of that normalisation
  // projects g onto the same mean-free space
  remove_mean<double>(X, X->b + X->nvel, X->ncell, 25);
  if (X->vel_singular) remove_vel_means<double>(X, g, X->b);
  int rc = STOKES_OK;
  launch_fill<double>(X->x, 0.0, X->n, X->s);
  rc = krylov(X, tol, max_iter, st);
  finish_solution(X, X->x, X->c, 1.0, lu, lp);
  launch_pack_vel(g, xu, 1.0, X->t, X->s);
  grad_impl(X, X->t, lu, dmu_cell, dmu_edge, drho_cell, dgamma_cell);
  hip_ok(X, hipStreamSynchronize(X->s));
  return finish(X, rc);
}

int stokes_set_history(stokes_ctx *X, double *buf, int cap) {
  if (!X || cap < 0) return STOKES_EINVAL;
  X->hist = (buf && cap > 0) ? buf : nullptr;
  X->hist_cap = X->hist ? cap : 0;
  return STOKES_OK;
}

int stokes_set_timing(stokes_ctx *X, int enable) {
  if (!X) return STOKES_EINVAL;
  if (enable && X->ev.empty()) {
    X->ev.resize(2 * kEventPool);
    for (auto &e : X->ev)
      if (hipEventCreate(&e) != hipSuccess) return STOKES_EDEVICE;
    X->vev.resize(2 * kEventPool);
    X->vev_kind.resize(kEventPool);
    for (auto &e : X->vev)
      if (hipEventCreate(&e) != hipSuccess) return STOKES_EDEVICE;
  }
  fold_events(X);
  fold_vevents(X);
  if (enable < 0 || enable > 2) return STOKES_EINVAL;
  X->timing = enable;
  X->t_ms = 0.0;
  X->launches = 0;
  X->bytes = 0.0;
  for (int k = 0; k < 2; k++) {
    X->vc_ms[k] = X->vc_bytes[k] = 0.0;
    X->vc_count[k] = 0;
  }
  return STOKES_OK;
}

int stokes_vcycle_time(stokes_ctx *X, int pressure, double *ms_total, long *cycles,
                       double *bytes_total) {
  if (!X || (pressure != 0 && pressure != 1)) return STOKES_EINVAL;
  fold_vevents(X);
  if (ms_total) *ms_total = X->vc_ms[pressure];
  if (cycles) *cycles = X->vc_count[pressure];
  if (bytes_total) *bytes_total = X->vc_bytes[pressure];
  return STOKES_OK;
}

int stokes_kernel_time(stokes_ctx *X, double *ms_total, long *launches, double *bytes_total) {
  if (!X) return STOKES_EINVAL;
  fold_events(X);
  if (ms_total) *ms_total = X->t_ms;
  if (launches) *launches = X->launches;
  if (bytes_total) *bytes_total = X->bytes;
  return STOKES_OK;
}

const char *stokes_strerror(int code) {
  switch (code) {
    case STOKES_OK: return "ok";
    case STOKES_EINVAL: return "invalid argument";
    case STOKES_ENOMEM: return "workspace too small";
    case STOKES_EDEVICE: return "HIP runtime error";
    case STOKES_ENOCONV: return "not converged within max_iter";
    case STOKES_EBREAKDOWN: return "Krylov breakdown";
    case STOKES_ENONFINITE: return "non-finite residual";
    case STOKES_EINCOMPAT: return "right-hand side incompatible with the null space";
    default: return "unknown status";
  }
}

}  // extern "C"
