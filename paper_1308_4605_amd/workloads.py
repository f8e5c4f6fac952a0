"""Seeded synthetic inputs for the variable-coefficient MAC Stokes solver.

This module only draws input data (coefficient fields, forcing fields, target
fields) and describes the array layout of the C ABI.  It holds none of the
solver's arithmetic: no face/edge averaging, no operators, no rescaling.  Both
the GPU path and the CPU oracle receive exactly these bytes.

The workloads follow the paper's own kind of test problems (Sec. "Results": smooth
variable coefficients, viscosity/density contrasts, random right-hand sides on
no-slip or periodic unit domains) at the five sizes the benchmark and the tests
use.  Seeds: workload k uses base seed 1000*k; sub-streams +1 coefficients,
+2 forcing, +3 second/target solve, +4 finite-difference directions.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

PERIODIC = 0
NOSLIP = 1
FREESLIP = 2
NOSLIP_FREESLIP = 3   # no-slip at the low end of the axis, free-slip at the high end
FREESLIP_NOSLIP = 4   # free-slip low, no-slip high


def end_is_noslip(bc, side):
    """Whether the wall at the low (side 0) or high (side 1) end of an axis
    with condition bc is no-slip."""
    return bc == NOSLIP or (bc == NOSLIP_FREESLIP and side == 0) or (
        bc == FREESLIP_NOSLIP and side == 1)

P1, P2, P3, P4, P5 = 1, 2, 3, 4, 5
GMRES_LEFT, FGMRES = 0, 1
FP64, MG_FP32 = 0, 1
EDGE_ARITH, EDGE_HARMONIC, EDGE_GIVEN = 0, 1, 2


# ---------------------------------------------------------------------------
# layout of the ABI arrays
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Layout:
    """Shapes of the flat ABI arrays (C order, x fastest).

    Velocity component k lives on the faces normal to axis k and has one more
    entry along k when that axis has walls, no-slip or free-slip (the wall
    faces, held at 0).
    Edge family m is parallel to axis m; it has one more entry along each of
    the other axes that has walls.  Families are stored in the order m = 2, 1, 0
    (3D) or m = 2 only (2D, where the edges are the grid nodes).
    """

    dim: int
    n: Tuple[int, int, int]
    bc: Tuple[int, int, int]

    def _np(self, dims):
        dims = tuple(int(x) for x in dims)
        return (dims[2], dims[1], dims[0]) if self.dim == 3 else (dims[1], dims[0])

    @property
    def cell_shape(self):
        return self._np(self.n)

    def wall(self, a):
        """1 when axis a has walls (no-slip or free-slip), else 0."""
        return 1 if (a < self.dim and self.bc[a] != PERIODIC) else 0

    def face_dims(self, k):
        return tuple(self.n[a] + (self.wall(a) if a == k else 0) for a in range(3))

    def face_shape(self, k):
        return self._np(self.face_dims(k))

    def edge_dims(self, m):
        return tuple(self.n[a] + (self.wall(a) if a != m else 0) for a in range(3))

    def edge_shape(self, m):
        return self._np(self.edge_dims(m))

    @property
    def edge_families(self) -> List[int]:
        return [2, 1, 0] if self.dim == 3 else [2]

    @property
    def ncell(self):
        return int(np.prod(self.n[: self.dim]))

    @property
    def face_counts(self):
        return [int(np.prod(self.face_dims(k)[: self.dim])) for k in range(self.dim)]

    @property
    def nvel(self):
        return int(sum(self.face_counts))

    @property
    def face_offsets(self):
        offs, o = [], 0
        for c in self.face_counts:
            offs.append(o)
            o += c
        return offs

    @property
    def nedge(self):
        return int(sum(int(np.prod(self.edge_dims(m)[: self.dim])) for m in self.edge_families))

    def split_vel(self, u):
        """Views of the d components of a flat velocity array."""
        out = []
        for k, (o, c) in enumerate(zip(self.face_offsets, self.face_counts)):
            out.append(u[o:o + c].reshape(self.face_shape(k)))
        return out

    def wall_mask(self):
        """Flat bool mask of stored velocity entries that are wall faces."""
        parts = []
        for k in range(self.dim):
            m = np.zeros(self.face_shape(k), dtype=bool)
            if self.wall(k):
                ax = self.dim - 1 - k  # numpy axis of grid axis k
                idx = [slice(None)] * self.dim
                idx[ax] = 0
                m[tuple(idx)] = True
                idx[ax] = -1
                m[tuple(idx)] = True
            parts.append(m.ravel())
        return np.concatenate(parts)

    def face_centres(self, k, h):
        """Coordinates (x, y[, z]) of the faces of component k, numpy-shaped."""
        axes = []
        for a in range(self.dim):
            dims = self.face_dims(k)[a]
            if a == k:
                axes.append(np.arange(dims) * h)
            else:
                axes.append((np.arange(dims) + 0.5) * h)
        grids = np.meshgrid(*axes[::-1], indexing="ij")
        return grids[::-1]

    def singular_components(self, theta):
        """Velocity components with a constant null space: theta = 0, the
        component's own axis periodic and no axis with no-slip walls."""
        if theta != 0.0 or any(end_is_noslip(self.bc[a], s) for a in range(self.dim)
                               for s in (0, 1)):
            return []
        return [k for k in range(self.dim) if self.bc[k] == PERIODIC]

    def cell_centres(self, h):
        axes = [(np.arange(self.n[a]) + 0.5) * h for a in range(self.dim)]
        grids = np.meshgrid(*axes[::-1], indexing="ij")
        return grids[::-1]


def make_layout(dim, n, bc) -> Layout:
    n3 = tuple(int(x) for x in n) + (1,) * (3 - len(n))
    bc3 = tuple(int(x) for x in bc) + (0,) * (3 - len(bc))
    if dim == 2:
        n3 = (n3[0], n3[1], 1)
        bc3 = (bc3[0], bc3[1], 0)
    return Layout(dim, n3, bc3)


# ---------------------------------------------------------------------------
# random fields
# ---------------------------------------------------------------------------

def _wavevectors(rng, dim, K, kmax):
    r = int(math.floor(kmax))
    rngs = [range(-r, r + 1)] * dim
    cand = np.array(np.meshgrid(*rngs, indexing="ij")).reshape(dim, -1).T
    nrm = np.sqrt((cand ** 2).sum(1))
    cand = cand[(nrm > 0) & (nrm <= kmax)]
    pick = rng.choice(len(cand), size=K, replace=False)
    return cand[pick]


def smooth_field_modes(rng, dim, K, kmax):
    """K distinct integer wavevectors 0 < |k| <= kmax, N(0,1) amplitudes,
    U[0, 2 pi) phases."""
    ks = _wavevectors(rng, dim, K, kmax)
    amp = rng.standard_normal(K)
    ph = rng.uniform(0.0, 2.0 * np.pi, K)
    return ks, amp, ph


def eval_modes(modes, coords_1d):
    """sum_k a_k cos(2 pi k.x + phi_k) on the tensor grid of the 1D coordinate
    arrays (x, y[, z]); returns a numpy-ordered array."""
    ks, amp, ph = modes
    dim = len(coords_1d)
    shape = tuple(len(c) for c in coords_1d[::-1])
    acc = np.zeros(shape, dtype=np.complex128)
    for kv, a, p in zip(ks, amp, ph):
        term = a * np.exp(1j * p)
        fac = None
        for ax in range(dim):
            e = np.exp(2j * np.pi * kv[ax] * coords_1d[ax])
            sh = [1] * dim
            sh[dim - 1 - ax] = len(e)
            e = e.reshape(sh)
            fac = e if fac is None else fac * e
        acc += term * fac
    return acc.real


def _minmax(v, lo, hi):
    vmin, vmax = float(v.min()), float(v.max())
    return lo + (hi - lo) * (v - vmin) / (vmax - vmin)


def _axes_cell(lay: Layout, h):
    return [(np.arange(lay.n[a]) + 0.5) * h for a in range(lay.dim)]


def _axes_face(lay: Layout, k, h):
    ax = []
    for a in range(lay.dim):
        dims = lay.face_dims(k)[a]
        ax.append(np.arange(dims) * h if a == k else (np.arange(dims) + 0.5) * h)
    return ax


def smooth_face_field(rng, lay: Layout, h, K, kmax, remove_mean=True):
    """Independent smooth random field per velocity component, evaluated at the
    face centres; wall faces set to 0; optional per-component mean removal."""
    parts = []
    for k in range(lay.dim):
        modes = smooth_field_modes(rng, lay.dim, K, kmax)
        v = eval_modes(modes, _axes_face(lay, k, h))
        parts.append(v.ravel())
    u = np.concatenate(parts)
    u[lay.wall_mask()] = 0.0
    if remove_mean is True:
        u = _remove_component_means(lay, u)
    elif remove_mean:
        u = _remove_component_means(lay, u, comps=tuple(remove_mean))
    return u


def _remove_component_means(lay: Layout, u, comps=None):
    """Subtract the interior mean of each velocity component (of `comps`
    only, when given)."""
    u = u.copy()
    wm = lay.wall_mask()
    for k, (o, c) in enumerate(zip(lay.face_offsets, lay.face_counts)):
        if comps is not None and k not in comps:
            continue
        seg = u[o:o + c]
        interior = ~wm[o:o + c]
        seg[interior] -= seg[interior].mean()
    return u


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    n: Tuple[int, int, int]
    bc: Tuple[int, int, int]
    h: float
    theta: float
    precond: int
    krylov: int
    precision: int
    edge_avg: int
    rho: np.ndarray          # cells, flat
    mu: np.ndarray           # cells, flat
    bu: np.ndarray           # velocity RHS, flat (walls 0)
    bp: np.ndarray           # pressure RHS, flat
    extra: Dict[str, np.ndarray] = dataclasses.field(default_factory=dict)

    @property
    def layout(self) -> Layout:
        return make_layout(self.dim, self.n, self.bc)

    def params(self, **over):
        p = dict(dim=self.dim, n=self.n, bc=self.bc, h=self.h, theta=self.theta,
                 precond=self.precond, krylov=self.krylov, precision=self.precision,
                 restart=10, nu_pre=2, nu_post=2, nu_coarse=8, vcycles=1,
                 rescale_c=0.0, edge_avg=self.edge_avg)
        p.update(over)
        return p


def _n3(dim, n):
    if isinstance(n, int):
        n = (n,) * dim
    return tuple(n) + (1,) * (3 - len(n))


def periodic_smooth_2d(seed=1000, n=32, dt=1e-2):
    """2D periodic unit square, unsteady (theta = 1/dt, rho = 1),
    mu = 10^s with s a smooth 8-mode field (|k| <= 4) in [-0.5, 0.5]
    (contrast 10), smooth 8-mode forcing per face component, means removed."""
    dim = 2
    n3 = _n3(dim, n)
    lay = make_layout(dim, n3, (PERIODIC, PERIODIC))
    h = 1.0 / n3[0]
    rc = np.random.default_rng(seed + 1)
    s = _minmax(eval_modes(smooth_field_modes(rc, dim, 8, 4), _axes_cell(lay, h)), -0.5, 0.5)
    mu = np.power(10.0, s).ravel()
    rho = np.ones(lay.ncell)
    rf = np.random.default_rng(seed + 2)
    bu = smooth_face_field(rf, lay, h, 8, 4)
    return Workload("2d-periodic-smooth", dim, lay.n, lay.bc, h, 1.0 / dt, P1, GMRES_LEFT, FP64,
                    EDGE_ARITH, rho, mu, bu, np.zeros(lay.ncell))


def discs_2d(seed=2000, n=1024, ndisc=64, mu_in=1e3):
    """2D no-slip unit square, steady (theta = 0), rho = 1, mu = 1e3 inside 64
    random discs (radius U[0.02, 0.05], centres U[0,1]^2) and 1 outside,
    harmonic edge averaging, i.i.d. N(0,1) forcing on interior faces.
    Flexible GMRES: on these sharp jumps left-preconditioned GMRES(10)
    minimises a preconditioned residual that stagnates far above the true
    residual's tolerance, while the flexible form converges."""
    dim = 2
    n3 = _n3(dim, n)
    lay = make_layout(dim, n3, (NOSLIP, NOSLIP))
    h = 1.0 / n3[0]
    rc = np.random.default_rng(seed + 1)
    cx = rc.uniform(0, 1, ndisc)
    cy = rc.uniform(0, 1, ndisc)
    rad = rc.uniform(0.02, 0.05, ndisc)
    X, Y = lay.cell_centres(h)
    inside = np.zeros(lay.cell_shape, dtype=bool)
    for a, b, r in zip(cx, cy, rad):
        inside |= (X - a) ** 2 + (Y - b) ** 2 <= r * r
    mu = np.where(inside, mu_in, 1.0).ravel()
    rho = np.ones(lay.ncell)
    rf = np.random.default_rng(seed + 2)
    bu = rf.standard_normal(lay.nvel)
    bu[lay.wall_mask()] = 0.0
    return Workload("2d-noslip-discs", dim, lay.n, lay.bc, h, 0.0, P2, FGMRES, FP64,
                    EDGE_HARMONIC, rho, mu, bu, np.zeros(lay.ncell))


def _tanh_profile(z, r, width):
    return 0.5 * (r + 1.0) + 0.5 * (r - 1.0) * np.tanh((z - 0.5) / width)


def layers_3d(seed=3000, n=128, dt=1e-2, rho_ratio=1e2, mu_ratio=1e4, noise=1e-2,
              precision=MG_FP32):
    """3D no-slip unit cube, unsteady (theta = 1/dt), two layers split at
    z = 0.5 by a tanh profile of width 2h (heavy, viscous fluid on top):
    rho contrast 1e2, mu contrast 1e4.  Forcing: gravity -rho(z_face) e_z
    evaluated from the same profile at the z-face centres, plus 1e-2 N(0,1)
    noise on every interior face."""
    dim = 3
    n3 = _n3(dim, n)
    lay = make_layout(dim, n3, (NOSLIP, NOSLIP, NOSLIP))
    h = 1.0 / n3[0]
    width = 2.0 * h
    Z = lay.cell_centres(h)[2]
    rho = _tanh_profile(Z, rho_ratio, width).ravel()
    mu = _tanh_profile(Z, mu_ratio, width).ravel()
    rf = np.random.default_rng(seed + 2)
    bu = noise * rf.standard_normal(lay.nvel)
    zf = lay.face_centres(2, h)[2]
    o = lay.face_offsets[2]
    bu[o:o + lay.face_counts[2]] += -_tanh_profile(zf, rho_ratio, width).ravel()
    bu[lay.wall_mask()] = 0.0
    return Workload("3d-noslip-layers", dim, lay.n, lay.bc, h, 1.0 / dt, P1, FGMRES, precision,
                    EDGE_ARITH, rho, mu, bu, np.zeros(lay.ncell))


def contrast_periodic_3d(seed=4000, n=256, contrast=1e6, precision=MG_FP32):
    """3D periodic unit cube, steady (theta = 0), rho = 1,
    mu = exp(ln(contrast) u) with u a smooth 16-mode field (|k| <= 6) in [0, 1];
    forcing: smooth 16-mode field per component with the means removed (the
    periodic steady problem needs zero-mean forcing)."""
    dim = 3
    n3 = _n3(dim, n)
    lay = make_layout(dim, n3, (PERIODIC, PERIODIC, PERIODIC))
    h = 1.0 / n3[0]
    rc = np.random.default_rng(seed + 1)
    u01 = _minmax(eval_modes(smooth_field_modes(rc, dim, 16, 6), _axes_cell(lay, h)), 0.0, 1.0)
    mu = np.exp(np.log(contrast) * u01).ravel()
    rho = np.ones(lay.ncell)
    rf = np.random.default_rng(seed + 2)
    bu = smooth_face_field(rf, lay, h, 16, 6)
    return Workload("3d-periodic-contrast", dim, lay.n, lay.bc, h, 0.0, P2, FGMRES, precision,
                    EDGE_ARITH, rho, mu, bu, np.zeros(lay.ncell))


def log_viscosity_field(rng, lay: Layout, sigma_cells=5.0):
    """N(0,1) white noise smoothed by a Gaussian of sigma = 5 cells (reflecting
    ends), normalised to zero mean and unit standard deviation."""
    from scipy.ndimage import gaussian_filter

    w = rng.standard_normal(lay.cell_shape)
    s = gaussian_filter(w, sigma=sigma_cells, mode="reflect")
    s = (s - s.mean()) / s.std()
    return s.ravel()


def adjoint_3d(seed=5000, n=128, dt=1e-2, precision=FP64):
    """3D no-slip unit cube, unsteady (theta = 1/dt), rho = 1, mu = exp(s) with
    s a Gaussian-smoothed N(0,1) field; smooth forcing (8 modes, |k| <= 4).
    extra['s'] holds the log-viscosity; extra['s2'], extra['bu2'] the second
    draw used to make the target velocity."""
    dim = 3
    n3 = _n3(dim, n)
    lay = make_layout(dim, n3, (NOSLIP, NOSLIP, NOSLIP))
    h = 1.0 / n3[0]
    rc = np.random.default_rng(seed + 1)
    s = log_viscosity_field(rc, lay)
    rf = np.random.default_rng(seed + 2)
    bu = smooth_face_field(rf, lay, h, 8, 4, remove_mean=False)
    bu[lay.wall_mask()] = 0.0
    rt = np.random.default_rng(seed + 3)
    s2 = log_viscosity_field(rt, lay)
    bu2 = smooth_face_field(rt, lay, h, 8, 4, remove_mean=False)
    bu2[lay.wall_mask()] = 0.0
    w = Workload("3d-noslip-adjoint", dim, lay.n, lay.bc, h, 1.0 / dt, P1, GMRES_LEFT, precision,
                 EDGE_ARITH, np.ones(lay.ncell), np.exp(s), bu, np.zeros(lay.ncell))
    w.extra.update(s=s, s2=s2, bu2=bu2)
    return w


def fd_directions(seed, lay: Layout, count):
    """Seeded unit directions in log-viscosity space and in forcing space."""
    r = np.random.default_rng(seed + 4)
    ds = r.standard_normal((count, lay.ncell))
    ds /= np.linalg.norm(ds, axis=1, keepdims=True)
    df = r.standard_normal((count, lay.nvel))
    df[:, lay.wall_mask()] = 0.0
    df /= np.linalg.norm(df, axis=1, keepdims=True)
    return ds, df


def bubble(dim=3, n=32, r_mu=100.0, r_rho=100.0, theta=0.0, seed=6000):
    """The paper's bubble test problem (Sec. "Results", eq. varcoeff_def): a sphere
    (disk in 2D) of radius L/4 at the centre of the unit cube (square) with
    no-slip walls; mu = f(x; r_mu), rho = f(x; r_rho) with
    f(x; r) = (r+1)/2 + (r-1)/2 tanh(d/eps) + 0.1 R, d the signed distance to
    the interface (positive outside), eps = h, R ~ U(0,1) per cell.  So the
    bubble holds ~1 and the surrounding fluid ~r.  Steady by default.
    The right-hand side is left to the caller (the paper uses b = M x for a
    random x); extra['x_u'], extra['x_p'] hold such a seeded random x."""
    n3 = _n3(dim, n)
    lay = make_layout(dim, n3, (NOSLIP,) * dim)
    h = 1.0 / n3[0]
    cc = lay.cell_centres(h)
    d = np.sqrt(sum((c - 0.5) ** 2 for c in cc)) - 0.25
    rng = np.random.default_rng(seed + 1)

    def f(r):
        return (0.5 * (r + 1) + 0.5 * (r - 1) * np.tanh(d / h) + 0.1 * rng.uniform(0, 1, d.shape)).ravel()

    mu = f(r_mu)
    rho = f(r_rho)
    rx = np.random.default_rng(seed + 3)
    xu = rx.standard_normal(lay.nvel)
    xu[lay.wall_mask()] = 0.0
    xp = rx.standard_normal(lay.ncell)
    w = Workload(f"{dim}d-bubble-r{r_mu:g}", dim, lay.n, lay.bc, h, theta, P1, GMRES_LEFT, FP64,
                 EDGE_ARITH, rho, mu, np.zeros(lay.nvel), np.zeros(lay.ncell))
    w.extra.update(x_u=xu, x_p=xp)
    return w


WORKLOADS = {
    "2d-periodic-smooth": periodic_smooth_2d,
    "2d-noslip-discs": discs_2d,
    "3d-noslip-layers": layers_3d,
    "3d-periodic-contrast": contrast_periodic_3d,
    "3d-noslip-adjoint": adjoint_3d,
    "bubble": bubble,
}


def random_coefficients(seed, lay: Layout, mu_range=(0.5, 2.0), rho_range=(0.5, 2.0)):
    """Generic small-test coefficients: i.i.d. uniform cell values."""
    r = np.random.default_rng(seed)
    mu = r.uniform(*mu_range, lay.ncell)
    rho = r.uniform(*rho_range, lay.ncell)
    return rho, mu


def random_bulk_viscosity(seed, lay: Layout, gamma_range=(0.0, 2.0)):
    """Bulk viscosity per cell for small tests: i.i.d. uniform, >= 0."""
    return np.random.default_rng(seed).uniform(*gamma_range, lay.ncell)


def random_velocity(seed, lay: Layout, remove_mean=False):
    r = np.random.default_rng(seed)
    u = r.standard_normal(lay.nvel)
    u[lay.wall_mask()] = 0.0
    if remove_mean:
        u = _remove_component_means(lay, u)
    return u


def random_cells(seed, lay: Layout, remove_mean=False):
    r = np.random.default_rng(seed)
    p = r.standard_normal(lay.ncell)
    if remove_mean:
        p = p - p.mean()
    return p
