"""Thin ctypes binding of libstokes_mi355x.so (include/stokes.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  PyTorch supplies device memory (the workspace and the caller's
arrays) and the HIP stream.  There is no CPU fallback: if the library is
missing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstokes_mi355x.so")

STOKES_OK = 0
STOKES_EINVAL = -1
STOKES_ENOMEM = -2
STOKES_EDEVICE = -3
STOKES_ENOCONV = -4
STOKES_EBREAKDOWN = -5
STOKES_ENONFINITE = -6
STOKES_EINCOMPAT = -7

# names declared in include/stokes.h
ABI_FUNCTIONS = (
    "stokes_sizes", "stokes_workspace_bytes", "stokes_create", "stokes_apply", "stokes_residual",
    "stokes_boundary_rhs", "stokes_precond",
    "stokes_vel_subsolve", "stokes_p_subsolve", "stokes_vel_mg_solve", "stokes_p_mg_solve",
    "stokes_solve", "stokes_solve_static", "stokes_adjoint_solve",
    "stokes_grad", "stokes_rescale", "stokes_set_timing", "stokes_kernel_time", "stokes_destroy",
    "stokes_set_history", "stokes_vcycle_time",
    "stokes_strerror",
)


class StokesParams(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("bc", ctypes.c_int * 3), ("theta", ctypes.c_double), ("precond", ctypes.c_int),
                ("precision", ctypes.c_int), ("krylov", ctypes.c_int), ("restart", ctypes.c_int),
                ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int), ("nu_coarse", ctypes.c_int),
                ("vcycles", ctypes.c_int), ("rescale_c", ctypes.c_double),
                ("edge_avg", ctypes.c_int), ("bulk", ctypes.c_int), ("scaling", ctypes.c_int),
                ("extended", ctypes.c_int)]


class StokesStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("precond_applies", ctypes.c_int), ("scalar_vcycles", ctypes.c_int),
                ("rel_res_true", ctypes.c_double), ("rel_res_est", ctypes.c_double),
                ("rel_res_unscaled", ctypes.c_double), ("history_len", ctypes.c_int),
                ("t_total", ctypes.c_double), ("t_precond", ctypes.c_double),
                ("t_krylov", ctypes.c_double)]

    def as_dict(self, history=None):
        out = {f: getattr(self, f) for f, _ in self._fields_}
        if history is not None:
            out["history"] = [history[i] for i in range(self.history_len)]
        return out


class StokesError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


_lib = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_1308_4605_amd.build.build() "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.c_void_p
        PP = ctypes.POINTER(StokesParams)
        L.stokes_sizes.argtypes = [PP, ctypes.POINTER(ctypes.c_size_t),
                                   ctypes.POINTER(ctypes.c_size_t),
                                   ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int)]
        L.stokes_workspace_bytes.argtypes = [PP]
        L.stokes_workspace_bytes.restype = ctypes.c_size_t
        L.stokes_create.argtypes = [PP, dp, dp, dp, dp, dp, ctypes.c_size_t, vp,
                                    ctypes.POINTER(ctypes.c_void_p)]
        L.stokes_apply.argtypes = [vp, dp, dp, dp, dp]
        L.stokes_precond.argtypes = [vp, dp, dp, dp, dp]
        L.stokes_residual.argtypes = [vp, dp, dp, dp, dp, dp, dp, ctypes.c_int]
        L.stokes_boundary_rhs.argtypes = [vp, dp, dp, dp, dp]
        L.stokes_vel_subsolve.argtypes = [vp, dp, dp]
        L.stokes_p_subsolve.argtypes = [vp, dp, dp]
        for f in ("stokes_vel_mg_solve", "stokes_p_mg_solve"):
            getattr(L, f).argtypes = [vp, dp, dp, ctypes.c_double, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        L.stokes_solve.argtypes = [vp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(StokesStats)]
        L.stokes_solve_static.argtypes = L.stokes_solve.argtypes
        L.stokes_adjoint_solve.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp,
                                           ctypes.c_double, ctypes.c_int,
                                           ctypes.POINTER(StokesStats)]
        L.stokes_grad.argtypes = [vp, dp, dp, dp, dp, dp, dp]
        L.stokes_rescale.argtypes = [vp]
        L.stokes_rescale.restype = ctypes.c_double
        L.stokes_set_timing.argtypes = [vp, ctypes.c_int]
        L.stokes_set_history.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        L.stokes_vcycle_time.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_long),
                                         ctypes.POINTER(ctypes.c_double)]
        L.stokes_kernel_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_long),
                                         ctypes.POINTER(ctypes.c_double)]
        L.stokes_destroy.argtypes = [vp]
        L.stokes_strerror.argtypes = [ctypes.c_int]
        L.stokes_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().stokes_strerror(int(code)).decode()


def make_params(dim, n, bc, h, theta, precond=1, precision=0, krylov=0, restart=10, nu_pre=2,
                nu_post=2, nu_coarse=8, vcycles=1, rescale_c=0.0, edge_avg=0, bulk=0,
                scaling=0, extended=0, **_ignored):
    p = StokesParams()
    p.dim = int(dim)
    n = tuple(n) + (1,) * (3 - len(n))
    bc = tuple(bc) + (0,) * (3 - len(bc))
    for a in range(3):
        p.n[a] = int(n[a])
        p.bc[a] = int(bc[a])
    p.h, p.theta = float(h), float(theta)
    p.precond, p.precision, p.krylov, p.restart = int(precond), int(precision), int(krylov), int(restart)
    p.nu_pre, p.nu_post, p.nu_coarse, p.vcycles = int(nu_pre), int(nu_post), int(nu_coarse), int(vcycles)
    p.rescale_c, p.edge_avg = float(rescale_c), int(edge_avg)
    p.bulk = int(bulk)
    p.scaling, p.extended = int(scaling), int(extended)
    return p


def stokes_sizes(params: StokesParams):
    nv, nc, ne = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    nl = ctypes.c_int()
    rc = lib().stokes_sizes(ctypes.byref(params), ctypes.byref(nv), ctypes.byref(nc),
                            ctypes.byref(ne), ctypes.byref(nl))
    if rc:
        raise StokesError(rc, "stokes_sizes")
    return nv.value, nc.value, ne.value, nl.value


def stokes_workspace_bytes(params: StokesParams) -> int:
    return int(lib().stokes_workspace_bytes(ctypes.byref(params)))


def _ptr(t):
    if t is None:
        return None
    import torch

    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), (t.device, t.dtype)
    return ctypes.c_void_p(t.data_ptr())


class Stokes:
    """One solver context: coefficients, multigrid hierarchy and Krylov
    workspace on the current HIP device, all in one caller-owned workspace
    tensor.  Methods take and return torch float64 CUDA tensors in the ABI
    layout (flat arrays).  gamma: bulk viscosity per cell (the stress with
    (gamma - 2/3 mu)(div u) I), or None for the incompressible stress form."""

    def __init__(self, params: dict, rho, mu, mu_edges=None, stream=None, gamma=None):
        import torch

        self.params = dict(params, bulk=0 if gamma is None else 1)
        self.bulk = gamma is not None
        self.p = make_params(**self.params)
        self.nvel, self.ncell, self.nedge, self.nlevels = stokes_sizes(self.p)
        self.ws_bytes = stokes_workspace_bytes(self.p)
        dev = rho.device
        self.device = dev
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        rc = lib().stokes_create(ctypes.byref(self.p), _ptr(rho), _ptr(mu), _ptr(mu_edges),
                                 _ptr(gamma), ctypes.c_void_p(self.workspace.data_ptr()),
                                 self.ws_bytes,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc:
            raise StokesError(rc, "stokes_create")
        self._h = h
        self.c = lib().stokes_rescale(h)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().stokes_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, n):
        import torch

        return torch.empty(n, dtype=torch.float64, device=self.device)

    def apply(self, xu, xp):
        yu, yp = self._new(self.nvel), self._new(self.ncell)
        rc = lib().stokes_apply(self._h, _ptr(xu), _ptr(xp), _ptr(yu), _ptr(yp))
        if rc:
            raise StokesError(rc, "stokes_apply")
        return yu, yp

    def residual(self, bu, bp, xu, xp, extended=False):
        """r = b - M x (FP64, or double-double rounded once when extended)."""
        ru, rp = self._new(self.nvel), self._new(self.ncell)
        rc = lib().stokes_residual(self._h, _ptr(bu), _ptr(bp), _ptr(xu), _ptr(xp), _ptr(ru),
                                   _ptr(rp), 1 if extended else 0)
        if rc:
            raise StokesError(rc, "stokes_residual")
        return ru, rp

    def precond(self, bu, bp):
        zu, zp = self._new(self.nvel), self._new(self.ncell)
        rc = lib().stokes_precond(self._h, _ptr(bu), _ptr(bp), _ptr(zu), _ptr(zp))
        if rc:
            raise StokesError(rc, "stokes_precond")
        return zu, zp

    def boundary_rhs(self, un, ut):
        """Boundary terms (cu, cp) of prescribed wall velocities: normal values
        un on the wall faces, tangential values ut on the wall edges."""
        cu, cp = self._new(self.nvel), self._new(self.ncell)
        rc = lib().stokes_boundary_rhs(self._h, _ptr(un), _ptr(ut), _ptr(cu), _ptr(cp))
        if rc:
            raise StokesError(rc, "stokes_boundary_rhs")
        return cu, cp

    def vel_subsolve(self, r):
        e = self._new(self.nvel)
        rc = lib().stokes_vel_subsolve(self._h, _ptr(r), _ptr(e))
        if rc:
            raise StokesError(rc, "stokes_vel_subsolve")
        return e

    def p_subsolve(self, r):
        e = self._new(self.ncell)
        rc = lib().stokes_p_subsolve(self._h, _ptr(r), _ptr(e))
        if rc:
            raise StokesError(rc, "stokes_p_subsolve")
        return e

    def _mg_solve(self, fn, r, n, tol, max_cycles):
        e = self._new(n)
        cyc, rel = ctypes.c_int(), ctypes.c_double()
        rc = getattr(lib(), fn)(self._h, _ptr(r), _ptr(e), float(tol), int(max_cycles),
                                ctypes.byref(cyc), ctypes.byref(rel))
        if rc not in (STOKES_OK, STOKES_ENOCONV):
            raise StokesError(rc, fn)
        return e, cyc.value, rel.value, rc

    def vel_mg_solve(self, r, tol=1e-10, max_cycles=200):
        """Velocity multigrid run to ||r - A e|| <= tol ||r||: (e, cycles, rel_res, rc)."""
        return self._mg_solve("stokes_vel_mg_solve", r, self.nvel, tol, max_cycles)

    def p_mg_solve(self, r, tol=1e-10, max_cycles=200):
        """Pressure multigrid run to ||r - L e|| <= tol ||r||: (e, cycles, rel_res, rc)."""
        return self._mg_solve("stokes_p_mg_solve", r, self.ncell, tol, max_cycles)

    def solve(self, bu, bp, tol=1e-8, max_iter=1000, x0=None, check=True, out=None,
              history=False):
        """Returns (xu, xp, stats, rc); history=True adds the per-iteration
        residual estimates to stats["history"]."""
        if out is not None:
            xu, xp = out
        else:
            xu, xp = self._new(self.nvel), self._new(self.ncell)
        if x0 is not None:
            xu.copy_(x0[0])
            xp.copy_(x0[1])
        st, buf = StokesStats(), None
        if history:
            buf = (ctypes.c_double * (int(max_iter) + 1))()
            lib().stokes_set_history(self._h, buf, int(max_iter) + 1)
        try:
            rc = lib().stokes_solve(self._h, _ptr(bu), _ptr(bp), _ptr(xu), _ptr(xp), float(tol),
                                    int(max_iter), 1 if x0 is not None else 0, ctypes.byref(st))
        finally:
            if history:
                lib().stokes_set_history(self._h, None, 0)
        if check and rc:
            raise StokesError(rc, "stokes_solve")
        return xu, xp, st.as_dict(buf), rc

    def solve_static(self, bu, bp, tol=1e-8, max_iter=1000, check=True):
        """stokes_solve_static: the solve with its Krylov storage in the
        library's static device array (no allocation in the library).
        Returns (xu, xp, stats, rc)."""
        xu, xp = self._new(self.nvel), self._new(self.ncell)
        st = StokesStats()
        rc = lib().stokes_solve_static(self._h, _ptr(bu), _ptr(bp), _ptr(xu), _ptr(xp),
                                       float(tol), int(max_iter), 0, ctypes.byref(st))
        if check and rc:
            raise StokesError(rc, "stokes_solve_static")
        return xu, xp, st.as_dict(), rc

    def adjoint(self, xu, xp, gu, gp, tol=1e-8, max_iter=1000, check=True):
        lu, lp = self._new(self.nvel), self._new(self.ncell)
        dmc, dme, drho = self._new(self.ncell), self._new(self.nedge), self._new(self.ncell)
        dg = self._new(self.ncell) if self.bulk else None
        st = StokesStats()
        rc = lib().stokes_adjoint_solve(self._h, _ptr(xu), _ptr(xp), _ptr(gu), _ptr(gp), _ptr(lu),
                                        _ptr(lp), _ptr(dmc), _ptr(dme), _ptr(drho), _ptr(dg),
                                        float(tol), int(max_iter), ctypes.byref(st))
        if check and rc:
            raise StokesError(rc, "stokes_adjoint_solve")
        out = dict(lu=lu, lp=lp, dmu_cell=dmc, dmu_edge=dme, drho_cell=drho,
                   stats=st.as_dict(), rc=rc)
        if self.bulk:
            out["dgamma_cell"] = dg
        return out

    def grad(self, xu, lu):
        dmc, dme, drho = self._new(self.ncell), self._new(self.nedge), self._new(self.ncell)
        dg = self._new(self.ncell) if self.bulk else None
        rc = lib().stokes_grad(self._h, _ptr(xu), _ptr(lu), _ptr(dmc), _ptr(dme), _ptr(drho),
                               _ptr(dg))
        if rc:
            raise StokesError(rc, "stokes_grad")
        out = dict(dmu_cell=dmc, dmu_edge=dme, drho_cell=drho)
        if self.bulk:
            out["dgamma_cell"] = dg
        return out

    def set_timing(self, enable):
        """0 / False: off; 1 / True: per-launch and per-V-cycle events (the
        V-cycles run kernel by kernel); 2: per-V-cycle events only."""
        rc = lib().stokes_set_timing(self._h, int(enable))
        if rc:
            raise StokesError(rc, "stokes_set_timing")

    def vcycle_time(self, pressure: bool):
        """(ms, cycles, algorithmic bytes) of the timed finest-level V-cycles."""
        ms, n, b = ctypes.c_double(), ctypes.c_long(), ctypes.c_double()
        rc = lib().stokes_vcycle_time(self._h, 1 if pressure else 0, ctypes.byref(ms),
                                      ctypes.byref(n), ctypes.byref(b))
        if rc:
            raise StokesError(rc, "stokes_vcycle_time")
        return ms.value, n.value, b.value

    def kernel_time(self):
        ms, n, b = ctypes.c_double(), ctypes.c_long(), ctypes.c_double()
        rc = lib().stokes_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b))
        if rc:
            raise StokesError(rc, "stokes_kernel_time")
        return ms.value, n.value, b.value
