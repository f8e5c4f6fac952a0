"""ctypes wrapper of the plain FP64 CPU oracle (stokes_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU product path never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stokes_oracle.c")
_LIB = os.path.join(_HERE, "libstokes_oracle.so")

ORC_OK, ORC_EINVAL, ORC_ENOMEM, ORC_ENOCONV, ORC_EBREAKDOWN, ORC_ENONFINITE, ORC_EINCOMPAT = (
    0, -1, -2, -4, -5, -6, -7)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP grid loops)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
            "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("bc", ctypes.c_int * 3), ("theta", ctypes.c_double),
                ("precond", ctypes.c_int), ("krylov", ctypes.c_int), ("restart", ctypes.c_int),
                ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int), ("nu_coarse", ctypes.c_int),
                ("vcycles", ctypes.c_int), ("rescale_c", ctypes.c_double),
                ("edge_avg", ctypes.c_int), ("scaling", ctypes.c_int),
                ("extended", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("precond_applies", ctypes.c_int), ("scalar_vcycles", ctypes.c_int),
                ("rel_res_true", ctypes.c_double), ("rel_res_est", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(ctypes.c_double)
        L.orc_create.argtypes = [ctypes.POINTER(_Params), P, P, P, P,
                                 ctypes.POINTER(ctypes.c_void_p)]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        for f in ("orc_nvel", "orc_ncell", "orc_nedge"):
            getattr(L, f).argtypes = [ctypes.c_void_p]
            getattr(L, f).restype = ctypes.c_size_t
        L.orc_nlevels.argtypes = [ctypes.c_void_p]
        L.orc_rescale.argtypes = [ctypes.c_void_p]
        L.orc_rescale.restype = ctypes.c_double
        L.orc_apply.argtypes = [ctypes.c_void_p, P, P, P, P]
        L.orc_residual.argtypes = [ctypes.c_void_p, P, P, P, P, P, P, ctypes.c_int]
        L.orc_diag_scaling.argtypes = [ctypes.c_void_p, P]
        L.orc_precond.argtypes = [ctypes.c_void_p, P, P, P, P]
        L.orc_boundary_rhs.argtypes = [ctypes.c_void_p, P, P, P, P]
        L.orc_vel_subsolve.argtypes = [ctypes.c_void_p, P, P]
        L.orc_p_subsolve.argtypes = [ctypes.c_void_p, P, P]
        for f in ("orc_vel_mg_solve", "orc_p_mg_solve"):
            getattr(L, f).argtypes = [ctypes.c_void_p, P, P, ctypes.c_double, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        L.orc_vel_sweep.argtypes = [ctypes.c_void_p, P, P]
        L.orc_p_sweep.argtypes = [ctypes.c_void_p, P, P]
        L.orc_level_coef.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, P, ctypes.c_size_t]
        L.orc_level_dims.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int * 3]
        for f in ("orc_restrict_faces", "orc_prolong_add_faces", "orc_restrict_cells",
                  "orc_prolong_add_cells"):
            getattr(L, f).argtypes = [ctypes.c_void_p, ctypes.c_int, P, P]
        L.orc_level_sizes.argtypes = [ctypes.c_void_p, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_size_t),
                                      ctypes.POINTER(ctypes.c_size_t)]
        L.orc_solve.argtypes = [ctypes.c_void_p, P, P, P, P, ctypes.c_double, ctypes.c_int,
                                ctypes.c_int, ctypes.POINTER(Stats)]
        L.orc_adjoint.argtypes = [ctypes.c_void_p, P, P, P, P, P, P, P, P, P, P,
                                  ctypes.c_double, ctypes.c_int, ctypes.POINTER(Stats)]
        L.orc_grad.argtypes = [ctypes.c_void_p, P, P, P, P, P, P]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel())


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} returned {code}")
        self.code = code


class Oracle:
    """One oracle context: coefficients, hierarchy and solver parameters.
    gamma: bulk viscosity per cell (stress form with (gamma - 2/3 mu)(div u) I),
    or None for the incompressible stress form."""

    def __init__(self, dim, n, bc, h, theta, rho, mu, edges=None, precond=1, krylov=0,
                 restart=10, nu_pre=2, nu_post=2, nu_coarse=8, vcycles=1, rescale_c=0.0,
                 edge_avg=0, gamma=None, scaling=0, extended=0, **_ignored):
        L = lib()
        p = _Params()
        p.dim = dim
        n = tuple(n) + (1,) * (3 - len(n))
        bc = tuple(bc) + (0,) * (3 - len(bc))
        for a in range(3):
            p.n[a] = int(n[a])
            p.bc[a] = int(bc[a])
        p.h, p.theta = float(h), float(theta)
        p.precond, p.krylov, p.restart = precond, krylov, restart
        p.nu_pre, p.nu_post, p.nu_coarse, p.vcycles = nu_pre, nu_post, nu_coarse, vcycles
        p.rescale_c, p.edge_avg = float(rescale_c), edge_avg
        p.scaling, p.extended = int(scaling), int(extended)
        self._rho, self._mu = _f64(rho), _f64(mu)
        self._edges = None if edges is None else _f64(edges)
        self._gamma = None if gamma is None else _f64(gamma)
        self.bulk = gamma is not None
        h_ = ctypes.c_void_p()
        rc = L.orc_create(ctypes.byref(p), _p(self._rho), _p(self._mu), _p(self._edges),
                          _p(self._gamma), ctypes.byref(h_))
        if rc != ORC_OK:
            raise OracleError(rc, "create")
        self._h = h_
        self.dim, self.theta = dim, theta
        self.nvel = L.orc_nvel(h_)
        self.ncell = L.orc_ncell(h_)
        self.nedge = L.orc_nedge(h_)
        self.nlevels = L.orc_nlevels(h_)
        self.c = L.orc_rescale(h_)

    @classmethod
    def from_workload(cls, w, **over):
        p = w.params(**over)
        return cls(rho=w.rho, mu=w.mu, **p)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    def apply(self, xu, xp):
        xu, xp = _f64(xu), _f64(xp)
        yu, yp = np.empty(self.nvel), np.empty(self.ncell)
        rc = lib().orc_apply(self._h, _p(xu), _p(xp), _p(yu), _p(yp))
        if rc:
            raise OracleError(rc, "apply")
        return yu, yp

    def residual(self, bu, bp, xu, xp, extended=False):
        """r = b - M x (caller's coefficients), FP64 or __float128 rounded once."""
        bu, bp, xu, xp = _f64(bu), _f64(bp), _f64(xu), _f64(xp)
        ru, rp = np.empty(self.nvel), np.empty(self.ncell)
        rc = lib().orc_residual(self._h, _p(bu), _p(bp), _p(xu), _p(xp), _p(ru), _p(rp),
                                1 if extended else 0)
        if rc:
            raise OracleError(rc, "residual")
        return ru, rp

    def diag_scaling(self):
        """The diagonal scaling S of the rescaled unknowns [faces | cells]."""
        s = np.empty(self.nvel + self.ncell)
        rc = lib().orc_diag_scaling(self._h, _p(s))
        if rc:
            raise OracleError(rc, "diag_scaling")
        return s

    def precond(self, bu, bp):
        bu, bp = _f64(bu), _f64(bp)
        zu, zp = np.empty(self.nvel), np.empty(self.ncell)
        rc = lib().orc_precond(self._h, _p(bu), _p(bp), _p(zu), _p(zp))
        if rc:
            raise OracleError(rc, "precond")
        return zu, zp

    def vel_subsolve(self, r):
        r = _f64(r)
        e = np.empty(self.nvel)
        rc = lib().orc_vel_subsolve(self._h, _p(r), _p(e))
        if rc:
            raise OracleError(rc, "vel_subsolve")
        return e

    def p_subsolve(self, r):
        r = _f64(r)
        e = np.empty(self.ncell)
        rc = lib().orc_p_subsolve(self._h, _p(r), _p(e))
        if rc:
            raise OracleError(rc, "p_subsolve")
        return e

    def boundary_rhs(self, un, ut):
        """Boundary terms (cu, cp) of the affine operator for prescribed wall
        velocities: normal values un on the wall faces (velocity layout) and
        tangential values ut on the wall edges (edge layout)."""
        un, ut = _f64(un), _f64(ut)
        cu, cp = np.empty(self.nvel), np.empty(self.ncell)
        rc = lib().orc_boundary_rhs(self._h, _p(un), _p(ut), _p(cu), _p(cp))
        if rc:
            raise OracleError(rc, "boundary_rhs")
        return cu, cp

    def _mg_solve(self, fn, r, n, tol, max_cycles):
        r = _f64(r)
        e = np.empty(n)
        cyc, rel = ctypes.c_int(), ctypes.c_double()
        rc = getattr(lib(), fn)(self._h, _p(r), _p(e), float(tol), int(max_cycles),
                                ctypes.byref(cyc), ctypes.byref(rel))
        if rc not in (ORC_OK, ORC_ENOCONV):
            raise OracleError(rc, fn)
        return e, cyc.value, rel.value, rc

    def vel_mg_solve(self, r, tol=1e-10, max_cycles=200):
        """Stand-alone velocity multigrid: V-cycles to ||r - A e|| <= tol ||r||.
        Returns (e, cycles, rel_res, rc)."""
        return self._mg_solve("orc_vel_mg_solve", r, self.nvel, tol, max_cycles)

    def p_mg_solve(self, r, tol=1e-10, max_cycles=200):
        """Stand-alone pressure multigrid, as vel_mg_solve for L_rho e = r."""
        return self._mg_solve("orc_p_mg_solve", r, self.ncell, tol, max_cycles)

    def vel_sweep(self, rhs, phi):
        rhs, phi = _f64(rhs), _f64(phi).copy()
        lib().orc_vel_sweep(self._h, _p(rhs), _p(phi))
        return phi

    def p_sweep(self, rhs, phi):
        rhs, phi = _f64(rhs), _f64(phi).copy()
        lib().orc_p_sweep(self._h, _p(rhs), _p(phi))
        return phi

    def level_dims(self, level):
        out = (ctypes.c_int * 3)()
        rc = lib().orc_level_dims(self._h, level, out)
        if rc:
            raise OracleError(rc, "level_dims")
        return tuple(out)

    def level_sizes(self, level):
        """(nvel, ncell) of multigrid level `level`."""
        nv, nc = ctypes.c_size_t(), ctypes.c_size_t()
        rc = lib().orc_level_sizes(self._h, level, ctypes.byref(nv), ctypes.byref(nc))
        if rc:
            raise OracleError(rc, "level_sizes")
        return nv.value, nc.value

    def _transfer(self, fn, level, src, dst_size, add_to=None):
        src = _f64(src)
        dst = np.zeros(dst_size) if add_to is None else _f64(add_to).copy()
        rc = getattr(lib(), fn)(self._h, level, _p(src), _p(dst))
        if rc:
            raise OracleError(rc, fn)
        return dst

    def restrict_faces(self, level, rf):
        """Face restriction of a level-`level` velocity field to level + 1."""
        return self._transfer("orc_restrict_faces", level, rf, self.level_sizes(level + 1)[0])

    def prolong_add_faces(self, level, ec, phif=None):
        """phif + P ec: face prolongation of a level + 1 field onto level `level`."""
        return self._transfer("orc_prolong_add_faces", level, ec, self.level_sizes(level)[0],
                              phif)

    def restrict_cells(self, level, rf):
        return self._transfer("orc_restrict_cells", level, rf, self.level_sizes(level + 1)[1])

    def prolong_add_cells(self, level, ec, pf=None):
        return self._transfer("orc_prolong_add_cells", level, ec, self.level_sizes(level)[1], pf)

    def level_coef(self, level, which, count):
        out = np.empty(count)
        rc = lib().orc_level_coef(self._h, level, which, _p(out), count)
        if rc:
            raise OracleError(rc, "level_coef")
        return out

    def solve(self, bu, bp, tol=1e-8, max_iter=1000, x0=None, check=True):
        bu, bp = _f64(bu), _f64(bp)
        if x0 is not None:
            xu, xp = _f64(x0[0]).copy(), _f64(x0[1]).copy()
        else:
            xu, xp = np.zeros(self.nvel), np.zeros(self.ncell)
        st = Stats()
        rc = lib().orc_solve(self._h, _p(bu), _p(bp), _p(xu), _p(xp), tol, max_iter,
                             1 if x0 is not None else 0, ctypes.byref(st))
        if check and rc:
            raise OracleError(rc, "solve")
        return xu, xp, st.as_dict(), rc

    def adjoint(self, xu, xp, gu, gp, tol=1e-8, max_iter=1000, check=True):
        xu, xp, gu, gp = _f64(xu), _f64(xp), _f64(gu), _f64(gp)
        lu, lp = np.empty(self.nvel), np.empty(self.ncell)
        dmc, dme, drho = np.empty(self.ncell), np.empty(self.nedge), np.empty(self.ncell)
        dg = np.empty(self.ncell) if self.bulk else None
        st = Stats()
        rc = lib().orc_adjoint(self._h, _p(xu), _p(xp), _p(gu), _p(gp), _p(lu), _p(lp),
                               _p(dmc), _p(dme), _p(drho), _p(dg), tol, max_iter,
                               ctypes.byref(st))
        if check and rc:
            raise OracleError(rc, "adjoint")
        out = dict(lu=lu, lp=lp, dmu_cell=dmc, dmu_edge=dme, drho_cell=drho,
                   stats=st.as_dict(), rc=rc)
        if self.bulk:
            out["dgamma_cell"] = dg
        return out

    def grad(self, xu, lu):
        xu, lu = _f64(xu), _f64(lu)
        dmc, dme, drho = np.empty(self.ncell), np.empty(self.nedge), np.empty(self.ncell)
        dg = np.empty(self.ncell) if self.bulk else None
        rc = lib().orc_grad(self._h, _p(xu), _p(lu), _p(dmc), _p(dme), _p(drho), _p(dg))
        if rc:
            raise OracleError(rc, "grad")
        out = dict(dmu_cell=dmc, dmu_edge=dme, drho_cell=drho)
        if self.bulk:
            out["dgamma_cell"] = dg
        return out


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP grid loops from now on."""
    lib().orc_set_threads(int(n))
