"""MI355X (gfx950) variable-coefficient MAC Stokes solver.

Block-preconditioned GMRES / flexible GMRES for the staggered-grid Stokes
saddle-point system of Cai, Nonaka, Bell, Griffith and Donev
(arXiv:1308.4605), with an FP32-multigrid preconditioner option and a
hand-written adjoint.  The solver lives in libstokes_mi355x.so (HIP kernels +
C ABI, include/stokes.h); this package is its Python binding.
"""
from . import workloads  # noqa: F401  (input generators; no solver arithmetic)

__all__ = ["workloads", "stokes", "autograd"]


def __getattr__(name):
    if name in ("stokes", "autograd", "build"):
        import importlib

        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
