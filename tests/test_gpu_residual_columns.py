"""The 3D FP32 velocity residual by columns along z (a thread carries the
values two planes share) against the residual by cells
(STOKES_RESIDUAL_COLUMNS=0 at create time).

Both forms load the same values and run the same row arithmetic, so every
result must agree bit for bit: the V-cycle (its residual before the
restriction), two V-cycles per subsolve (the residual between them), P5 (the
residual with the pressure gradient), and whole FGMRES solves.  The grids have at least 2^21 cells, where the columns are used:
periodic, every wall kind, alpha, the bulk term, and z extents that are not a
multiple of the column length (one partial column that wraps; a partial last
column against a wall), a y extent that is not a multiple of 8 (threads not
banded by XCD), with the default column length, with columns of 3 cells, and
with a length beyond every z extent (one column per thread, the whole axis).
"""
import os

import numpy as np
import pytest

from gpu_common import N, T, params
from paper_1308_4605_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ctx(p, rho, mu, gamma, columns):
    """columns: None for the library's default column length, else the value
    of STOKES_RESIDUAL_COLUMNS at create time ("0": by cells)."""
    from paper_1308_4605_amd.stokes import Stokes

    old = os.environ.pop("STOKES_RESIDUAL_COLUMNS", None)
    if columns is not None:
        os.environ["STOKES_RESIDUAL_COLUMNS"] = columns
    try:
        return Stokes(p, T(rho), T(mu), gamma=None if gamma is None else T(gamma))
    finally:
        os.environ.pop("STOKES_RESIDUAL_COLUMNS", None)
        if old is not None:
            os.environ["STOKES_RESIDUAL_COLUMNS"] = old


# (n, bc, theta, bulk, precond, vcycles)
CASES = [((128, 128, 128), (0, 0, 0), 0.0, False, W.P2, 1),
         ((128, 128, 128), (1, 0, 2), 30.0, False, W.P2, 1),
         ((128, 128, 128), (0, 1, 0), 10.0, True, W.P1, 2),
         ((1024, 512, 4), (0, 0, 0), 0.0, False, W.P2, 1),
         ((8, 512, 516), (0, 0, 1), 0.0, False, W.P5, 1),
         ((256, 128, 64), (3, 4, 0), 5.0, True, W.P5, 2),
         ((1024, 4, 512), (0, 0, 0), 0.0, False, W.P2, 1)]


@pytest.mark.parametrize("n,bc,theta,bulk,precond,vcycles", CASES)
@pytest.mark.parametrize("columns", [None, "3", "99999999999"])
def test_columns_equal_cells(n, bc, theta, bulk, precond, vcycles, columns):
    print(f"residual columns {columns or 'default'} {n} {bc} theta={theta} bulk={bulk} "
          f"P{precond} vcycles={vcycles}", flush=True)
    lay = W.make_layout(3, n, bc)
    rho, mu = W.random_coefficients(91, lay, mu_range=(0.1, 10.0))
    gamma = W.random_bulk_viscosity(92, lay) if bulk else None
    p, _ = params(3, n, bc, theta, precision=W.MG_FP32, krylov=W.FGMRES, precond=precond,
                  vcycles=vcycles)
    a = _ctx(p, rho, mu, gamma, columns)
    b = _ctx(p, rho, mu, gamma, "0")
    r = W.random_velocity(93, lay, remove_mean=lay.singular_components(theta))
    ea, eb = N(a.vel_subsolve(T(r))), N(b.vel_subsolve(T(r)))
    print(f"  subsolve: max |columns - cells| = {np.abs(ea - eb).max():.3e}", flush=True)
    assert np.all(np.isfinite(ea))
    assert np.array_equal(ea, eb)
    bu, bp = T(W.random_velocity(94, lay)), T(W.random_cells(95, lay))
    (ua, pa), (ub, pb) = a.precond(bu, bp), b.precond(bu, bp)
    print(f"  precond: max |columns - cells| = {np.abs(N(ua) - N(ub)).max():.3e}", flush=True)
    assert np.array_equal(N(ua), N(ub)) and np.array_equal(N(pa), N(pb))
    a.close()
    b.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", [W.MG_FP32, W.FP64])
def test_columns_solve_equal_cells(precision):
    """FGMRES(10) with P2 on the contrast-1e6 periodic field at 128^3: the
    same iterates and solution with either form (the FP64 form keeps the
    residual by cells, so its solve checks that the switch leaves it alone)."""
    print(f"residual columns solve contrast 1e6 128^3 precision={precision}", flush=True)
    w = W.contrast_periodic_3d(n=128, contrast=1e6, precision=precision)
    p = w.params(krylov=W.FGMRES)
    a = _ctx(p, w.rho, w.mu, None, None)
    b = _ctx(p, w.rho, w.mu, None, "0")
    xa, pa, sa, ra = a.solve(T(w.bu), T(w.bp), tol=1e-8, max_iter=500)
    xb, pb, sb, rb = b.solve(T(w.bu), T(w.bp), tol=1e-8, max_iter=500)
    print(f"  iters columns {sa['iters']} cells {sb['iters']}", flush=True)
    assert ra == 0 and rb == 0
    assert sa["iters"] == sb["iters"]
    assert np.array_equal(N(xa), N(xb)) and np.array_equal(N(pa), N(pb))
    a.close()
    b.close()
