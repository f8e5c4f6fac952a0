"""The finest-level velocity V-cycle of a colour-split FP32 hierarchy,
recorded at create as a HIP graph and replayed, against the same V-cycle
launched kernel by kernel (STOKES_VGRAPH=0 at create time).

The graph holds the same kernels with the same arguments in the same order,
so every replay must equal the eager result bit for bit.  Replays are
interleaved with other work of the library on the same stream (operator
applications, solves) and with host synchronisations, and each one is
checked.
"""
import os

import numpy as np
import pytest

from gpu_common import N, T, params, rel
from paper_1308_4605_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ctx(p, rho, mu, gamma, graph):
    from paper_1308_4605_amd.stokes import Stokes

    old = os.environ.get("STOKES_VGRAPH")
    os.environ["STOKES_VGRAPH"] = "1" if graph else "0"
    try:
        return Stokes(p, T(rho), T(mu), gamma=None if gamma is None else T(gamma))
    finally:
        if old is None:
            del os.environ["STOKES_VGRAPH"]
        else:
            os.environ["STOKES_VGRAPH"] = old


# colour-split finest levels (FP32, n0 >= 128): periodic, walls, alpha, bulk
CASES = [((128, 32, 32), (0, 0, 0), 0.0, False), ((128, 64, 16), (1, 0, 2), 30.0, False),
         ((256, 32), (0, 1), 0.0, False), ((128, 32, 32), (0, 0, 0), 10.0, True)]


@pytest.mark.parametrize("n,bc,theta,bulk", CASES)
def test_graph_replays_equal_eager(n, bc, theta, bulk):
    import torch

    dim = len(n)
    print(f"vgraph replays {n} {bc} theta={theta} bulk={bulk}", flush=True)
    lay = W.make_layout(dim, n, bc)
    rho, mu = W.random_coefficients(81, lay, mu_range=(0.1, 10.0))
    gamma = W.random_bulk_viscosity(82, lay) if bulk else None
    p, _ = params(dim, n, bc, theta, precision=W.MG_FP32, krylov=W.FGMRES, precond=W.P2)
    a = _ctx(p, rho, mu, gamma, True)
    b = _ctx(p, rho, mu, gamma, False)
    xu, xp = T(W.random_velocity(83, lay)), T(W.random_cells(84, lay))
    for rep in range(4):
        r = W.random_velocity(85 + rep, lay, remove_mean=lay.singular_components(theta))
        ea = N(a.vel_subsolve(T(r)))
        eb = N(b.vel_subsolve(T(r)))
        print(f"  replay {rep}: max |graph - eager| = {np.abs(ea - eb).max():.3e}", flush=True)
        assert np.all(np.isfinite(ea))
        assert np.array_equal(ea, eb)
        # other work on the stream between replays, then a host sync
        a.apply(xu, xp)
        a.precond(xu, xp)
        torch.cuda.synchronize()
    a.close()
    b.close()


@pytest.mark.timeout(300)
def test_graph_solve_equals_eager():
    """FGMRES(10) with P2 on the contrast-1e6 periodic field at 128^3: the
    graph replays inside the solve give the eager solve's iterates."""
    print("vgraph solve contrast 1e6 128^3", flush=True)
    w = W.contrast_periodic_3d(n=128, contrast=1e6, precision=W.MG_FP32)
    p = w.params()
    a = _ctx(p, w.rho, w.mu, None, True)
    b = _ctx(p, w.rho, w.mu, None, False)
    for rep in range(2):
        xa, pa, sa, ra = a.solve(T(w.bu), T(w.bp), tol=1e-8, max_iter=500)
        xb, pb, sb, rb = b.solve(T(w.bu), T(w.bp), tol=1e-8, max_iter=500)
        print(f"  solve {rep}: iters graph {sa['iters']} eager {sb['iters']} "
              f"rel diff u {rel(N(xa), N(xb)):.2e}", flush=True)
        assert ra == 0 and rb == 0
        assert sa["iters"] == sb["iters"]
        assert np.array_equal(N(xa), N(xb)) and np.array_equal(N(pa), N(pb))
    a.close()
    b.close()
