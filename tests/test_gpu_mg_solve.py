"""The stand-alone multigrid solvers on the GPU (the velocity and pressure
V-cycle run to convergence, Sec. "The effect of the number of multigrid cycles") against the oracle: FP64 cycle counts
equal the oracle's (+-1) and the solutions agree to the tolerance; the FP32
hierarchy, used as iterative refinement under FP64 residuals, reaches the same
FP64 tolerances; and the coupled solver costs at most three split solves in
scalar V-cycles (tests/golden/paper_claims.json)."""
import json
import os

import numpy as np
import pytest

import oracle
from gpu_common import N, T, pair, params, rel
from paper_1308_4605_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_claims.json")))

CASES = [
    # dim, n, bc, theta
    (2, (64, 64), (1, 1), 0.0),
    (2, (128, 64), (0, 1), 10.0),
    (2, (64, 64), (0, 0), 0.0),
    (3, (32, 32, 32), (1, 1, 1), 100.0),
    (3, (32, 16, 32), (0, 1, 0), 0.0),
    (3, (32, 32, 32), (0, 0, 0), 0.0),
]


def _ctx(dim, n, bc, theta, precision):
    krylov = W.FGMRES if precision == W.MG_FP32 else W.GMRES_LEFT
    p, lay = params(dim, n, bc, theta, precision=precision, krylov=krylov)
    rho, mu = W.random_coefficients(31, lay, mu_range=(0.1, 10.0))
    g, _ = pair(p, rho, mu)
    o = oracle.Oracle(rho=rho, mu=mu, **dict(p, precision=W.FP64, krylov=W.GMRES_LEFT))
    return g, o, lay


@pytest.mark.parametrize("precision", [W.FP64, W.MG_FP32])
@pytest.mark.parametrize("dim,n,bc,theta", CASES)
def test_vel_mg_solve_parity(dim, n, bc, theta, precision):
    print(f"vel mg solve {dim}D n={n} bc={bc} theta={theta} precision={precision}", flush=True)
    g, o, lay = _ctx(dim, n, bc, theta, precision)
    r = W.random_velocity(32, lay)
    e, cyc, q, rc = g.vel_mg_solve(T(r), tol=1e-10, max_cycles=300)
    oe, ocyc, oq, orc = o.vel_mg_solve(r, tol=1e-10, max_cycles=300)
    print(f"  gpu {cyc} cycles rel {q:.2e}; oracle {ocyc} cycles rel {oq:.2e}", flush=True)
    assert rc == orc == oracle.ORC_OK and q <= 1e-10
    if precision == W.FP64:
        assert abs(cyc - ocyc) <= 1
        assert rel(N(e), oe) <= 1e-9
    else:
        assert cyc <= ocyc + 3
        assert rel(N(e), oe) <= 1e-8


@pytest.mark.parametrize("precision", [W.FP64, W.MG_FP32])
@pytest.mark.parametrize("dim,n,bc,theta", CASES)
def test_p_mg_solve_parity(dim, n, bc, theta, precision):
    print(f"p mg solve {dim}D n={n} bc={bc} precision={precision}", flush=True)
    g, o, lay = _ctx(dim, n, bc, theta, precision)
    r = W.random_cells(33, lay, remove_mean=True)
    e, cyc, q, rc = g.p_mg_solve(T(r), tol=1e-10, max_cycles=300)
    oe, ocyc, oq, orc = o.p_mg_solve(r, tol=1e-10, max_cycles=300)
    print(f"  gpu {cyc} cycles rel {q:.2e}; oracle {ocyc} cycles rel {oq:.2e}", flush=True)
    assert rc == orc == oracle.ORC_OK and q <= 1e-10
    assert abs(float(N(e).mean())) <= 1e-12 * float(np.abs(N(e)).max())
    if precision == W.FP64:
        assert abs(cyc - ocyc) <= 1
        assert rel(N(e), oe) <= 1e-9
    else:
        assert cyc <= ocyc + 3
        assert rel(N(e), oe) <= 1e-8


def test_mg_solve_limits():
    g, o, lay = _ctx(2, (64, 64), (1, 1), 1.0, W.FP64)
    r = W.random_velocity(34, lay)
    _, cyc, q, rc = g.vel_mg_solve(T(r), tol=1e-14, max_cycles=2)
    assert rc == oracle.ORC_ENOCONV and cyc == 2 and q > 1e-14
    e, cyc, q, rc = g.vel_mg_solve(T(np.zeros(lay.nvel)), tol=1e-8)
    assert rc == 0 and cyc == 0 and not bool(e.any())


def test_vel_mg_solve_full_size_layers():
    """128^3 no-slip layers (contrast 1e4 in mu): the GPU solution's residual,
    evaluated with the oracle's own operator, meets the tolerance."""
    print("vel mg solve 128^3 layers", flush=True)
    w = W.layers_3d()
    for prec in (W.FP64, W.MG_FP32):
        p = w.params(precision=prec, krylov=W.FGMRES if prec == W.MG_FP32 else W.GMRES_LEFT)
        g, o = pair(p, w.rho, w.mu)
        e, cyc, q, rc = g.vel_mg_solve(T(w.bu), tol=1e-8, max_cycles=300)
        yu, _ = o.apply(N(e), np.zeros(w.layout.ncell))
        true = np.linalg.norm(w.bu - yu) / np.linalg.norm(w.bu)
        print(f"  precision {prec}: {cyc} cycles, reported {q:.2e}, oracle-checked {true:.2e}",
              flush=True)
        assert rc == 0 and true <= 1e-8 * (1 + 1e-6)


@pytest.mark.parametrize("precision", [W.FP64, W.MG_FP32])
def test_coupled_costs_at_most_three_split_solves_64(precision):
    gold = GOLD["coupled_vs_split"]
    w = W.bubble(3, 64, 100.0, 100.0)
    krylov = W.FGMRES if precision == W.MG_FP32 else W.GMRES_LEFT
    p = w.params(precision=precision, krylov=krylov, restart=30)
    g, o = pair(p, w.rho, w.mu)
    bu, bp = o.apply(w.extra["x_u"], w.extra["x_p"])
    bp = bp - bp.mean()
    _, _, st, rc = g.solve(T(bu), T(bp), tol=1e-8, max_iter=500)
    assert rc == 0
    us, cv, _, rc1 = g.vel_mg_solve(T(bu), tol=1e-8, max_cycles=500)
    _, mdu = g.apply(us, T(np.zeros(w.layout.ncell)))  # pressure part of M [u*; 0] is -D u*
    _, cp, _, rc2 = g.p_mg_solve(mdu - T(bp), tol=1e-8, max_cycles=500)
    assert rc1 == rc2 == 0
    split = 3 * cv + cp
    ratio = st["scalar_vcycles"] / split
    print(f"64^3 bubble precision {precision}: coupled {st['scalar_vcycles']} split {split} "
          f"ratio {ratio:.2f}", flush=True)
    assert gold["min_ratio_scalar_vcycles"] <= ratio <= gold["max_ratio_scalar_vcycles"]


@pytest.mark.parametrize("dim,n", [(2, (512, 512)), (3, (128, 128, 128))])
@pytest.mark.parametrize("precision", [W.FP64, W.MG_FP32])
def test_vcycle_contraction_at_box_sizes(dim, n, precision):
    """Constant-coefficient steady no-slip subproblems at 512^2 and 128^3: the
    velocity V-cycle contracts the residual by at least 1/0.105 (2D) / 1/0.15
    (3D) per cycle and the pressure V-cycle by at least tenfold (the same
    bounds the oracle is pinned to at 128^2 / 32^3), so the stand-alone
    multigrid reaches 1e-10 within ceil(log(1e-10) / log(rate)) + 1 cycles."""
    import math

    rate = {2: 0.105, 3: 0.15}[dim]
    krylov = W.FGMRES if precision == W.MG_FP32 else W.GMRES_LEFT
    p, lay = params(dim, n, (1,) * dim, 0.0, precision=precision, krylov=krylov)
    g, _ = pair(p, np.ones(lay.ncell), np.ones(lay.ncell))
    _, cv, qv, rcv = g.vel_mg_solve(T(W.random_velocity(35, lay)), tol=1e-10, max_cycles=100)
    _, cp, qp, rcp = g.p_mg_solve(T(W.random_cells(36, lay, remove_mean=True)), tol=1e-10,
                                  max_cycles=100)
    print(f"{dim}D {n} precision={precision}: velocity {cv} cycles, pressure {cp} cycles",
          flush=True)
    assert rcv == rcp == 0
    assert cv <= math.ceil(math.log(1e-10) / math.log(rate)) + 1
    assert cp <= 11
