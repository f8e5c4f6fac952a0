"""The oracle's stand-alone multigrid solvers (the velocity and pressure
V-cycle run to convergence, Sec. "The effect of the number of multigrid cycles") pinned against dense direct solves of
the operators assembled from the oracle's own M by unit vectors, against the
V-cycle contraction bounds, and against the paper's statement that the coupled
solver costs at most 2-3 times the scalar V-cycles of a split (projection)
solve (tests/golden/paper_claims.json)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from mac_helpers import assemble, interior_index
from paper_1308_4605_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_claims.json")))


def _params(dim, n, bc, theta, **kw):
    lay = W.make_layout(dim, n, bc)
    p = dict(dim=dim, n=lay.n, bc=lay.bc, h=1.0 / lay.n[0], theta=theta, precond=W.P1,
             precision=W.FP64, krylov=W.GMRES_LEFT, restart=10, nu_pre=2, nu_post=2, nu_coarse=8,
             vcycles=1, rescale_c=0.0, edge_avg=W.EDGE_ARITH)
    p.update(kw)
    return p, lay


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dim,n,bc,theta", [(2, (16, 16), (1, 1), 1.0), (2, (16, 8), (0, 1), 10.0),
                                            (3, (8, 8, 8), (0, 0, 0), 100.0),
                                            (3, (8, 8, 8), (1, 0, 1), 0.0)])
def test_vel_mg_solve_matches_dense_solve(dim, n, bc, theta):
    p, lay = _params(dim, n, bc, theta)
    rho, mu = W.random_coefficients(21, lay, mu_range=(0.1, 10.0))
    o = oracle.Oracle(rho=rho, mu=mu, **p)
    M, nv = assemble(o, lay)
    A = M[:nv, :nv]
    vel, _ = interior_index(lay)
    r = W.random_velocity(22, lay)
    x = np.linalg.solve(A, r[vel])
    e, cyc, rel, rc = o.vel_mg_solve(r, tol=1e-12, max_cycles=100)
    assert rc == oracle.ORC_OK and rel <= 1e-12 and cyc > 0
    assert _rel(e[vel], x) <= 1e-9
    assert np.all(e[lay.wall_mask()] == 0.0)
    # the reported residual is the true one
    assert np.linalg.norm(r[vel] - A @ e[vel]) / np.linalg.norm(r[vel]) == pytest.approx(rel, rel=1e-3)


@pytest.mark.parametrize("dim,n", [(2, (16, 16)), (3, (8, 8, 8))])
def test_vel_mg_solve_singular_periodic_steady(dim, n):
    """Periodic and theta = 0: A annihilates constant components; the solve
    returns the mean-free solution of the projected right-hand side."""
    p, lay = _params(dim, n, (0,) * dim, 0.0)
    rho, mu = W.random_coefficients(23, lay, mu_range=(0.1, 10.0))
    o = oracle.Oracle(rho=rho, mu=mu, **p)
    M, nv = assemble(o, lay)
    A = M[:nv, :nv]
    r = W.random_velocity(24, lay, remove_mean=True)
    x = np.linalg.lstsq(A, r, rcond=1e-12)[0]
    comps = np.split(x, dim)
    x = np.concatenate([c - c.mean() for c in comps])
    e, cyc, rel, rc = o.vel_mg_solve(r, tol=1e-12, max_cycles=200)
    assert rc == oracle.ORC_OK
    assert max(abs(c.mean()) for c in np.split(e, dim)) <= 1e-12 * np.abs(e).max()
    assert _rel(e, x) <= 1e-8


@pytest.mark.parametrize("dim,n,bc", [(2, (16, 16), (0, 0)), (2, (16, 16), (1, 1)),
                                      (3, (8, 8, 8), (1, 1, 0))])
def test_p_mg_solve_matches_dense_solve(dim, n, bc):
    """rho = 1: L_rho = D G with D = -M_pu and G = M_up taken from the
    assembled M; the solution is the mean-free one."""
    p, lay = _params(dim, n, bc, 1.0)
    _, mu = W.random_coefficients(25, lay, mu_range=(0.5, 2.0))
    o = oracle.Oracle(rho=np.ones(lay.ncell), mu=mu, **p)
    M, nv = assemble(o, lay)
    G = M[:nv, nv:]
    D = -M[nv:, :nv]
    L = D @ G
    r = W.random_cells(26, lay, remove_mean=True)
    x = np.linalg.lstsq(L, r, rcond=1e-12)[0]
    x -= x.mean()
    e, cyc, rel, rc = o.p_mg_solve(r, tol=1e-12, max_cycles=100)
    assert rc == oracle.ORC_OK and rel <= 1e-12
    assert abs(e.mean()) <= 1e-12 * np.abs(e).max()
    assert _rel(e, x) <= 1e-9


@pytest.mark.parametrize("dim", [2, 3])
def test_mg_solve_cycles_follow_vcycle_contraction(dim):
    """Constant-coefficient no-slip stress form: the V-cycle contracts by less
    than 0.105 (2D) / 0.15 (3D) per cycle (pinned in test_oracle_solvers), so
    reaching 1e-10 takes at most ceil(log(1e-10) / log(rate)) + 1 cycles."""
    rate = {2: 0.105, 3: 0.15}[dim]
    n = (64, 64) if dim == 2 else (16, 16, 16)
    p, lay = _params(dim, n, (1,) * dim, 0.0)
    o = oracle.Oracle(rho=np.ones(lay.ncell), mu=np.ones(lay.ncell), **p)
    r = W.random_velocity(27, lay)
    _, cyc, rel, rc = o.vel_mg_solve(r, tol=1e-10, max_cycles=100)
    assert rc == oracle.ORC_OK
    assert cyc <= math.ceil(math.log(1e-10) / math.log(rate)) + 1, cyc
    _, cyc4, _, _ = o.vel_mg_solve(r, tol=1e-4, max_cycles=100)
    assert cyc4 < cyc


def test_mg_solve_limits_and_errors():
    p, lay = _params(2, (16, 16), (1, 1), 1.0)
    rho, mu = W.random_coefficients(28, lay)
    o = oracle.Oracle(rho=rho, mu=mu, **p)
    r = W.random_velocity(29, lay)
    e, cyc, rel, rc = o.vel_mg_solve(r, tol=1e-14, max_cycles=2)
    assert rc == oracle.ORC_ENOCONV and cyc == 2 and rel > 1e-14
    e, cyc, rel, rc = o.vel_mg_solve(np.zeros(lay.nvel), tol=1e-8)
    assert rc == oracle.ORC_OK and cyc == 0 and not e.any()
    with pytest.raises(oracle.OracleError):
        o.vel_mg_solve(r, tol=0.0)
    with pytest.raises(oracle.OracleError):
        o.p_mg_solve(W.random_cells(1, lay), tol=1e-8, max_cycles=-1)


def split_cost(o, w, bu, bp, tol):
    """Scalar V-cycles of one projection step with multigrid run to the
    tolerance: u* = A^{-1} b_u, then phi = L_rho^{-1} (-(D u* + b_p))."""
    us, cv, _, rc1 = o.vel_mg_solve(bu, tol=tol, max_cycles=500)
    _, mdu = o.apply(us, np.zeros(w.layout.ncell))  # pressure part of M [u*; 0] is -D u*
    _, cp, _, rc2 = o.p_mg_solve(mdu - bp, tol=tol, max_cycles=500)
    assert rc1 == rc2 == oracle.ORC_OK
    return w.dim * cv + cp


@pytest.mark.parametrize("dim,n,r", [(3, 32, 100.0), (3, 32, 2.0), (2, 128, 100.0), (2, 128, 2.0)])
def test_coupled_costs_at_most_three_split_solves(dim, n, r):
    g = GOLD["coupled_vs_split"]
    w = W.bubble(dim, n, r, r)
    o = oracle.Oracle.from_workload(w, restart=30)
    bu, bp = o.apply(w.extra["x_u"], w.extra["x_p"])
    bp = bp - bp.mean()
    _, _, st, rc = o.solve(bu, bp, tol=1e-8, max_iter=500)
    assert rc == oracle.ORC_OK
    split = split_cost(o, w, bu, bp, 1e-8)
    ratio = st["scalar_vcycles"] / split
    print(f"{dim}D n={n} contrast {r}: coupled {st['scalar_vcycles']} split {split} ratio {ratio:.2f}")
    assert g["min_ratio_scalar_vcycles"] <= ratio <= g["max_ratio_scalar_vcycles"]
