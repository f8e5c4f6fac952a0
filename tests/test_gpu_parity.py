"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
identical seeded inputs.  Sizes span several workgroups with ragged tails
(non-power-of-two axes), both boundary conditions, 2D and 3D, and the
degenerate 2-cell grid.

Bars (norm-wise over the stored arrays, whose wall entries are 0 on both
sides):
  - FP64 operator applies and gradient contractions: 1e-12 relative;
  - FP64 V-cycles and preconditioners (composites of ~10^2 stencil passes whose
    FP64 rounding differs only in operation order and fused multiply-adds):
    1e-11 relative;
  - FP32 preconditioner against the FP64 oracle: 1e-4 relative (FP32 unit
    roundoff 6e-8 amplified by the V-cycle's condition);
  - solves: iteration counts within +-1 of the oracle, true residual of the
    rescaled system <= tol checked with the oracle's own M;
  - adjoint gradients: 1e-6 relative of the oracle's FP64 adjoint.
"""
import numpy as np
import pytest

import oracle
from gpu_common import N, T, pair, params, rel, scaled_residual
from paper_1308_4605_amd import workloads as W

pytestmark = pytest.mark.gpu

OPS = [
    (2, (32, 32), (0, 0)), (2, (48, 32), (1, 1)), (2, (192, 64), (0, 1)), (2, (2, 2), (1, 1)),
    (3, (16, 16, 16), (1, 1, 1)), (3, (16, 16, 16), (0, 0, 0)), (3, (48, 40, 8), (1, 0, 1)),
    (3, (32, 48, 16), (0, 1, 0)), (3, (24, 16, 16), (1, 1, 1)), (3, (2, 2, 2), (0, 0, 0)),
    # free-slip walls (2), alone and mixed
    (2, (48, 32), (2, 2)), (2, (64, 32), (0, 2)), (3, (16, 16, 16), (2, 2, 2)),
    (3, (48, 40, 8), (2, 0, 1)), (3, (32, 16, 16), (2, 1, 0)),
    # one axis with different walls: 3 = no-slip low / free-slip high, 4 = the reverse
    (2, (64, 32), (0, 3)), (2, (48, 32), (4, 1)), (3, (32, 16, 16), (4, 0, 3)),
    (3, (16, 16, 16), (3, 4, 2)),
    # rows of >= 128 colour positions (two faces per thread), full and partial chunks
    (2, (320, 64), (0, 1)), (2, (256, 32), (1, 0)), (3, (256, 16, 16), (1, 0, 2)),
]


def _coefs(lay, seed=1):
    return W.random_coefficients(seed, lay, mu_range=(0.2, 5.0), rho_range=(0.5, 2.0))


@pytest.mark.parametrize("dim,n,bc", OPS)
@pytest.mark.parametrize("edge_avg", [W.EDGE_ARITH, W.EDGE_HARMONIC, W.EDGE_GIVEN])
def test_apply_parity(dim, n, bc, edge_avg):
    print(f"apply {dim} {n} {bc} edge={edge_avg}", flush=True)
    p, lay = params(dim, n, bc, 30.0, edge_avg=edge_avg)
    rho, mu = _coefs(lay)
    edges = np.random.default_rng(3).uniform(0.3, 3.0, lay.nedge) if edge_avg == W.EDGE_GIVEN else None
    g, o = pair(p, rho, mu, edges)
    xu = W.random_velocity(5, lay)
    xp = W.random_cells(6, lay)
    # wall entries of the input are ignored (read as 0)
    xu_dirty = xu.copy()
    xu_dirty[lay.wall_mask()] = 7.0
    yu, yp = g.apply(T(xu_dirty), T(xp))
    ou, op = o.apply(xu, xp)
    assert rel(N(yu), ou) <= 1e-12
    assert rel(N(yp), op) <= 1e-12
    assert np.all(N(yu)[lay.wall_mask()] == 0.0)


@pytest.mark.parametrize("dim,n,bc", OPS)
@pytest.mark.parametrize("theta", [0.0, 40.0])
def test_subsolver_parity(dim, n, bc, theta):
    print(f"subsolve {dim} {n} {bc} theta={theta}", flush=True)
    p, lay = params(dim, n, bc, theta)
    rho, mu = _coefs(lay, 2)
    g, o = pair(p, rho, mu)
    r = W.random_velocity(7, lay, remove_mean=lay.singular_components(theta))
    e = N(g.vel_subsolve(T(r)))
    assert rel(e, o.vel_subsolve(r)) <= 1e-11
    q = W.random_cells(8, lay, remove_mean=True)
    assert rel(N(g.p_subsolve(T(q))), o.p_subsolve(q)) <= 1e-11


@pytest.mark.parametrize("dim,n,bc,theta", [(2, (48, 32), (1, 1), 25.0), (3, (16, 16, 16), (0, 0, 0), 0.0),
                                            (3, (48, 40, 8), (1, 0, 1), 100.0), (2, (32, 32), (0, 0), 0.0),
                                            (2, (48, 32), (2, 2), 0.0), (3, (32, 16, 16), (2, 0, 2), 0.0),
                                            (3, (16, 16, 16), (2, 1, 2), 40.0),
                                            (2, (64, 32), (0, 3), 0.0),
                                            (3, (32, 16, 16), (4, 0, 3), 20.0)])
@pytest.mark.parametrize("precond", [W.P1, W.P2, W.P3, W.P4, W.P5])
def test_precond_parity(dim, n, bc, theta, precond):
    print(f"precond P{precond} {dim} {n} {bc} theta={theta}", flush=True)
    p, lay = params(dim, n, bc, theta, precond=precond)
    rho, mu = _coefs(lay, 3)
    g, o = pair(p, rho, mu)
    bu = W.random_velocity(9, lay, remove_mean=lay.singular_components(theta))
    bp = W.random_cells(10, lay, remove_mean=True)
    zu, zp = g.precond(T(bu), T(bp))
    ou, op = o.precond(bu, bp)
    assert rel(N(zu), ou) <= 1e-11
    assert rel(N(zp), op) <= 1e-11


SOLVES = [
    # (name, workload builder at reduced size, overrides)
    ("periodic-smooth-32", lambda: W.periodic_smooth_2d(n=32), {}),
    ("discs-128-c100", lambda: W.discs_2d(n=128, mu_in=1e2), {}),
    ("layers-32", lambda: W.layers_3d(n=32, precision=W.FP64), dict(krylov=W.GMRES_LEFT)),
    ("contrast-32", lambda: W.contrast_periodic_3d(n=32, contrast=1e3, precision=W.FP64), {}),
    ("adjoint-cfg-32", lambda: W.adjoint_3d(n=32), {}),
]


@pytest.mark.parametrize("name,mk,over", SOLVES, ids=[s[0] for s in SOLVES])
@pytest.mark.parametrize("krylov", [W.GMRES_LEFT, W.FGMRES])
def test_solve_parity_fp64(name, mk, over, krylov):
    print(f"solve {name} krylov={krylov}", flush=True)
    w = mk()
    p = w.params(**over)
    p.update(krylov=krylov, precision=W.FP64)
    g, o = pair(p, w.rho, w.mu)
    xu, xp, st, rc = g.solve(T(w.bu), T(w.bp), tol=1e-8, max_iter=500)
    ou, op, ost, orc = o.solve(w.bu, w.bp, tol=1e-8, max_iter=500)
    print(f"  gpu iters {st['iters']} oracle iters {ost['iters']}", flush=True)
    assert abs(st["iters"] - ost["iters"]) <= 1
    assert scaled_residual(o, o.c, w.bu, w.bp, N(xu), N(xp)) <= 1e-8 * (1 + 1e-6)
    assert rel(N(xu), ou) <= 1e-5
    assert rel(N(xp), op) <= 1e-5


@pytest.mark.parametrize("name,mk,over", SOLVES[:4], ids=[s[0] for s in SOLVES[:4]])
def test_mixed_precision_solve(name, mk, over):
    """FP32 multigrid inside FP64 FGMRES reaches the FP64 tolerance; error
    against the FP64 oracle and the iteration penalty are printed."""
    print(f"mixed {name}", flush=True)
    w = mk()
    p = w.params(**over)
    p.update(krylov=W.FGMRES, precision=W.MG_FP32)
    g, o = pair(p, w.rho, w.mu)
    # preconditioner itself: FP32 against the FP64 oracle
    bu = W.random_velocity(11, w.layout, remove_mean=w.layout.singular_components(w.theta))
    bp = W.random_cells(12, w.layout, remove_mean=True)
    zu, zp = g.precond(T(bu), T(bp))
    ou, op = o.precond(bu, bp)
    assert rel(N(zu), ou) <= 1e-4 and rel(N(zp), op) <= 1e-4
    xu, xp, st, rc = g.solve(T(w.bu), T(w.bp), tol=1e-8, max_iter=500)
    po = dict(p, precision=W.FP64)
    o64 = oracle.Oracle(rho=w.rho, mu=w.mu, **po)
    ou, op, ost, orc = o64.solve(w.bu, w.bp, tol=1e-8, max_iter=500)
    err_u, err_p = rel(N(xu), ou), rel(N(xp), op)
    print(f"  fp32-mg iters {st['iters']} fp64 oracle iters {ost['iters']} err_u {err_u:.2e} "
          f"err_p {err_p:.2e}", flush=True)
    assert scaled_residual(o64, o64.c, w.bu, w.bp, N(xu), N(xp)) <= 1e-8 * (1 + 1e-6)
    assert st["iters"] <= ost["iters"] + 3
    assert err_u <= 1e-5 and err_p <= 1e-5


@pytest.mark.parametrize("dim,n,bc,theta", [(2, (32, 32), (1, 1), 100.0), (3, (16, 16, 16), (1, 1, 1), 100.0),
                                            (2, (32, 32), (0, 0), 0.0), (3, (16, 16, 16), (0, 1, 0), 10.0),
                                            (2, (32, 32), (2, 2), 0.0), (3, (16, 16, 16), (2, 0, 1), 10.0)])
@pytest.mark.parametrize("edge_avg", [W.EDGE_ARITH, W.EDGE_HARMONIC])
def test_grad_contraction_parity(dim, n, bc, theta, edge_avg):
    print(f"grad {dim} {n} {bc}", flush=True)
    p, lay = params(dim, n, bc, theta, edge_avg=edge_avg)
    rho, mu = _coefs(lay, 4)
    g, o = pair(p, rho, mu)
    u = W.random_velocity(13, lay)
    lam = W.random_velocity(14, lay)
    gg = g.grad(T(u), T(lam))
    og = o.grad(u, lam)
    for k in ("dmu_cell", "dmu_edge", "drho_cell"):
        assert rel(N(gg[k]), og[k]) <= 1e-12, k


@pytest.mark.parametrize("precision,krylov", [(W.FP64, W.GMRES_LEFT), (W.MG_FP32, W.FGMRES)])
def test_adjoint_parity(precision, krylov):
    """Adjoint solve + strain contraction: within 1e-6 of the oracle's FP64
    adjoint (both solved to 1e-12)."""
    w = W.adjoint_3d(n=16)
    p = w.params(precision=precision, krylov=krylov)
    g, o = pair(p, w.rho, w.mu)
    xu, xp, st, rc = g.solve(T(w.bu), T(w.bp), tol=1e-12, max_iter=1000)
    ou, op, ost, orc = oracle.Oracle(rho=w.rho, mu=w.mu, **dict(p, precision=W.FP64)).solve(
        w.bu, w.bp, tol=1e-12, max_iter=1000)
    target = 0.5 * ou
    gu = ou - target
    gp = np.zeros(w.layout.ncell)
    ga = g.adjoint(xu, xp, T(N(xu) - target), T(gp), tol=1e-12, max_iter=1000)
    oa = oracle.Oracle(rho=w.rho, mu=w.mu, **dict(p, precision=W.FP64, krylov=W.GMRES_LEFT)).adjoint(
        ou, op, gu, gp, tol=1e-12, max_iter=1000)
    for k in ("lu", "dmu_cell", "dmu_edge", "drho_cell"):
        r = rel(N(ga[k]), oa[k])
        print(f"  {k} rel {r:.2e}", flush=True)
        assert r <= 1e-6, k


def test_error_paths():
    from paper_1308_4605_amd.stokes import Stokes, StokesError, STOKES_EINCOMPAT, STOKES_ENOCONV, STOKES_EINVAL

    p, lay = params(2, (32, 32), (1, 1), 0.0)
    rho, mu = _coefs(lay, 5)
    g, o = pair(p, rho, mu)
    bp = np.ones(lay.ncell)
    with pytest.raises(StokesError) as e:
        g.solve(T(np.zeros(lay.nvel)), T(bp))
    assert e.value.code == STOKES_EINCOMPAT
    xu, xp, st, rc = g.solve(T(W.random_velocity(1, lay)), T(np.zeros(lay.ncell)), tol=1e-14,
                             max_iter=3, check=False)
    assert rc == STOKES_ENOCONV and st["iters"] == 3
    bad = rho.copy()
    bad[5] = -1.0
    with pytest.raises(StokesError) as e:
        Stokes(p, T(bad), T(mu))
    assert e.value.code == STOKES_EINVAL
    # zero right-hand side: zero solution, no iterations
    xu, xp, st, rc = g.solve(T(np.zeros(lay.nvel)), T(np.zeros(lay.ncell)))
    assert rc == 0 and st["iters"] == 0 and np.all(N(xu) == 0)


FREESLIP = [
    # dim, n, bc, theta
    (2, (64, 64), (2, 2), 0.0),
    (3, (32, 32, 32), (2, 0, 2), 0.0),
    (3, (32, 32, 32), (2, 2, 1), 10.0),
    (2, (64, 64), (0, 3), 0.0),
    (3, (32, 32, 32), (0, 4, 0), 0.0),
]


@pytest.mark.parametrize("dim,n,bc,theta", FREESLIP)
@pytest.mark.parametrize("precond", [W.P1, W.P2])
@pytest.mark.parametrize("precision,krylov", [(W.FP64, W.GMRES_LEFT), (W.FP64, W.FGMRES),
                                              (W.MG_FP32, W.FGMRES)])
def test_solve_parity_freeslip(dim, n, bc, theta, precond, precision, krylov):
    """Free-slip walls (zero normal velocity, no tangential momentum flux),
    variable coefficients, b = M x for a seeded x (Sec. "Results" protocol)."""
    print(f"free-slip solve {dim} {n} {bc} theta={theta} P{precond} prec={precision} kry={krylov}",
          flush=True)
    p, lay = params(dim, n, bc, theta, precond=precond, precision=precision, krylov=krylov)
    rho, mu = W.random_coefficients(41, lay, mu_range=(0.2, 5.0), rho_range=(0.5, 2.0))
    g, _ = pair(p, rho, mu)
    o = oracle.Oracle(rho=rho, mu=mu, **dict(p, precision=W.FP64))
    xu0 = W.random_velocity(42, lay, remove_mean=lay.singular_components(theta))
    bu, bp = o.apply(xu0, W.random_cells(43, lay))
    bp = bp - bp.mean()
    xu, xp, st, rc = g.solve(T(bu), T(bp), tol=1e-9, max_iter=600)
    ou, op, ost, orc = o.solve(bu, bp, tol=1e-9, max_iter=600)
    print(f"  gpu iters {st['iters']} oracle iters {ost['iters']}", flush=True)
    assert rc == 0 and orc == 0
    if precision == W.FP64:
        assert abs(st["iters"] - ost["iters"]) <= 1
    assert scaled_residual(o, o.c, bu, bp, N(xu), N(xp)) <= 1e-9 * (1 + 1e-6)
    assert rel(N(xu), ou) <= 1e-6


LONG_ROWS = [
    # dim, n, bc, theta: rows of >= 128 faces (the finest velocity level of an FP32 hierarchy
    # is stored colour-split there), odd row lengths on x-walls, partial last waves
    (2, (256, 32), (1, 1), 0.0), (2, (320, 64), (0, 1), 25.0), (3, (128, 16, 16), (1, 0, 2), 10.0),
    (3, (256, 8, 8), (0, 0, 0), 0.0), (3, (128, 16, 16), (2, 1, 4), 0.0),
]


@pytest.mark.parametrize("dim,n,bc,theta", LONG_ROWS)
@pytest.mark.parametrize("precond", [W.P1, W.P2, W.P5])
def test_fp32_precond_parity_long_rows(dim, n, bc, theta, precond):
    """FP32 preconditioner and velocity subsolver against the FP64 oracle (1e-4) on grids
    whose finest velocity level runs in the colour-split storage order."""
    print(f"fp32 long rows P{precond} {dim} {n} {bc} theta={theta}", flush=True)
    p, lay = params(dim, n, bc, theta, precond=precond, precision=W.MG_FP32, krylov=W.FGMRES)
    rho, mu = _coefs(lay, 5)
    g, o = pair(p, rho, mu)
    bu = W.random_velocity(15, lay, remove_mean=lay.singular_components(theta))
    bp = W.random_cells(16, lay, remove_mean=True)
    zu, zp = g.precond(T(bu), T(bp))
    ou, op = o.precond(bu, bp)
    assert rel(N(zu), ou) <= 1e-4
    assert rel(N(zp), op) <= 1e-4
    assert np.all(N(zu)[lay.wall_mask()] == 0.0)
    assert rel(N(g.vel_subsolve(T(bu))), o.vel_subsolve(bu)) <= 1e-4


ODD_COARSE = [
    # wall axes may coarsen to an odd extent; here the coarsest level (129 x 2 x 2 = 516 cells,
    # 257 x 2 = 514 in 2D) is larger than the single-workgroup tail, so the grid kernels run on
    # it and clear the iterate with a fill instead of starting the sweep from uncleared memory
    (3, (516, 8, 8), (1, 0, 0), 0.0), (3, (516, 8, 8), (2, 1, 0), 10.0),
    (2, (1028, 8), (3, 0), 0.0), (2, (1028, 8), (1, 1), 25.0),
]


@pytest.mark.parametrize("dim,n,bc,theta", ODD_COARSE)
@pytest.mark.parametrize("precision", [W.FP64, W.MG_FP32])
def test_precond_parity_odd_coarse_level(dim, n, bc, theta, precision):
    """Preconditioner against the oracle on grids whose coarsest level has an odd extent and
    runs outside the coarse tail (FP64 1e-11, FP32 multigrid 1e-4)."""
    print(f"odd coarse {dim} {n} {bc} theta={theta} prec={precision}", flush=True)
    kry = W.FGMRES if precision == W.MG_FP32 else W.GMRES_LEFT
    p, lay = params(dim, n, bc, theta, precond=W.P1, precision=precision, krylov=kry)
    rho, mu = _coefs(lay, 7)
    g, o = pair(p, rho, mu)
    bu = W.random_velocity(17, lay, remove_mean=lay.singular_components(theta))
    bp = W.random_cells(18, lay, remove_mean=True)
    zu, zp = g.precond(T(bu), T(bp))
    ou, op = o.precond(bu, bp)
    tol = 1e-11 if precision == W.FP64 else 1e-4
    assert rel(N(zu), ou) <= tol
    assert rel(N(zp), op) <= tol
    assert np.all(N(zu)[lay.wall_mask()] == 0.0)


@pytest.mark.parametrize("krylov", [W.GMRES_LEFT, W.FGMRES])
@pytest.mark.parametrize("restart", [16, 32])
def test_solve_parity_long_restart(krylov, restart):
    """Restart lengths beyond 12 (the GPU Arnoldi then keeps its basis
    transform in device memory instead of the kernel arguments)."""
    print(f"long restart {restart} krylov={krylov}", flush=True)
    w = W.contrast_periodic_3d(n=32, contrast=1e3, precision=W.FP64)
    p = w.params(krylov=krylov, precision=W.FP64, restart=restart)
    g, o = pair(p, w.rho, w.mu)
    xu, xp, st, rc = g.solve(T(w.bu), T(w.bp), tol=1e-8, max_iter=500)
    ou, op, ost, orc = o.solve(w.bu, w.bp, tol=1e-8, max_iter=500)
    print(f"  gpu iters {st['iters']} oracle iters {ost['iters']}", flush=True)
    assert rc == 0 and orc == 0
    assert abs(st["iters"] - ost["iters"]) <= 1
    assert rel(N(xu), ou) <= 1e-5 and rel(N(xp), op) <= 1e-5
