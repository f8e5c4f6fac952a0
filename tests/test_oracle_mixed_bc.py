"""Walls of one axis with different conditions (Sec. "Staggered-grid Discretization": a condition is
specified at each domain boundary): no-slip at one end, free-slip at the
other.  Pinned by the open channel, whose discrete solution is known in
closed form (the shear stress falls linearly from zero at the free surface,
one-sided half-cell difference at the no-slip bed, given edge viscosities),
by manufactured solutions meeting both wall conditions at second order, and
by the boundary terms reading tangential wall data at the no-slip end only.
The operator pins (D = -G^T, D G, symmetry, the constant-viscosity identity
against a Kronecker Laplacian with one Dirichlet and one Neumann end, the
energy form) and the dense direct solves run on mixed grids in
test_oracle_operators.py and test_oracle_solvers.py."""
import numpy as np
import pytest

import oracle
from paper_1308_4605_amd import workloads as W


def _open_channel_exact(mu_e, h, f, bed_low):
    """x-velocity at the cell rows of a channel with a no-slip bed and a
    free-slip surface, driven by the uniform body force f along x.  Edge rows
    0..n carry mu_e; with the bed at edge row 0 the stress on edge row j is
    tau_j = f h (n - j) (zero at the surface), and u rises from the bed by
    tau h / mu per row (half a cell at the bed)."""
    n = len(mu_e) - 1
    if not bed_low:
        u = _open_channel_exact(mu_e[::-1], h, f, True)
        return u[::-1]
    tau = f * h * (n - np.arange(n + 1))
    u = np.empty(n)
    u[0] = tau[0] * h / (2 * mu_e[0])
    for j in range(1, n):
        u[j] = u[j - 1] + tau[j] * h / mu_e[j]
    return u


@pytest.mark.parametrize("bc_y", [W.NOSLIP_FREESLIP, W.FREESLIP_NOSLIP])
@pytest.mark.parametrize("krylov", [W.GMRES_LEFT, W.FGMRES])
def test_open_channel_2d_exact(bc_y, krylov):
    n = (16, 32)
    lay = W.make_layout(2, n, (W.PERIODIC, bc_y))
    h = 1.0 / n[0]
    rng = np.random.default_rng(71)
    mu_nodes = rng.uniform(0.2, 5.0, n[1] + 1)
    edges = np.repeat(mu_nodes[:, None], n[0], axis=1).ravel()
    o = oracle.Oracle(2, lay.n, lay.bc, h, 0.0, np.ones(lay.ncell),
                      rng.uniform(0.2, 5.0, lay.ncell), edges=edges, edge_avg=W.EDGE_GIVEN,
                      precond=W.P2, krylov=krylov)
    f = 1.3
    bu = np.zeros(lay.nvel)
    lay.split_vel(bu)[0][...] = f
    xu, xp, st, rc = o.solve(bu, np.zeros(lay.ncell), tol=1e-13, max_iter=500)
    assert rc == oracle.ORC_OK
    ux, uy = lay.split_vel(xu)
    uex = _open_channel_exact(mu_nodes, h, f, bc_y == W.NOSLIP_FREESLIP)
    scale = np.abs(uex).max()
    assert np.abs(ux - uex[:, None]).max() <= 1e-10 * scale
    assert np.abs(uy).max() <= 1e-10 * scale


def test_open_channel_3d_exact():
    """Bed at the top of z (free-slip low, no-slip high), flow along y."""
    n = (8, 8, 16)
    lay = W.make_layout(3, n, (W.PERIODIC, W.PERIODIC, W.FREESLIP_NOSLIP))
    h = 1.0 / n[0]
    rng = np.random.default_rng(72)
    mu_z = rng.uniform(0.2, 5.0, n[2] + 1)
    edges = np.ones(lay.nedge)
    fam, o_ = {}, 0
    for m in lay.edge_families:
        c = int(np.prod(lay.edge_shape(m)))
        fam[m] = edges[o_:o_ + c].reshape(lay.edge_shape(m))
        o_ += c
    fam[0][...] = mu_z[:, None, None]   # x-parallel edges carry the y-z shear
    fam[1][...] = mu_z[:, None, None]
    o = oracle.Oracle(3, lay.n, lay.bc, h, 0.0, np.ones(lay.ncell), np.ones(lay.ncell),
                      edges=edges, edge_avg=W.EDGE_GIVEN, precond=W.P2)
    f = 0.7
    bu = np.zeros(lay.nvel)
    lay.split_vel(bu)[1][...] = f
    xu, xp, st, rc = o.solve(bu, np.zeros(lay.ncell), tol=1e-13, max_iter=500)
    assert rc == oracle.ORC_OK
    ux, uy, uz = lay.split_vel(xu)
    uex = _open_channel_exact(mu_z, h, f, False)
    scale = np.abs(uex).max()
    assert np.abs(uy - uex[:, None, None]).max() <= 1e-10 * scale
    assert max(np.abs(ux).max(), np.abs(uz).max()) <= 1e-10 * scale


def _mms_channel(dim, n, bc_y, theta):
    """Divergence-free flow, periodic along x (and z), zero velocity on the
    no-slip wall of y, zero normal velocity and zero normal derivative of the
    tangential velocity on the free-slip wall: psi-type fields with the
    profile g(s) = 3 s^2 - 5 s^3 + 2 s^4 (g = g' = 0 at s = 0, g = g'' = 0 at
    s = 1), s the distance from the no-slip wall."""
    import sympy as sp

    X = sp.symbols("x y z")[:dim]
    pi = sp.pi
    s = X[1] if bc_y == W.NOSLIP_FREESLIP else 1 - X[1]
    g = 3 * s ** 2 - 5 * s ** 3 + 2 * s ** 4
    gy = sp.diff(g, X[1])
    if dim == 2:
        u = [sp.sin(2 * pi * X[0]) * gy, -2 * pi * sp.cos(2 * pi * X[0]) * g]
    else:
        u = [sp.sin(2 * pi * X[0]) * gy,
             -2 * pi * (sp.cos(2 * pi * X[0]) + sp.cos(2 * pi * X[2])) * g,
             sp.sin(2 * pi * X[2]) * gy]
    assert sp.simplify(sum(sp.diff(u[k], X[k]) for k in range(dim))) == 0
    p = sp.sin(2 * pi * X[0]) * sp.cos(pi * X[1])
    mu = 1 + sp.Rational(1, 2) * sp.sin(2 * pi * X[0]) * X[1]
    rho = 1 + X[1] ** 2
    f = []
    for k in range(dim):
        dtau = sum(sp.diff(mu * (sp.diff(u[k], X[l]) + sp.diff(u[l], X[k])), X[l])
                   for l in range(dim))
        f.append(theta * rho * u[k] - dtau + sp.diff(p, X[k]))
    lam = lambda e: sp.lambdify(X, e, "numpy")
    bc = (W.PERIODIC, bc_y) + ((W.PERIODIC,) if dim == 3 else ())
    lay = W.make_layout(dim, (n,) * dim, bc)
    h = 1.0 / n
    cc = lay.cell_centres(h)
    cell = lambda e: np.broadcast_to(lam(e)(*cc), lay.cell_shape).ravel()
    bu, ue = [], []
    for k in range(dim):
        fc = lay.face_centres(k, h)
        bu.append(np.broadcast_to(lam(f[k])(*fc), lay.face_shape(k)).ravel())
        ue.append(np.broadcast_to(lam(u[k])(*fc), lay.face_shape(k)).ravel())
    bu, ue = np.concatenate(bu), np.concatenate(ue)
    wm = lay.wall_mask()
    bu[wm] = 0.0
    o = oracle.Oracle(dim, lay.n, lay.bc, h, theta, cell(rho), cell(mu), precond=W.P1)
    xu, xp, st, rc = o.solve(bu, np.zeros(lay.ncell), tol=1e-11, max_iter=3000)
    assert rc == oracle.ORC_OK
    eu = np.abs(xu - ue)[~wm].max()
    pe = cell(p)
    ep = np.sqrt(np.mean(((xp - xp.mean()) - (pe - pe.mean())) ** 2))
    return eu, ep


@pytest.mark.parametrize("dim,ns,bc_y,theta", [
    (2, (16, 32, 64), W.NOSLIP_FREESLIP, 0.0), (2, (32, 64, 128), W.FREESLIP_NOSLIP, 30.0),
    (3, (8, 16), W.NOSLIP_FREESLIP, 0.0)])
def test_mixed_walls_manufactured_second_order(dim, ns, bc_y, theta):
    errs = [_mms_channel(dim, n, bc_y, theta) for n in ns]
    for (eu0, ep0), (eu1, ep1) in zip(errs[:-1], errs[1:]):
        assert np.log2(eu0 / eu1) >= 1.8, errs
        assert np.log2(ep0 / ep1) >= 1.5, errs


def test_boundary_terms_read_the_no_slip_end_only():
    """Tangential wall data is read on the no-slip wall of an axis and
    ignored on its free-slip wall; a mixed axis gives, at each end, the
    boundary terms of the corresponding uniform axis."""
    lay = W.make_layout(2, (16, 16), (W.PERIODIC, W.NOSLIP_FREESLIP))
    h = 1.0 / 16
    rho, mu = W.random_coefficients(73, lay)
    mk = lambda bc: oracle.Oracle(2, lay.n, (0, bc), h, 4.0, rho, mu)
    om, on, of = mk(W.NOSLIP_FREESLIP), mk(W.NOSLIP), mk(W.FREESLIP)
    rng = np.random.default_rng(74)
    un = np.zeros(lay.nvel)
    ut = rng.standard_normal(lay.nedge)
    nodes = ut.reshape(lay.edge_shape(2))
    cm = om.boundary_rhs(un, ut)[0]
    cn = on.boundary_rhs(un, ut)[0]
    cf = of.boundary_rhs(un, ut)[0]
    ux = lambda c: lay.split_vel(c)[0]
    np.testing.assert_allclose(ux(cm)[0], ux(cn)[0], rtol=0, atol=1e-12)    # bed row: no-slip
    np.testing.assert_allclose(ux(cm)[-1], ux(cf)[-1], rtol=0, atol=1e-12)  # surface row
    assert not ux(cf).any()
    nodes[-1, :] += 5.0   # surface data changes nothing
    np.testing.assert_array_equal(om.boundary_rhs(un, ut)[0], cm)
