"""The oracle's smoothers (Appendix C: multicolour Gauss-Seidel, per sweep
red then black faces of x, then of y[, then of z] for the velocity, red then
black cells for the pressure) against the same sweeps written out on the
dense matrices assembled from M: phi_q += (r_q - (A phi)_q) / A_qq over the
faces of one colour of one component at a time.  This pins the smoother's
diagonal (wall weights per wall end, bulk term) and its ordering, neither of
which changes a converged solution."""
import numpy as np
import pytest

import oracle
from mac_helpers import assemble, interior_index
from paper_1308_4605_amd import workloads as W

GRIDS = [
    (2, (8, 8), (0, 0), False), (2, (8, 4), (1, 1), False), (2, (8, 8), (2, 0), False),
    (2, (8, 8), (0, 3), False), (2, (8, 8), (4, 1), True),
    (3, (4, 4, 4), (1, 1, 1), False), (3, (4, 4, 4), (3, 2, 0), True),
    (3, (4, 8, 4), (0, 4, 1), False),
]


def _face_keys(lay):
    """(component, parity of i0 + i1 + i2) of every stored velocity entry."""
    comp, par = [], []
    for k in range(lay.dim):
        shape = lay.face_shape(k)
        idx = np.indices(shape)  # numpy axes (z,) y, x
        comp.append(np.full(int(np.prod(shape)), k))
        par.append((sum(idx[a] for a in range(lay.dim)) % 2).ravel())
    return np.concatenate(comp), np.concatenate(par)


@pytest.mark.parametrize("dim,n,bc,bulk", GRIDS)
def test_velocity_sweep_is_dense_multicolour_gauss_seidel(dim, n, bc, bulk):
    lay = W.make_layout(dim, n, bc)
    h = 1.0 / lay.n[0]
    rho, mu = W.random_coefficients(81, lay)
    gamma = W.random_bulk_viscosity(82, lay) if bulk else None
    o = oracle.Oracle(dim, lay.n, lay.bc, h, 3.0, rho, mu, gamma=gamma)
    M, nv = assemble(o, lay)
    A = M[:nv, :nv]
    vel, _ = interior_index(lay)
    comp, par = _face_keys(lay)
    rhs = W.random_velocity(83, lay)
    phi0 = W.random_velocity(84, lay)
    x = phi0[vel].copy()
    b = rhs[vel]
    for k in range(dim):
        for colour in (0, 1):
            sel = np.nonzero((comp[vel] == k) & (par[vel] == colour))[0]
            r = b[sel] - A[sel] @ x
            x[sel] += r / np.diag(A)[sel]
    got = o.vel_sweep(rhs, phi0)
    expect = phi0.copy()
    expect[vel] = x
    assert np.abs(got - expect).max() <= 1e-12 * np.abs(expect).max()


@pytest.mark.parametrize("dim,n,bc,bulk", GRIDS)
def test_pressure_sweep_is_dense_red_black_gauss_seidel(dim, n, bc, bulk):
    lay = W.make_layout(dim, n, bc)
    h = 1.0 / lay.n[0]
    rho, mu = W.random_coefficients(85, lay)
    o1 = oracle.Oracle(dim, lay.n, lay.bc, h, 1.0, rho, mu)
    o0 = oracle.Oracle(dim, lay.n, lay.bc, h, 0.0, rho, mu)
    M1, nv = assemble(o1, lay)
    M0, _ = assemble(o0, lay)
    rho_f = np.diag(M1[:nv, :nv] - M0[:nv, :nv])   # theta = 1: the face densities
    G, mD = M1[:nv, nv:], M1[nv:, :nv]
    Lr = (-mD) @ np.diag(1.0 / rho_f) @ G          # L_rho = D rho_f^{-1} G
    par = (sum(np.indices(lay.cell_shape)[a] for a in range(dim)) % 2).ravel()
    rhs = W.random_cells(86, lay)
    phi0 = W.random_cells(87, lay)
    x = phi0.copy()
    for colour in (0, 1):
        sel = np.nonzero(par == colour)[0]
        x[sel] += (rhs[sel] - Lr[sel] @ x) / np.diag(Lr)[sel]
    got = o1.p_sweep(rhs, phi0)
    assert np.abs(got - x).max() <= 1e-12 * np.abs(x).max()
