"""Bulk viscosity (Sec. "Preconditioners": for div u = g != 0 the stress gains
(gamma - 2/3 mu)(div u) I; eq. Schur_app_bulk: the Schur approximation uses
gamma + 4/3 mu in place of 2 mu; Appendix A: the constant-coefficient symbol).
The oracle's bulk term is pinned by the grad-div operator it must reduce to
when mu = 0, by the Navier-Lame form of the constant-coefficient operator, by
the Fourier symbol, by the exactness of the Schur approximation, by symmetry
and definiteness, by manufactured compressible flows converging at second
order, and by finite differences of the bulk-viscosity gradient."""
import numpy as np
import pytest

import oracle
from mac_helpers import assemble, blocks, rel, textbook_vector_laplacian
from paper_1308_4605_amd import workloads as W

CASES = [
    (2, (8, 8), (0, 0)),
    (2, (8, 8), (1, 1)),
    (2, (8, 4), (0, 1)),
    (2, (8, 8), (2, 1)),
    (3, (4, 4, 4), (1, 1, 1)),
    (3, (4, 4, 4), (0, 0, 0)),
    (3, (4, 8, 4), (2, 0, 1)),
]


def _mk(dim, n, bc, theta, rho, mu, gamma, **kw):
    lay = W.make_layout(dim, n, bc)
    h = 1.0 / lay.n[0]
    return oracle.Oracle(dim, lay.n, lay.bc, h, theta, rho, mu, gamma=gamma, **kw), lay, h


@pytest.mark.parametrize("dim,n,bc", CASES)
def test_bulk_term_alone_is_grad_gamma_div(dim, n, bc):
    """mu = 0: the viscous operator is the gradient of gamma div u, so
    A = -G diag(gamma) D with the staggered G and D (pinned on their own as
    D = -G^T and D G = textbook Laplacian)."""
    lay = W.make_layout(dim, n, bc)
    gamma = W.random_bulk_viscosity(1, lay, (0.5, 3.0))
    o, lay, h = _mk(dim, n, bc, 0.0, np.ones(lay.ncell), np.zeros(lay.ncell), gamma)
    M, nv = assemble(o, lay)
    A, G, mD, _ = blocks(M, nv)
    np.testing.assert_allclose(A, -G @ np.diag(gamma) @ (-mD), rtol=0, atol=1e-12 / h ** 2)


@pytest.mark.parametrize("dim,n,bc", CASES)
def test_constant_coefficient_navier_lame_form(dim, n, bc):
    """Constant mu0, gamma0: div tau = mu0 lap u + (mu0/3 + gamma0) grad div u
    (the Navier-Lame form of the compressible viscous term), discretely
    mu0 L + (mu0/3 + gamma0) G D with L the textbook Laplace-form vector
    Laplacian and its wall rules.  Pins the -2/3 coefficient."""
    mu0, g0 = 1.3, 0.45
    lay = W.make_layout(dim, n, bc)
    o, lay, h = _mk(dim, n, bc, 0.0, np.ones(lay.ncell), np.full(lay.ncell, mu0),
                    np.full(lay.ncell, g0))
    M, nv = assemble(o, lay)
    A, G, mD, _ = blocks(M, nv)
    L = textbook_vector_laplacian(lay, h)
    np.testing.assert_allclose(-A, mu0 * L + (mu0 / 3.0 + g0) * G @ (-mD), rtol=0,
                               atol=1e-11 * (mu0 + g0) / h ** 2)


@pytest.mark.parametrize("dim,n,bc", CASES)
def test_bulk_operator_symmetric_and_semidefinite(dim, n, bc):
    """M = M^T for variable rho, mu, gamma; -L_mu stays positive semidefinite
    for gamma >= 0 (gamma = 0 included: 2 |e|^2 - 2/3 (tr e)^2 >= 0 for d <= 3).
    A per-cell mistake in the bulk term (wrong cell, wrong sign) breaks one of
    the two."""
    lay = W.make_layout(dim, n, bc)
    rho, mu = W.random_coefficients(3, lay)
    for gamma in (W.random_bulk_viscosity(4, lay), np.zeros(lay.ncell)):
        o, lay, h = _mk(dim, n, bc, 2.0, rho, mu, gamma)
        M, nv = assemble(o, lay)
        assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
        o0, *_ = _mk(dim, n, bc, 0.0, rho, mu, gamma)
        M0, _ = assemble(o0, lay)
        ev = np.linalg.eigvalsh(M0[:nv, :nv])
        assert ev.min() >= -1e-10 * ev.max()


@pytest.mark.parametrize("dim,mode", [(2, (1, 2)), (2, (3, 0)), (3, (1, 2, 1))])
def test_periodic_bulk_operator_matches_fourier_symbol(dim, mode):
    """Constant coefficients, periodic: the viscous symbol is
    (4/3 mu0 + gamma0) G_k D_k + mu0 sum_{l != k} G_l D_l on the diagonal and
    (mu0/3 + gamma0) G_k D_l off it (Appendix A, bulk-viscosity case)."""
    n, h = 8, 1.0 / 8
    theta, rho0, mu0, g0 = 3.0, 1.1, 0.7, 0.4
    lay = W.make_layout(dim, (n,) * dim, (0,) * dim)
    o, lay, h = _mk(dim, lay.n, lay.bc, theta, np.full(lay.ncell, rho0),
                    np.full(lay.ncell, mu0), np.full(lay.ncell, g0))
    kap = [2 * np.pi * mode[a] / n for a in range(dim)]
    Dh = np.array([(np.exp(1j * kap[a]) - 1) / h for a in range(dim)])
    Gh = np.array([(1 - np.exp(-1j * kap[a])) / h for a in range(dim)])
    Lm = np.zeros((dim, dim), complex)
    for k in range(dim):
        for l in range(dim):
            if k == l:
                Lm[k, k] = (4 * mu0 / 3 + g0) * Gh[k] * Dh[k] + mu0 * sum(
                    Gh[b] * Dh[b] for b in range(dim) if b != k)
            else:
                Lm[k, l] = (mu0 / 3 + g0) * Gh[k] * Dh[l]
    Ms = np.zeros((dim + 1, dim + 1), complex)
    Ms[:dim, :dim] = theta * rho0 * np.eye(dim) - Lm
    Ms[:dim, dim] = Gh
    Ms[dim, :dim] = -Dh
    rng = np.random.default_rng(12)
    amp = rng.standard_normal(dim + 1) + 1j * rng.standard_normal(dim + 1)

    def wave(dims):
        axes = [np.arange(dims[a]) for a in range(dim)]
        grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
        return np.exp(1j * sum(kap[a] * grids[a] for a in range(dim))).ravel()

    xu = np.concatenate([amp[k] * wave(lay.face_dims(k)) for k in range(dim)])
    xp = amp[dim] * wave(lay.n)
    y = np.concatenate(o.apply(xu.real, xp.real)) + 1j * np.concatenate(o.apply(xu.imag, xp.imag))
    out = Ms @ amp
    expect = np.concatenate([out[k] * wave(lay.face_dims(k)) for k in range(dim)]
                            + [out[dim] * wave(lay.n)])
    assert rel(y, expect) < 1e-13


@pytest.mark.parametrize("dim,n", [(2, (8, 8)), (3, (4, 4, 4))])
@pytest.mark.parametrize("theta", [0.0, 7.0])
def test_bulk_schur_approximation_exact_periodic_constant(dim, n, theta):
    """S = -D A^{-1} G inverted on the mean-free space equals
    -theta rho0 L_p^{-1} + (gamma0 + 4/3 mu0) I for periodic constant
    coefficients (eq. Schur_app_bulk); 2 mu0 in its place does not."""
    rho0, mu0, g0 = 1.2, 0.9, 0.25  # gamma0 + 4/3 mu0 = 1.45, 2 mu0 = 1.8
    lay = W.make_layout(dim, n, (0,) * dim)
    o, lay, h = _mk(dim, lay.n, lay.bc, theta, np.full(lay.ncell, rho0),
                    np.full(lay.ncell, mu0), np.full(lay.ncell, g0))
    M, nv = assemble(o, lay)
    A, G, mD = M[:nv, :nv], M[:nv, nv:], M[nv:, :nv]
    if theta == 0.0:
        # the constant velocity modes are in A's null space; G's range is
        # orthogonal to them, so a least-squares solve is exact there
        S = mD @ np.linalg.lstsq(A, G, rcond=None)[0]
    else:
        S = mD @ np.linalg.solve(A, G)
    Lp = (-mD) @ G
    P0 = np.eye(lay.ncell) - 1.0 / lay.ncell
    approx = -theta * rho0 * np.linalg.pinv(Lp) + (g0 + 4 * mu0 / 3) * np.eye(lay.ncell)
    assert rel(P0 @ approx @ S @ P0, P0) < 1e-11
    wrong = -theta * rho0 * np.linalg.pinv(Lp) + 2 * mu0 * np.eye(lay.ncell)
    assert rel(P0 @ wrong @ S @ P0, P0) > 1e-2


@pytest.mark.parametrize("dim,n", [(2, (16, 16)), (3, (8, 8, 8))])
def test_bulk_preconditioners_exact_periodic_constant(dim, n):
    """With (near-)exact subsolvers and the exact Schur approximation of
    eq. Schur_app_bulk: P1^{-1} M = I (one GMRES iteration) and the block
    triangular P2, P3 give (P^{-1} M - I)^2 = 0 (at most two)."""
    lay = W.make_layout(dim, n, (0,) * dim)
    iters = {}
    for P in (W.P1, W.P2, W.P3):
        o, lay, h = _mk(dim, lay.n, lay.bc, 30.0, np.full(lay.ncell, 1.4),
                        np.full(lay.ncell, 0.8), np.full(lay.ncell, 1.5), precond=P, vcycles=40)
        xu = W.random_velocity(5, lay)
        xp = W.random_cells(6, lay, remove_mean=True)
        bu, bp = o.apply(xu, xp)
        if P == W.P1:
            zu, zp = o.precond(bu, bp)
            assert rel(zu, xu) < 1e-10 and rel(zp, xp) < 1e-10
        _, _, st, rc = o.solve(bu, bp, tol=1e-9)
        iters[P] = st["iters"]
    assert iters[W.P1] == 1 and iters[W.P2] <= 2 and iters[W.P3] <= 2, iters


def _mms_fields(dim, periodic):
    import sympy as sp

    X = sp.symbols("x y z")[:dim]
    pi = sp.pi
    if periodic:
        if dim == 2:
            u = [sp.sin(2 * pi * X[0]) * sp.cos(2 * pi * X[1]),
                 sp.cos(2 * pi * X[0]) + sp.sin(2 * pi * X[1])]
        else:
            u = [sp.sin(2 * pi * X[0]) * sp.cos(2 * pi * X[1]),
                 sp.sin(2 * pi * X[1]) * sp.cos(2 * pi * X[2]),
                 sp.sin(2 * pi * X[2]) + sp.cos(2 * pi * X[0])]
        p = sp.sin(2 * pi * X[0]) * sp.sin(4 * pi * X[1])
        mu = 1 + sp.Rational(1, 2) * sp.sin(2 * pi * X[0]) * sp.cos(2 * pi * X[1])
        gamma = 1 + sp.Rational(1, 2) * sp.cos(2 * pi * X[0] + 2 * pi * X[1])
        rho = 2 + sp.cos(2 * pi * X[0] + 2 * pi * X[1])
    else:
        s = 1
        for a in range(dim):
            s = s * sp.sin(pi * X[a])
        if dim == 2:
            u = [s * (1 + X[1]), s * sp.cos(pi * X[0])]
        else:
            u = [s * (1 + X[1]), s * sp.cos(pi * X[2]), s * X[0]]
        p = sp.cos(pi * X[0]) * sp.cos(2 * pi * X[1])
        mu = 1 + sp.Rational(1, 2) * X[0] * X[1]
        gamma = sp.Rational(1, 2) + X[0] ** 2
        rho = 1 + X[1] ** 2
    return X, u, p, mu, gamma, rho


def _discrete_div(lay, h, ue):
    """Staggered divergence of face values (numpy, periodic wrap or walls)."""
    out = np.zeros(lay.cell_shape)
    for k, c in enumerate(lay.split_vel(ue)):
        ax = lay.dim - 1 - k
        if lay.wall(k):
            out += np.diff(c, axis=ax) / h
        else:
            out += (np.roll(c, -1, axis=ax) - c) / h
    return out.ravel()


def _mms_case(dim, n, periodic, theta):
    import sympy as sp

    X, u, p, mu, gamma, rho = _mms_fields(dim, periodic)
    div = sum(sp.diff(u[k], X[k]) for k in range(dim))
    f = []
    for k in range(dim):
        dtau = 0
        for l in range(dim):
            tau = mu * (sp.diff(u[k], X[l]) + sp.diff(u[l], X[k]))
            if l == k:
                tau += (gamma - sp.Rational(2, 3) * mu) * div
            dtau += sp.diff(tau, X[l])
        f.append(theta * rho * u[k] - dtau + sp.diff(p, X[k]))
    lam = lambda e: sp.lambdify(X, e, "numpy")
    bc = (0 if periodic else 1,) * dim
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
    # b_p = -g with g the discrete divergence of the exact face velocities
    bp = -_discrete_div(lay, h, ue)
    o = oracle.Oracle(dim, lay.n, lay.bc, h, theta, cell(rho), cell(mu), gamma=cell(gamma),
                      precond=W.P1)
    xu, xp, st, rc = o.solve(bu, bp, tol=1e-11, max_iter=3000)
    assert rc == oracle.ORC_OK
    eu = np.abs(xu - ue)[~wm].max()
    pe = cell(p)
    ep = np.sqrt(np.mean(((xp - xp.mean()) - (pe - pe.mean())) ** 2))
    return eu, ep


@pytest.mark.parametrize("dim,ns,periodic,theta", [
    (2, (16, 32, 64), True, 0.0), (2, (16, 32, 64), False, 0.0), (2, (16, 32, 64), False, 40.0),
    (3, (8, 16), True, 10.0), (3, (8, 16), False, 0.0)])
def test_compressible_manufactured_solution_second_order(dim, ns, periodic, theta):
    """Variable mu, gamma, rho; div u != 0 (b_p = -D u_exact); no-slip walls or
    periodic: velocity and pressure converge at second order."""
    errs = [_mms_case(dim, n, periodic, theta) for n in ns]
    for (eu0, ep0), (eu1, ep1) in zip(errs[:-1], errs[1:]):
        assert np.log2(eu0 / eu1) >= 1.8, errs
        assert np.log2(ep0 / ep1) >= (1.8 if periodic else 1.5), errs


@pytest.mark.parametrize("dim,n,bc,theta", [(2, (16, 16), (1, 1), 50.0),
                                            (3, (8, 8, 8), (2, 1, 0), 0.0)])
def test_bulk_gradients_match_central_differences(dim, n, bc, theta):
    """dL/dgamma and dL/dmu (with the -2/3 mu inside the bulk coefficient)
    from the adjoint match central differences of
    L = 1/2 ||u - u_target||^2 + 1/2 ||p - p_target||^2 for a compressible
    right-hand side.  The pressure term matters: with div u prescribed the
    bulk stress is a gradient, so gamma moves only p (and dL/dgamma of a
    velocity-only loss is zero)."""
    lay = W.make_layout(dim, n, bc)
    h = 1.0 / lay.n[0]
    rho, mu = W.random_coefficients(7, lay)
    gamma = W.random_bulk_viscosity(8, lay)
    f = W.random_velocity(9, lay)
    g = W.random_cells(10, lay, remove_mean=True)
    target = 0.01 * W.random_velocity(11, lay)
    ptarget = 0.01 * W.random_cells(13, lay)

    def loss(mu_, gamma_):
        o = oracle.Oracle(dim, lay.n, lay.bc, h, theta, rho, mu_, gamma=gamma_, precond=W.P1)
        xu, xp, st, rc = o.solve(f, -g, tol=1e-13, max_iter=5000)
        L = 0.5 * np.sum((xu - target) ** 2) + 0.5 * np.sum((xp - ptarget) ** 2)
        return L, o, xu, xp

    L0, o, xu, xp = loss(mu, gamma)
    adj = o.adjoint(xu, xp, xu - target, xp - ptarget, tol=1e-13, max_iter=5000)
    assert np.linalg.norm(adj["dgamma_cell"]) > 1e-3 * np.linalg.norm(adj["dmu_cell"])
    rng = np.random.default_rng(12)
    eps = 1e-6
    for _ in range(3):
        d = rng.standard_normal(lay.ncell)
        d /= np.linalg.norm(d)
        fd = (loss(mu, gamma + eps * d)[0] - loss(mu, gamma - eps * d)[0]) / (2 * eps)
        gg = adj["dgamma_cell"] @ d
        assert abs(fd - gg) <= 1e-5 * abs(fd) + 1e-7 * np.linalg.norm(adj["dgamma_cell"]), (fd, gg)
        fd = (loss(mu + eps * d, gamma)[0] - loss(mu - eps * d, gamma)[0]) / (2 * eps)
        gm = adj["dmu_cell"] @ d
        assert abs(fd - gm) <= 1e-5 * abs(fd) + 1e-7 * np.linalg.norm(adj["dmu_cell"]), (fd, gm)


def test_bulk_coarse_coefficient_is_cell_mean():
    """The bulk coefficient of a coarse level is the mean of its 2^d fine
    cells (like the cell viscosity, Appendix C), scaled by c on level 0:
    a linear field stays the same linear field on every level."""
    dim, n = 2, (16, 16)
    lay = W.make_layout(dim, n, (1, 0))
    h = 1.0 / 16
    cc = lay.cell_centres(h)
    gamma = (1.0 + 0.3 * cc[0] + 0.2 * cc[1]).ravel()
    mu = np.ones(lay.ncell)
    o = oracle.Oracle(dim, lay.n, lay.bc, h, 0.0, np.ones(lay.ncell), mu, gamma=gamma,
                      rescale_c=2.0)
    for l in range(o.nlevels):
        nl = o.level_dims(l)
        ll = W.make_layout(dim, nl[:dim], (1, 0))
        ccl = ll.cell_centres(h * 2 ** l)
        got = o.level_coef(l, 4, ll.ncell)
        exp = 2.0 * ((1.0 + 0.3 * ccl[0] + 0.2 * ccl[1]).ravel() - 2.0 / 3.0)
        assert rel(got, exp) < 1e-14


def test_bulk_invalid_inputs():
    lay = W.make_layout(2, (8, 8), (1, 1))
    h = 1.0 / 8
    rho, mu = W.random_coefficients(1, lay)
    for bad in (-1e-3, np.nan, np.inf):
        gamma = np.ones(lay.ncell)
        gamma[5] = bad
        with pytest.raises(oracle.OracleError):
            oracle.Oracle(2, lay.n, lay.bc, h, 0.0, rho, mu, gamma=gamma)
    o = oracle.Oracle(2, lay.n, lay.bc, h, 0.0, rho, mu)
    assert "dgamma_cell" not in o.grad(W.random_velocity(1, lay), W.random_velocity(2, lay))
