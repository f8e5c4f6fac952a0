"""Pins of the oracle's solver path (multigrid subsolvers, preconditioners,
GMRES/FGMRES) against exact solutions, closed forms and the paper's stated
properties (arXiv:1308.4605, Sec. "Preconditioners", Sec. "Multigrid Subsolvers", Appendices A-C)."""
import numpy as np
import pytest

import oracle
from mac_helpers import assemble, interior_index, rel
from paper_1308_4605_amd import workloads as W


def _mk(dim, n, bc, theta, rho, mu, **kw):
    lay = W.make_layout(dim, n, bc)
    h = 1.0 / lay.n[0]
    return oracle.Oracle(dim, lay.n, lay.bc, h, theta, rho, mu, **kw), lay, h


# ---------------------------------------------------------------------------
# FFT exact solve (Appendix A symbols), periodic constant coefficients
# ---------------------------------------------------------------------------

def fft_exact_solve(lay, h, theta, rho0, mu0, bu, bp):
    """Solve M x = b mode by mode with the Appendix A symbols, an independent
    exact solver for the periodic constant-coefficient problem.  Mode 0:
    p = 0 and u = b_u / (theta rho0) (or 0 when theta = 0)."""
    dim = lay.dim
    comps = [np.fft.fftn(c) for c in lay.split_vel(bu)]
    ph = np.fft.fftn(bp.reshape(lay.cell_shape))
    shape = lay.cell_shape
    freqs = np.meshgrid(*[np.fft.fftfreq(s) * s for s in shape], indexing="ij")
    # numpy axis order is (z,) y, x; grid axis a is numpy axis dim-1-a
    kap = [2 * np.pi * freqs[dim - 1 - a] / lay.n[a] for a in range(dim)]
    Dh = [(np.exp(1j * kap[a]) - 1) / h for a in range(dim)]
    Gh = [(1 - np.exp(-1j * kap[a])) / h for a in range(dim)]
    out_u = [np.zeros(shape, complex) for _ in range(dim)]
    out_p = np.zeros(shape, complex)
    it = np.nditer(np.zeros(shape), flags=["multi_index"])
    for _ in it:
        idx = it.multi_index
        Msym = np.zeros((dim + 1, dim + 1), complex)
        for k in range(dim):
            for l in range(dim):
                if k == l:
                    Msym[k, k] = theta * rho0 - mu0 * (2 * Gh[k][idx] * Dh[k][idx] +
                                                       sum(Gh[b][idx] * Dh[b][idx] for b in range(dim) if b != k))
                else:
                    Msym[k, l] = -mu0 * Gh[k][idx] * Dh[l][idx]
            Msym[k, dim] = Gh[k][idx]
            Msym[dim, k] = -Dh[k][idx]
        rhs = np.array([comps[k][idx] for k in range(dim)] + [ph[idx]])
        if all(i == 0 for i in idx):
            sol = np.zeros(dim + 1, complex)
            if theta > 0:
                sol[:dim] = rhs[:dim] / (theta * rho0)
        else:
            sol = np.linalg.solve(Msym, rhs)
        for k in range(dim):
            out_u[k][idx] = sol[k]
        out_p[idx] = sol[dim]
    u = np.concatenate([np.fft.ifftn(c).real.ravel() for c in out_u])
    p = np.fft.ifftn(out_p).real.ravel()
    return u, p


@pytest.mark.parametrize("dim,n,theta", [(2, 32, 0.0), (2, 32, 100.0), (3, 16, 0.0), (3, 16, 100.0)])
@pytest.mark.parametrize("precond", [W.P1, W.P2, W.P3])
def test_gmres_matches_fft_exact_solution(dim, n, theta, precond):
    rho0, mu0 = 1.0, 1.0
    lay = W.make_layout(dim, (n,) * dim, (0,) * dim)
    h = 1.0 / n
    o, lay, h = _mk(dim, lay.n, lay.bc, theta, np.full(lay.ncell, rho0), np.full(lay.ncell, mu0),
                    precond=precond)
    bu = W.smooth_face_field(np.random.default_rng(3), lay, h, 8, 4, remove_mean=True)
    bp = np.zeros(lay.ncell)
    xu, xp, st, rc = o.solve(bu, bp, tol=1e-12)
    eu, ep = fft_exact_solve(lay, h, theta, rho0, mu0, bu, bp)
    assert rel(xu, eu) < 1e-9
    assert rel(xp - xp.mean(), ep - ep.mean()) < 1e-9


# ---------------------------------------------------------------------------
# dense direct solve on 8x8 (and 4^3), variable coefficients
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n,bc,theta", [
    (2, (8, 8), (1, 1), 0.0), (2, (8, 8), (0, 0), 30.0), (2, (8, 8), (0, 1), 0.0),
    (2, (8, 8), (0, 0), 0.0), (3, (4, 4, 4), (1, 1, 1), 10.0), (3, (4, 4, 4), (1, 0, 0), 0.0),
    (2, (8, 8), (2, 2), 0.0), (2, (8, 8), (0, 2), 0.0), (3, (4, 4, 4), (2, 1, 2), 10.0),
    (3, (4, 4, 4), (2, 2, 0), 0.0), (2, (8, 8), (0, 3), 0.0), (3, (4, 4, 4), (4, 2, 3), 10.0)])
@pytest.mark.parametrize("precond,krylov", [(W.P1, W.GMRES_LEFT), (W.P2, W.GMRES_LEFT),
                                            (W.P3, W.GMRES_LEFT), (W.P5, W.GMRES_LEFT),
                                            (W.P1, W.FGMRES), (W.P4, W.FGMRES)])
def test_gmres_matches_dense_direct_solve(dim, n, bc, theta, precond, krylov):
    lay = W.make_layout(dim, n, bc)
    rho, mu = W.random_coefficients(17, lay, mu_range=(0.1, 10.0), rho_range=(0.5, 3.0))
    o, lay, h = _mk(dim, lay.n, lay.bc, theta, rho, mu, precond=precond, krylov=krylov)
    singular_u = lay.singular_components(theta)
    bu = W.random_velocity(5, lay, remove_mean=singular_u)
    bp = W.random_cells(6, lay, remove_mean=True)
    xu, xp, st, rc = o.solve(bu, bp, tol=1e-12, max_iter=2000)
    assert st["rel_res_true"] <= 1e-12
    M, nv = assemble(o, lay)
    vel, pr = interior_index(lay)
    b = np.concatenate([bu, bp])[np.concatenate([vel, pr])]
    # pin the null space: minimum-norm solution of the consistent system
    x = np.linalg.lstsq(M, b, rcond=None)[0]
    xu_d = np.zeros(lay.nvel)
    xu_d[vel] = x[:nv]
    xp_d = x[nv:]
    if singular_u:
        xu_d = W._remove_component_means(lay, xu_d, comps=singular_u)
    sv = np.linalg.svd(M, compute_uv=False)
    sv = sv[sv > 1e-12 * sv[0]]
    tol = max(10 * 1e-12 * sv[0] / sv[-1], 1e-10)
    assert rel(xu, xu_d) < tol
    assert rel(xp - xp.mean(), xp_d - xp_d.mean()) < tol


# ---------------------------------------------------------------------------
# manufactured solutions: global second order (Sec. "Staggered-grid Discretization")
# ---------------------------------------------------------------------------

def _mms_fields(dim, periodic, freeslip=False):
    """Exact velocity, pressure, viscosity, density as sympy expressions and
    the forcing f = theta rho u - div(mu (grad u + grad u^T)) + grad p."""
    import sympy as sp

    X = sp.symbols("x y z")[:dim]
    pi = sp.pi
    if freeslip:
        # divergence free; zero normal velocity and zero normal derivative of
        # the tangential components on every wall (both shear terms vanish)
        c = [sp.cos(pi * X[a]) for a in range(dim)]
        sn = [sp.sin(pi * X[a]) for a in range(dim)]
        if dim == 2:
            u = [sn[0] * c[1], -c[0] * sn[1]]
        else:
            u = [sn[0] * c[1] * c[2], c[0] * sn[1] * c[2], -2 * c[0] * c[1] * sn[2]]
        p = sp.cos(pi * X[0]) * sp.cos(2 * pi * X[1])
        mu = 1 + sp.Rational(1, 2) * X[0] * X[1]
        rho = 1 + X[1] ** 2
        return X, u, p, mu, rho
    if periodic:
        if dim == 2:
            psi = sp.sin(2 * pi * X[0]) * sp.cos(2 * pi * X[1]) / (2 * pi)
            u = [sp.diff(psi, X[1]), -sp.diff(psi, X[0])]
        else:
            a = sp.sin(2 * pi * X[0]) * sp.sin(2 * pi * X[1]) * sp.sin(2 * pi * X[2])
            u = [sp.cos(2 * pi * X[1]) * sp.sin(2 * pi * X[2]),
                 sp.sin(2 * pi * X[0]) * sp.cos(2 * pi * X[2]),
                 sp.cos(2 * pi * X[0]) * sp.sin(2 * pi * X[1])]
            del a
        p = sp.sin(2 * pi * X[0]) * sp.sin(4 * pi * X[1])
        mu = 1 + sp.Rational(1, 2) * sp.sin(2 * pi * X[0]) * sp.cos(2 * pi * X[1])
        rho = 2 + sp.cos(2 * pi * X[0] + 2 * pi * X[1])
    else:
        if dim == 2:
            psi = sp.sin(pi * X[0]) ** 2 * sp.sin(pi * X[1]) ** 2
            u = [sp.diff(psi, X[1]), -sp.diff(psi, X[0])]
        else:
            s = [sp.sin(pi * X[a]) ** 2 for a in range(3)]
            # u = curl(0, 0, psi) + curl(psi2, 0, 0) with psi vanishing with
            # its normal derivative on the walls: divergence free, zero on walls
            psi = s[0] * s[1] * s[2]
            u = [sp.diff(psi, X[1]), -sp.diff(psi, X[0]) + sp.diff(psi, X[2]), -sp.diff(psi, X[1])]
        p = sp.cos(pi * X[0]) * sp.cos(2 * pi * X[1])
        mu = 1 + sp.Rational(1, 2) * X[0] * X[1]
        rho = 1 + X[1] ** 2
    return X, u, p, mu, rho


def _mms_case(dim, n, periodic, theta, freeslip=False):
    import sympy as sp

    X, u, p, mu, rho = _mms_fields(dim, periodic, freeslip)
    f = []
    for k in range(dim):
        div_tau = sum(sp.diff(mu * (sp.diff(u[k], X[l]) + sp.diff(u[l], X[k])), X[l]) for l in range(dim))
        f.append(theta * rho * u[k] - div_tau + sp.diff(p, X[k]))
    g = sum(sp.diff(u[k], X[k]) for k in range(dim))
    assert sp.simplify(g) == 0
    lam = lambda e: sp.lambdify(X, e, "numpy")
    bc = (0 if periodic else (2 if freeslip else 1),) * dim
    lay = W.make_layout(dim, (n,) * dim, bc)
    h = 1.0 / n
    cc = lay.cell_centres(h)
    mu_c = np.broadcast_to(lam(mu)(*cc), lay.cell_shape).ravel()
    rho_c = np.broadcast_to(lam(rho)(*cc), lay.cell_shape).ravel()
    bu, ue = [], []
    for k in range(dim):
        fc = lay.face_centres(k, h)
        bu.append(np.broadcast_to(lam(f[k])(*fc), lay.face_shape(k)).ravel())
        ue.append(np.broadcast_to(lam(u[k])(*fc), lay.face_shape(k)).ravel())
    bu = np.concatenate(bu)
    ue = np.concatenate(ue)
    wm = lay.wall_mask()
    bu[wm] = 0.0
    pe = np.broadcast_to(lam(p)(*cc), lay.cell_shape).ravel()
    o = oracle.Oracle(dim, lay.n, lay.bc, h, theta, rho_c, mu_c, precond=W.P1)
    xu, xp, st, rc = o.solve(bu, np.zeros(lay.ncell), tol=1e-11, max_iter=3000)
    eu = np.abs(xu - ue)[~wm].max()
    ep = np.sqrt(np.mean(((xp - xp.mean()) - (pe - pe.mean())) ** 2))
    return eu, ep


@pytest.mark.parametrize("dim,ns,periodic,theta,freeslip", [
    (2, (16, 32, 64), True, 0.0, False), (2, (16, 32, 64), False, 0.0, False),
    (2, (16, 32, 64), False, 50.0, False), (3, (8, 16), True, 10.0, False),
    (3, (8, 16), False, 0.0, False), (2, (16, 32, 64), False, 0.0, True),
    (3, (8, 16), False, 10.0, True)])
def test_manufactured_solution_second_order(dim, ns, periodic, theta, freeslip):
    errs = [_mms_case(dim, n, periodic, theta, freeslip) for n in ns]
    for (eu0, ep0), (eu1, ep1) in zip(errs[:-1], errs[1:]):
        ou = np.log2(eu0 / eu1)
        op = np.log2(ep0 / ep1)
        assert ou >= 1.8, (errs, ou)
        assert op >= (1.8 if periodic else 1.5), (errs, op)


# ---------------------------------------------------------------------------
# multigrid subsolvers (Sec. "Multigrid Subsolvers", Appendix C)
# ---------------------------------------------------------------------------

def _vel_op(o, lay, u):
    return o.apply(u, np.zeros(lay.ncell))[0]


def _ratios_above_roundoff(hist, floor=1e-11):
    """per-cycle reductions while the residual is still above roundoff"""
    out = [hist[0]]
    for i in range(1, len(hist)):
        if hist[i - 1] > floor:
            out.append(hist[i] / hist[i - 1])
    return out


def _vcycle_reduction(o, lay, r, cycles, op, sub):
    e = np.zeros_like(r)
    out = []
    for _ in range(cycles):
        res = r - op(e)
        e = e + sub(res)
        out.append(np.linalg.norm(r - op(e)) / np.linalg.norm(r))
    return out


# Per-cycle contraction bounds.  The paper states at least one order of
# magnitude per V-cycle and about a dozen cycles to near roundoff (subsection
# "The effect of the number of smoothing sweeps", read off its figure for
# 512^2 and 128^3).  The paper pin here is the dozen cycles: both dimensions
# must reach 1e-10 after 12 cycles.  The per-cycle bounds are regression
# bounds measured on this oracle, not paper values: 2D stays <= 0.1; 3D
# starts near 0.03 and settles at about 0.14 (geometric mean over 12 cycles
# 0.11).  The transfers themselves are pinned directly in
# test_oracle_transfers.py; the alternatives tried for 3D (full-weighting
# tangential restriction, reversed colour order after coarse correction) both
# contract more slowly (0.19 and 0.22), so the tensor readings stand.
RATE = {2: 0.105, 3: 0.15}


@pytest.mark.parametrize("dim,n", [(2, 128), (3, 32)])
def test_velocity_vcycle_contracts_tenfold(dim, n):
    """Constant-coefficient steady no-slip stress-form velocity problem
    (Sec. "The effect of the number of smoothing sweeps"): per-cycle residual reduction and 12 cycles to 1e-10."""
    lay = W.make_layout(dim, (n,) * dim, (1,) * dim)
    o, lay, h = _mk(dim, lay.n, lay.bc, 0.0, np.ones(lay.ncell), np.ones(lay.ncell), rescale_c=1.0)
    r = W.random_velocity(1, lay)
    hist = _vcycle_reduction(o, lay, r, 12, lambda u: _vel_op(o, lay, u), o.vel_subsolve)
    ratios = _ratios_above_roundoff(hist)
    assert max(ratios) < RATE[dim], ratios
    assert hist[-1] < 1e-10, hist


@pytest.mark.parametrize("dim,n,bc", [(2, 128, 1), (3, 32, 1), (2, 64, 0)])
def test_pressure_vcycle_contracts_tenfold(dim, n, bc):
    lay = W.make_layout(dim, (n,) * dim, (bc,) * dim)
    o, lay, h = _mk(dim, lay.n, lay.bc, 0.0, np.ones(lay.ncell), np.ones(lay.ncell), rescale_c=1.0)

    def lrho(p):
        gp = o.apply(np.zeros(lay.nvel), p)[0]  # G p (A*0 = 0)
        return -o.apply(gp, np.zeros(lay.ncell))[1]  # D G p with rho = 1

    r = W.random_cells(2, lay, remove_mean=True)
    hist = _vcycle_reduction(o, lay, r, 12, lrho, o.p_subsolve)
    ratios = _ratios_above_roundoff(hist)
    assert max(ratios) < RATE[dim], ratios
    assert hist[-1] < 1e-10, hist


def test_vcycle_is_linear():
    """A fixed number of V-cycles is a constant linear operator (needed for
    left-preconditioned GMRES, Sec. "Results")."""
    dim, n, bc = 3, (8, 8, 8), (1, 0, 1)
    lay = W.make_layout(dim, n, bc)
    rho, mu = W.random_coefficients(2, lay)
    o, lay, h = _mk(dim, lay.n, lay.bc, 20.0, rho, mu)
    a, b = W.random_velocity(3, lay), W.random_velocity(4, lay)
    ea, eb, eab = o.vel_subsolve(a), o.vel_subsolve(b), o.vel_subsolve(2.0 * a - 3.0 * b)
    assert rel(eab, 2.0 * ea - 3.0 * eb) < 1e-13
    pa, pb = W.random_cells(5, lay, True), W.random_cells(6, lay, True)
    qa, qb, qab = o.p_subsolve(pa), o.p_subsolve(pb), o.p_subsolve(pa + 0.5 * pb)
    assert rel(qab, qa + 0.5 * qb) < 1e-13


def test_coarse_coefficients_of_linear_fields():
    """Coarsening (Appendix C): cell values are means of 2^d fine cells and
    edge values means of the two overlaid fine edges (3D) or injected nodes
    (2D); applied to linear fields they reproduce the field at the coarse
    positions.  Face alpha = mean of overlaid faces: linear in the tangential
    directions -> exact."""
    for dim in (2, 3):
        n = (16,) * dim
        lay = W.make_layout(dim, n, (0,) * dim)
        h = 1.0 / 16
        cc = lay.cell_centres(h)
        coef = [0.3, -0.7, 0.45][:dim]
        mu = (2.0 + sum(c * x for c, x in zip(coef, cc))).ravel()
        rho = np.ones(lay.ncell)
        o, lay, h = _mk(dim, lay.n, lay.bc, 1.0, rho, mu, rescale_c=1.0)
        for lvl in range(1, o.nlevels):
            nl = o.level_dims(lvl)
            ll = W.make_layout(dim, nl[:dim], (0,) * dim)
            hl = h * 2 ** lvl
            got = o.level_coef(lvl, 2, ll.ncell)
            ccl = ll.cell_centres(hl)
            exp = (2.0 + sum(c * x for c, x in zip(coef, ccl))).ravel()
            assert rel(got, exp) < 1e-14


# ---------------------------------------------------------------------------
# preconditioners with (near-)exact subsolvers (Sec. "Preconditioners", Appendix B)
# ---------------------------------------------------------------------------

EXACT = dict(vcycles=40)


@pytest.mark.parametrize("dim,n", [(2, (16, 16)), (3, (8, 8, 8))])
def test_p1_is_exact_for_periodic_constant_coefficients(dim, n):
    """P1^{-1} M = I for periodic constant coefficients with exact
    subsolvers (Appendix B): the Schur approximation -theta L_rho^{-1} + 2 mu0
    is then exact."""
    lay = W.make_layout(dim, n, (0,) * dim)
    o, lay, h = _mk(dim, lay.n, lay.bc, 50.0, np.full(lay.ncell, 1.5), np.full(lay.ncell, 0.8),
                    precond=W.P1, **EXACT)
    xu = W.random_velocity(3, lay)
    xp = W.random_cells(4, lay, remove_mean=True)
    zu, zp = o.precond(*o.apply(xu, xp))
    assert rel(zu, xu) < 1e-10
    assert rel(zp, xp) < 1e-10
    xs, ps, st, rc = o.solve(*o.apply(xu, xp), tol=1e-9)
    assert st["iters"] == 1


@pytest.mark.parametrize("dim,n,bc", [(2, (16, 16), (1, 1)), (3, (8, 8, 8), (1, 0, 1))])
def test_inviscid_preconditioners_exact(dim, n, bc):
    """mu = 0 (inviscid) with any boundary condition and variable density:
    P1^{-1} M = I and (P2^{-1} M - I)^2 = 0 (Appendix B), so GMRES takes one
    iteration with P1 and two with P2, P3."""
    lay = W.make_layout(dim, n, bc)
    rho, _ = W.random_coefficients(8, lay)
    mu = np.zeros(lay.ncell)
    res = {}
    for P in (W.P1, W.P2, W.P3):
        o, lay, h = _mk(dim, lay.n, lay.bc, 25.0, rho, mu, precond=P, rescale_c=1.0, **EXACT)
        xu = W.random_velocity(3, lay)
        xp = W.random_cells(4, lay, remove_mean=True)
        bu, bp = o.apply(xu, xp)
        zu, zp = o.precond(bu, bp)
        if P == W.P1:
            assert rel(zu, xu) < 1e-10 and rel(zp, xp) < 1e-10
        if P == W.P2:
            # (P^{-1}M - I)^2 x = 0
            du, dp = zu - xu, zp - xp
            wu, wp = o.precond(*o.apply(du, dp))
            assert np.linalg.norm(wu - du) < 1e-9 * np.linalg.norm(xu)
            assert np.linalg.norm(wp - dp) < 1e-9 * np.linalg.norm(xp)
            assert np.linalg.norm(du) > 1e-3 * np.linalg.norm(xu)  # P2 is not exact
        _, _, st, rc = o.solve(bu, bp, tol=1e-9)
        res[P] = st["iters"]
    assert res[W.P1] == 1
    assert res[W.P2] <= 2 and res[W.P3] <= 2


def test_schur_approximation_is_exact_periodic_constant():
    """S = -D A^{-1} G inverted on the mean-free space equals
    -theta rho0 L_p^{-1} + 2 mu0 I for periodic constant coefficients
    (eq. Schur_app_varDen_varVis with the factor 2 of Appendix A)."""
    dim, n = 2, (8, 8)
    theta, rho0, mu0 = 7.0, 1.2, 0.9
    lay = W.make_layout(dim, n, (0, 0))
    o, lay, h = _mk(dim, lay.n, lay.bc, theta, np.full(lay.ncell, rho0), np.full(lay.ncell, mu0))
    M, nv = assemble(o, lay)
    A, G, mD = M[:nv, :nv], M[:nv, nv:], M[nv:, :nv]
    S = mD @ np.linalg.solve(A, G)  # -D A^{-1} G
    Lp = (-mD) @ G
    P0 = np.eye(lay.ncell) - 1.0 / lay.ncell  # projector on mean-free cells
    Sinv_approx = -theta * rho0 * np.linalg.pinv(Lp) + 2 * mu0 * np.eye(lay.ncell)
    assert rel(P0 @ Sinv_approx @ S @ P0, P0) < 1e-12


# ---------------------------------------------------------------------------
# spectra (Appendix B.1)
# ---------------------------------------------------------------------------

def test_saddle_inertia_and_schur_clustering_32():
    """32^2 no-slip steady constant viscosity: N_dof = 3008, M has 1024
    eigenvalues <= 0 (the pressure count); S~^{-1} S = 2 mu0 D L_mu^{-1} G has
    one zero eigenvalue and about 4 (n_c - 1) = 124 non-unit eigenvalues
    (Appendix B.1; golden values in tests/golden/spectrum_32.json)."""
    import json, os

    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "spectrum_32.json")))
    nc = gold["n_c"]
    lay = W.make_layout(2, (nc, nc), (1, 1))
    o, lay, h = _mk(2, lay.n, lay.bc, 0.0, np.ones(lay.ncell), np.ones(lay.ncell), rescale_c=1.0)
    M, nv = assemble(o, lay)
    assert M.shape[0] == gold["n_dof"]
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    scale = np.abs(ev).max()
    assert int((ev <= 1e-9 * scale).sum()) == gold["nonpositive_eigs_M"]
    A, G, mD = M[:nv, :nv], M[:nv, nv:], M[nv:, :nv]
    S = mD @ np.linalg.solve(A, G)
    lam = np.sort(np.linalg.eigvals(2.0 * S).real)
    zero = np.abs(lam) < 1e-8
    assert zero.sum() == 1
    nonunit = (np.abs(lam - 1.0) > 1e-6) & ~zero
    assert 0 < nonunit.sum() <= gold["nonunit_bound"]
    assert lam[~zero].min() > 0.0 and lam.max() <= 1.0 + 1e-8


def test_bubble_schur_spectrum_32():
    """32^2 no-slip steady bubble, viscosity contrast 100 (App. B.1): about 87%
    of the N_dof eigenvalues of the exactly-preconditioned operator lie in
    (0.99, 1.01), and the rest stay near unity (tests/golden/spectrum_32.json)."""
    import json, os

    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "spectrum_32.json")))["bubble_contrast_100"]
    w = W.bubble(2, 32, 100.0, 100.0)
    lay = w.layout
    o, lay, h = _mk(2, lay.n, lay.bc, 0.0, w.rho, w.mu, rescale_c=1.0)
    M, nv = assemble(o, lay)
    A, G, mD = M[:nv, :nv], M[:nv, nv:], M[nv:, :nv]
    lam = np.linalg.eigvals(np.diag(2.0 * w.mu) @ (mD @ np.linalg.solve(A, G)))
    assert np.abs(lam.imag).max() <= 1e-8 * np.abs(lam).max()
    lam = lam.real
    zero = np.abs(lam) < 1e-8
    assert zero.sum() == 1
    near = ((lam > 0.99) & (lam < 1.01)).sum() + nv
    frac = near / (nv + lay.ncell)
    assert abs(frac - gold["fraction_in_0.99_1.01"]) <= gold["fraction_tolerance"], frac
    assert lam[~zero].min() > 0.2 and lam.max() < 2.0


# ---------------------------------------------------------------------------
# adjoint (M = M^T, Sec. "Preconditioners")
# ---------------------------------------------------------------------------

def _loss_and_grad(dim, n, bc, theta, s, f, target, tol):
    lay = W.make_layout(dim, n, bc)
    o, lay, h = _mk(dim, lay.n, lay.bc, theta, np.ones(lay.ncell), np.exp(s), precond=W.P1)
    xu, xp, st, rc = o.solve(f, np.zeros(lay.ncell), tol=tol, max_iter=5000)
    r = xu - target
    L = 0.5 * r @ r
    return L, o, xu, xp, r


@pytest.mark.parametrize("dim,n,bc,theta", [(2, (16, 16), (1, 1), 100.0), (3, (8, 8, 8), (1, 1, 1), 100.0),
                                            (2, (16, 16), (0, 1), 0.0), (2, (16, 16), (2, 2), 0.0),
                                            (3, (8, 8, 8), (2, 1, 2), 100.0)])
def test_adjoint_gradient_matches_central_differences(dim, n, bc, theta):
    """dL/ds (mu = exp(s)) and dL/df from the adjoint solve match central
    finite differences of L = 1/2 ||u - u_target||^2 with forward solves at
    1e-13 (the adjoint of a symmetric M reuses the forward solver).  The FD
    quotient at step 1e-6 is itself limited by the 1e-13 solves, so the bound
    is 1e-5 relative plus 1e-7 of the gradient norm."""
    lay = W.make_layout(dim, n, bc)
    h = 1.0 / lay.n[0]
    rng = np.random.default_rng(42)
    s = 0.5 * rng.standard_normal(lay.ncell)
    f = W.random_velocity(43, lay)
    target = W.random_velocity(44, lay) * 0.01
    L0, o, xu, xp, r = _loss_and_grad(dim, n, bc, theta, s, f, target, 1e-13)
    adj = o.adjoint(xu, xp, r, np.zeros(lay.ncell), tol=1e-13, max_iter=5000)
    gs = adj["dmu_cell"] * np.exp(s)
    gf = adj["lu"]
    eps = 1e-6
    for t in range(4):
        ds = rng.standard_normal(lay.ncell)
        ds /= np.linalg.norm(ds)
        Lp = _loss_and_grad(dim, n, bc, theta, s + eps * ds, f, target, 1e-13)[0]
        Lm = _loss_and_grad(dim, n, bc, theta, s - eps * ds, f, target, 1e-13)[0]
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - gs @ ds) <= 1e-5 * abs(fd) + 1e-7 * np.linalg.norm(gs), (fd, gs @ ds)
        df = W.random_velocity(100 + t, lay)
        df /= np.linalg.norm(df)
        Lp = _loss_and_grad(dim, n, bc, theta, s, f + eps * df, target, 1e-13)[0]
        Lm = _loss_and_grad(dim, n, bc, theta, s, f - eps * df, target, 1e-13)[0]
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - gf @ df) <= 1e-5 * abs(fd) + 1e-7 * np.linalg.norm(gf), (fd, gf @ df)


def test_density_gradient_matches_finite_difference():
    dim, n, bc, theta = 2, (8, 8), (1, 0), 40.0
    lay = W.make_layout(dim, n, bc)
    h = 1.0 / lay.n[0]
    rho, mu = W.random_coefficients(4, lay)
    f = W.random_velocity(5, lay)
    target = 0.01 * W.random_velocity(6, lay)

    def loss(rho_):
        o = oracle.Oracle(dim, lay.n, lay.bc, h, theta, rho_, mu)
        xu, xp, st, rc = o.solve(f, np.zeros(lay.ncell), tol=1e-13, max_iter=5000)
        return 0.5 * np.sum((xu - target) ** 2), o, xu, xp

    L0, o, xu, xp = loss(rho)
    adj = o.adjoint(xu, xp, xu - target, np.zeros(lay.ncell), tol=1e-13, max_iter=5000)
    rng = np.random.default_rng(0)
    for _ in range(3):
        d = rng.standard_normal(lay.ncell)
        d /= np.linalg.norm(d)
        fd = (loss(rho + 1e-6 * d)[0] - loss(rho - 1e-6 * d)[0]) / 2e-6
        g = adj["drho_cell"] @ d
        assert abs(fd - g) <= 1e-6 * abs(fd) + 1e-9, (fd, g)


# ---------------------------------------------------------------------------
# error paths
# ---------------------------------------------------------------------------

def test_invalid_sizes_and_incompatible_rhs():
    lay = W.make_layout(2, (12, 12), (1, 1))
    with pytest.raises(oracle.OracleError) as e:
        oracle.Oracle(2, lay.n, lay.bc, 1 / 12, 0.0, np.ones(lay.ncell), np.ones(lay.ncell))
    assert e.value.code == oracle.ORC_EINVAL
    lay = W.make_layout(2, (8, 8), (1, 1))
    o, lay, h = _mk(2, lay.n, lay.bc, 0.0, np.ones(lay.ncell), np.ones(lay.ncell))
    bp = np.ones(lay.ncell)
    with pytest.raises(oracle.OracleError) as e:
        o.solve(np.zeros(lay.nvel), bp)
    assert e.value.code == oracle.ORC_EINCOMPAT
    xu, xp, st, rc = o.solve(W.random_velocity(1, lay), np.zeros(lay.ncell), tol=1e-14, max_iter=3,
                             check=False)
    assert rc == oracle.ORC_ENOCONV and st["iters"] == 3
