"""Solver statistics and the differentiable solve with given edge
viscosities, on the GPU: the residual history (one entry per Arnoldi step,
ending at the last Givens estimate), the residual of the caller's unscaled
system against the oracle's operator, the timers, and dL/dmu_edge through
autograd against the oracle's FP64 adjoint."""
import numpy as np
import pytest

import oracle
from gpu_common import N, T, pair, params, rel
from paper_1308_4605_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,krylov", [(W.FP64, W.GMRES_LEFT), (W.MG_FP32, W.FGMRES)])
def test_stats_history_unscaled_residual_and_timers(precision, krylov):
    p, lay = params(3, (32, 32, 32), (1, 0, 2), 20.0, precond=W.P2, precision=precision,
                    krylov=krylov, restart=5)
    rho, mu = W.random_coefficients(91, lay, mu_range=(0.2, 5.0))
    g, o = pair(p, rho, mu)
    bu = W.random_velocity(92, lay)
    bp = W.random_cells(93, lay, remove_mean=True)
    xu, xp, st, rc = g.solve(T(bu), T(bp), tol=1e-9, max_iter=300, history=True)
    assert rc == 0
    h = st["history"]
    print(f"  {st['iters']} iterations, {st['restarts']} cycles, t_total {st['t_total']:.3f} s, "
          f"t_precond {st['t_precond']:.3f} s", flush=True)
    assert len(h) == st["history_len"] == st["iters"]
    assert h[-1] == st["rel_res_est"]
    # the Givens estimate never increases within a restart cycle
    assert all(h[i + 1] <= h[i] * (1 + 1e-12) for i in range(4))
    yu, yp = o.apply(N(xu), N(xp))
    true = np.sqrt(np.sum((bu - yu) ** 2) + np.sum((bp - yp) ** 2)) / np.sqrt(
        np.sum(bu ** 2) + np.sum(bp ** 2))
    assert abs(st["rel_res_unscaled"] - true) <= 1e-3 * true
    assert 0.0 < st["t_precond"] <= st["t_total"]
    assert st["t_krylov"] == pytest.approx(st["t_total"] - st["t_precond"])
    # no history requested: nothing is written and the count is 0
    _, _, st2, _ = g.solve(T(bu), T(bp), tol=1e-9, max_iter=300)
    assert st2["history_len"] == 0 and st2["iters"] == st["iters"]


def test_autograd_given_edge_viscosity_matches_oracle():
    import torch

    from paper_1308_4605_amd.autograd import stokes_solve

    dim, n, bc = 3, (16, 16, 16), (1, 2, 0)
    p, lay = params(dim, n, bc, 10.0, edge_avg=W.EDGE_GIVEN)
    rho, mu = W.random_coefficients(94, lay)
    edges = np.random.default_rng(95).uniform(0.3, 3.0, lay.nedge)
    f = W.random_velocity(96, lay)
    ut = 0.01 * W.random_velocity(97, lay)
    mu_t, e_t, f_t = T(mu).requires_grad_(True), T(edges).requires_grad_(True), T(f)
    u, pr = stokes_solve(mu_t, T(rho), f_t, p, tol=1e-12, max_iter=3000, mu_edge=e_t)
    L = 0.5 * torch.sum((u - T(ut)) ** 2)
    L.backward()
    o = oracle.Oracle(rho=rho, mu=mu, edges=edges, **p)
    ou, op, _, _ = o.solve(f, np.zeros(lay.ncell), tol=1e-12, max_iter=3000)
    adj = o.adjoint(ou, op, ou - ut, np.zeros(lay.ncell), tol=1e-12, max_iter=3000)
    assert rel(N(e_t.grad), adj["dmu_edge"]) <= 1e-6
    assert rel(N(mu_t.grad), adj["dmu_cell"]) <= 1e-6



def _vcycle_bytes_model(dim, n, bc, theta, vel, s=8, nu=(2, 2, 8)):
    """The documented byte model of one finest-level V-cycle (stokes.h,
    stokes_vcycle_time), from the array sizes of each level."""
    total, levels, dims = 0.0, [], []
    m = list(n)
    while True:
        levels.append(W.make_layout(dim, tuple(m), bc))
        dims.append(tuple(m))
        if min(m) == 2:
            break
        m = [x // 2 for x in m]
    for l, lay in enumerate(levels):
        nv, nc, ne = lay.nvel, lay.ncell, lay.nedge
        coarsest = l == len(levels) - 1
        sweeps = nu[2] if coarsest else nu[0] + nu[1]
        edges = {m_: int(np.prod(lay.edge_dims(m_)[:dim])) for m_ in lay.edge_families}
        if vel:
            # levels of at most 512 cells form the coarse tail, applied as its
            # matrix (first tail level's nv squared, plus its input and output)
            if nc <= 512:
                total += s * (nv * nv + 2.0 * nv)
                break
            # above it the first sweep starts from uncleared memory (every
            # extent even) and reads only the components it has written
            in_tail = False
            zf = (not in_tail) and all(x % 2 == 0 for x in dims[l]) and \
                (nu[2] if coarsest else nu[0]) > 0
            b = 0 if zf else nv
            sw = first = done = 0.0
            for k in range(dim):
                e = sum(c for m_, c in edges.items() if m_ != k)
                fk = lay.face_counts[k]
                # a colour pass needs only its colour's half of rhs_k, alpha_k
                # and the written u_k
                coef = (1 if theta else 0.5) * fk + nc + e
                sw += 2 * (nv + coef + 0.5 * fk)
                first += (done + coef + 0.5 * fk) + (done + 0.5 * fk + coef + 0.5 * fk)
                done += fk
            b += first + (sweeps - 1) * sw if zf else sweeps * sw
            if not coarsest:
                nvc = levels[l + 1].nvel
                b += 3 * nv + (nv if theta else 0) + nc + ne + nv + nvc + nvc + 2 * nv
        else:
            zf = nc > 512 and all(x % 2 == 0 for x in dims[l]) and \
                (nu[2] if coarsest else nu[0]) > 0
            if zf:
                b = (nv + nc) + (nv + 1.5 * nc) + (sweeps - 1) * 2 * (nv + 2 * nc)
            else:
                b = nc + sweeps * 2 * (nv + 2 * nc)
            if not coarsest:
                ncc = levels[l + 1].ncell
                b += nv + 3 * nc + nc + ncc + ncc + 2 * nc
        total += s * b
    return total


@pytest.mark.parametrize("dim,n,bc", [
    (3, (32, 32, 32), (1, 1, 1)),  # coarse tail below 16^3; first sweeps from uncleared memory
    (3, (516, 8, 8), (1, 0, 0)),   # no tail; odd coarsest extent (129), which keeps the fill
    (2, (256, 256), (0, 0)),       # periodic 2D, tail from 16^2
])
@pytest.mark.parametrize("mode", [1, 2])
def test_vcycle_timing_counts_and_bytes(dim, n, bc, mode):
    """The V-cycle timer counts one velocity and one pressure cycle per P1
    application and reports the bytes of the documented cycle model, with
    per-launch events (mode 1) and with per-V-cycle events only (mode 2)."""
    p, lay = params(dim, n, bc, 10.0, precond=W.P1)
    rho, mu = W.random_coefficients(98, lay)
    g, _ = pair(p, rho, mu)
    bu = W.random_velocity(99, lay)
    g.set_timing(mode)
    g.precond(T(bu), T(np.zeros(lay.ncell)))
    g.precond(T(bu), T(np.zeros(lay.ncell)))
    msv, cv, bv = g.vcycle_time(False)
    msp, cp, bpr = g.vcycle_time(True)
    g.set_timing(False)
    assert cv == 2 and cp == 2 and msv > 0 and msp > 0
    assert bv / cv == pytest.approx(_vcycle_bytes_model(dim, n, bc, 10.0, True), rel=1e-12)
    assert bpr / cp == pytest.approx(_vcycle_bytes_model(dim, n, bc, 10.0, False), rel=1e-12)
