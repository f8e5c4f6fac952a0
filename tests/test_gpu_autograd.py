"""The differentiable solve (torch.autograd.Function over the hand-written
adjoint) against central finite differences (step 1e-6, solves at 1e-13) and
against the oracle's FP64 adjoint, in the FP64 and FP32-multigrid forms.

Loss: L = 1/2 ||u - u_target||^2 over the faces, mu = exp(s), u_target the
solution for a second seeded draw; directions are seeded unit vectors in
s-space and in forcing space.
"""
import numpy as np
import pytest

import oracle
from gpu_common import N, T, rel
from paper_1308_4605_amd import workloads as W

pytestmark = pytest.mark.gpu

# The central-difference quotient at step 1e-6 is limited by the 1e-13 solves:
# its error is about tol * cond * L / eps, which grows with the grid.  For unit
# directions the bound is 1e-5 of the quotient plus 1e-6 of the gradient norm
# (random directions in n dimensions see |g.d| ~ |g| / sqrt(n)).
FD_TOL_REL, FD_TOL_ABS = 1e-5, 1e-6


def _setup(n, precision):
    import torch

    from paper_1308_4605_amd.autograd import stokes_solve

    w = W.adjoint_3d(n=n, precision=precision)
    krylov = W.FGMRES if precision == W.MG_FP32 else W.GMRES_LEFT
    params = w.params(precision=precision, krylov=krylov)
    rho = T(w.rho)
    with torch.no_grad():
        ut, _ = stokes_solve(T(np.exp(w.extra["s2"])), rho, T(w.extra["bu2"]), params, tol=1e-13)

    def loss(s, f):
        u, p = stokes_solve(torch.exp(s), rho, f, params, tol=1e-13, max_iter=5000)
        return 0.5 * torch.sum((u - ut) ** 2)

    return w, params, loss, ut


def _check_fd(w, loss, ns, nf):
    import torch

    s = T(w.extra["s"]).requires_grad_(True)
    f = T(w.bu).requires_grad_(True)
    L = loss(s, f)
    L.backward()
    gs, gf = s.grad.detach(), f.grad.detach()
    ds, df = W.fd_directions(5000, w.layout, max(ns, nf))
    eps = 1e-6
    worst = 0.0
    gn_s, gn_f = float(torch.linalg.norm(gs)), float(torch.linalg.norm(gf))
    with torch.no_grad():
        for i in range(ns):
            d = T(ds[i])
            fd = (float(loss(s + eps * d, f)) - float(loss(s - eps * d, f))) / (2 * eps)
            ad = float(gs @ d)
            err = abs(fd - ad)
            worst = max(worst, err / gn_s)
            assert err <= FD_TOL_REL * abs(fd) + FD_TOL_ABS * gn_s, (i, fd, ad)
        for i in range(nf):
            d = T(df[i])
            fd = (float(loss(s, f + eps * d)) - float(loss(s, f - eps * d))) / (2 * eps)
            ad = float(gf @ d)
            err = abs(fd - ad)
            worst = max(worst, err / gn_f)
            assert err <= FD_TOL_REL * abs(fd) + FD_TOL_ABS * gn_f, (i, fd, ad)
    print(f"  worst |FD - adjoint| / |gradient| {worst:.2e}", flush=True)
    return gs, gf


@pytest.mark.parametrize("precision", [W.FP64, W.MG_FP32])
def test_autograd_matches_fd_and_oracle_small(precision):
    print(f"autograd small precision={precision}", flush=True)
    w, params, loss, ut = _setup(16, precision)
    gs, gf = _check_fd(w, loss, 6, 6)
    # oracle FP64 adjoint on the same problem
    o = oracle.Oracle(rho=w.rho, mu=np.exp(w.extra["s"]), **dict(params, precision=W.FP64,
                                                                  krylov=W.GMRES_LEFT))
    ou, op, _, _ = o.solve(w.bu, w.bp, tol=1e-13, max_iter=5000)
    adj = o.adjoint(ou, op, ou - N(ut), np.zeros(w.layout.ncell), tol=1e-13, max_iter=5000)
    mu = np.exp(w.extra["s"])
    assert rel(N(gs), adj["dmu_cell"] * mu) <= 1e-6
    assert rel(N(gf), adj["lu"]) <= 1e-6


@pytest.mark.parametrize("precision,ns,nf", [(W.FP64, 20, 20), (W.MG_FP32, 20, 20)])
def test_autograd_full_size_fd(precision, ns, nf):
    """The 128^3 no-slip unsteady workload with mu = exp(s), s a smoothed
    Gaussian field: gradients in s and in the forcing against central
    differences on seeded directions."""
    print(f"autograd 128^3 precision={precision}", flush=True)
    w, params, loss, ut = _setup(128, precision)
    _check_fd(w, loss, ns, nf)
