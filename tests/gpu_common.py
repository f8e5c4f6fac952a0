"""Shared helpers of the GPU parity tests (test infrastructure)."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1308_4605_amd import workloads as W


def dev():
    import torch

    return torch.device("cuda:0")


def T(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev())


def N(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def params(dim, n, bc, theta, **kw):
    lay = W.make_layout(dim, n, bc)
    p = dict(dim=dim, n=lay.n, bc=lay.bc, h=1.0 / lay.n[0], theta=theta, precond=W.P1,
             precision=W.FP64, krylov=W.GMRES_LEFT, restart=10, nu_pre=2, nu_post=2, nu_coarse=8,
             vcycles=1, rescale_c=0.0, edge_avg=W.EDGE_ARITH)
    p.update(kw)
    return p, lay


def pair(p, rho, mu, edges=None, gamma=None):
    """GPU context and oracle context on identical inputs (gamma: bulk
    viscosity or None)."""
    from paper_1308_4605_amd.stokes import Stokes

    g = Stokes(p, T(rho), T(mu), None if edges is None else T(edges),
               gamma=None if gamma is None else T(gamma))
    o = oracle.Oracle(rho=rho, mu=mu, edges=edges, gamma=gamma, **p)
    return g, o


def scaled_residual(o, c, bu, bp, xu, xp):
    """||b' - M' x'|| / ||b'|| of the rescaled system, with the oracle's M."""
    yu, yp = o.apply(xu, xp)
    ru, rp = c * (bu - yu), bp - yp
    nb = np.sqrt(np.sum((c * bu) ** 2) + np.sum(bp ** 2))
    return float(np.sqrt(np.sum(ru ** 2) + np.sum(rp ** 2)) / nb)
