"""torch.autograd wrapper of the Stokes solve with the hand-written adjoint.

forward:  (mu_cell, rho_cell, f_u[, gamma_cell, b_p, mu_edge]) -> (u, p), the
          solution of M x = (f_u, b_p) (b_p = -g, zero when not given); with
          gamma_cell the stress carries the bulk-viscosity term
          (gamma - 2/3 mu)(div u) I; mu_edge is the edge (3D) / node (2D)
          viscosity when the parameters ask for given edges (STOKES_EDGE_GIVEN)
backward: one adjoint solve M lambda = (dL/du, dL/dp) with the same
          preconditioner and a fresh Krylov space (M = M^T), then the
          strain-contraction kernel; the Krylov basis of the forward solve is
          not kept.  dL/df = lambda_u, dL/db_p = lambda_p; dL/dmu_cell,
          dL/dmu_edge, dL/drho_cell and dL/dgamma_cell come from the library
          (the chain rule through derived edge viscosities included).

All arithmetic runs in libstokes_mi355x.so; this file only marshals tensors.
Parametrisations such as mu = exp(s) are ordinary torch ops in the caller's
graph.
"""
from __future__ import annotations

import torch

from .stokes import Stokes


class StokesSolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu_cell, rho_cell, f_u, gamma_cell, b_p, mu_edge, params, tol=1e-10,
                max_iter=2000):
        gamma = None if gamma_cell is None else gamma_cell.detach().contiguous()
        edges = None if mu_edge is None else mu_edge.detach().contiguous()
        S = Stokes(params, rho_cell.detach().contiguous(), mu_cell.detach().contiguous(),
                   edges, gamma=gamma)
        if b_p is None:
            bp = torch.zeros(S.ncell, dtype=torch.float64, device=f_u.device)
        else:
            bp = b_p.detach().contiguous()
        xu, xp, st, rc = S.solve(f_u.detach().contiguous(), bp, tol=tol, max_iter=max_iter)
        ctx.S = S
        ctx.tol, ctx.max_iter = tol, max_iter
        ctx.stats = st
        ctx.save_for_backward(xu, xp)
        return xu, xp

    @staticmethod
    def backward(ctx, gu, gp):
        xu, xp = ctx.saved_tensors
        S = ctx.S
        if gu is None:
            gu = torch.zeros_like(xu)
        if gp is None:
            gp = torch.zeros_like(xp)
        res = S.adjoint(xu, xp, gu.contiguous(), gp.contiguous(), tol=ctx.tol,
                        max_iter=ctx.max_iter)
        ctx.adjoint_stats = res["stats"]
        dgamma = res.get("dgamma_cell") if ctx.needs_input_grad[3] else None
        dbp = res["lp"] if ctx.needs_input_grad[4] else None
        dedge = res["dmu_edge"] if ctx.needs_input_grad[5] else None
        return (res["dmu_cell"], res["drho_cell"], res["lu"], dgamma, dbp, dedge, None, None,
                None)


def stokes_solve(mu_cell, rho_cell, f_u, params, tol=1e-10, max_iter=2000, gamma_cell=None,
                 b_p=None, mu_edge=None):
    """Differentiable solve: returns (u, p).  gamma_cell: bulk viscosity (or
    None); b_p: pressure right-hand side -g for div u = g (or None = 0);
    mu_edge: given edge viscosity (params edge_avg = STOKES_EDGE_GIVEN)."""
    return StokesSolveFn.apply(mu_cell, rho_cell, f_u, gamma_cell, b_p, mu_edge, params, tol,
                               max_iter)
