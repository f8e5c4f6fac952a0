"""Test-side helpers: dense assembly of the oracle's operators from unit
vectors, and textbook operators built independently (Kronecker sums of 1D
second-difference matrices) to pin the oracle against."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from paper_1308_4605_amd import workloads as W


def interior_index(lay: W.Layout):
    """Indices of the unknowns in a flat [velocity | pressure] vector."""
    wm = lay.wall_mask()
    vel = np.nonzero(~wm)[0]
    pr = lay.nvel + np.arange(lay.ncell)
    return vel, pr


def assemble(o, lay: W.Layout):
    """Dense M over the unknowns (interior faces then cells) from o.apply."""
    vel, pr = interior_index(lay)
    idx = np.concatenate([vel, pr])
    N = len(idx)
    M = np.zeros((N, N))
    x = np.zeros(lay.nvel + lay.ncell)
    for j, q in enumerate(idx):
        x[:] = 0.0
        x[q] = 1.0
        yu, yp = o.apply(x[: lay.nvel], x[lay.nvel:])
        y = np.concatenate([yu, yp])
        M[:, j] = y[idx]
    return M, len(vel)


def second_diff_1d(n, h, kind):
    """1D second-difference matrices.
    kind = 'periodic'   : circulant (1, -2, 1)/h^2 on n points;
           'dirichlet'  : n-1 interior nodes of a vertex grid with zero ends;
           'wall_cc'    : n cell-centred points, zero value on the walls half a
                          cell outside (ghost = -adjacent: ends -3);
           'neumann_cc' : n cell-centred points, zero flux at the walls (ends -1)."""
    if kind == "periodic":
        m = n
        A = sp.diags([np.ones(m - 1), -2 * np.ones(m), np.ones(m - 1)], [-1, 0, 1]).tolil()
        A[0, m - 1] += 1.0
        A[m - 1, 0] += 1.0
    elif kind == "dirichlet":
        m = n - 1
        A = sp.diags([np.ones(m - 1), -2 * np.ones(m), np.ones(m - 1)], [-1, 0, 1]).tolil()
    elif kind == "wall_cc":
        m = n
        A = sp.diags([np.ones(m - 1), -2 * np.ones(m), np.ones(m - 1)], [-1, 0, 1]).tolil()
        A[0, 0] = -3.0
        A[m - 1, m - 1] = -3.0
    elif kind == "neumann_cc":
        m = n
        A = sp.diags([np.ones(m - 1), -2 * np.ones(m), np.ones(m - 1)], [-1, 0, 1]).tolil()
        A[0, 0] = -1.0
        A[m - 1, m - 1] = -1.0
    elif kind in ("wall_neumann_cc", "neumann_wall_cc"):
        # zero value half a cell out at one end, zero flux at the other
        m = n
        A = sp.diags([np.ones(m - 1), -2 * np.ones(m), np.ones(m - 1)], [-1, 0, 1]).tolil()
        lo, hi = (-3.0, -1.0) if kind == "wall_neumann_cc" else (-1.0, -3.0)
        A[0, 0] = lo
        A[m - 1, m - 1] = hi
    else:
        raise ValueError(kind)
    return (A.tocsr() / (h * h))


def kron_sum(mats):
    """sum_a I x ... x T_a x ... x I with mats ordered (x, y[, z]) and the
    flattened order x fastest (so z is the slowest Kronecker factor)."""
    dims = [m.shape[0] for m in mats]
    total = None
    for a, T in enumerate(mats):
        ops = []
        for b in reversed(range(len(mats))):
            ops.append(T if b == a else sp.identity(dims[b], format="csr"))
        K = ops[0]
        for o in ops[1:]:
            K = sp.kron(K, o, format="csr")
        total = K if total is None else total + K
    return total


def textbook_vector_laplacian(lay: W.Layout, h):
    """Laplace-form vector Laplacian per component (no coupling), on the
    interior unknowns of each component, with the wall rules (normal
    direction: Dirichlet nodes; tangential: zero wall value half a cell out
    at no-slip walls, zero normal derivative at free-slip walls)."""
    blocks = []
    for k in range(lay.dim):
        mats = []
        for a in range(lay.dim):
            n = lay.n[a]
            if lay.bc[a] == W.PERIODIC:
                mats.append(second_diff_1d(n, h, "periodic"))
            elif a == k:
                mats.append(second_diff_1d(n, h, "dirichlet"))
            else:
                lo, hi = (W.end_is_noslip(lay.bc[a], s) for s in (0, 1))
                kind = {(True, True): "wall_cc", (False, False): "neumann_cc",
                        (True, False): "wall_neumann_cc", (False, True): "neumann_wall_cc"}[(lo, hi)]
                mats.append(second_diff_1d(n, h, kind))
        blocks.append(kron_sum(mats))
    return sp.block_diag(blocks, format="csr").toarray()


def textbook_cell_laplacian(lay: W.Layout, h):
    mats = []
    for a in range(lay.dim):
        kind = "periodic" if lay.bc[a] == W.PERIODIC else "neumann_cc"
        mats.append(second_diff_1d(lay.n[a], h, kind))
    return kron_sum(mats).toarray()


def blocks(M, nv):
    return M[:nv, :nv], M[:nv, nv:], M[nv:, :nv], M[nv:, nv:]


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
