"""stokes_solve_static (the solve for callers that cannot allocate: its
Krylov storage in the library's static device array) against stokes_solve
on the same contexts, through the C ABI.  Two static calls run back to back,
the second on a smaller grid (so it starts on the first one's leftovers);
both must equal the workspace solve bit for bit (same kernels, same
reduction grids, same order of operations).  A context whose Krylov storage
exceeds the array gets STOKES_ENOMEM before anything is launched."""
import numpy as np
import pytest

from gpu_common import T
from paper_1308_4605_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ctx(w, **over):
    from paper_1308_4605_amd.stokes import Stokes

    return Stokes(w.params(**over), T(w.rho), T(w.mu))


def test_static_solve_equals_workspace_solve_twice():
    import torch

    cases = [
        # larger first: FP32 multigrid inside FGMRES (Z stored in FP32)
        (W.contrast_periodic_3d(n=32, contrast=1e3, precision=W.MG_FP32),
         dict(precision=W.MG_FP32, krylov=W.FGMRES)),
        # then smaller: plain FP64, left GMRES (no Z), no-slip walls
        (W.layers_3d(n=16, precision=W.FP64), dict(precision=W.FP64, krylov=W.GMRES_LEFT)),
    ]
    ctxs = [_ctx(w, **over) for w, over in cases]
    static = []
    for (w, _), S in zip(cases, ctxs):
        print(f"static solve {w.name} n={S.nvel + S.ncell}", flush=True)
        static.append(S.solve_static(T(w.bu), T(w.bp), tol=1e-8, max_iter=2000))
    for (w, _), S, (su, sp, sst, src) in zip(cases, ctxs, static):
        xu, xp, st, rc = S.solve(T(w.bu), T(w.bp), tol=1e-8, max_iter=2000)
        print(f"  {w.name}: static iters {sst['iters']} res {sst['rel_res_true']:.3e}; "
              f"workspace iters {st['iters']} res {st['rel_res_true']:.3e}", flush=True)
        assert src == rc == 0
        assert sst["iters"] == st["iters"] and sst["rel_res_true"] == st["rel_res_true"]
        assert torch.equal(su, xu) and torch.equal(sp, xp)
        S.close()


def test_static_solve_rejects_storage_beyond_the_array():
    from paper_1308_4605_amd.stokes import STOKES_ENOMEM

    lay = W.make_layout(3, (128, 64, 64), (0, 0, 0))
    w = W.Workload(name="too-large", dim=3, n=lay.n, bc=lay.bc, h=1.0 / 128, theta=10.0,
                   precond=W.P1, krylov=W.FGMRES, precision=W.FP64, edge_avg=W.EDGE_ARITH,
                   rho=np.ones(lay.ncell), mu=np.ones(lay.ncell),
                   bu=np.zeros(lay.nvel), bp=np.zeros(lay.ncell))
    S = _ctx(w)
    print(f"static solve beyond the array: n={S.nvel + S.ncell}", flush=True)
    _, _, _, rc = S.solve_static(T(w.bu), T(w.bp), check=False)
    assert rc == STOKES_ENOMEM
    S.close()
