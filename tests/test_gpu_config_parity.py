"""Parity at the workloads' own scale, against the FP64 oracle:

  - the 1e6-contrast periodic steady field (the headline workload's
    coefficients) at 32^3: iteration counts within +-1 for left GMRES and
    FGMRES in FP64, and the FP32-multigrid form's iteration penalty and error;
    at 64^3 the same for FGMRES;
  - the headline workload itself at 256^3: the FP64 FGMRES iterate after a
    fixed number of Arnoldi steps, element for element;
  - the two-layer unsteady workload at 128^3, both forms solved to 1e-8 and
    their error against the oracle's FP64 solution stated;
  - the adjoint workload at 64^3: adjoint velocity and gradients within 1e-6
    of the oracle's FP64 adjoint, both forms.

The oracle takes tens of seconds to minutes at these sizes, so each test
carries its own time limit.
"""
import numpy as np
import pytest

import oracle
from gpu_common import N, T, pair, rel, scaled_residual
from paper_1308_4605_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
@pytest.mark.parametrize("krylov", [W.GMRES_LEFT, W.FGMRES])
def test_contrast_1e6_iteration_parity_32(krylov):
    print(f"contrast 1e6 32^3 krylov={krylov}", flush=True)
    w = W.contrast_periodic_3d(n=32, contrast=1e6, precision=W.FP64)
    p = w.params(krylov=krylov, precision=W.FP64)
    g, o = pair(p, w.rho, w.mu)
    xu, xp, st, rc = g.solve(T(w.bu), T(w.bp), tol=1e-8, max_iter=3000)
    ou, op, ost, orc = o.solve(w.bu, w.bp, tol=1e-8, max_iter=3000)
    eu, ep = rel(N(xu), ou), rel(N(xp), op)
    print(f"  gpu iters {st['iters']} oracle iters {ost['iters']} err u {eu:.2e} p {ep:.2e}",
          flush=True)
    assert rc == 0 and orc == 0
    assert abs(st["iters"] - ost["iters"]) <= 1
    assert scaled_residual(o, o.c, w.bu, w.bp, N(xu), N(xp)) <= 1e-8 * (1 + 1e-6)
    assert eu <= 1e-6 and ep <= 1e-6
    if krylov == W.FGMRES:
        # the FP32-multigrid form of the same solve: its iteration penalty and
        # its error against the FP64 oracle
        g32, _ = pair(dict(p, precision=W.MG_FP32), w.rho, w.mu)
        yu, yp, st32, rc32 = g32.solve(T(w.bu), T(w.bp), tol=1e-8, max_iter=3000)
        e32u, e32p = rel(N(yu), ou), rel(N(yp), op)
        print(f"  fp32-mg iters {st32['iters']} (oracle fp64 {ost['iters']}) err u {e32u:.2e} "
              f"p {e32p:.2e}", flush=True)
        assert rc32 == 0
        assert scaled_residual(o, o.c, w.bu, w.bp, N(yu), N(yp)) <= 1e-8 * (1 + 1e-6)
        assert st32["iters"] <= 1.05 * ost["iters"] + 3
        assert e32u <= 1e-5 and e32p <= 1e-5


@pytest.mark.timeout(900)
def test_contrast_1e6_iteration_parity_64():
    """The same field at 64^3 with FGMRES(10): the FP64 GPU solve within +-1
    iteration of the oracle, and both GPU forms' errors against the oracle's
    solution."""
    print("contrast 1e6 64^3 FGMRES", flush=True)
    w = W.contrast_periodic_3d(n=64, contrast=1e6, precision=W.FP64)
    p = w.params(krylov=W.FGMRES, precision=W.FP64)
    g, o = pair(p, w.rho, w.mu)
    xu, xp, st, rc = g.solve(T(w.bu), T(w.bp), tol=1e-8, max_iter=3000)
    ou, op, ost, orc = o.solve(w.bu, w.bp, tol=1e-8, max_iter=3000)
    eu, ep = rel(N(xu), ou), rel(N(xp), op)
    print(f"  gpu iters {st['iters']} oracle iters {ost['iters']} err u {eu:.2e} p {ep:.2e}",
          flush=True)
    assert rc == 0 and orc == 0
    assert abs(st["iters"] - ost["iters"]) <= 1
    assert eu <= 1e-6 and ep <= 1e-6
    g32, _ = pair(dict(p, precision=W.MG_FP32), w.rho, w.mu)
    yu, yp, st32, rc32 = g32.solve(T(w.bu), T(w.bp), tol=1e-8, max_iter=3000)
    e32u, e32p = rel(N(yu), ou), rel(N(yp), op)
    print(f"  fp32-mg iters {st32['iters']} err u {e32u:.2e} p {e32p:.2e}", flush=True)
    assert rc32 == 0
    assert scaled_residual(o, o.c, w.bu, w.bp, N(yu), N(yp)) <= 1e-8 * (1 + 1e-6)
    assert st32["iters"] <= 1.05 * ost["iters"] + 3
    assert e32u <= 1e-5 and e32p <= 1e-5


@pytest.mark.timeout(900)
def test_contrast_256_fixed_iterations_fp64():
    """The headline workload at full size: three FGMRES(10) steps with the P2
    preconditioner in FP64 on both sides; the iterates agree element for
    element (norm-wise 1e-9) and so do the true residuals."""
    print("contrast 256^3 fixed iterations fp64", flush=True)
    w = W.contrast_periodic_3d(n=256, precision=W.FP64)
    p = w.params(precision=W.FP64, krylov=W.FGMRES)
    g, o = pair(p, w.rho, w.mu)
    k = 3
    xu, xp, st, rc = g.solve(T(w.bu), T(w.bp), tol=1e-12, max_iter=k, check=False)
    print(f"  gpu rc {rc} res {st['rel_res_true']:.6e}", flush=True)
    ou, op, ost, orc = o.solve(w.bu, w.bp, tol=1e-12, max_iter=k, check=False)
    eu, ep = rel(N(xu), ou), rel(N(xp), op)
    print(f"  oracle rc {orc} res {ost['rel_res_true']:.6e}; iterate err u {eu:.2e} p {ep:.2e}",
          flush=True)
    assert rc == orc == oracle.ORC_ENOCONV and st["iters"] == ost["iters"] == k
    assert eu <= 1e-9 and ep <= 1e-9
    assert abs(st["rel_res_true"] - ost["rel_res_true"]) <= 1e-9 * ost["rel_res_true"]


@pytest.mark.timeout(1200)
def test_layers_128_both_forms_against_oracle():
    """The two-layer unsteady no-slip workload at 128^3 (P1): the plain FP64
    solver (left GMRES) and the FP32-multigrid / FP64-FGMRES form, each solved
    to 1e-8, against the oracle's FP64 solution."""
    print("layers 128^3 both forms", flush=True)
    from paper_1308_4605_amd.stokes import Stokes

    w = W.layers_3d(n=128, precision=W.FP64)
    p64 = w.params(precision=W.FP64, krylov=W.GMRES_LEFT)
    o = oracle.Oracle(rho=w.rho, mu=w.mu, **p64)
    ou, op, ost, orc = o.solve(w.bu, w.bp, tol=1e-8, max_iter=3000)
    assert orc == 0
    print(f"  oracle iters {ost['iters']}", flush=True)
    for prec, kry in ((W.FP64, W.GMRES_LEFT), (W.MG_FP32, W.FGMRES)):
        S = Stokes(w.params(precision=prec, krylov=kry), T(w.rho), T(w.mu))
        xu, xp, st, rc = S.solve(T(w.bu), T(w.bp), tol=1e-8, max_iter=3000)
        eu, ep = rel(N(xu), ou), rel(N(xp), op)
        r = scaled_residual(o, o.c, w.bu, w.bp, N(xu), N(xp))
        print(f"  precision {prec}: iters {st['iters']} err u {eu:.2e} p {ep:.2e} "
              f"oracle-checked residual {r:.2e}", flush=True)
        assert rc == 0 and r <= 1e-8 * (1 + 1e-6)
        if prec == W.FP64:
            assert abs(st["iters"] - ost["iters"]) <= 1
            assert eu <= 1e-6 and ep <= 1e-6
        else:
            assert eu <= 1e-5 and ep <= 1e-5
        S.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,krylov", [(W.FP64, W.GMRES_LEFT), (W.MG_FP32, W.FGMRES)])
def test_adjoint_parity_64(precision, krylov):
    """Adjoint solve and strain contraction on the adjoint workload at 64^3,
    within 1e-6 of the oracle's FP64 adjoint (all solves to 1e-12)."""
    print(f"adjoint 64^3 precision={precision}", flush=True)
    w = W.adjoint_3d(n=64)
    p = w.params(precision=precision, krylov=krylov)
    g, _ = pair(p, w.rho, w.mu)
    po = dict(p, precision=W.FP64, krylov=W.GMRES_LEFT)
    o = oracle.Oracle(rho=w.rho, mu=w.mu, **po)
    ou, op, _, _ = o.solve(w.bu, w.bp, tol=1e-12, max_iter=3000)
    target = w.extra["bu2"]
    xu, xp, st, rc = g.solve(T(w.bu), T(w.bp), tol=1e-12, max_iter=3000)
    ga = g.adjoint(xu, xp, T(N(xu) - target), T(np.zeros(w.layout.ncell)), tol=1e-12,
                   max_iter=3000)
    oa = o.adjoint(ou, op, ou - target, np.zeros(w.layout.ncell), tol=1e-12, max_iter=3000)
    for k in ("lu", "dmu_cell", "dmu_edge", "drho_cell"):
        r = rel(N(ga[k]), oa[k])
        print(f"  {k} rel {r:.2e}", flush=True)
        assert r <= 1e-6, k
