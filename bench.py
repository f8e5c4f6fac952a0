#!/usr/bin/env python3
"""Benchmark: Stokes solves/s to a 1e-8 true relative residual on one MI355X.

One step = one full solve (block-preconditioned flexible GMRES(10) with one
FP32 multigrid V-cycle per subsolver, FP64 Krylov/M/residuals) of the 3D
periodic steady workload with a 1e6 viscosity contrast on 256^3 cells, inputs
resident in HBM.  The plain FP64 solver (same preconditioner, FP64 multigrid)
is timed beside it, and the FP32-MG solution is compared with the FP64 one.

The JSON line also carries
  - roofline: the finest-level velocity Gauss-Seidel colour pass (the
    dominant kernel), algorithmic bytes per launch / average launch time,
    timed with HIP events on the solver's stream during one more solve after
    the timed ones (the events stay out of the timed region);
  - vcycle_aggregate: whole finest-level V-cycles (velocity, pressure when
    the preconditioner runs one), their algorithmic bytes over all levels /
    their time, from HIP events on the solver's stream;
  - cpu_baseline: the FP64 CPU oracle on a bounded sample of the same
    workload (one Arnoldi step), scaled to solves/s with the iteration count
    of the FP64 solve, plus fully measured oracle solves (the 2D periodic
    32^2 workload, median of 3 on all threads and on one thread, and the
    headline coefficients at 32^3) and the CPU model;
  - oracle_parity: the GPU solutions' error against the oracle's FP64
    solution on those measured inputs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
KERNEL_SRC = os.path.join(ROOT, "paper_1308_4605_amd", "csrc", "stokes_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_vel_gs_3d-periodic-contrast-256.json")


def _kernel_source_sha():
    import hashlib

    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _measured_traffic(n):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None when it was taken on other kernel
    source or another size."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != _kernel_source_sha() or t.get("n") != n:
        return None
    return t.get("hbm_bytes_per_launch")


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _adjoint_timing(torch, dev, W, Stokes, n=128, reps=2):
    """Forward solve + adjoint solve with gradients on the 128^3 no-slip
    unsteady workload (mu = exp(s)), loss 1/2 ||u - u_target||^2, in the FP64
    and FP32-multigrid forms; the FP32-MG gradient is compared with FP64."""
    w = W.adjoint_3d(n=n)
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    rho, mu, bu, bp = T(w.rho), T(w.mu), T(w.bu), T(w.bp)
    out, grads = {}, {}
    for name, prec, kry in (("fp64", W.FP64, W.GMRES_LEFT), ("fp32mg", W.MG_FP32, W.FGMRES)):
        S = Stokes(w.params(precision=prec, krylov=kry), rho, mu)
        S2 = Stokes(w.params(precision=prec, krylov=kry), rho, T(np.exp(w.extra["s2"])))
        ut, _, _, _ = S2.solve(T(w.extra["bu2"]), bp, tol=1e-10)
        S2.close()
        res = None
        for r in range(reps + 1):  # first repetition is a warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xu, xp, st, _ = S.solve(bu, bp, tol=1e-10)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            res = S.adjoint(xu, xp, xu - ut, torch.zeros_like(xp), tol=1e-10)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        out[name] = {"forward_ms": 1e3 * (t1 - t0), "adjoint_ms": 1e3 * (t2 - t1),
                     "forward_iters": st["iters"], "adjoint_iters": res["stats"]["iters"]}
        grads[name] = res["dmu_cell"] * mu  # dL/ds with mu = exp(s)
        S.close()
    out["workload"] = f"3d-noslip-adjoint-{n}"
    out["tol"] = 1e-10
    out["fp32mg_vs_fp64_grad_rel_diff"] = float(torch.linalg.norm(grads["fp32mg"] - grads["fp64"])
                                                / torch.linalg.norm(grads["fp64"]))
    _log(f"adjoint: {out}")
    return out


def _split_baseline(torch, dev, Stokes, params, rho, mu, bu, bp, tol, coupled_sv):
    """One projection step with the multigrid solvers run to the same
    tolerance (the split-method reference of the V-cycle study):
    u* = A^{-1} b_u, then phi = L_rho^{-1}(-(D u* + b_p)); scalar V-cycles
    d * velocity cycles + pressure cycles, against the coupled solve's."""
    S = Stokes(params, rho, mu)
    S.vel_mg_solve(bu, tol=tol, max_cycles=500)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    us, cv, qv, rcv = S.vel_mg_solve(bu, tol=tol, max_cycles=500)
    _, mdu = S.apply(us, torch.zeros_like(bp))  # pressure part of M [u*; 0] is -D u*
    _, cp, qp, rcp = S.p_mg_solve(mdu - bp, tol=tol, max_cycles=500)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0)
    S.close()
    sv = params["dim"] * cv + cp
    out = {"velocity_cycles": cv, "pressure_cycles": cp, "scalar_vcycles": sv, "ms": ms,
           "rel_res": [qv, qp], "converged": rcv == 0 and rcp == 0,
           "coupled_scalar_vcycles": coupled_sv, "coupled_over_split": coupled_sv / sv}
    _log(f"split baseline: {out}")
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_measured(torch, dev, W, Stokes, tol):
    """Fully measured oracle solves (not extrapolated), with the GPU forms
    compared against the oracle's FP64 solution on the same inputs:
      - the 2D periodic 32^2 workload (P1, left GMRES): median of 3 oracle
        solves on all threads and on one thread, and the GPU solve beside it;
      - the headline workload's coefficients (contrast 1e6, P2, FGMRES) at
        32^3: one oracle solve, and the FP32-multigrid and FP64 GPU solves'
        error against it."""
    import oracle

    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    rel = lambda a, b: float(np.linalg.norm(a.cpu().numpy() - b) / np.linalg.norm(b))
    nthreads = oracle.threads()
    out = {"cores": nthreads, "cpu_model": _cpu_model()}

    w1 = W.periodic_smooth_2d(n=32)
    o1 = oracle.Oracle.from_workload(w1)

    def med3():
        ts = []
        for _ in range(3):
            t = time.perf_counter()
            ou, op, ost, _ = o1.solve(w1.bu, w1.bp, tol=tol)
            ts.append(time.perf_counter() - t)
        return sorted(ts)[1], ou, op, ost

    t_all, ou1, op1, ost1 = med3()
    oracle.set_threads(1)
    t_one, _, _, _ = med3()
    oracle.set_threads(nthreads)
    S1 = Stokes(w1.params(), T(w1.rho), T(w1.mu))
    S1.solve(T(w1.bu), T(w1.bp), tol=tol)
    gts = []
    for _ in range(5):
        torch.cuda.synchronize()
        t = time.perf_counter()
        xu, xp, st1, _ = S1.solve(T(w1.bu), T(w1.bp), tol=tol)
        torch.cuda.synchronize()
        gts.append(time.perf_counter() - t)
    S1.close()
    out["2d-periodic-smooth-32"] = {
        "oracle_s_median_of_3": t_all, "oracle_s_1_thread_median_of_3": t_one,
        "oracle_iters": ost1["iters"], "gpu_s_median_of_5": sorted(gts)[2],
        "gpu_iters": st1["iters"], "gpu_rel_err_u": rel(xu, ou1), "gpu_rel_err_p": rel(xp, op1)}

    w4 = W.contrast_periodic_3d(n=32, precision=W.FP64)
    p4 = w4.params(precision=W.FP64, krylov=W.FGMRES)
    o4 = oracle.Oracle(rho=w4.rho, mu=w4.mu, **p4)
    t = time.perf_counter()
    ou, op, ost, _ = o4.solve(w4.bu, w4.bp, tol=tol, max_iter=3000)
    t4 = time.perf_counter() - t
    del o4
    rec = {"oracle_s": t4, "oracle_iters": ost["iters"]}
    for name, prec in (("fp32mg", W.MG_FP32), ("fp64", W.FP64)):
        S = Stokes(dict(p4, precision=prec), T(w4.rho), T(w4.mu))
        xu, xp, st, _ = S.solve(T(w4.bu), T(w4.bp), tol=tol, max_iter=3000)
        rec[name] = {"iters": st["iters"], "rel_err_u": rel(xu, ou), "rel_err_p": rel(xp, op)}
        S.close()
    out["3d-periodic-contrast-32"] = rec
    _log(f"oracle measured: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="cells per axis (default: the 256^3 workload)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle sample")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 solver")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with a plain 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--profile-solve", action="store_true",
                    help="only one FP32-multigrid solve of the workload (then the calibration "
                         "copy if asked), no JSON line: the program the counter runs profile")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is designed but not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1308_4605_amd import workloads as W
    from paper_1308_4605_amd.stokes import Stokes

    if not torch.cuda.is_available():
        print("bench.py: no HIP device visible", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")

    t0 = time.time()
    w = W.contrast_periodic_3d(n=args.n, precision=W.MG_FP32)
    _log(f"workload {w.name} n={args.n} generated in {time.time() - t0:.1f}s")
    lay = w.layout
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    rho, mu, bu, bp = T(w.rho), T(w.mu), T(w.bu), T(w.bp)

    if args.profile_solve:
        S = Stokes(w.params(precision=W.MG_FP32, krylov=W.FGMRES), rho, mu)
        _, _, st, rc = S.solve(bu, bp, tol=args.tol, max_iter=3000)
        torch.cuda.synchronize()
        _log(f"profiled solve: rc {rc}, iters {st['iters']}, rel_res {st['rel_res_true']:.2e}")
        S.close()
        if args.calib_copy:
            _calibration_copy(torch, dev)
        return

    def timed_solves(params, steps, warmup, timing):
        S = Stokes(params, rho, mu)
        xu = torch.empty(S.nvel, dtype=torch.float64, device=dev)
        xp = torch.empty(S.ncell, dtype=torch.float64, device=dev)
        st = None
        for i in range(warmup):
            _, _, st, rc = S.solve(bu, bp, tol=args.tol, max_iter=3000, out=(xu, xp))
            _log(f"warmup {i}: iters {st['iters']} rel_res {st['rel_res_true']:.2e}")
        torch.cuda.synchronize()
        t = time.perf_counter()
        its = []
        for i in range(steps):
            _, _, st, rc = S.solve(bu, bp, tol=args.tol, max_iter=3000, out=(xu, xp))
            its.append(st["iters"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        kt = None
        if timing:
            # two more solves outside the timed region: per-launch events for
            # the colour-pass bandwidth, then per-V-cycle events only (the
            # V-cycles as the timed solves run them) for the V-cycle rate
            S.set_timing(1)
            S.solve(bu, bp, tol=args.tol, max_iter=3000, out=(xu, xp))
            k = S.kernel_time()
            S.set_timing(2)
            S.solve(bu, bp, tol=args.tol, max_iter=3000, out=(xu, xp))
            kt = (k, S.vcycle_time(False), S.vcycle_time(True))
            S.set_timing(0)
        S.close()
        return el, st, its, kt, xu, xp

    p32 = w.params(precision=W.MG_FP32, krylov=W.FGMRES)
    el, st, its, kt, xu32, xp32 = timed_solves(p32, args.steps, args.warmup, True)
    ms_per_step = 1e3 * el / args.steps
    value = args.steps / el
    _log(f"FP32-MG FGMRES: {ms_per_step:.1f} ms/solve, iters {its}, rel_res {st['rel_res_true']:.2e}")

    split = _split_baseline(torch, dev, Stokes, p32, rho, mu, bu, bp, args.tol, st["scalar_vcycles"])

    (ms_k, launches, bytes_k), vc_vel, vc_p = kt
    avg_ms = ms_k / max(launches, 1)

    def vcycle_rate(t):
        ms, cycles, nbytes = t
        if cycles == 0:
            return None
        gbs = nbytes / (ms * 1e-3) / 1e9
        return {"cycles": cycles, "avg_ms": ms / cycles, "alg_bytes_per_cycle": nbytes / cycles,
                "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}

    vcycles = {"velocity": vcycle_rate(vc_vel), "pressure": vcycle_rate(vc_p),
               "note": "whole V-cycles from the finest level (all levels, the finest "
                       "level's cycle replayed as its recorded HIP graph), HIP events on the "
                       "solver stream; algorithmic bytes = every array each kernel reads or "
                       "writes, once per kernel"}
    achieved = (bytes_k / max(launches, 1)) / (avg_ms * 1e-3) / 1e9 if launches else 0.0

    fp64 = None
    if not args.no_fp64:
        p64 = w.params(precision=W.FP64, krylov=W.FGMRES)
        el64, st64, its64, _, xu64, xp64 = timed_solves(p64, max(1, args.steps - 1), 1, False)
        n64 = max(1, args.steps - 1)
        err_u = float(torch.linalg.norm(xu32 - xu64) / torch.linalg.norm(xu64))
        err_p = float(torch.linalg.norm(xp32 - xp64) / torch.linalg.norm(xp64))
        fp64 = {"solves_per_s": n64 / el64, "ms_per_solve": 1e3 * el64 / n64, "iters": its64[-1],
                "rel_res_true": st64["rel_res_true"],
                "fp32mg_vs_fp64_rel_err_u": err_u, "fp32mg_vs_fp64_rel_err_p": err_p}
        _log(f"FP64 FGMRES: {fp64['ms_per_solve']:.1f} ms/solve, iters {its64}, "
             f"err u {err_u:.2e} p {err_p:.2e}")
        del xu64, xp64

    adjoint = None
    if not args.no_adjoint:
        adjoint = _adjoint_timing(torch, dev, W, Stokes)

    cpu = None
    if not args.no_cpu:
        import oracle

        o = oracle.Oracle.from_workload(w, precision=W.FP64, krylov=W.FGMRES)
        k_it = 1
        t = time.perf_counter()
        o.solve(w.bu, w.bp, tol=args.tol, max_iter=k_it, check=False)
        t_cpu = time.perf_counter() - t
        iters_ref = fp64["iters"] if fp64 else st["iters"]
        cpu = {"value": 1.0 / (t_cpu / k_it * iters_ref), "unit": "solves/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"FP64 oracle FGMRES(10)+P2 on the same {args.n}^3 workload, {k_it} Arnoldi "
                         f"step(s) plus the two true-residual evaluations ({t_cpu:.1f} s), scaled by "
                         f"the {iters_ref} iterations of the FP64 solve"}
        _log(f"CPU oracle: {t_cpu:.1f}s for {k_it} iteration(s) on {cpu['cores']} threads")
        del o
        # fully measured oracle solves beside the extrapolation, and the GPU
        # forms' error against the oracle on those inputs
        cpu["measured"] = _oracle_measured(torch, dev, W, Stokes, args.tol)
        cpu["cpu_model"] = cpu["measured"]["cpu_model"]

    # device copy ceiling: a plain 1 GiB read + 1 GiB write on the same GPU
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * (1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    _log(f"device copy: {copy_gbs:.0f} GB/s")

    sv = st["scalar_vcycles"]
    line = {
        "metric": "Stokes solves/s to 1e-8 rel resid (FP32-MG in FP64 FGMRES)",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 multigrid / f64 krylov",
        "data": "synthetic",
        "config": {"workload": f"3d-periodic-contrast-{args.n}", "grid": f"{args.n}^3",
                   "bc": "periodic", "theta": 0.0, "viscosity_contrast": 1e6, "precond": "P2",
                   "krylov": "FGMRES(10)", "vcycles_per_subsolve": 1, "tol": args.tol},
        "iters": st["iters"],
        "scalar_vcycles_per_solve": sv,
        "scalar_vcycles_per_s": sv * value,
        "rel_res_true": st["rel_res_true"],
        "fp64": fp64,
        "speedup_fp32mg_vs_fp64": (value / fp64["solves_per_s"]) if fp64 else None,
        "roofline": {"kernel": "velocity Gauss-Seidel colour pass, finest level (k_vel_gs)",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": _measured_traffic(args.n),
                     "copy_ceiling": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "avg_launch_us": 1e3 * avg_ms, "launches": launches,
                     "bytes_per_launch": bytes_k / max(launches, 1)},
        "vcycle_aggregate": vcycles,
        "split_baseline": split,
        "adjoint": adjoint,
        "cpu_baseline": cpu,
        "oracle_parity": None if cpu is None else {
            "note": "GPU solutions against the FP64 oracle's solution on the same inputs "
                    "(relative 2-norm error), from cpu_baseline.measured",
            "3d-periodic-contrast-32": cpu["measured"]["3d-periodic-contrast-32"],
            "2d-periodic-smooth-32": {k: cpu["measured"]["2d-periodic-smooth-32"][k]
                                      for k in ("gpu_iters", "oracle_iters", "gpu_rel_err_u",
                                                "gpu_rel_err_p")}},
    }
    print(json.dumps(line), flush=True)
    if args.calib_copy:
        _calibration_copy(torch, dev)


def _calibration_copy(torch, dev):
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    _log("calibration copy: 1 GiB read + 1 GiB write")


if __name__ == "__main__":
    main()
