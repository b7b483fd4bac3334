"""Benchmark of the FSE-Shooting hot path on one MI355X.

One step = one pass of the hot path over the von Karman beam workload
(147 DOF, d = 2, 64 trajectories, H = 15, S1 = 512, full sensitivities):
inverse DFT, consistent a_0 / Phi_0, Newmark integration with per-step Newton,
sensitivity propagation, DFT + rotation + residual, and the Jacobian of Eq. (22).
value = trajectory-steps/s = S~ * S1 / (time per step).

Prints ONE JSON line.  Extra fields: the roofline of the dominant kernel (the
fused trajectory kernel: state integration + sensitivity propagation), the FP64
oracle timed on the host cores on a bounded sample, and the shooting solve time to
||R|| < 1e-8 (measured outside the timed region).

`--calibrate-copy` instead times a plain device-to-device copy of known size; its
FETCH_SIZE / WRITE_SIZE counters scale the counters of the fused kernel to bytes.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ARC_POINTS = 10
ARC_DS = 0.5


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-krylov", action="store_true")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "k_fused_c2_traffic.json"))
    ap.add_argument("--calibrate-copy", action="store_true")
    return ap.parse_args()


FUSED_SRC = [os.path.join(ROOT, "paper_2508_06302_amd", "csrc", f) for f in ("k_fused.hip", "band_ldlt.h")]


def fused_source_hash():
    """Hash of the sources the fused kernel is compiled from (counters taken on other
    sources are not used)."""
    h = hashlib.sha256()
    for f in FUSED_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def calibrate_copy():
    """A plain 1 GiB device-to-device copy, run 5 times (the counter-scaling reference)."""
    import torch
    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / 5
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": 5,
                      "GBps_read_plus_write": 2 * nbytes / el / 1e9}), flush=True)


def read_traffic(path):
    """HBM bytes per launch of the fused kernel from counter runs, or None when absent or
    taken on a different kernel source."""
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except Exception:
        return None
    if t.get("k_fused_source_sha256_16") != fused_source_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(wl, Z0, tables, budget_s=20.0):
    """The oracle as it stands on a bounded sample: whole trajectories with sensitivities."""
    from oracle import shooting as osh
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    done = 0
    t0 = time.perf_counter()
    s = 0
    while time.perf_counter() - t0 < budget_s and s < tables.Stilde:
        osh.evaluate(wl.system, wl.torus, wl.omega, Z0, sens=True, tables=tables, samples=[s])
        done += 1
        s += 1
    el = time.perf_counter() - t0
    return {"value": done * wl.torus.S1 / el, "unit": "trajectory-steps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{done} of {tables.Stilde} trajectories of the same workload, each the "
                      f"full {wl.torus.S1}-step integration with sensitivities, {el:.1f} s"}


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_precision(fse, torch, wl, prec, steps, warmup, solve):
    """Throughput of the residual + Jacobian step and the continuation solve in one
    precision mode; returns a dict (kernel times from HIP events on the library stream)."""
    progress(f"precision {prec}: {warmup} warmup + {steps} timed steps")
    tr = wl.torus
    ctx = fse.fse_init_torus(wl.system, tr, precision=prec)
    U, St, bw, kt = fse.fse_get_layout(ctx)
    Z0 = wl.initial_iterate(kt)
    om = wl.omega[None]
    Zd = torch.tensor(Z0[None], dtype=torch.float64, device="cuda")

    def step():
        return fse.fse_shooting_residual_jacobian(ctx, om, Zd, want_J=True)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    kern_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        tm = fse.fse_last_timing(ctx)          # HIP events around the launch, on its stream
        kern_ms.append(tm["state_ms"] + tm["sens_ms"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ncw, tune_ms = fse.fse_get_tuning(ctx)
    res = {"ctx": ctx, "U": U, "St": St, "bw": bw, "Z0": Z0, "ms_per_step": 1e3 * el / steps,
           "tuning": {"column_waves_per_workgroup": ncw, "tuned_launch_ms": [float(x) for x in tune_ms]},
           "value": St * tr.S1 / (el / steps), "kernel_ms": float(np.mean(kern_ms)),
           "fused": tm["sens_launches"] == 1 and tm["sens_ms"] < 0.05 * tm["state_ms"]}
    progress(f"precision {prec}: {res['ms_per_step']:.1f} ms per step")
    if prec == fse.FSE_PREC_FP64:
        # the trajectories alone (states, no sensitivities): same workload and step count
        for _ in range(warmup):
            fse.fse_integrate_batch(ctx, om, Zd)
        torch.cuda.synchronize()
        st_ms = []
        t0 = time.perf_counter()
        for _ in range(steps):
            fse.fse_integrate_batch(ctx, om, Zd)
            st_ms.append(fse.fse_last_timing(ctx)["state_ms"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res["state_only"] = {"value": St * tr.S1 / (el / steps), "unit": "trajectory-steps/s",
                             "ms_per_step": 1e3 * el / steps, "kernel_ms_per_launch": float(np.mean(st_ms))}
        progress(f"precision {prec}: state only {res['state_only']['ms_per_step']:.1f} ms per step")
    if solve:
        # shooting solve: natural-parameter continuation in the forcing amplitude
        # f1 = f2 = 0.1 ... 0.5 N at the same omega, secant predictor, ||R||_2 < 1e-8 per point
        amps = [0.1, 0.2, 0.3, 0.4, 0.5]
        params = np.array([[*wl.omega, a, a] for a in amps])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        try:
            Zs, its, rns = fse.fse_continuation(ctx, params, Z0 * amps[0], tol=1e-8, maxit=15)
            ok = True
        except fse.FseError as ex:
            Zs, its, rns, ok = ex.Z, ex.iters, ex.rnorm, str(ex)
        torch.cuda.synchronize()
        res["solve"] = {"time_s": time.perf_counter() - t1,
                        "newton_iterations": [int(i) for i in its],
                        "final_residuals": [float(r) for r in rns], "converged": ok is True}
        res["Z_solution"] = Zs[-1].clone() if ok is True else None
        progress(f"precision {prec}: amplitude continuation {res['solve']['time_s']:.1f} s")
        if ok is True:
            # pseudo-arclength continuation in omega_1 (tangent predictor, orthogonal
            # corrector) from the 0.3 N torus: ARC_POINTS points, step ARC_DS in the 2-norm of
            # [Z(0); omega_1], ||R||_2 < 1e-8 per point
            fse.fse_set_forcing(ctx, [amps[2]] * wl.system.e)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            try:
                _, oms, steps, cits, crn = fse.fse_arclength(ctx, wl.omega, Zs[2], ARC_DS, ARC_POINTS,
                                                             tol=1e-8, maxit=8)
                aok = True
            except fse.FseError as ex:
                oms, steps, cits, crn, aok = ex.omega, ex.steps, ex.iters, ex.rnorm, str(ex)
            torch.cuda.synchronize()
            el2 = time.perf_counter() - t2
            progress(f"precision {prec}: arclength {el2:.1f} s")
            res["arclength"] = {"time_s": el2, "points": ARC_POINTS, "s_per_point": el2 / ARC_POINTS,
                                "corrections": [int(i) for i in cits],
                                "omega1": [float(o[0]) for o in oms], "final_residuals": [float(r) for r in crn],
                                "converged": aok is True}
        fse.fse_set_forcing(ctx, [1.0] * wl.system.e)
    return res


def krylov_solve(fse, torch, amp=0.1):
    """Matrix-free Newton-Krylov on the three-frequency beam (84 966 unknowns, where the dense
    Jacobian would take 57.8 GB) from the linear response at amp N: time to ||R||_2 < 1e-8."""
    from fse_inputs import workload
    wl = workload("C4")
    ctx = fse.fse_init_torus(wl.system, wl.torus)
    U, St, bw, kt = fse.fse_get_layout(ctx)
    fse.fse_set_forcing(ctx, [amp] * wl.system.e)
    Z = torch.tensor(wl.initial_iterate(kt) * amp, dtype=torch.float64, device="cuda")
    progress("three-frequency beam: Newton-Krylov")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist, gits = [], []
    for _ in range(10):
        rn, its, _ = fse.fse_newton_krylov_step(ctx, wl.omega, Z, rtol=1e-8, restart=30, maxit=300)
        hist.append(rn)
        gits.append(its)
        if rn < 1e-8:
            break
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    progress(f"three-frequency beam: {len(hist)} Newton steps, {el:.1f} s")
    return {"workload": "von Karman beam, 147 DOF, d=3 (omega_1 (1, sqrt2, sqrt3)), 32x32 trajectories, "
                        f"H=8x8 (U={U}), S1=512, forcing {amp} N, from the linear response",
            "unknowns": int(2 * wl.system.n * U), "time_s": el,
            "newton_residuals": [float(h) for h in hist], "gmres_iterations": [int(g) for g in gits],
            "converged": bool(hist[-1] < 1e-8), "gmres": "restart 30, rtol 1e-8, harmonic-block preconditioner"}


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard trajectories or sensitivity columns across GPUs)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2508_06302_amd as fse
    from fse_inputs import workload
    torch.cuda.set_device(0)
    wl = workload("C2")
    tr = wl.torus
    solve = not args.no_solve
    plain = run_precision(fse, torch, wl, fse.FSE_PREC_FP64, args.steps, args.warmup, solve)
    mixed = None if args.no_mixed else run_precision(fse, torch, wl, fse.FSE_PREC_MIXED_FP32, args.steps,
                                                     args.warmup, solve)
    U, St, bw, Z0 = plain["U"], plain["St"], plain["bw"], plain["Z0"]
    n = wl.system.n
    traj_steps = St * tr.S1
    bytes_per_traj_step = 6 * n * (2 * n) * 8          # read + write Q, U, A (FP64)
    alg_bytes = bytes_per_traj_step * traj_steps
    achieved = alg_bytes / (plain["kernel_ms"] * 1e-3) / 1e9
    traffic = read_traffic(args.traffic)
    out = {
        "metric": "trajectory-steps/s and shooting solve time @||R||<1e-8, mixed vs plain FP64",
        "value": plain["value"], "unit": "trajectory-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": plain["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "von Karman clamped-clamped beam, 50 elements (147 DOF), d=2, "
                               "64 trajectories, H=15 (U=31), S1=512, full sensitivities, "
                               "plain FP64, one continuation point; one step = residual and "
                               "Jacobian of the shooting problem",
                   "n": n, "Stilde": St, "U": U, "S1": tr.S1, "half_band": bw},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_fused (state + sensitivities)" if plain["fused"] else "k_state + k_sens",
                     "kernel_ms_per_launch": plain["kernel_ms"],
                     "algorithmic_bytes_per_launch": alg_bytes},
        "autotuner": plain["tuning"],
        "state_only": plain["state_only"],
    }
    if mixed is not None:
        out["mixed"] = {"value": mixed["value"], "ms_per_step": mixed["ms_per_step"],
                        "kernel_ms_per_launch": mixed["kernel_ms"],
                        "dtype": "f64 arithmetic, f32 sensitivity storage"}
    if solve:
        path = "forcing amplitude 0.1 -> 0.5 N in 5 points from the linear response at 0.1 N, secant predictor"
        out["shooting_solve"] = {"path": path, "fp64": plain["solve"]}
        if "arclength" in plain:
            out["arclength_continuation"] = {
                "path": f"omega_1 from {wl.omega[0]:g} rad/s at 0.3 N, {ARC_POINTS} points, step {ARC_DS} "
                        "(2-norm of [Z(0); omega_1]), tangent predictor and orthogonal corrector",
                "fp64": plain["arclength"]}
            if mixed is not None and "arclength" in mixed:
                out["arclength_continuation"]["mixed"] = mixed["arclength"]
        if mixed is not None:
            out["shooting_solve"]["mixed"] = mixed["solve"]
            zp, zm = plain.get("Z_solution"), mixed.get("Z_solution")
            if zp is not None and zm is not None:
                out["shooting_solve"]["mixed_vs_fp64_torus_rel_diff"] = float((zm - zp).norm() / zp.norm())
    if solve and not args.no_krylov:
        out["krylov_solve"] = krylov_solve(fse, torch)
    if not args.no_cpu_baseline:
        from oracle import shooting as osh
        tb = osh.TorusTables(tr)
        progress("oracle on the host cores (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(wl, Z0, tb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
