"""Benchmark of the FSE-Shooting hot path on one MI355X.

Headline workload: the 1872-DOF synthetic shell (12 x 24 triangle mesh, 6 DOF per node, half band
89, lumped mass), d = 2, 128 trajectories on the 1-torus, H = 20 (U = 41), S1 = 1024 Newmark steps,
full sensitivities (3744 columns per trajectory), plain FP64.  One step = one pass of the hot path
for one continuation point: inverse DFT, consistent a_0 and the sensitivity seeds, the batched
Newmark integration with the per-step chord iteration, the sensitivity propagation, DFT +
rotation + residual, and one matrix-free Jacobian product J v from the stored sensitivities.
value = trajectory-steps/s = S~ * S1 / (time per step), inputs resident in HBM.

Prints ONE JSON line.  Besides the headline: the roofline of the dominant kernel (the wide-band
sensitivity sweep), the mixed-precision throughput of the same workload, the 147-DOF beam
(throughput, roofline of the fused kernel, shooting solve and arclength continuation times in
both precisions), the three-frequency beam with 8 continuation points in one launch and its
Newton-Krylov solve, and the FP64 oracle timed on the host cores on a bounded sample.

`--calibrate-copy` instead times a plain device-to-device copy of known size; its
FETCH_SIZE / WRITE_SIZE counters scale the counters of the profiled kernels to bytes.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3
ARC_POINTS = 10
ARC_DS = 0.5
CSRC = os.path.join(ROOT, "paper_2508_06302_amd", "csrc")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-beam", action="store_true", help="skip the 147-DOF beam fields")
    ap.add_argument("--no-c4", action="store_true", help="skip the three-frequency beam fields")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--shell-solve", action="store_true",
                    help="also time a shell solve in both precisions (about a minute)")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--sweep", choices=["train", "learned", "secant"],
                    help="run one phase of the 200-point shell sweep instead of the benchmark")
    ap.add_argument("--sweep-dir", default=os.path.join(ROOT, "sweep_results"),
                    help="where a sweep phase writes its results")
    ap.add_argument("--sweep-in", default=None,
                    help="where a sweep phase reads the training results (default: --sweep-dir)")
    ap.add_argument("--sweep-precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--sweep-deadline", type=float, default=1000.0,
                    help="seconds after which a sweep phase stops and saves the points it has solved")
    return ap.parse_args()


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def read_traffic(name, files):
    """HBM bytes per launch of a profiled kernel from its counter summary, or None when absent or
    taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except Exception:
        return None
    if t.get("source_sha256_16") != source_hash(files):
        return None
    return t.get("bytes_per_launch")


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


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------- host baseline
_ORACLE_INPUT = None


def _oracle_init(payload):
    """Pool initializer: the shell's inputs, built once by the parent."""
    global _ORACLE_INPUT
    _ORACLE_INPUT = payload


def _oracle_steps(args):
    """One worker of the host baseline: the oracle integrates `steps` Newmark steps of trajectory
    s with all sensitivity columns, on one BLAS thread; returns (steps done, seconds)."""
    s, steps = args
    from threadpoolctl import threadpool_limits
    from oracle import newmark
    sysm, omega, S1, phases, zbar0 = _ORACLE_INPUT
    with threadpool_limits(1):
        t0 = time.perf_counter()
        newmark.integrate(sysm, omega, S1, phases[:, s], zbar0[:, s], sens=True, steps=steps)
        return steps, time.perf_counter() - t0


def cpu_baseline(steps_per_worker=1):
    """The oracle as it stands, on the host cores: trajectories of the same shell workload with all
    sensitivity columns, the first `steps_per_worker` Newmark steps each (a whole trajectory takes
    minutes), one process per trajectory with one BLAS thread each, at 1 worker and at as many
    workers as the host share has cores (at most 16).  value = trajectory-steps/s at that count."""
    from multiprocessing import get_context
    from fse_inputs import workload
    from oracle import shooting
    cpus = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    workers = max(1, min(16, cpus))
    try:
        model = [l.split(":", 1)[1].strip() for l in subprocess.run(["lscpu"], capture_output=True, text=True)
                 .stdout.splitlines() if l.startswith("Model name")][0]
    except Exception:
        model = "unknown"
    wl = workload("C3")
    tb = shooting.TorusTables(wl.torus)
    n = wl.system.n
    zbar0 = wl.initial_iterate(tb.table).reshape(2 * n, tb.U) @ tb.G.T
    payload = (wl.system, wl.omega, wl.torus.S1, tb.phases, zbar0)
    out = {}
    ctx = get_context("spawn")
    for nw in sorted({1, workers}):
        progress(f"oracle: starting {nw} worker(s)")
        with ctx.Pool(nw, initializer=_oracle_init, initargs=(payload,)) as pool:
            pool.map(_oracle_steps, [(0, 1)] * nw)          # imports and first touch outside the clock
            t0 = time.perf_counter()
            res = pool.map(_oracle_steps, [(s * 7 % 128, steps_per_worker) for s in range(nw)])
            el = time.perf_counter() - t0
        out[nw] = (sum(r[0] for r in res) / el, el)
        progress(f"oracle: {nw} worker(s), {out[nw][0]:.3f} trajectory-steps/s")
    v, el = out[workers]
    return {"value": v, "unit": "trajectory-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} trajectories of the shell workload, the first {steps_per_worker} Newmark step(s) "
                      f"each with all 3744 sensitivity columns, one process per trajectory on one BLAS thread "
                      f"({el:.1f} s wall)",
            "one_core": {"value": out[1][0], "wall_s": out[1][1]},
            "host": {"cpu_model": model, "cpus_available": cpus}}


# ----------------------------------------------------------------------------- shell (headline)
def sweep_flops_per_traj_step(sysm, bw):
    """Algorithmic FP64 work of one sensitivity step of one trajectory on the wide-band path: the
    right-hand side w1^2 M P2 + w1 D P1 (lumped M, sparse D), forward and backward substitution with
    the banded unit lower factor, the pivot scaling and the updates of P1, P2 (5 flops per entry)."""
    n = sysm.n
    nnzD = int(np.count_nonzero(sysm.D))
    nnzL = n * bw - bw * (bw + 1) // 2
    return 2 * n * (2 * n + 2 * nnzD + 4 * nnzL + n + 5 * n)


def run_shell(fse, torch, prec, steps, warmup):
    from fse_inputs import workload
    wl = workload("C3")
    progress(f"shell: init (precision {prec})")
    ctx = fse.fse_init_torus(wl.system, wl.torus, precision=prec)
    U, St, bw, kt = fse.fse_get_layout(ctx)
    Z0 = torch.tensor(wl.initial_iterate(kt), dtype=torch.float64, device="cuda")
    v = torch.randn_like(Z0)

    def step():
        R, rn = fse.fse_shooting_residual_matfree(ctx, wl.omega, Z0)
        Jv = fse.fse_jacobian_apply(ctx, v)
        return rn, Jv

    for i in range(warmup):
        step()
        progress(f"shell: warmup {i + 1}/{warmup}")
    torch.cuda.synchronize()
    kms, kl, st = [], [], []
    t0 = time.perf_counter()
    for i in range(steps):
        rn, _ = step()
        path, ms, nl = fse.fse_last_kernel_timing(ctx)
        kms.append(ms)
        kl.append(nl)
        st.append(fse.fse_last_timing(ctx)["state_ms"])
        progress(f"shell: step {i + 1}/{steps} |R| {rn:.3e}")
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    mx, tot = fse.fse_step_stats(ctx)
    return {"ctx": ctx, "wl": wl, "Z0": Z0, "U": U, "St": St, "bw": bw, "path": path,
            "s_per_step": el, "value": St * wl.torus.S1 / el, "rnorm": rn,
            "sweep_ms_per_launch": float(np.mean(kms)) / float(np.mean(kl)) if np.mean(kl) > 0 else None,
            "sweep_launches": int(np.mean(kl)), "state_ms": float(np.mean(st)),
            "chord_iterations": {"max_per_step": mx, "mean_per_step": tot / (St * wl.torus.S1)}}


def shell_solve(fse, torch, wl, prec, a=10.0, w_ratio=0.95):
    """Time to solution on the shell: from the linear harmonic start at forcing scale a (loads 40a
    and 20a N) and omega_1 = w_ratio x the first natural frequency, Newton-Krylov with Jacobian
    reuse (the sweep's solver: one sensitivity evaluation, then chord steps) to ||R||_2 < 1e-8,
    the residual FP64 in both precisions."""
    from fse_inputs import workload
    wn = 2 * np.pi * 100.0
    w = workload("C3", omega1=w_ratio * wn)
    ctx = fse.fse_init_torus(w.system, w.torus, precision=prec)
    U, St, bw, kt = fse.fse_get_layout(ctx)
    fse.fse_set_forcing(ctx, np.array([a, a]))
    Z = torch.tensor(w.initial_iterate(kt) * a, dtype=torch.float64, device="cuda")
    _, r0, _ = fse.fse_shooting_residual_jacobian(ctx, w.omega[None], Z[None])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = {}
    its, full, rn, ok = chord_solve(fse, torch, ctx, w.omega, Z, st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    progress(f"shell solve (precision {prec}): {its} corrections, ||R|| {rn:.3e}, {el:.1f} s")
    return {"time_s": el, "start_residual": float(r0[0]), "final_residual": float(rn), "corrections": its,
            "sensitivity_evaluations": sum(1 for k, _ in st["gmres"] if k == "full"), "converged": bool(ok),
            "point": f"omega_1 = {w_ratio} omega_n, loads {40 * a:g} and {20 * a:g} N"}, Z


# ----------------------------------------------------------------------------- 147-DOF beam
def run_beam(fse, torch, prec, steps, warmup, solve):
    """Throughput of the residual + dense Jacobian step on the 147-DOF beam and its solves."""
    from fse_inputs import workload
    wl = workload("C2")
    tr = wl.torus
    ctx = fse.fse_init_torus(wl.system, tr, precision=prec)
    U, St, bw, kt = fse.fse_get_layout(ctx)
    Z0 = wl.initial_iterate(kt)
    om = wl.omega[None]
    Zd = torch.tensor(Z0[None], dtype=torch.float64, device="cuda")
    step = lambda: fse.fse_shooting_residual_jacobian(ctx, om, Zd, want_J=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    kern = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        kern.append(fse.fse_last_kernel_timing(ctx)[1])
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    n = wl.system.n
    alg = 6 * n * (2 * n) * 8 * St * tr.S1
    kms = float(np.mean(kern))
    res = {"value": St * tr.S1 / el, "ms_per_step": 1e3 * el, "kernel_ms_per_launch": kms,
           "roofline": {"bound": "hbm", "achieved": alg / (kms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": alg / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "kernel": "k_fused", "algorithmic_bytes_per_launch": alg}}
    progress(f"beam (precision {prec}): {res['ms_per_step']:.1f} ms per step")
    if solve:
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
        res["solve"] = {"time_s": time.perf_counter() - t1, "newton_iterations": [int(i) for i in its],
                        "final_residuals": [float(r) for r in rns], "converged": ok is True}
        res["Z_solution"] = Zs[-1].clone() if ok is True else None
        if ok is True:
            fse.fse_set_forcing(ctx, [amps[2]] * wl.system.e)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            try:
                _, oms, _, cits, crn = fse.fse_arclength(ctx, wl.omega, Zs[2], ARC_DS, ARC_POINTS, tol=1e-8, maxit=8)
                aok = True
            except fse.FseError as ex:
                oms, cits, crn, aok = ex.omega, ex.iters, ex.rnorm, str(ex)
            torch.cuda.synchronize()
            el2 = time.perf_counter() - t2
            res["arclength"] = {"time_s": el2, "points": ARC_POINTS, "corrections": [int(i) for i in cits],
                                "omega1": [float(o[0]) for o in oms], "converged": aok is True}
        progress(f"beam (precision {prec}): solves done")
    return res


# ----------------------------------------------------------------------------- 3-frequency beam
def run_c4(fse, torch, steps, warmup, solve):
    """Eight continuation points (omega_1 from 36.5 to 40.0 rad/s, below the first resonance at
    44.55 rad/s where the 1 N linear start stays within the step Newton's reach) of the
    three-frequency beam in one launch: 8 x 1024 trajectories of 512 steps with full sensitivities."""
    from fse_inputs import workload
    w1s = np.linspace(36.5, 40.0, 8)
    wls = [workload("C4", omega1=float(w)) for w in w1s]
    tr = wls[0].torus
    ctx = fse.fse_init_torus(wls[0].system, tr, max_batch=8)
    U, St, bw, kt = fse.fse_get_layout(ctx)
    om = np.stack([w.omega for w in wls])
    Zs = np.stack([w.initial_iterate(kt) for w in wls])
    for _ in range(warmup):
        fse.fse_integrate_batch(ctx, om, Zs, want_phi=True)
    torch.cuda.synchronize()
    kern = []
    t0 = time.perf_counter()
    for _ in range(steps):
        fse.fse_integrate_batch(ctx, om, Zs, want_phi=True)
        kern.append(fse.fse_last_kernel_timing(ctx)[1])
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    n = wls[0].system.n
    W = 8 * St
    alg = 6 * n * (2 * n) * 8 * W * tr.S1
    kms = float(np.mean(kern))
    out = {"workload": "von Karman beam, 147 DOF, d=3 (omega_1 (1, sqrt2, sqrt3)), 32x32 trajectories, H=8x8 "
                       f"(U={U}), S1=512, 8 continuation points omega_1 = 36.5..40.0 rad/s in one launch, "
                       "full sensitivities, FP64",
           "value": W * tr.S1 / el, "unit": "trajectory-steps/s", "s_per_launch": el, "kernel_ms_per_launch": kms,
           "roofline": {"bound": "hbm", "achieved": alg / (kms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": alg / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, "kernel": "k_fused",
                        "algorithmic_bytes_per_launch": alg}}
    progress(f"three-frequency beam, 8 points: {el:.2f} s per launch")
    del ctx
    torch.cuda.empty_cache()
    if solve:
        out["krylov_solve"] = krylov_solve(fse, torch)
    return out


def krylov_solve(fse, torch, amp=0.1):
    """Matrix-free Newton-Krylov on the three-frequency beam (84 966 unknowns, where the dense
    Jacobian would take 57.8 GB) from the linear response at amp N: time to ||R||_2 < 1e-8."""
    from fse_inputs import workload
    wl = workload("C4")
    ctx = fse.fse_init_torus(wl.system, wl.torus)
    U, St, bw, kt = fse.fse_get_layout(ctx)
    fse.fse_set_forcing(ctx, [amp] * wl.system.e)
    Z = torch.tensor(wl.initial_iterate(kt) * amp, dtype=torch.float64, device="cuda")
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
    progress(f"three-frequency beam Newton-Krylov: {len(hist)} steps, {el:.1f} s")
    return {"point": "omega_1 = 40 rad/s, forcing 0.1 N, from the linear response", "unknowns": int(2 * wl.system.n * U),
            "time_s": el, "newton_residuals": [float(h) for h in hist], "gmres_iterations": [int(g) for g in gits],
            "converged": bool(hist[-1] < 1e-8)}


# ----------------------------------------------------------------------------- shell sweep
SWEEP_W = (0.93, 0.97)       # omega_1 / omega_n (first natural frequency 100 Hz)
SWEEP_A = (6.0, 14.0)        # forcing amplitude scale a: loads 40 a and 20 a N
SWEEP_RATIO = 2 ** -0.5      # omega_2 / omega_1
SWEEP_TOL = 1e-8
SWEEP_EPOCHS = 10000         # full-batch AdamW steps of the predictor's training


def sweep_points():
    """The 200 points of the shell sweep as (omega_1 / omega_n, a).  Training: a 10 x 10 grid over
    the box, amplitude rows visited as a serpentine in frequency (frequency sweeps up and down at
    rising amplitude).  Evaluation: a second 10 x 10 grid strictly inside the box, interleaved
    with the first (grid coordinates 0.45 + 0.9 k), visited as a serpentine in the opposite
    amplitude direction, so that it starts next to the last training point."""
    def axis(lo, hi, t):
        return lo + (hi - lo) * np.asarray(t) / 9.0

    gi = np.arange(10)
    ge = 0.45 + 0.9 * np.arange(10)
    train, evalp = [], []
    for r, k in enumerate(gi):
        ws = axis(*SWEEP_W, gi if r % 2 == 0 else gi[::-1])
        train += [(w, axis(*SWEEP_A, k)) for w in ws]
    for r, k in enumerate(ge[::-1]):
        ws = axis(*SWEEP_W, ge if r % 2 == 0 else ge[::-1])
        evalp += [(w, axis(*SWEEP_A, k)) for w in ws]
    return np.array(train), np.array(evalp)


def chord_solve(fse, torch, ctx, om, Z, st, rate=0.25, max_steps=30, rtol=1e-4):
    """Newton-Krylov with Jacobian reuse for one point (omega host [2], Z torch [2n][U] in place):
    chord steps with the stored Jacobian, and a full Newton-Krylov step (new sensitivities) when
    none is stored or when the last step contracted ||R|| by less than `rate` (after a check of
    ||R|| from the states alone, so that no sensitivities are computed at a converged iterate).  When a step does
    not lower ||R||_2 by 1 % below the best iterate so far, the next step is a full Newton step from
    that best iterate; if its update does not lower it either, the point ends there (not
    converged, Z = the best iterate).  Stops at the first iterate with ||R||_2 < SWEEP_TOL, which
    is the one returned.  -> (corrections, of which full Newton steps, final ||R||, converged)."""
    Zk = torch.empty_like(Z)
    Zb = torch.empty_like(Z)
    its = refr = 0
    prev, best = None, np.inf
    redo = from_best = False
    refresh = not st.get("have_J", False)
    st["gmres"] = []
    while True:
        Zk.copy_(Z)
        if refresh and st.get("have_J", False):
            # a refresh costs a sensitivity evaluation: first see, from the states alone, whether
            # the iterate has already converged
            _, rc, _ = fse.fse_shooting_residual_jacobian(ctx, np.asarray(om)[None], Z[None])
            progress(f"  check: ||R|| {rc[0]:.3e}")
            if rc[0] < SWEEP_TOL:
                return its, refr, float(rc[0]), True
        if refresh:
            rn, g, _ = fse.fse_newton_krylov_step(ctx, om, Z, rtol=rtol, restart=30, maxit=120)
            st["have_J"] = True
            refr += 1
        else:
            rn, g, _ = fse.fse_newton_krylov_chord_step(ctx, om, Z, rtol=rtol, restart=30, maxit=120)
        st["gmres"].append(("full" if refresh else "chord", int(g)))
        progress(f"  {'full' if refresh else 'chord'} step: ||R|| {rn:.3e} before, {g} GMRES iterations")
        if rn < SWEEP_TOL:
            Z.copy_(Zk)
            return its, refr - (1 if refresh else 0), rn, True
        if its >= max_steps or not np.isfinite(rn):
            Z.copy_(Zb)
            return its, refr - (1 if refresh else 0), best, False
        if redo:
            # a full step from the best iterate (whose residual this is): judge its update next
            redo, from_best, refresh = False, True, False
        elif rn < 0.99 * best:
            best, from_best = rn, False
            Zb.copy_(Zk)
            refresh = prev is not None and rn > rate * prev
            prev = rn
        elif from_best:
            # not even a fresh Newton step from the best iterate lowers ||R||: the floor is here
            Z.copy_(Zb)
            return its, refr - (1 if refresh else 0), best, False
        else:
            Z.copy_(Zb)
            redo, refresh = True, True
        its += 1


def _sweep_ctx(fse, torch, prec):
    from fse_inputs import workload
    wl = workload("C3")
    ctx = fse.fse_init_torus(wl.system, wl.torus, precision=prec)
    U, St, bw, kt = fse.fse_get_layout(ctx)
    wn = 2 * np.pi * 100.0
    return wl, ctx, kt, wn


def _sweep_params(wn, pt):
    """Point (omega_1 / omega_n, a) -> (omega [2], amplitudes [2], continuation vector, features)."""
    w1 = pt[0] * wn
    om = np.array([w1, SWEEP_RATIO * w1])
    amp = np.array([pt[1], pt[1]])
    return om, amp, np.concatenate([om, amp]), np.array([w1, SWEEP_RATIO, pt[1]])


def run_sweep(fse, torch, phase, sweep_dir, sweep_in, prec_name, deadline):
    """One phase of the 200-point shell sweep; prints one JSON line.
    train:   the 100 training points with the secant predictor (point 0 from its linear harmonic
             response); writes the converged tori (FP32) and the last two (FP64) to sweep_dir, and
             resumes after the points already in sweep_in.
    learned: POD (rank 64) of the training tori, the MLP 3 -> 256 -> 256 -> 64 trained on the GPU
             (SWEEP_EPOCHS steps),
             then the 100 evaluation points, each from the better of the secant and the learned
             (BF16 matrix-core inference) prediction by ||R||.
    secant:  the 100 evaluation points with the secant predictor alone.
    The evaluation phases read the training results from sweep_in, start from the last two
    training points and solve every point to
    ||R||_2 < 1e-8 with the same Newton-Krylov iteration with Jacobian reuse.  A phase still
    running `deadline` seconds after its start stops and reports (and saves) the points it has."""
    prec = fse.FSE_PREC_MIXED_FP32 if prec_name == "mixed" else fse.FSE_PREC_FP64
    os.makedirs(sweep_dir, exist_ok=True)
    train, evalp = sweep_points()
    progress(f"sweep {phase}: init ({prec_name})")
    wl, ctx, kt, wn = _sweep_ctx(fse, torch, prec)
    N = 2 * wl.system.n * ctx.U
    st = {}
    recs = []
    t_all = time.perf_counter()
    done = 0
    if phase == "train":
        pts = train
        Zs = torch.empty((len(pts), 2 * wl.system.n, ctx.U), dtype=torch.float32, device="cuda")
        prev = os.path.join(sweep_in, "train_mixed.json") if prec_name == "mixed" else None
        if os.path.exists(os.path.join(sweep_in, "train_points.npy")):
            # resume: keep the points solved by an earlier run of this phase
            done = len(np.load(os.path.join(sweep_in, "train_points.npy")))
            Zs[:done].copy_(torch.from_numpy(np.load(os.path.join(sweep_in, "train_Z_f32.npy"))))
            last = np.load(os.path.join(sweep_in, "train_last2.npy"))
            hist = [(_sweep_params(wn, train[done - 2])[2], torch.tensor(last[0], device="cuda")),
                    (_sweep_params(wn, train[done - 1])[2], torch.tensor(last[1], device="cuda"))]
            recs = json.load(open(prev))["records"] if prev and os.path.exists(prev) else []
            progress(f"sweep train: resuming after {done} points")
        else:
            om0, amp0, _, _ = _sweep_params(wn, pts[0])
            from fse_inputs import workload
            Zlin = workload("C3", omega1=om0[0]).initial_iterate(kt) * pts[0][1]
            Z = torch.tensor(Zlin, dtype=torch.float64, device="cuda")
            hist = []
    else:
        last = np.load(os.path.join(sweep_in, "train_last2.npy"))
        train = np.load(os.path.join(sweep_in, "train_points.npy"))
        hist = [(_sweep_params(wn, train[-2])[2], torch.tensor(last[0], device="cuda")),
                (_sweep_params(wn, train[-1])[2], torch.tensor(last[1], device="cuda"))]
        pts = evalp
        prev = os.path.join(sweep_in, f"{phase}_{prec_name}.json")
        if os.path.exists(prev) and os.path.exists(os.path.join(sweep_in, f"{phase}_{prec_name}_last2.npy")):
            # resume after the evaluation points an earlier run of this phase solved
            recs = json.load(open(prev))["records"]
            done = len(recs)
            last = np.load(os.path.join(sweep_in, f"{phase}_{prec_name}_last2.npy"))
            hist = [(_sweep_params(wn, evalp[done - 2])[2], torch.tensor(last[0], device="cuda")),
                    (_sweep_params(wn, evalp[done - 1])[2], torch.tensor(last[1], device="cuda"))]
            progress(f"sweep {phase}: resuming after {done} points")
        lp = None
        if phase == "learned":
            X = torch.tensor(np.load(os.path.join(sweep_in, "train_Z_f32.npy")), device="cuda").double()
            feats = np.array([_sweep_params(wn, p)[3] for p in train])
            lp = fse.fse_learned_create(ctx, n_in=3, hidden=256, rank=64)
            rng = np.random.default_rng(7)
            params = []
            for fi, fo in ((3, 256), (256, 256), (256, 64)):
                params += [rng.normal(scale=(1.0 / fi) ** 0.5, size=(fo, fi)).ravel(), np.zeros(fo)]
            lp.set_params(np.concatenate(params).astype(np.float32))
            t0 = time.perf_counter()
            sig = lp.fit_pod(X)
            loss = lp.train(feats, X, epochs=SWEEP_EPOCHS, lr=1e-3, wd=1e-5)
            torch.cuda.synchronize()
            t_train = time.perf_counter() - t0
            mean, modes = lp.get_pod()
            Xc = X.reshape(len(train), N) - mean
            proj_err = float((Xc - (Xc @ modes) @ modes.T).norm() / Xc.norm())
            del X, Xc
            torch.cuda.empty_cache()
            progress(f"sweep learned: POD + MLP in {t_train:.1f} s, loss {loss[0]:.3e} -> {loss[-1]:.3e}")
    for j, pt in enumerate(pts):
        if j < done:
            continue
        if time.perf_counter() - t_all > deadline:
            progress(f"sweep {phase}: deadline reached after {j} points")
            break
        om, amp, pvec, feat = _sweep_params(wn, pt)
        fse.fse_set_forcing(ctx, amp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = {"omega_ratio": float(pt[0]), "a": float(pt[1])}
        if len(hist) >= 2:
            Z = fse.fse_secant_predict(ctx, hist[-2][0], hist[-1][0], pvec, hist[-2][1], hist[-1][1])
        elif len(hist) == 1:
            Z = hist[-1][1].clone()
        if phase == "learned":
            _, rs, _ = fse.fse_shooting_residual_jacobian(ctx, om[None], Z[None])
            Zl = lp.predict_batch(feat[None], bf16=True)[0]
            _, rl, _ = fse.fse_shooting_residual_jacobian(ctx, om[None], Zl[None])
            rec["R_secant"], rec["R_learned"] = float(rs[0]), float(rl[0])
            rec["learned_used"] = bool(np.isfinite(rl[0]) and rl[0] < rs[0])
            if rec["learned_used"]:
                Z = Zl
        its, full, rn, ok = chord_solve(fse, torch, ctx, om, Z, st)
        torch.cuda.synchronize()
        rec.update({"corrections": its, "full_newton_steps": full, "R_final": rn, "converged": ok,
                    "seconds": time.perf_counter() - t0, "gmres": st["gmres"]})
        recs.append(rec)
        if phase == "train":
            Zs[j].copy_(Z)
        hist = (hist + [(pvec, Z.clone())])[-2:]
        progress(f"sweep {phase} {j + 1}/{len(pts)}: {its} corrections ({full} full), ||R|| {rn:.2e}, "
                 f"{rec['seconds']:.1f} s" + (f", learned {rec['learned_used']}" if phase == "learned" else ""))
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    if phase == "train":
        np.save(os.path.join(sweep_dir, "train_Z_f32.npy"), Zs[:len(recs)].cpu().numpy())
        np.save(os.path.join(sweep_dir, "train_points.npy"), pts[:len(recs)])
        np.save(os.path.join(sweep_dir, "train_last2.npy"), np.stack([h[1].cpu().numpy() for h in hist]))
    else:
        np.save(os.path.join(sweep_dir, f"{phase}_{prec_name}_last2.npy"),
                np.stack([h[1].cpu().numpy() for h in hist]))
    total += sum(r["seconds"] for r in recs[:done])   # the earlier runs' share
    c = np.array([r["corrections"] for r in recs], float)
    sec = np.array([r["seconds"] for r in recs])
    out = {"metric": "Newton corrections and seconds per point to ||R||_2 < 1e-8 (shell sweep)",
           "phase": phase, "precision": prec_name, "points": len(recs),
           "corrections_per_point": float(c.mean()),
           "full_newton_steps_per_point": float(np.mean([r["full_newton_steps"] for r in recs])),
           "seconds_per_point": float(sec.mean()), "seconds_total": float(sec.sum()), "wall_s": total,
           "max_final_residual": float(max(r["R_final"] for r in recs)),
           "not_converged": int(sum(1 for r in recs if not r.get("converged", True))),
           "config": {"workload": "synthetic shell 1872 DOF, d=2, 128 trajectories, H=20, S1=1024",
                      "box": {"omega1_over_omega_n": SWEEP_W, "a": SWEEP_A, "omega2_over_omega1": SWEEP_RATIO}},
           "records": recs}
    if phase == "learned":
        out.update({"learned_used_fraction": float(np.mean([r["learned_used"] for r in recs])),
                    "train_s": t_train, "loss_first_last": [float(loss[0]), float(loss[-1])],
                    "pod_sigma_first_last": [float(sig[0]), float(sig[-1])], "pod_projection_error": proj_err,
                    "median_R_secant": float(np.median([r["R_secant"] for r in recs])),
                    "median_R_learned": float(np.median([r["R_learned"] for r in recs]))})
    json.dump(out, open(os.path.join(sweep_dir, f"{phase}_{prec_name}.json"), "w"))
    print(json.dumps({k: v for k, v in out.items() if k != "records"}), flush=True)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard trajectories or sensitivity columns across GPUs)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2508_06302_amd as fse
    torch.cuda.set_device(0)
    if args.sweep:
        run_sweep(fse, torch, args.sweep, args.sweep_dir, args.sweep_in or args.sweep_dir, args.sweep_precision,
                  args.sweep_deadline)
        return
    sh = run_shell(fse, torch, fse.FSE_PREC_FP64, args.steps, args.warmup)
    wl, St, bw = sh["wl"], sh["St"], sh["bw"]
    n, S1 = wl.system.n, wl.torus.S1
    fl_ts = sweep_flops_per_traj_step(wl.system, bw)
    flops_launch = fl_ts * St
    achieved = flops_launch / (sh["sweep_ms_per_launch"] * 1e-3) / 1e12
    traffic = read_traffic("k_wide_sweep_shell_traffic.json", ["k_wide.hip"])
    out = {
        "metric": "trajectory-steps/s and shooting solve time @||R||<1e-8, mixed vs plain FP64",
        "value": sh["value"], "unit": "trajectory-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * sh["s_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "synthetic shell, 12 x 24 triangle mesh, 6 DOF per node (1872 DOF, half band 89, "
                               "lumped mass), d=2, 128 trajectories, H=20 (U=41), S1=1024, full sensitivities "
                               "(3744 columns per trajectory), plain FP64, one continuation point; one step = "
                               "residual with sensitivities and one matrix-free Jacobian product",
                   "n": n, "Stilde": St, "U": sh["U"], "S1": S1, "half_band": bw},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFS, "traffic": traffic,
                     "kernel": "k_wide_sweep (FP64 matrix cores; one launch per Newmark step)",
                     "kernel_ms_per_launch": sh["sweep_ms_per_launch"], "launches_per_step": sh["sweep_launches"],
                     "algorithmic_flops_per_launch": flops_launch,
                     "algorithmic_bytes_per_launch": 4 * n * (2 * n) * 8 * St},
        "state_chain_ms": sh["state_ms"], "chord_iterations": sh["chord_iterations"],
        "residual_norm_at_start": sh["rnorm"],
    }
    del sh["ctx"]
    torch.cuda.empty_cache()
    if not args.no_mixed:
        mx = run_shell(fse, torch, fse.FSE_PREC_MIXED_FP32, max(1, args.steps // 2), args.warmup)
        out["mixed"] = {"value": mx["value"], "ms_per_step": 1e3 * mx["s_per_step"],
                        "speedup_vs_fp64": mx["value"] / sh["value"],
                        "sweep_ms_per_launch": mx["sweep_ms_per_launch"],
                        "sweep_frac_of_fp32_peak": fl_ts * St / (mx["sweep_ms_per_launch"] * 1e-3) / 1e12 / FP32_PEAK_TFS,
                        "dtype": "FP32 factor, FP32 matrix-core sweeps and FP32 sensitivity storage; FP64 states "
                                 "and residuals"}
        del mx["ctx"]
        torch.cuda.empty_cache()
    if args.shell_solve:
        s64, Z64 = shell_solve(fse, torch, wl, fse.FSE_PREC_FP64)
        s32, Z32 = shell_solve(fse, torch, wl, fse.FSE_PREC_MIXED_FP32)
        out["shell_solve"] = {"fp64": s64, "mixed": s32, "speedup_mixed_vs_fp64": s64["time_s"] / s32["time_s"],
                              "mixed_vs_fp64_torus_rel_diff": float((Z32 - Z64).norm() / Z64.norm())}
    def guarded(name, fn):
        """Secondary fields: a failure is recorded in the line instead of losing it."""
        try:
            fn()
        except Exception as ex:  # noqa: BLE001
            out[name] = {"error": f"{type(ex).__name__}: {ex}"}
            progress(f"{name} failed: {ex}")

    def beam_fields():
        b64 = run_beam(fse, torch, fse.FSE_PREC_FP64, 5, 1, not args.no_solve)
        beam = {"workload": "von Karman clamped-clamped beam, 50 elements (147 DOF), d=2, 64 trajectories, H=15 "
                            "(U=31), S1=512, full sensitivities; step = residual and dense Jacobian",
                "fp64": {k: v for k, v in b64.items() if k not in ("Z_solution",)}}
        if not args.no_mixed:
            b32 = run_beam(fse, torch, fse.FSE_PREC_MIXED_FP32, 5, 1, not args.no_solve)
            beam["mixed"] = {k: v for k, v in b32.items() if k not in ("Z_solution",)}
            zp, zm = b64.get("Z_solution"), b32.get("Z_solution")
            if zp is not None and zm is not None:
                beam["mixed_vs_fp64_torus_rel_diff"] = float((zm - zp).norm() / zp.norm())
        out["beam"] = beam
        torch.cuda.empty_cache()

    def c4_fields():
        out["three_frequency_beam"] = run_c4(fse, torch, 1, 1, not args.no_solve)

    def cpu_fields():
        progress("oracle on the host cores (bounded sample)")
        out["cpu_baseline"] = cpu_baseline()

    if not args.no_beam:
        guarded("beam", beam_fields)
    if not args.no_c4:
        guarded("three_frequency_beam", c4_fields)
    if not args.no_cpu_baseline:
        guarded("cpu_baseline", cpu_fields)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
