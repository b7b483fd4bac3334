"""FSE-Shooting on one MI355X: Python binding of libfse.so (include/fse.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device arrays are torch tensors on the current CUDA (HIP) device; the library
works on torch's current stream.  There is no CPU fallback: without the built
library or without a GPU every call raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib

__all__ = ["FseError", "Context", "fse_init_torus", "fse_get_layout", "fse_integrate_batch",
           "fse_step_stats", "fse_shooting_residual_jacobian", "fse_newton_step",
           "fse_newton_solve", "fse_lyapunov", "fse_last_timing", "fse_set_forcing", "fse_set_newmark", "fse_set_contacts",
           "fse_secant_predict", "fse_continuation", "fse_residual_domega", "Learned",
           "fse_learned_create", "fse_continuation_learned", "fse_residual_dp", "fse_arclength",
           "fse_shooting_residual_matfree", "fse_jacobian_apply", "fse_newton_krylov_step",
           "fse_hypertime_residual_jacobian", "fse_hypertime_newton_step", "fse_multiple_residual_jacobian",
           "fse_multiple_newton_step", "fse_get_tuning", "FSE_PREC_FP64",
           "FSE_PREC_MIXED_FP32"]

FSE_PREC_FP64 = 0
FSE_PREC_MIXED_FP32 = 1


class FseError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_lib.FSE_STATUS.get(status, status)}: {msg}")
        self.status = status


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("FSE-Shooting needs a GPU (HIP device); none is available")
    return torch


def _csr(A):
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    ptr = np.zeros(n + 1, np.int32)
    idx, val = [], []
    for i in range(n):
        nz = np.flatnonzero(A[i])
        idx.append(nz.astype(np.int32))
        val.append(A[i, nz])
        ptr[i + 1] = ptr[i] + len(nz)
    return ptr, np.concatenate(idx).astype(np.int32), np.concatenate(val).astype(np.float64)


def _p(arr, ct):
    return arr.ctypes.data_as(C.POINTER(ct))


class Context:
    """Owns an fse_ctx; keeps the host arrays alive for the duration of init."""

    def __init__(self, handle, lib, n, d, U, St, bw, ktable):
        self.h, self.lib = handle, lib
        self.n, self.d, self.U, self.Stilde, self.half_band = n, d, U, St, bw
        self.ktable = ktable

    def check(self, status):
        if status != 0:
            msg = self.lib.fse_last_error(self.h).decode()
            raise FseError(status, msg)

    def bind_stream(self):
        torch = _torch()
        self.check(self.lib.fse_set_stream(self.h, C.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def __del__(self):
        try:
            if self.h:
                self.lib.fse_destroy(self.h)
                self.h = None
        except Exception:
            pass


def fse_init_torus(system, torus, max_batch=1, precision=FSE_PREC_FP64, step_tol=1e-12,
                   step_maxit=30) -> Context:
    """system: fse_inputs.System (dense M, D, K; COO tensors); torus: fse_inputs.Torus."""
    lib = _lib.load()
    _torch()
    n = system.n
    Mp, Mi, Mv = _csr(system.M)
    Dp, Di, Dv = _csr(system.D)
    Kp, Ki, Kv = _csr(system.K)
    t2i = np.ascontiguousarray(system.t2_idx, dtype=np.int32)
    t2v = np.ascontiguousarray(system.t2_val, dtype=np.float64)
    t3i = np.ascontiguousarray(system.t3_idx, dtype=np.int32)
    t3v = np.ascontiguousarray(system.t3_val, dtype=np.float64)
    F = np.ascontiguousarray(system.F, dtype=np.float64)
    sysc = _lib.FseSystem(n, _p(Mp, C.c_int32), _p(Mi, C.c_int32), _p(Mv, C.c_double),
                          _p(Dp, C.c_int32), _p(Di, C.c_int32), _p(Dv, C.c_double),
                          _p(Kp, C.c_int32), _p(Ki, C.c_int32), _p(Kv, C.c_double),
                          len(t2v), _p(t2i, C.c_int32), _p(t2v, C.c_double),
                          len(t3v), _p(t3i, C.c_int32), _p(t3v, C.c_double),
                          F.shape[0], _p(F, C.c_double))
    klen = np.array([len(k) for k in torus.K] or [0], np.int32)
    klist = np.concatenate([np.asarray(k, np.int32) for k in torus.K] or [np.zeros(1, np.int32)])
    klist = np.ascontiguousarray(klist, dtype=np.int32)
    S = np.array(list(torus.S) or [1], np.int32)
    desc = _lib.FseTorusDesc(torus.d, torus.e, _p(klen, C.c_int32), _p(klist, C.c_int32),
                             _p(S, C.c_int32), torus.S1, step_tol, step_maxit, max_batch, precision)
    h = C.c_void_p()
    st = lib.fse_init_torus(C.byref(sysc), C.byref(desc), C.byref(h))
    if st != 0:
        msg = lib.fse_last_error(h).decode() if h else "init failed"
        if h:
            lib.fse_destroy(h)
        raise FseError(st, msg)
    U, St, bw = C.c_int32(), C.c_int32(), C.c_int32()
    lib.fse_get_layout(h, C.byref(U), C.byref(St), C.byref(bw), None)
    kt = np.zeros(((U.value + 1) // 2, max(torus.d - 1, 1)), np.int32)
    lib.fse_get_layout(h, None, None, None, _p(kt, C.c_int32))
    ctx = Context(h, lib, n, torus.d, U.value, St.value, bw.value, kt[:, : torus.d - 1])
    ctx.e = int(F.shape[0])
    ctx.bind_stream()
    beta, gamma = getattr(torus, "beta", 0.25), getattr(torus, "gamma", 0.5)
    if (beta, gamma) != (0.25, 0.5):
        fse_set_newmark(ctx, beta, gamma)
    if len(getattr(system, "con_k", ())):
        fse_set_contacts(ctx, system.con_dof, system.con_dir, system.con_gap, system.con_k)
    return ctx


def fse_get_layout(ctx: Context):
    return ctx.U, ctx.Stilde, ctx.half_band, ctx.ktable.copy()


def _omega(omega, B, d):
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64).reshape(B, d))
    return om


def _dev(x, shape):
    torch = _torch()
    t = torch.as_tensor(x, dtype=torch.float64, device="cuda").reshape(shape).contiguous()
    return t


def _inout(t, numel, name):
    """An array the library updates in place: a contiguous float64 CUDA tensor of numel entries."""
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
            and t.numel() == numel):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of {numel} entries (updated in place)")
    return C.c_void_p(t.data_ptr())


def fse_integrate_batch(ctx: Context, omega, Z0, want_phi=False):
    """omega [B][d] (host), Z0 [B][2n][U] -> zT [B][2n][S~], Phi [B][S~][2n][2n] or None."""
    torch = _torch()
    ctx.bind_stream()
    B = int(np.asarray(omega).reshape(-1, ctx.d).shape[0])
    om = _omega(omega, B, ctx.d)
    z0 = _dev(Z0, (B, 2 * ctx.n, ctx.U))
    zT = torch.empty((B, 2 * ctx.n, ctx.Stilde), dtype=torch.float64, device="cuda")
    phi = (torch.empty((B, ctx.Stilde, 2 * ctx.n, 2 * ctx.n), dtype=torch.float64, device="cuda")
           if want_phi else None)
    ctx.check(ctx.lib.fse_integrate_batch(ctx.h, B, _p(om, C.c_double), C.c_void_p(z0.data_ptr()),
                                          C.c_void_p(zT.data_ptr()),
                                          C.c_void_p(phi.data_ptr()) if phi is not None else None))
    return zT, phi


def fse_step_stats(ctx: Context):
    mx, tot = C.c_int32(), C.c_int64()
    ctx.check(ctx.lib.fse_step_stats(ctx.h, C.byref(mx), C.byref(tot)))
    return mx.value, tot.value


def fse_shooting_residual_jacobian(ctx: Context, omega, Z0, want_J=False):
    """-> (R [B][2n][U], ||R||_2 [B], J [B][2nU][2nU] or None)."""
    torch = _torch()
    ctx.bind_stream()
    B = int(np.asarray(omega).reshape(-1, ctx.d).shape[0])
    om = _omega(omega, B, ctx.d)
    z0 = _dev(Z0, (B, 2 * ctx.n, ctx.U))
    R = torch.empty_like(z0)
    rn = np.zeros(B)
    N = 2 * ctx.n * ctx.U
    J = torch.empty((B, N, N), dtype=torch.float64, device="cuda") if want_J else None
    ctx.check(ctx.lib.fse_shooting_residual_jacobian(
        ctx.h, B, _p(om, C.c_double), C.c_void_p(z0.data_ptr()), C.c_void_p(R.data_ptr()),
        _p(rn, C.c_double), C.c_void_p(J.data_ptr()) if J is not None else None, None))
    return R, rn, J


def _omega_inout(omega, d, e):
    """Host copy of omega [d] for a call that updates the unknown frequencies omega[e:] in place.
    With d > e the caller's omega must be a writable contiguous float64 ndarray of d entries
    (the updated frequencies are written back into it); anything else raises TypeError, so
    Z(0) and omega can never drift apart."""
    if d > e and not (isinstance(omega, np.ndarray) and omega.dtype == np.float64
                      and omega.size == d and omega.flags.writeable and omega.flags.c_contiguous):
        raise TypeError("with unknown frequencies (d > e) omega must be a writable contiguous "
                        "float64 numpy array of d entries; it is updated in place")
    return np.ascontiguousarray(np.asarray(omega, dtype=np.float64).reshape(d)).copy()


def _omega_back(omega, om):
    if isinstance(omega, np.ndarray) and omega.dtype == np.float64 and omega.size == om.size \
            and omega.flags.writeable and omega.flags.c_contiguous:
        omega.reshape(-1)[:] = om


def fse_newton_step(ctx: Context, omega, Z0):
    """Z0 (torch cuda tensor [2n][U], updated in place) -> ||R||_2 before the update.
    For d > e the unknown frequencies omega[e:] are updated in place (numpy float64 array)."""
    ctx.bind_stream()
    om = _omega_inout(omega, ctx.d, ctx.e)
    rn = C.c_double()
    ctx.check(ctx.lib.fse_newton_step(ctx.h, _p(om, C.c_double), _inout(Z0, 2 * ctx.n * ctx.U, "Z0"),
                                      C.byref(rn)))
    _omega_back(omega, om)
    return rn.value


def fse_newton_solve(ctx: Context, omega, Z0, tol=1e-8, maxit=20):
    """Z0 (torch cuda tensor, in place) -> (iterations, final ||R||_2).  For d > e the
    unknown frequencies omega[e:] are updated in place (numpy float64 array)."""
    ctx.bind_stream()
    om = _omega_inout(omega, ctx.d, ctx.e)
    it, rn = C.c_int32(), C.c_double()
    st = ctx.lib.fse_newton_solve(ctx.h, _p(om, C.c_double), _inout(Z0, 2 * ctx.n * ctx.U, "Z0"),
                                  tol, maxit, C.byref(it), C.byref(rn))
    _omega_back(omega, om)
    ctx.check(st)
    return it.value, rn.value


def fse_residual_domega(ctx: Context, omega, Z0):
    """-> (R [B][2n][U], dR/d omega_u [B][2nU][d-e]) for the unknown base frequencies."""
    torch = _torch()
    ctx.bind_stream()
    B = int(np.asarray(omega).reshape(-1, ctx.d).shape[0])
    om = _omega(omega, B, ctx.d)
    z0 = _dev(Z0, (B, 2 * ctx.n, ctx.U))
    R = torch.empty_like(z0)
    nu = ctx.d - ctx.e
    dR = torch.empty((B, 2 * ctx.n * ctx.U, max(nu, 1)), dtype=torch.float64, device="cuda")
    ctx.check(ctx.lib.fse_shooting_residual_jacobian(
        ctx.h, B, _p(om, C.c_double), C.c_void_p(z0.data_ptr()), C.c_void_p(R.data_ptr()), None,
        None, C.c_void_p(dR.data_ptr())))
    return R, dR


def fse_lyapunov(ctx: Context, omega, Z0, N_Ly=1000, Q0=None):
    ctx.bind_stream()
    om = _omega(omega, 1, ctx.d)
    z0 = _dev(Z0, (2 * ctx.n, ctx.U))
    q0 = _dev(Q0, (2 * ctx.n, 2 * ctx.n)) if Q0 is not None else None
    sig = np.zeros(2 * ctx.n)
    ctx.check(ctx.lib.fse_lyapunov(ctx.h, _p(om, C.c_double), C.c_void_p(z0.data_ptr()), N_Ly,
                                   C.c_void_p(q0.data_ptr()) if q0 is not None else None,
                                   _p(sig, C.c_double)))
    return sig


def fse_last_timing(ctx: Context):
    ms = np.zeros(4)
    nl = C.c_int32()
    ctx.check(ctx.lib.fse_last_timing(ctx.h, _p(ms, C.c_double), C.byref(nl)))
    return {"total_ms": ms[0], "state_ms": ms[1], "sens_ms": ms[2], "idft_ms": ms[3],
            "sens_launches": nl.value}


def fse_last_kernel_timing(ctx: Context):
    """-> (path of the last integration: 0 generic, 1 fused, 2 wide-band; summed duration [ms]
    of its dominant kernel's launches from HIP events on the context stream; launch count)."""
    path, ms, nl = C.c_int32(), C.c_double(), C.c_int32()
    ctx.check(ctx.lib.fse_last_kernel_timing(ctx.h, C.byref(path), C.byref(ms), C.byref(nl)))
    return path.value, ms.value, nl.value


def fse_get_tuning(ctx: Context):
    """-> (column waves per fused work-group in use, timed launches [ms] for 1 and 2 waves)."""
    ncw = C.c_int32()
    ms = np.zeros(2, np.float32)
    ctx.check(ctx.lib.fse_get_tuning(ctx.h, C.byref(ncw), _p(ms, C.c_float)))
    return ncw.value, ms


def fse_set_newmark(ctx: Context, beta, gamma):
    ctx.check(ctx.lib.fse_set_newmark(ctx.h, float(beta), float(gamma)))


def fse_set_contacts(ctx: Context, dof, direction, gap, stiffness):
    """Unilateral penalty contacts (host arrays of equal length m; m = 0 removes them)."""
    dof = np.ascontiguousarray(dof, dtype=np.int32).reshape(-1)
    dr = np.ascontiguousarray(direction, dtype=np.int32).reshape(-1)
    g = np.ascontiguousarray(gap, dtype=np.float64).reshape(-1)
    k = np.ascontiguousarray(stiffness, dtype=np.float64).reshape(-1)
    m = dof.size
    if not (dr.size == g.size == k.size == m):
        raise ValueError("contact arrays must have equal lengths")
    ctx.check(ctx.lib.fse_set_contacts(ctx.h, m, _p(dof, C.c_int32), _p(dr, C.c_int32), _p(g, C.c_double),
                                       _p(k, C.c_double)))


def fse_set_forcing(ctx: Context, amp):
    """Forcing amplitudes (host [e]) multiplying the unit load vectors."""
    a = np.ascontiguousarray(np.asarray(amp, dtype=np.float64).reshape(ctx.e))
    ctx.bind_stream()
    ctx.check(ctx.lib.fse_set_forcing(ctx.h, _p(a, C.c_double)))


def fse_secant_predict(ctx: Context, p_prev, p_cur, p_next, Z_prev, Z_cur):
    """-> Z_next [2n][U] (torch cuda) = Z_cur + tau (Z_cur - Z_prev)."""
    torch = _torch()
    ctx.bind_stream()
    pp = [np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel()) for x in (p_prev, p_cur, p_next)]
    zp = _dev(Z_prev, (2 * ctx.n, ctx.U))
    zc = _dev(Z_cur, (2 * ctx.n, ctx.U))
    zn = torch.empty_like(zc)
    ctx.check(ctx.lib.fse_secant_predict(ctx.h, len(pp[0]), _p(pp[0], C.c_double), _p(pp[1], C.c_double),
                                         _p(pp[2], C.c_double), C.c_void_p(zp.data_ptr()),
                                         C.c_void_p(zc.data_ptr()), C.c_void_p(zn.data_ptr())))
    return zn


def fse_continuation(ctx: Context, params, Z_init, tol=1e-8, maxit=20):
    """params host [P][d+e] (omega then forcing amplitudes) -> (Z [P][2n][U] torch cuda,
    iterations [P], final ||R|| [P]).  Raises FseError on a failed point (its iteration
    count is -1 in the error's .iters)."""
    torch = _torch()
    ctx.bind_stream()
    pr = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, ctx.d + ctx.e))
    P = pr.shape[0]
    z0 = _dev(Z_init, (2 * ctx.n, ctx.U))
    Z = torch.zeros((P, 2 * ctx.n, ctx.U), dtype=torch.float64, device="cuda")
    it = np.zeros(P, np.int32)
    rn = np.zeros(P)
    st = ctx.lib.fse_continuation(ctx.h, P, _p(pr, C.c_double), C.c_void_p(z0.data_ptr()), float(tol),
                                  int(maxit), C.c_void_p(Z.data_ptr()), _p(it, C.c_int32), _p(rn, C.c_double))
    if st != 0:
        err = FseError(st, ctx.lib.fse_last_error(ctx.h).decode())
        err.iters, err.rnorm, err.Z = it, rn, Z
        raise err
    return Z, it, rn


def fse_residual_dp(ctx: Context, omega, Z0):
    """omega host [B][d], Z0 [B][2n][U] -> (R, dR/dp) torch cuda [B][2n][U], p = omega_1 along
    the frequency conditions (forcing ratios fixed, unknown frequencies held)."""
    torch = _torch()
    ctx.bind_stream()
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64).reshape(-1, ctx.d))
    B = om.shape[0]
    Z = _dev(Z0, (B, 2 * ctx.n, ctx.U))
    R = torch.empty((B, 2 * ctx.n, ctx.U), dtype=torch.float64, device="cuda")
    dRdp = torch.empty_like(R)
    ctx.check(ctx.lib.fse_residual_dp(ctx.h, B, _p(om, C.c_double), C.c_void_p(Z.data_ptr()),
                                      C.c_void_p(R.data_ptr()), C.c_void_p(dRdp.data_ptr())))
    return R, dRdp


def fse_arclength(ctx: Context, omega0, Z_init, ds, npts, tol=1e-8, maxit=8):
    """Pseudo-arclength continuation in omega_1 from (omega0, Z_init): npts points ->
    (Z [P][2n][U] torch cuda, omega [P][d], steps [P], corrections [P], ||R|| [P]).  Raises
    FseError on a failed point, with the valid points attached (.Z, .omega, .iters...)."""
    torch = _torch()
    ctx.bind_stream()
    om0 = np.ascontiguousarray(np.asarray(omega0, dtype=np.float64).reshape(ctx.d))
    P = int(npts)
    z0 = _dev(Z_init, (2 * ctx.n, ctx.U))
    Z = torch.zeros((P, 2 * ctx.n, ctx.U), dtype=torch.float64, device="cuda")
    om = np.zeros((P, ctx.d))
    steps = np.zeros(P)
    it = np.zeros(P, np.int32)
    rn = np.zeros(P)
    st = ctx.lib.fse_arclength(ctx.h, P, _p(om0, C.c_double), C.c_void_p(z0.data_ptr()), float(ds), float(tol),
                               int(maxit), C.c_void_p(Z.data_ptr()), _p(om, C.c_double), _p(steps, C.c_double),
                               _p(it, C.c_int32), _p(rn, C.c_double))
    if st != 0:
        err = FseError(st, ctx.lib.fse_last_error(ctx.h).decode())
        err.Z, err.omega, err.steps, err.iters, err.rnorm = Z, om, steps, it, rn
        raise err
    return Z, om, steps, it, rn


def fse_shooting_residual_matfree(ctx: Context, omega, Z0):
    """omega host [d], Z0 [2n][U] -> (R torch cuda [2n][U], ||R||); keeps the sensitivities for
    fse_jacobian_apply."""
    torch = _torch()
    ctx.bind_stream()
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64).reshape(ctx.d))
    z = _dev(Z0, (2 * ctx.n, ctx.U))
    R = torch.empty((2 * ctx.n, ctx.U), dtype=torch.float64, device="cuda")
    rn = C.c_double()
    ctx.check(ctx.lib.fse_shooting_residual_matfree(ctx.h, _p(om, C.c_double), C.c_void_p(z.data_ptr()),
                                                    C.c_void_p(R.data_ptr()), C.byref(rn)))
    return R, rn.value


def fse_jacobian_apply(ctx: Context, v):
    """J v with the sensitivities of the last fse_shooting_residual_matfree."""
    torch = _torch()
    ctx.bind_stream()
    x = _dev(v, (2 * ctx.n, ctx.U))
    out = torch.empty_like(x)
    ctx.check(ctx.lib.fse_jacobian_apply(ctx.h, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr())))
    return out


def fse_jacobian_apply_noalloc(ctx: Context, v, out):
    """J v into the caller's out (torch cuda [2n][U]) without any device allocation (the library's
    fixed per-GPU scratch); the sensitivities of the last fse_shooting_residual_matfree."""
    ctx.bind_stream()
    x = _dev(v, (2 * ctx.n, ctx.U))
    ctx.check(ctx.lib.fse_jacobian_apply_noalloc(ctx.h, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr())))
    return out


def fse_newton_krylov_step(ctx: Context, omega, Z0, rtol=1e-10, restart=30, maxit=300, precond=True):
    """Z0 (torch cuda [2n][U], updated in place) <- Z0 + dZ with J dZ = -R by GMRES ->
    (||R|| before, GMRES iterations, relative linear residual).  For d > e the unknown
    frequencies omega[e:] are updated in place (numpy float64 array), as in fse_newton_step."""
    _torch()
    ctx.bind_stream()
    om = _omega_inout(omega, ctx.d, ctx.e)
    rn = C.c_double()
    its = C.c_int32()
    rel = C.c_double()
    st = ctx.lib.fse_newton_krylov_step(ctx.h, _p(om, C.c_double), _inout(Z0, 2 * ctx.n * ctx.U, "Z0"), float(rtol),
                                        int(restart), int(maxit), int(bool(precond)), C.byref(rn),
                                        C.byref(its), C.byref(rel))
    ctx.check(st)
    _omega_back(omega, om)
    return rn.value, its.value, rel.value


def fse_newton_krylov_chord_step(ctx: Context, omega, Z0, rtol=1e-10, restart=30, maxit=300, precond=True):
    """Simplified Newton step with the stored Jacobian (that of the last matrix-free
    evaluation): Z0 (torch cuda [2n][U], in place) <- Z0 + dZ with J_stored dZ = -R(omega, Z0),
    R from the states alone -> (||R|| before, GMRES iterations, relative linear residual)."""
    _torch()
    ctx.bind_stream()
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64).reshape(ctx.d))
    rn = C.c_double()
    its = C.c_int32()
    rel = C.c_double()
    st = ctx.lib.fse_newton_krylov_chord_step(ctx.h, _p(om, C.c_double), _inout(Z0, 2 * ctx.n * ctx.U, "Z0"), float(rtol),
                                              int(restart), int(maxit), int(bool(precond)), C.byref(rn),
                                              C.byref(its), C.byref(rel))
    ctx.check(st)
    return rn.value, its.value, rel.value


def fse_hypertime_residual_jacobian(ctx: Context, omega, zbar0, want_J=False):
    """Hyper-time shooting (samples as unknowns): omega [B][d], zbar0 [B][2n][S~] ->
    (R torch cuda [B][2n][S~], ||R|| [B], J [B][2nS~][2nS~] or None)."""
    torch = _torch()
    ctx.bind_stream()
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64).reshape(-1, ctx.d))
    B = om.shape[0]
    z = _dev(zbar0, (B, 2 * ctx.n, ctx.Stilde))
    R = torch.empty_like(z)
    rn = np.zeros(B)
    Nh = 2 * ctx.n * ctx.Stilde
    J = torch.empty((B, Nh, Nh), dtype=torch.float64, device="cuda") if want_J else None
    ctx.check(ctx.lib.fse_hypertime_residual_jacobian(ctx.h, B, _p(om, C.c_double), C.c_void_p(z.data_ptr()),
                                                      C.c_void_p(R.data_ptr()), _p(rn, C.c_double),
                                                      C.c_void_p(J.data_ptr()) if J is not None else None))
    return R, rn, J


def fse_multiple_residual_jacobian(ctx: Context, M, omega, Zs, want_J=False):
    """Multiple shooting over M segments: omega [d], Zs [M][2n][U] -> (R torch cuda [M][2n][U],
    ||R||_2, J [M 2nU][M 2nU] or None)."""
    torch = _torch()
    ctx.bind_stream()
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64).reshape(ctx.d))
    z = _dev(Zs, (int(M), 2 * ctx.n, ctx.U))
    R = torch.empty_like(z)
    rn = C.c_double()
    NM = int(M) * 2 * ctx.n * ctx.U
    J = torch.empty((NM, NM), dtype=torch.float64, device="cuda") if want_J else None
    ctx.check(ctx.lib.fse_multiple_residual_jacobian(ctx.h, int(M), _p(om, C.c_double), C.c_void_p(z.data_ptr()),
                                                     C.c_void_p(R.data_ptr()), C.byref(rn),
                                                     C.c_void_p(J.data_ptr()) if J is not None else None))
    return R, rn.value, J


def fse_multiple_newton_step(ctx: Context, M, omega, Zs):
    """Zs (torch cuda [M][2n][U], updated in place) <- one dense Newton step -> ||R|| before.
    For d > e the unknown frequencies omega[e:] are updated in place (numpy float64 array)."""
    _torch()
    ctx.bind_stream()
    om = _omega_inout(omega, ctx.d, ctx.e)
    rn = C.c_double()
    ctx.check(ctx.lib.fse_multiple_newton_step(ctx.h, int(M), _p(om, C.c_double), _inout(Zs, int(M) * 2 * ctx.n * ctx.U, "Zs"),
                                               C.byref(rn)))
    _omega_back(omega, om)
    return rn.value


def fse_hypertime_newton_step(ctx: Context, omega, zbar0):
    """zbar0 (torch cuda [2n][S~], updated in place) <- one dense Newton step -> ||R|| before.
    For d > e the unknown frequencies omega[e:] are updated in place (numpy float64 array)."""
    _torch()
    ctx.bind_stream()
    om = _omega_inout(omega, ctx.d, ctx.e)
    rn = C.c_double()
    ctx.check(ctx.lib.fse_hypertime_newton_step(ctx.h, _p(om, C.c_double), _inout(zbar0, 2 * ctx.n * ctx.Stilde, "zbar0"),
                                                C.byref(rn)))
    _omega_back(omega, om)
    return rn.value


class Learned:
    """Owns an fse_learned (POD + MLP predictor) bound to a Context."""

    def __init__(self, ctx: Context, handle, n_in, hidden, rank):
        self.ctx, self.h = ctx, handle
        self.n_in, self.hidden, self.rank = n_in, hidden, rank
        self.num_params = int(ctx.lib.fse_learned_num_params(handle))

    def set_params(self, flat):
        a = np.ascontiguousarray(np.asarray(flat, dtype=np.float32).reshape(self.num_params))
        self.ctx.bind_stream()
        self.ctx.check(self.ctx.lib.fse_learned_set_params(self.h, _p(a, C.c_float)))

    def get_params(self):
        a = np.zeros(self.num_params, np.float32)
        self.ctx.check(self.ctx.lib.fse_learned_get_params(self.h, _p(a, C.c_float)))
        return a

    def fit_pod(self, X):
        """X: [m][2n][U] (or [m][N]) converged Z(0) -> singular values [min(m, rank)]."""
        ctx = self.ctx
        ctx.bind_stream()
        N = 2 * ctx.n * ctx.U
        Xd = _dev(X, (-1, N))
        m = Xd.shape[0]
        sig = np.zeros(min(m, self.rank))
        ctx.check(ctx.lib.fse_learned_fit_pod(self.h, m, C.c_void_p(Xd.data_ptr()), _p(sig, C.c_double)))
        return sig

    def get_pod(self):
        torch = _torch()
        ctx = self.ctx
        N = 2 * ctx.n * ctx.U
        mean = torch.empty(N, dtype=torch.float64, device="cuda")
        modes = torch.empty((N, self.rank), dtype=torch.float64, device="cuda")
        ctx.check(ctx.lib.fse_learned_get_pod(self.h, C.c_void_p(mean.data_ptr()), C.c_void_p(modes.data_ptr())))
        return mean, modes

    def loss_grad(self, x, t):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
        t = np.ascontiguousarray(np.asarray(t, dtype=np.float32))
        g = np.zeros(self.num_params, np.float32)
        loss = C.c_float()
        self.ctx.bind_stream()
        self.ctx.check(self.ctx.lib.fse_learned_loss_grad(self.h, x.shape[0], _p(x, C.c_float), _p(t, C.c_float),
                                                          C.byref(loss), _p(g, C.c_float)))
        return loss.value, g

    def fit(self, x, t, steps, lr=1e-3, wd=1e-4):
        """AdamW steps on normalised data (x [B][n_in], t [B][rank]) -> loss history."""
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
        t = np.ascontiguousarray(np.asarray(t, dtype=np.float32))
        hist = np.zeros(steps)
        self.ctx.bind_stream()
        self.ctx.check(self.ctx.lib.fse_learned_fit(self.h, x.shape[0], _p(x, C.c_float), _p(t, C.c_float),
                                                    int(steps), float(lr), float(wd), _p(hist, C.c_double)))
        return hist

    def train(self, P, X, epochs=2000, lr=1e-3, wd=1e-4):
        ctx = self.ctx
        ctx.bind_stream()
        N = 2 * ctx.n * ctx.U
        Pp = np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(-1, self.n_in))
        Xd = _dev(X, (-1, N))
        hist = np.zeros(epochs)
        ctx.check(ctx.lib.fse_learned_train(self.h, Pp.shape[0], _p(Pp, C.c_double), C.c_void_p(Xd.data_ptr()),
                                            int(epochs), float(lr), float(wd), _p(hist, C.c_double)))
        return hist

    def predict(self, p):
        torch = _torch()
        ctx = self.ctx
        ctx.bind_stream()
        pp = np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(self.n_in))
        Z = torch.empty((2 * ctx.n, ctx.U), dtype=torch.float64, device="cuda")
        ctx.check(ctx.lib.fse_learned_predict(self.h, _p(pp, C.c_double), C.c_void_p(Z.data_ptr())))
        return Z

    def forward(self, x, bf16=False):
        """Raw network outputs y [B][rank] (FP32 host) for normalised inputs x [B][n_in]."""
        _torch()
        self.ctx.bind_stream()
        xf = np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(-1, self.n_in))
        y = np.zeros((xf.shape[0], self.rank), np.float32)
        self.ctx.check(self.ctx.lib.fse_learned_forward(self.h, xf.shape[0], _p(xf, C.c_float), int(bool(bf16)),
                                                        _p(y, C.c_float)))
        return y

    def predict_batch(self, params, bf16=False):
        """Predictions Z [P][2n][U] (torch cuda) for parameters [P][n_in] in one batch."""
        torch = _torch()
        ctx = self.ctx
        ctx.bind_stream()
        pp = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, self.n_in))
        Z = torch.empty((pp.shape[0], 2 * ctx.n, ctx.U), dtype=torch.float64, device="cuda")
        ctx.check(ctx.lib.fse_learned_predict_batch(self.h, pp.shape[0], _p(pp, C.c_double), int(bool(bf16)),
                                                    C.c_void_p(Z.data_ptr())))
        return Z

    def __del__(self):
        try:
            if self.h:
                self.ctx.lib.fse_learned_destroy(self.h)
                self.h = None
        except Exception:
            pass


def fse_learned_create(ctx: Context, n_in=3, hidden=256, rank=64) -> Learned:
    h = C.c_void_p()
    ctx.bind_stream()
    ctx.check(ctx.lib.fse_learned_create(ctx.h, n_in, hidden, rank, C.byref(h)))
    return Learned(ctx, h, n_in, hidden, rank)


def fse_continuation_learned(ctx: Context, params, features, Z_init, learned: Learned, first_learned,
                             tol=1e-8, maxit=20):
    """As fse_continuation, with the learned predictor judged against the secant predictor
    from point first_learned on -> (Z, iterations, residuals, used_learned)."""
    torch = _torch()
    ctx.bind_stream()
    pr = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, ctx.d + ctx.e))
    ft = np.ascontiguousarray(np.asarray(features, dtype=np.float64).reshape(pr.shape[0], learned.n_in))
    P = pr.shape[0]
    z0 = _dev(Z_init, (2 * ctx.n, ctx.U))
    Z = torch.zeros((P, 2 * ctx.n, ctx.U), dtype=torch.float64, device="cuda")
    it = np.zeros(P, np.int32)
    rn = np.zeros(P)
    used = np.zeros(P, np.int32)
    st = ctx.lib.fse_continuation_learned(ctx.h, P, _p(pr, C.c_double), _p(ft, C.c_double), C.c_void_p(z0.data_ptr()),
                                          float(tol), int(maxit), learned.h, int(first_learned),
                                          C.c_void_p(Z.data_ptr()), _p(it, C.c_int32), _p(rn, C.c_double),
                                          _p(used, C.c_int32))
    if st != 0:
        err = FseError(st, ctx.lib.fse_last_error(ctx.h).decode())
        err.iters, err.rnorm, err.Z, err.used = it, rn, Z, used
        raise err
    return Z, it, rn, used
