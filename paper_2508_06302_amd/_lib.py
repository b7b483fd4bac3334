"""ctypes declarations of include/fse.h.  Loading fails loudly if libfse.so is absent."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfse.so")

FSE_STATUS = {0: "FSE_OK", 1: "FSE_E_INVAL", 2: "FSE_E_NOMEM", 3: "FSE_E_DEVICE",
              4: "FSE_E_NOCONV", 5: "FSE_E_SINGULAR", 6: "FSE_E_NAN", 7: "FSE_E_UNSUPPORTED"}

EXPORTS = ["fse_init_torus", "fse_get_layout", "fse_set_stream", "fse_integrate_batch",
           "fse_step_stats", "fse_shooting_residual_jacobian", "fse_newton_step",
           "fse_newton_solve", "fse_lyapunov", "fse_set_forcing", "fse_set_newmark", "fse_set_contacts", "fse_secant_predict",
           "fse_continuation", "fse_continuation_learned", "fse_residual_dp", "fse_arclength",
           "fse_shooting_residual_matfree", "fse_jacobian_apply", "fse_jacobian_apply_noalloc", "fse_newton_krylov_step",
           "fse_newton_krylov_chord_step",
           "fse_hypertime_residual_jacobian", "fse_hypertime_newton_step", "fse_multiple_residual_jacobian",
           "fse_multiple_newton_step", "fse_learned_create",
           "fse_learned_num_params", "fse_learned_inputs", "fse_learned_set_params",
           "fse_learned_get_params", "fse_learned_fit_pod", "fse_learned_get_pod",
           "fse_learned_loss_grad", "fse_learned_fit", "fse_learned_train", "fse_learned_predict",
           "fse_learned_forward", "fse_learned_predict_batch",
           "fse_learned_destroy", "fse_last_kernel_timing", "fse_get_tuning", "fse_last_timing", "fse_last_error", "fse_destroy"]

i32p = C.POINTER(C.c_int32)
f64p = C.POINTER(C.c_double)


class FseSystem(C.Structure):
    _fields_ = [("n", C.c_int32),
                ("M_ptr", i32p), ("M_idx", i32p), ("M_val", f64p),
                ("D_ptr", i32p), ("D_idx", i32p), ("D_val", f64p),
                ("K_ptr", i32p), ("K_idx", i32p), ("K_val", f64p),
                ("nnz2", C.c_int64), ("t2_idx", i32p), ("t2_val", f64p),
                ("nnz3", C.c_int64), ("t3_idx", i32p), ("t3_val", f64p),
                ("e", C.c_int32), ("F", f64p)]


class FseTorusDesc(C.Structure):
    _fields_ = [("d", C.c_int32), ("e", C.c_int32), ("K_len", i32p), ("K_list", i32p),
                ("S", i32p), ("S1", C.c_int32), ("step_tol", C.c_double),
                ("step_maxit", C.c_int32), ("max_batch", C.c_int32), ("precision", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libfse.so and declare every C-ABI signature.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with paper_2508_06302_amd.build.build()")
    # torch bundles its own HIP runtime (SONAME libamdhip64.so.7).  Importing torch first
    # makes libfse.so bind to that already-loaded runtime, so the process holds one HIP
    # runtime and torch's device pointers and streams are valid in the library.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.fse_init_torus.argtypes = [C.POINTER(FseSystem), C.POINTER(FseTorusDesc), C.POINTER(vp)]
    lib.fse_get_layout.argtypes = [vp, i32p, i32p, i32p, i32p]
    lib.fse_set_stream.argtypes = [vp, vp]
    lib.fse_integrate_batch.argtypes = [vp, C.c_int32, f64p, vp, vp, vp]
    lib.fse_step_stats.argtypes = [vp, i32p, C.POINTER(C.c_int64)]
    lib.fse_shooting_residual_jacobian.argtypes = [vp, C.c_int32, f64p, vp, vp, f64p, vp, vp]
    lib.fse_newton_step.argtypes = [vp, f64p, vp, f64p]
    lib.fse_newton_solve.argtypes = [vp, f64p, vp, C.c_double, C.c_int32, i32p, f64p]
    lib.fse_lyapunov.argtypes = [vp, f64p, vp, C.c_int32, vp, f64p]
    lib.fse_set_forcing.argtypes = [vp, f64p]
    lib.fse_set_newmark.argtypes = [vp, C.c_double, C.c_double]
    lib.fse_set_contacts.argtypes = [vp, C.c_int32, i32p, i32p, f64p, f64p]
    lib.fse_secant_predict.argtypes = [vp, C.c_int32, f64p, f64p, f64p, vp, vp, vp]
    lib.fse_continuation.argtypes = [vp, C.c_int32, f64p, vp, C.c_double, C.c_int32, vp, i32p, f64p]
    lib.fse_residual_dp.argtypes = [vp, C.c_int32, f64p, vp, vp, vp]
    lib.fse_shooting_residual_matfree.argtypes = [vp, f64p, vp, vp, f64p]
    lib.fse_jacobian_apply.argtypes = [vp, vp, vp]
    lib.fse_jacobian_apply_noalloc.argtypes = [vp, vp, vp]
    lib.fse_hypertime_residual_jacobian.argtypes = [vp, C.c_int32, f64p, vp, vp, f64p, vp]
    lib.fse_hypertime_newton_step.argtypes = [vp, f64p, vp, f64p]
    lib.fse_multiple_residual_jacobian.argtypes = [vp, C.c_int32, f64p, vp, vp, f64p, vp]
    lib.fse_multiple_newton_step.argtypes = [vp, C.c_int32, f64p, vp, f64p]
    lib.fse_newton_krylov_step.argtypes = [vp, f64p, vp, C.c_double, C.c_int32, C.c_int32, C.c_int32, f64p,
                                           i32p, f64p]
    lib.fse_newton_krylov_chord_step.argtypes = [vp, f64p, vp, C.c_double, C.c_int32, C.c_int32, C.c_int32,
                                                 f64p, i32p, f64p]
    lib.fse_arclength.argtypes = [vp, C.c_int32, f64p, vp, C.c_double, C.c_double, C.c_int32, vp, f64p,
                                  f64p, i32p, f64p]
    f32p = C.POINTER(C.c_float)
    lib.fse_continuation_learned.argtypes = [vp, C.c_int32, f64p, f64p, vp, C.c_double, C.c_int32, vp,
                                             C.c_int32, vp, i32p, f64p, i32p]
    lib.fse_learned_create.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(vp)]
    lib.fse_learned_num_params.argtypes = [vp]
    lib.fse_learned_num_params.restype = C.c_int64
    lib.fse_learned_inputs.argtypes = [vp]
    lib.fse_learned_inputs.restype = C.c_int32
    lib.fse_learned_set_params.argtypes = [vp, f32p]
    lib.fse_learned_get_params.argtypes = [vp, f32p]
    lib.fse_learned_fit_pod.argtypes = [vp, C.c_int32, vp, f64p]
    lib.fse_learned_get_pod.argtypes = [vp, vp, vp]
    lib.fse_learned_loss_grad.argtypes = [vp, C.c_int32, f32p, f32p, f32p, f32p]
    lib.fse_learned_fit.argtypes = [vp, C.c_int32, f32p, f32p, C.c_int32, C.c_double, C.c_double, f64p]
    lib.fse_learned_train.argtypes = [vp, C.c_int32, f64p, vp, C.c_int32, C.c_double, C.c_double, f64p]
    lib.fse_learned_predict.argtypes = [vp, f64p, vp]
    lib.fse_learned_forward.argtypes = [vp, C.c_int32, f32p, C.c_int32, f32p]
    lib.fse_learned_predict_batch.argtypes = [vp, C.c_int32, f64p, C.c_int32, vp]
    lib.fse_learned_destroy.argtypes = [vp]
    lib.fse_learned_destroy.restype = None
    lib.fse_last_kernel_timing.argtypes = [vp, i32p, f64p, i32p]
    lib.fse_get_tuning.argtypes = [vp, i32p, f32p]
    lib.fse_last_timing.argtypes = [vp, f64p, i32p]
    lib.fse_last_error.argtypes = [vp]
    lib.fse_last_error.restype = C.c_char_p
    lib.fse_destroy.argtypes = [vp]
    lib.fse_destroy.restype = None
    for name in EXPORTS:
        if name not in ("fse_last_error", "fse_destroy", "fse_learned_destroy", "fse_learned_num_params",
                        "fse_learned_inputs"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib
