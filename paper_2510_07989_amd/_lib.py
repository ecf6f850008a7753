"""ctypes declarations of libmot.so (the C ABI in include/mot.h)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmot.so")

MOT_OK, MOT_EINVAL, MOT_ENOMEM, MOT_ENOCONV, MOT_EHIP, MOT_ESTATE, MOT_ECANCEL = 0, -1, -2, -3, -4, -5, -6
MOT_FP64, MOT_MIXED, MOT_MIXED32 = 0, 1, 2
FAM_H, FAM_HAT, FAM_TILDE = 0, 1, 2
MED_EXT, MED_INT = 0, 1
OP_T, OP_K = 0, 1

_P = ctypes.c_void_p
_I = ctypes.c_int32
_D = ctypes.c_double


class MotMesh(ctypes.Structure):
    _fields_ = [("nv", _I), ("nf", _I), ("ne", _I), ("verts", _P), ("tris", _P), ("edges", _P)]


class MotPlaneWave(ctypes.Structure):
    _fields_ = [("amp", _D), ("pol", _D * 3), ("dir", _D * 3), ("width", _D), ("t0", _D)]


class MotOptions(ctypes.Structure):
    _fields_ = [("precision", _I), ("gmres_tol", _D), ("gmres_restart", _I), ("gmres_maxit", _I),
                ("cg_tol", _D), ("cg_maxit", _I), ("diameter", _D), ("keep_history", _I),
                ("max_steps", _I), ("mem_cap_bytes", ctypes.c_uint64), ("profile", _I),
                ("precond", _I), ("stream_split", _I), ("history_order", _I),
                ("hilo_lags", _I), ("mix_group", _I), ("spec_window", _I),
                ("recovery", _I), ("autotune", _I), ("graph", _I), ("tile_wg", _I), ("history_form", _I)]


class MotStepInfo(ctypes.Structure):
    _fields_ = [("step", _I), ("gmres_iters", _I), ("gmres_relres", _D), ("converged", _I)]


class MotInfo(ctypes.Structure):
    _fields_ = [("D", _D), ("Tmax", _D), ("dt", _D), ("kmax", _I), ("nlags", _I), ("ne", _I),
                ("n", _I), ("nrhs", _I), ("genus", _I), ("folded", _I), ("steps_done", _I),
                ("device_bytes", ctypes.c_uint64), ("setup_ms", _D), ("fold_ms", _D),
                ("gmres_iters_total", ctypes.c_int64), ("hist_ms", _D), ("hist_launches", ctypes.c_int64),
                ("q0_ms", _D), ("q0_launches", ctypes.c_int64), ("recover_ms", _D),
                ("precond_iters", _I), ("precond_resid", _D), ("peak_bytes", ctypes.c_uint64),
                ("tuned", _I), ("sched_hist", _I), ("sched_q0", _I), ("sched_pc", _I), ("tune_ms", _D),
                ("graph_windows", ctypes.c_int64), ("hist_wg", _I), ("q0_wg", _I)]


EXPORTS = ["mot_default_options", "mot_create", "mot_set_lag", "mot_set_lag_csr", "mot_step",
           "mot_run", "mot_get_matrix", "mot_get_info", "mot_reset", "mot_destroy",
           "mot_last_error", "mot_footprint", "mot_get_steps", "mot_run_batch",
           "mot_far_field", "mot_checkpoint_size", "mot_checkpoint", "mot_restore",
           "mot_step_norms", "mot_set_lag_device", "mot_step_norms_noalloc", "mot_cancel"]

_lib = None


def load():
    """Load libmot.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmot.so is not built (run __graft_entry__.build() or "
                           "python paper_2510_07989_amd/build.py)")
    # PyTorch ships its own HIP runtime with the same soname as the system one.
    # Loading torch first makes libmot bind to that runtime, so the process has
    # one HIP runtime and torch's streams and device tensors are valid handles
    # for the library (loaded the other way round, two runtimes would coexist).
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    lib.mot_default_options.argtypes = [ctypes.POINTER(MotOptions)]
    lib.mot_default_options.restype = None
    lib.mot_create.argtypes = [ctypes.POINTER(MotMesh), _D, _D, _D, _P, _P, _P, _P, _P, _I,
                               ctypes.POINTER(MotPlaneWave), ctypes.POINTER(MotOptions), _P,
                               ctypes.POINTER(_P)]
    lib.mot_create.restype = _I
    lib.mot_set_lag.argtypes = [_P, _I, _I, _I, _I, _P]
    lib.mot_set_lag_device.argtypes = [_P, _I, _I, _I, _I, _P, ctypes.c_int64]
    lib.mot_set_lag_device.restype = _I
    lib.mot_set_lag.restype = _I
    lib.mot_set_lag_csr.argtypes = [_P, _I, _I, _I, _I, _P, _P, _P]
    lib.mot_set_lag_csr.restype = _I
    lib.mot_step.argtypes = [_P, ctypes.POINTER(MotStepInfo)]
    lib.mot_step.restype = _I
    lib.mot_run.argtypes = [_P, _I, _P, _P, _P, _I, ctypes.POINTER(MotStepInfo)]
    lib.mot_run.restype = _I
    lib.mot_get_steps.argtypes = [_P, _I, _I, _P, _P, _P, _I]
    lib.mot_get_steps.restype = _I
    lib.mot_far_field.argtypes = [_P, _I, _I, _D, _I, _P, _P, _P]
    lib.mot_far_field.restype = _I
    lib.mot_checkpoint_size.argtypes = [_P, _I, ctypes.POINTER(ctypes.c_uint64)]
    lib.mot_checkpoint_size.restype = _I
    lib.mot_checkpoint.argtypes = [_P, _I, _P, ctypes.c_uint64]
    lib.mot_checkpoint.restype = _I
    lib.mot_restore.argtypes = [_P, _P, ctypes.c_uint64]
    lib.mot_restore.restype = _I
    lib.mot_step_norms.argtypes = [_P, _I, _I, _P]
    lib.mot_step_norms.restype = _I
    lib.mot_step_norms_noalloc.argtypes = [_P, _I, _I, _P]
    lib.mot_step_norms_noalloc.restype = _I
    lib.mot_run_batch.argtypes = [ctypes.POINTER(_P), _I, _I, ctypes.POINTER(_I)]
    lib.mot_run_batch.restype = _I
    lib.mot_cancel.argtypes = [_P]
    lib.mot_cancel.restype = _I
    lib.mot_get_matrix.argtypes = [_P, _I, _I, _P]
    lib.mot_get_matrix.restype = _I
    lib.mot_get_info.argtypes = [_P, ctypes.POINTER(MotInfo)]
    lib.mot_get_info.restype = _I
    lib.mot_reset.argtypes = [_P]
    lib.mot_reset.restype = _I
    lib.mot_destroy.argtypes = [_P]
    lib.mot_destroy.restype = None
    lib.mot_last_error.argtypes = [_P]
    lib.mot_last_error.restype = ctypes.c_char_p
    lib.mot_footprint.argtypes = [ctypes.POINTER(MotMesh), _D, _D, _D, _I, ctypes.c_int64,
                                  ctypes.POINTER(MotOptions), ctypes.POINTER(ctypes.c_uint64),
                                  ctypes.POINTER(ctypes.c_uint64)]
    lib.mot_footprint.restype = _I
    _lib = lib
    return lib
