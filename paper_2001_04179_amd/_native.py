"""ctypes declarations of the C ABI in ``include/rebk.h`` (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librebk.so")

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
U64 = ctypes.c_uint64
F64 = ctypes.c_double

# rebk_dtype_t
F64_T, F32_T, BF16_T, F16_T = 0, 1, 2, 3
DTYPES = {"f64": F64_T, "f32": F32_T, "bf16": BF16_T, "f16": F16_T}

# rebk_status_t
OK, NOT_CONVERGED, DIVERGED = 0, 1, 2
ERR_INVALID, ERR_HIP, ERR_OOM, ERR_TIMEOUT = -1, -2, -3, -4
STATUS_NAMES = {0: "ok", 1: "not_converged", 2: "diverged", -1: "invalid", -2: "hip_error", -3: "oom",
                -4: "timeout"}

# rebk_kernel_t
KERNELS = {"auto": 0, "workgroup": 1, "grid": 2, "pipe": 3}
KERNEL_NAMES = {v: k for k, v in KERNELS.items()}


class Result(ctypes.Structure):
    _fields_ = [("status", I32), ("kernel", I32), ("iterations", I64), ("rel_err", F64), ("time_ms", F64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("b_dev", P), ("x0_dev", P), ("z0_dev", P), ("k0", I64), ("max_iter", I64),
        ("x_ref_dev", P), ("tol", F64), ("check_every", I64), ("x_out_dev", P), ("z_out_dev", P),
        ("trace_j_dev", P), ("trace_i_dev", P), ("kernel", I32), ("grid_wgs", I32),
    ]


class RefineOpts(ctypes.Structure):
    _fields_ = [
        ("A_dev", P), ("lda", I64), ("b_dev", P), ("x0_dev", P), ("x_ref_dev", P), ("tol", F64),
        ("inner_iters", I64), ("max_outer", I32), ("kernel", I32), ("grid_wgs", I32),
        ("x_out_dev", P), ("z_out_dev", P), ("err_trace", P),
    ]


class BatchOpts(ctypes.Structure):
    _fields_ = [
        ("nrhs", P), ("b_dev", P), ("x0_dev", P), ("x_ref_dev", P), ("x_out_dev", P), ("z_out_dev", P),
        ("max_iter", I64), ("tol", F64), ("check_every", I64), ("threads", I32), ("lds_budget", I32),
        ("max_tile", I32), ("xcd_order", I32), ("z0_from_x0", I32), ("team", I32),
    ]


class BatchRhs(ctypes.Structure):
    _fields_ = [("iterations", I64), ("rel_err", F64), ("status", I32), ("tile", I32), ("team", I32)]


# name -> (restype, argtypes); every function declared in include/rebk.h
SIGNATURES = {
    "rebk_create": (ctypes.c_int, [ctypes.POINTER(P), P, I32, I32, I64, I64, I64, P, I64, P, I64, F64, U64, P]),
    "rebk_destroy": (None, [P]),
    "rebk_solve": (ctypes.c_int, [P, P, P, P, F64, I64, ctypes.POINTER(Result)]),
    "rebk_solve_ex": (ctypes.c_int, [P, ctypes.POINTER(SolveOpts), ctypes.POINTER(Result)]),
    "rebk_solve_ex_static": (ctypes.c_int, [P, ctypes.POINTER(SolveOpts), ctypes.POINTER(Result)]),
    "rebk_pipe_prepare": (ctypes.c_int, [P, ctypes.POINTER(F64)]),
    "rebk_pipe_release": (None, [P]),
    "rebk_get_weights": (ctypes.c_int, [P, P, P]),
    "rebk_get_thresholds": (ctypes.c_int, [P, P, P]),
    "rebk_get_info": (ctypes.c_int, [P] + [ctypes.POINTER(I64)] * 6),
    "rebk_sample_blocks": (ctypes.c_int, [P, U64, I64, I64, P, P]),
    "rebk_philox4x64_10": (ctypes.c_int, [U64, U64, U64, U64, U64, U64, I64, P, P]),
    "rebk_solve_refined": (ctypes.c_int, [P, ctypes.POINTER(RefineOpts), ctypes.POINTER(Result)]),
    "rebk_block_betas": (ctypes.c_int, [P, I32, F64, P, P, ctypes.POINTER(F64), ctypes.POINTER(I32)]),
    "rebk_batch_create": (ctypes.c_int, [ctypes.POINTER(P), I32, P, P, P]),
    "rebk_batch_destroy": (None, [P]),
    "rebk_batch_solve": (ctypes.c_int, [P, ctypes.POINTER(BatchOpts), P, ctypes.POINTER(F64)]),
    "rebk_batch_autotune": (ctypes.c_int, [P, ctypes.POINTER(BatchOpts), I64, ctypes.POINTER(I32),
                                           ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32),
                                           ctypes.POINTER(F64)]),
    "rebk_mlp_create": (ctypes.c_int, [ctypes.POINTER(P), I32, I32, P, I64, I64, F64, I32, U64, P]),
    "rebk_mlp_destroy": (None, [P]),
    "rebk_mlp_set_params": (ctypes.c_int, [P, P, P, P, P, P, P]),
    "rebk_mlp_get_params": (ctypes.c_int, [P, P, P, P, P, P, P]),
    "rebk_mlp_forward": (ctypes.c_int, [P, P, I32, F64, P, P]),
    "rebk_mlp_grad": (ctypes.c_int, [P, P, P, I32, F64, ctypes.POINTER(F64)]),
    "rebk_mlp_get_grads": (ctypes.c_int, [P, P, P, P, P, P, P]),
    "rebk_mlp_adam": (ctypes.c_int, [P, F64, F64, F64, F64]),
    "rebk_mlp_train_step": (ctypes.c_int, [P, P, P, I32, F64, F64, ctypes.POINTER(F64)]),
    "rebk_last_error": (ctypes.c_char_p, []),
    "rebk_version": (ctypes.c_char_p, []),
}

_lib = None


class NativeLibraryMissing(RuntimeError):
    pass


def load():
    """Load ``librebk.so``; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise NativeLibraryMissing(
            f"{LIB_PATH} is missing: build it with `python -m paper_2001_04179_amd.build` "
            "(the REBK path only runs in the HIP library)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().rebk_last_error().decode()


class RebkError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where} failed with {STATUS_NAMES.get(code, code)}: {last_error()}")


def check(code: int, where: str) -> int:
    if code < 0:
        raise RebkError(code, where)
    return code
