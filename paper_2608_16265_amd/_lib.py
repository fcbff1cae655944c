"""ctypes view of the C ABI declared in include/exa.h.

This module only loads the shared library and declares the signatures; it
fails loudly (ImportError) when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libexa.so")

EXA_OK, EXA_EINVAL, EXA_ENOMEM, EXA_ECOMPILE, EXA_EHIP, EXA_ESTATE = range(6)
KIND = {"obj": 0, "con": 1, "aug": 2}
OPCODE = {
    "const": 0, "data": 1, "var": 2, "param": 3,
    "neg": 10, "abs2": 11, "inv": 12, "sqrt": 13, "exp": 14, "log": 15, "sin": 16,
    "cos": 17, "tan": 18, "atan": 19, "sinh": 20, "cosh": 21, "tanh": 22, "log1p": 23,
    "expm1": 24, "add": 40, "sub": 41, "mul": 42, "div": 43, "pow": 44,
}

P_i32 = C.POINTER(C.c_int32)
P_i64 = C.POINTER(C.c_int64)
P_f64 = C.POINTER(C.c_double)


class PatternDesc(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("nnodes", C.c_int32),
        ("op", P_i32), ("a", P_i32), ("b", P_i32), ("off", P_i64), ("val", P_f64),
        ("ndata", C.c_int64), ("n_icols", C.c_int32), ("n_fcols", C.c_int32),
        ("icols", C.POINTER(P_i32)), ("fcols", C.POINTER(P_f64)),
        ("target", C.c_int32), ("row_icol", C.c_int32), ("row_off", C.c_int64),
        ("lcon", P_f64), ("ucon", P_f64),
    ]


class Options(C.Structure):
    _fields_ = [("host_only", C.c_int32), ("block", C.c_int32), ("epl", C.c_int32),
                ("autotune", C.c_int32), ("fuse", C.c_int32), ("eval_per_mode", C.c_int32),
                ("reserved", C.c_int32 * 2), ("cache_dir", C.c_char_p), ("max_device_bytes", C.c_int64)]


class BatchOptions(C.Structure):
    _fields_ = [("autotune", C.c_int32), ("block", C.c_int32), ("epl", C.c_int32),
                ("fuse", C.c_int32), ("units", C.c_int32), ("use_graph", C.c_int32),
                ("xcd_aware", C.c_int32), ("reserved", C.c_int32)]


class BatchIO(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("obj_weight", C.c_double),
                ("v", C.c_void_p), ("w", C.c_void_p), ("wx", C.c_void_p),
                ("f", C.c_void_p), ("g", C.c_void_p), ("c", C.c_void_p), ("jac", C.c_void_p),
                ("hess", C.c_void_p), ("jv", C.c_void_p), ("jtw", C.c_void_p), ("hv", C.c_void_p),
                ("lag", C.c_void_p), ("theta_bar", C.c_void_p)]


# exa_eval selection bits, by callback name (lag and adjoint: batched only)
EV = {"obj": 1 << 0, "grad": 1 << 1, "cons": 1 << 2, "jac": 1 << 3, "hess": 1 << 4,
      "jprod": 1 << 5, "jtprod": 1 << 6, "hprod": 1 << 7}
EV_BATCH = dict(EV, lag=1 << 8, adjoint=1 << 9)
UNITS = {"per_callback": 0, "jac_hess": 1, "one_pass": 2, "separate": 3}
UNSTAGED = 0x20     # OR'ed into units: each lane's own output stores


class EvalArgs(C.Structure):
    _fields_ = [("mask", C.c_uint32), ("reserved", C.c_uint32),
                ("x", C.c_void_p), ("y", C.c_void_p), ("obj_weight", C.c_double),
                ("v", C.c_void_p), ("w", C.c_void_p),
                ("f", C.c_void_p), ("g", C.c_void_p), ("c", C.c_void_p), ("jac", C.c_void_p),
                ("hess", C.c_void_p), ("jv", C.c_void_p), ("jtw", C.c_void_p), ("hv", C.c_void_p)]


CALLBACKS = ["obj", "grad", "cons", "jac", "hess", "jprod", "jtprod", "hprod", "adjoint", "jac_hess"]


class ExaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[exa status {code}] {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2608_16265_amd.build_lib`")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    sig = {
        "exa_last_error": (C.c_char_p, []),
        "exa_version": (C.c_char_p, []),
        "exa_create": (C.c_int32, [C.POINTER(PatternDesc), C.c_int32, C.c_int64, P_f64, P_f64,
                                   C.c_int64, P_f64, C.POINTER(Options), C.POINTER(vp)]),
        "exa_destroy": (C.c_int32, [vp]),
        "exa_dims": (C.c_int32, [vp, P_i64, P_i64, P_i64, P_i64]),
        "exa_bounds": (C.c_int32, [vp, P_f64, P_f64, P_f64, P_f64]),
        "exa_set_theta": (C.c_int32, [vp, vp, vp]),
        "exa_jac_structure": (C.c_int32, [vp, P_i32, P_i32]),
        "exa_hess_structure": (C.c_int32, [vp, P_i32, P_i32]),
        "exa_obj": (C.c_int32, [vp, vp, vp, vp]),
        "exa_obj_host": (C.c_int32, [vp, vp, P_f64, vp]),
        "exa_grad": (C.c_int32, [vp, vp, vp, vp]),
        "exa_cons": (C.c_int32, [vp, vp, vp, vp]),
        "exa_jac_coord": (C.c_int32, [vp, vp, vp, vp]),
        "exa_hess_coord": (C.c_int32, [vp, vp, vp, C.c_double, vp, vp]),
        "exa_jprod": (C.c_int32, [vp, vp, vp, vp, vp]),
        "exa_jac_hess_coord": (C.c_int32, [vp, vp, vp, C.c_double, vp, vp, vp]),
        "exa_jtprod": (C.c_int32, [vp, vp, vp, vp, vp]),
        "exa_hprod": (C.c_int32, [vp, vp, vp, C.c_double, vp, vp, vp]),
        "exa_hprod_noalloc": (C.c_int32, [vp, vp, vp, C.c_double, vp, vp, vp]),
        "exa_lag_grad": (C.c_int32, [vp, vp, vp, C.c_double, vp, vp]),
        "exa_csc_dims": (C.c_int32, [vp, C.c_int32, vp]),
        "exa_csc_structure": (C.c_int32, [vp, C.c_int32, vp, vp]),
        "exa_csc_values": (C.c_int32, [vp, C.c_int32, vp, vp, vp]),
        "exa_adjoint_theta": (C.c_int32, [vp, vp, vp, C.c_double, vp, vp, vp]),
        "exa_eval": (C.c_int32, [vp, C.POINTER(EvalArgs), vp]),
        "exa_eval_schedule": (C.c_int32, [vp, C.c_uint32, P_i64]),
        "exa_eval_set_schedule": (C.c_int32, [vp, C.c_uint32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
        "exa_eval_bytes": (C.c_int32, [vp, C.c_uint32, P_i64]),
        "exa_device_copy": (C.c_int32, [vp, vp, C.c_int64, vp]),
        "exa_eval_timing": (C.c_int32, [vp, C.c_int32]),
        "exa_eval_timing_read": (C.c_int32, [vp, P_f64]),
        "exa_counters": (C.c_int32, [vp, P_i64]),
        "exa_device_bytes": (C.c_int32, [vp, P_i64]),
        "exa_build_info": (C.c_int32, [vp, P_f64]),
        "exa_generated_source": (C.c_int32, [vp, C.c_char_p, C.c_int64, P_i64]),
        "exa_compile_check": (C.c_int32, [vp]),
        "exa_pattern_info": (C.c_int32, [vp, C.c_int32, P_i64]),
        "exa_kernel_bytes": (C.c_int32, [vp, C.c_int32, P_i64, P_i64]),
        "exa_schedule": (C.c_int32, [vp, C.c_int32, P_i64]),
        "exa_batch_create": (C.c_int32, [C.POINTER(vp), C.c_int32, C.POINTER(BatchOptions),
                                         C.POINTER(vp)]),
        "exa_batch_destroy": (C.c_int32, [vp]),
        "exa_batch_offsets": (C.c_int32, [vp, P_i64]),
        "exa_batch_set_theta": (C.c_int32, [vp, vp, vp]),
        "exa_batch_eval": (C.c_int32, [vp, C.c_uint32, C.POINTER(BatchIO), vp]),
        "exa_batch_schedule": (C.c_int32, [vp, C.c_uint32, P_i64]),
        "exa_batch_set_schedule": (C.c_int32, [vp, C.c_uint32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
        "exa_batch_bytes": (C.c_int32, [vp, C.c_uint32, P_i64]),
        "exa_batch_timing": (C.c_int32, [vp, C.c_int32]),
        "exa_batch_timing_read": (C.c_int32, [vp, P_f64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def check(status: int):
    if status != EXA_OK:
        raise ExaError(status, LIB.exa_last_error().decode())


def exported_symbols():
    """Names of the C ABI entry points this binding declares."""
    return ["exa_last_error", "exa_version", "exa_create", "exa_destroy", "exa_dims", "exa_bounds",
            "exa_set_theta", "exa_jac_structure", "exa_hess_structure", "exa_obj", "exa_obj_host", "exa_grad",
            "exa_cons", "exa_jac_coord", "exa_hess_coord", "exa_jac_hess_coord", "exa_jprod", "exa_jtprod", "exa_hprod",
            "exa_hprod_noalloc",
            "exa_lag_grad", "exa_csc_dims", "exa_csc_structure", "exa_csc_values",
            "exa_adjoint_theta", "exa_eval", "exa_eval_schedule", "exa_eval_set_schedule", "exa_eval_bytes", "exa_eval_timing", "exa_device_copy",
            "exa_eval_timing_read", "exa_counters", "exa_device_bytes", "exa_build_info",
            "exa_generated_source", "exa_compile_check",
            "exa_pattern_info", "exa_kernel_bytes", "exa_schedule", "exa_batch_create", "exa_batch_destroy",
            "exa_batch_offsets", "exa_batch_set_theta", "exa_batch_eval", "exa_batch_schedule",
            "exa_batch_set_schedule", "exa_batch_bytes", "exa_batch_timing", "exa_batch_timing_read"]
