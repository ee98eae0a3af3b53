"""ctypes declarations of the C ABI in include/lbm.h (argument marshalling only).

Loading fails loudly when liblbm_hip.so has not been built: there is no CPU
fallback for any entry point.
"""
from __future__ import annotations

import ctypes
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbm_hip.so")

LBM_OK, LBM_ERR_INVALID, LBM_ERR_OOM, LBM_ERR_DEVICE, LBM_ERR_STATE, LBM_ERR_NONFINITE = range(6)
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
PATTERN = {"ab": 0, "aa": 1}

# Every symbol the header declares, in header order.
EXPORTS = [
    "lbm_options_default", "lbm_create", "lbm_create_ex", "lbm_destroy", "lbm_query_buffer_sizes",
    "lbm_trajectory_bytes", "lbm_set_trajectory_buffer", "lbm_set_adjoint_buffer", "lbm_get_info",
    "lbm_set_stream", "lbm_step_kernel_name", "lbm_set_tau", "lbm_set_wall_velocity", "lbm_set_force_uniform",
    "lbm_set_force_field", "lbm_init_equilibrium", "lbm_step", "lbm_step_macros", "lbm_macros",
    "lbm_get_populations", "lbm_set_populations", "lbm_debug_stream_only",
    "lbm_forward_checkpointed", "lbm_adjoint", "lbm_adjoint_noalloc", "lbm_check_finite", "lbm_step_times", "lbm_sync",
    "lbm_device_bytes", "lbm_status_string", "lbm_last_error", "lbm_copy_f32",
]
# include/lbm_study.h
STUDY_EXPORTS = ["lbm_study_stream", "lbm_study_shift", "lbm_study_planes", "lbm_study_step"]


class LBMError(RuntimeError):
    def __init__(self, status: int, func: str, message: str):
        self.status = status
        super().__init__(f"{func} -> {status_name(status)}: {message}")


class lbm_options(ctypes.Structure):
    _fields_ = [
        ("storage", ctypes.c_int),
        ("pattern", ctypes.c_int),
        ("hip_stream", ctypes.c_void_p),
        ("block_x", ctypes.c_int),
        ("block_y", ctypes.c_int),
        ("timing_capacity", ctypes.c_int),
        ("check_interval", ctypes.c_int),
        ("device", ctypes.c_int),
        ("cells_per_lane", ctypes.c_int),
        ("gather_mode", ctypes.c_int),
        ("groups_per_cu", ctypes.c_int),
        ("population_dev", ctypes.c_void_p * 2),
    ]


class lbm_buffer_sizes(ctypes.Structure):
    _fields_ = [
        ("population_bytes", ctypes.c_size_t),
        ("population_arrays", ctypes.c_int),
        ("adjoint_bytes", ctypes.c_size_t),
        ("state_bytes", ctypes.c_size_t),
    ]


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded library; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"{_LIB_PATH} is missing: build it with `python -m paper_1309_1983_amd.build` "
            "(there is no CPU fallback)")
    L = ctypes.CDLL(_LIB_PATH)
    vp, ip, fp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(ctypes.c_void_p)
    c_int, c_float, c_size = ctypes.c_int, ctypes.c_float, ctypes.c_size_t
    sig = {
        "lbm_options_default": (None, [ctypes.POINTER(lbm_options)]),
        "lbm_create": (c_int, [c_int, c_int, c_int, c_float, vp, pp]),
        "lbm_create_ex": (c_int, [c_int, c_int, c_int, c_float, vp, ctypes.POINTER(lbm_options), pp]),
        "lbm_destroy": (None, [vp]),
        "lbm_query_buffer_sizes": (c_int, [c_int, c_int, c_int, ctypes.POINTER(lbm_options),
                                           ctypes.POINTER(lbm_buffer_sizes)]),
        "lbm_trajectory_bytes": (c_size, [c_int, c_int, c_int, c_int, c_int]),
        "lbm_set_trajectory_buffer": (c_int, [vp, vp, c_size]),
        "lbm_set_adjoint_buffer": (c_int, [vp, vp, c_size]),
        "lbm_get_info": (c_int, [vp, ip, ip, ip, ip, ip]),
        "lbm_set_stream": (c_int, [vp, vp]),
        "lbm_step_kernel_name": (c_int, [vp, ctypes.c_char_p, c_size]),
        "lbm_set_tau": (c_int, [vp, c_float]),
        "lbm_set_wall_velocity": (c_int, [vp, c_float, c_float, c_float]),
        "lbm_set_force_uniform": (c_int, [vp, c_float, c_float, c_float]),
        "lbm_set_force_field": (c_int, [vp, fp]),
        "lbm_init_equilibrium": (c_int, [vp, fp, fp]),
        "lbm_step": (c_int, [vp, c_int]),
        "lbm_step_macros": (c_int, [vp, c_int, fp, fp]),
        "lbm_macros": (c_int, [vp, fp, fp]),
        "lbm_get_populations": (c_int, [vp, fp]),
        "lbm_set_populations": (c_int, [vp, fp]),
        "lbm_debug_stream_only": (c_int, [vp, c_int]),
        "lbm_forward_checkpointed": (c_int, [vp, c_int, c_int]),
        "lbm_adjoint": (c_int, [vp, fp, fp, dp]),
        "lbm_adjoint_noalloc": (c_int, [vp, fp, fp, dp]),
        "lbm_check_finite": (c_int, [vp]),
        "lbm_step_times": (c_int, [vp, ctypes.POINTER(c_float), c_int, ip]),
        "lbm_sync": (c_int, [vp]),
        "lbm_device_bytes": (c_size, [vp]),
        "lbm_status_string": (ctypes.c_char_p, [c_int]),
        "lbm_last_error": (ctypes.c_char_p, []),
        "lbm_copy_f32": (c_int, [fp, fp, c_size, vp]),
        "lbm_study_stream": (c_int, [c_int, fp, fp, fp, c_size, c_int, c_int, c_int, c_int, vp]),
        "lbm_study_shift": (c_int, [fp, fp, c_int, c_int, c_int, vp]),
        "lbm_study_planes": (c_int, [c_int, fp, fp, fp, c_int, c_int, c_int, vp]),
        "lbm_study_step": (c_int, [fp, fp, vp, c_int, c_int, c_int, c_float, c_int, c_int, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def status_name(st: int) -> str:
    return lib().lbm_status_string(int(st)).decode()


def last_error() -> str:
    return lib().lbm_last_error().decode()


def check(st: int, func: str) -> None:
    if st != LBM_OK:
        raise LBMError(st, func, last_error())


def call(name: str, *args) -> None:
    """Call an entry point that returns lbm_status; raise LBMError on failure."""
    check(getattr(lib(), name)(*args), name)
