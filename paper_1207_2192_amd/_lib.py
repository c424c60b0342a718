"""ctypes declarations of the C ABI in include/llgdisk.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libllgdisk.so")

c_int, c_ll, c_ull, c_uint = ctypes.c_int, ctypes.c_longlong, ctypes.c_ulonglong, ctypes.c_uint
c_double, c_vp = ctypes.c_double, ctypes.c_void_p
P_double = ctypes.POINTER(ctypes.c_double)
P_int = ctypes.POINTER(ctypes.c_int)


class LLGParamsC(ctypes.Structure):
    _fields_ = [("alpha", c_double), ("c", c_double), ("hext", c_double * 3), ("temp", c_double),
                ("dtau", c_double), ("renorm", c_int), ("fd_factor", c_int),
                ("hac", c_double * 3), ("freq", c_double), ("phase", c_double),
                ("hpulse", c_double * 3), ("tpulse", c_double), ("wpulse", c_double), ("tau0", c_double)]


# name -> (restype, argtypes)
STEP_COUNTER = 2**64 - 1      # LLG_STEP_COUNTER

SIGNATURES = {
    "llg_params_from_si": (c_int, [c_double, c_double, c_double, c_double, c_double, c_double, c_double,
                                   c_double, ctypes.POINTER(LLGParamsC), P_double]),
    "llg_build_kernels": (c_int, [c_double, c_double, c_double, c_int, ctypes.POINTER(c_vp)]),
    "llg_batch_create": (c_int, [c_int, P_double, P_double, c_double, P_int, ctypes.POINTER(c_vp)]),
    "llg_disk_count": (c_int, [c_vp]),
    "llg_disk_info": (c_int, [c_vp, c_int, P_int, P_int, P_int]),
    "llg_disk_offset": (c_ll, [c_vp, c_int]),
    "llg_state_size": (c_ll, [c_vp]),
    "llg_disk_workgroups": (c_int, [c_vp, c_int]),
    "llg_tune": (c_int, [c_vp, c_int, c_int, P_int]),
    "llg_autotune": (c_int, [c_vp, c_vp, ctypes.POINTER(LLGParamsC), c_int, c_ll, c_vp, P_double]),
    "llg_launch_shape": (c_int, [c_vp, P_int, P_int, P_int, P_int]),
    "llg_set_on_chip": (c_int, [c_vp, c_int]),
    "llg_get_on_chip": (c_int, [c_vp]),
    "llg_debug_spin_limit": (c_int, [c_vp, ctypes.c_uint]),
    "llg_timing": (c_int, [c_vp, c_int]),
    "llg_last_launch_ms": (c_int, [c_vp, c_int, ctypes.POINTER(ctypes.c_float)]),
    "llg_demag_field": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "llg_rhs": (c_int, [c_vp, c_vp, c_vp, ctypes.POINTER(LLGParamsC), c_vp]),
    "llg_rk4_step": (c_int, [c_vp, c_vp, c_ll, ctypes.POINTER(LLGParamsC), c_vp]),
    "llg_heun_step": (c_int, [c_vp, c_vp, c_ll, c_ull, c_ull, c_uint, ctypes.POINTER(LLGParamsC), c_vp]),
    "llg_rk4_series": (c_int, [c_vp, c_vp, c_ll, ctypes.POINTER(LLGParamsC), c_ll, c_vp, c_vp]),
    "llg_heun_series": (c_int, [c_vp, c_vp, c_ll, c_ull, c_ull, c_uint, ctypes.POINTER(LLGParamsC), c_ll, c_vp,
                                c_vp]),
    "llg_power_spectrum": (c_int, [c_vp, c_int, c_ll, c_ll, c_ll, c_int, c_int, c_vp, c_vp, c_vp]),
    "llg_step_counter_set": (c_int, [c_vp, c_ull, c_vp]),
    "llg_step_counter_get": (c_int, [c_vp, ctypes.POINTER(c_ull), c_vp]),
    "llg_graph_create": (c_int, [c_vp, c_int, c_vp, c_ll, ctypes.POINTER(LLGParamsC), c_ull, c_uint,
                                 ctypes.POINTER(c_vp)]),
    "llg_graph_launch": (c_int, [c_vp, c_vp]),
    "llg_graph_destroy": (None, [c_vp]),
    "llg_relax": (c_int, [c_vp, c_vp, P_double, c_double, c_double, c_double, c_ll, ctypes.POINTER(LLGParamsC), c_vp,
                          c_vp]),
    "llg_rk4_record": (c_int, [c_vp, c_vp, c_ll, ctypes.POINTER(LLGParamsC), c_vp, c_vp]),
    "llg_rk4_vjp": (c_int, [c_vp, c_vp, c_ll, c_vp, c_vp, ctypes.POINTER(LLGParamsC), c_vp]),
    "llg_heun_record": (c_int, [c_vp, c_vp, c_ll, c_ull, c_ull, c_uint, ctypes.POINTER(LLGParamsC), c_vp, c_vp]),
    "llg_heun_vjp": (c_int, [c_vp, c_vp, c_ll, c_ull, c_ull, c_uint, c_vp, c_vp, ctypes.POINTER(LLGParamsC), c_vp]),
    "llg_core_position_vjp": (c_int, [c_vp, c_vp, c_double, c_vp, c_vp, c_vp, c_vp]),
    "llg_noise": (c_int, [c_vp, c_ull, c_ull, c_uint, c_vp, c_vp]),
    "llg_energy": (c_int, [c_vp, c_vp, ctypes.POINTER(LLGParamsC), c_vp, c_vp]),
    "llg_vortex_core_position": (c_int, [c_vp, c_vp, c_double, P_double, c_vp, c_vp]),
    "llg_mean_m": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "llg_noalloc_bytes": (c_ll, [c_vp]),
    "llg_rk4_step_noalloc": (c_int, [c_vp, c_vp, c_ll, ctypes.POINTER(LLGParamsC), c_vp]),
    "llg_check": (c_int, [c_vp, c_vp]),
    "llg_destroy": (None, [c_vp]),
    "llg_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libllgdisk.so from the package directory; fail loudly when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"lib_llgdisk is not built ({LIB_PATH} missing); "
                           "build it with `python -m paper_1207_2192_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class LLGError(RuntimeError):
    pass


def check(rc: int, what: str):
    if rc != 0:
        msg = load().llg_last_error()
        raise LLGError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")
