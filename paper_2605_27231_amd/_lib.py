"""ctypes declarations of the C ABI in include/sigw.h.

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation of any step.
"""
from __future__ import annotations

import ctypes as ct
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# SIGW_LIBRARY selects another build of the same library (e.g. the host
# sanitizer build of build.py --sanitize); there is no fallback either way
LIB_PATH = os.environ.get("SIGW_LIBRARY") or os.path.join(PKG, "libsigw.so")

SIGW_OK = 0
SIGW_E_INVALID = -1
SIGW_E_NOMEM = -2
SIGW_E_DEVICE = -3
SIGW_E_UNSUPPORTED = -4
SIGW_E_STATE = -5
SIGW_E_PENDING = -6

SIGW_F32 = 0
SIGW_F64 = 1

MAP_KINDS = {"gauss": 0, "local": 1, "exptail": 2, "nonlocal": 3}

# every entry point the header declares
EXPORTS = (
    "sigw_plan_desc_default", "sigw_plan_footprint", "sigw_plan_create", "sigw_plan_destroy",
    "sigw_kernel_table", "sigw_white_noise", "sigw_generate_field", "sigw_set_zeta",
    "sigw_set_phi_hat", "sigw_get_phi_hat", "sigw_source_convolutions", "sigw_spectrum",
    "sigw_spectrum_batch", "sigw_spectrum_enqueue", "sigw_spectrum_poll", "sigw_synchronize",
    "sigw_set_timing", "sigw_kernel_time", "sigw_last_error", "sigw_status_string",
    "sigw_graph_create", "sigw_graph_launch", "sigw_graph_results", "sigw_graph_destroy",
    "sigw_autotune", "sigw_plan_schedule", "sigw_plan_set_schedule", "sigw_spectrum_jackknife",
    "sigw_spectrum_adaptive", "sigw_plan_set_kernel_table", "sigw_spectrum_noalloc",
    "sigw_kernel_table_w", "sigw_stream_probe", "sigw_shell_modes",
)

SIGW_TUNE_FORCE = 1


class PlanDesc(ct.Structure):
    _fields_ = [
        ("N", ct.c_int32), ("L", ct.c_double), ("prec", ct.c_int32), ("n_slots", ct.c_int32),
        ("n_modes", ct.c_int32), ("n_alpha", ct.c_int32),
        ("u_min", ct.c_double), ("u_max", ct.c_double), ("u_p", ct.c_double),
        ("sigma_p", ct.c_double), ("A_p", ct.c_double), ("alpha_chunk", ct.c_int32),
        ("scratch_terms", ct.c_int32), ("batch", ct.c_int32), ("autotune", ct.c_int32),
    ]


class Lognormal(ct.Structure):
    _fields_ = [("A", ct.c_double), ("sigma", ct.c_double), ("k_star", ct.c_double)]


class NGMap(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("F_NL", ct.c_double), ("G_NL", ct.c_double),
                ("beta", ct.c_double), ("clip", ct.c_double), ("alpha_NL", ct.c_double),
                ("beta_NL", ct.c_double), ("k_NL", ct.c_double)]


class SigwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib() -> ct.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run `python -m paper_2605_27231_amd.build`)")
    L = ct.CDLL(LIB_PATH)
    P = ct.c_void_p
    D = ct.POINTER(ct.c_double)
    I64 = ct.POINTER(ct.c_int64)
    I32 = ct.POINTER(ct.c_int32)
    sig = {
        "sigw_plan_desc_default": [ct.POINTER(PlanDesc), ct.c_int32, ct.c_double, ct.c_int32],
        "sigw_plan_footprint": [ct.POINTER(PlanDesc), ct.POINTER(ct.c_size_t)],
        "sigw_plan_create": [ct.POINTER(PlanDesc), P, ct.POINTER(P)],
        "sigw_plan_destroy": [P],
        "sigw_kernel_table": [ct.POINTER(PlanDesc), ct.c_int32, D, D, D],
        "sigw_kernel_table_w": [ct.POINTER(PlanDesc), ct.c_double, ct.c_int32, D, D, D],
        "sigw_stream_probe": [ct.c_int32, P, ct.c_size_t, ct.c_int32, P, D],
        "sigw_shell_modes": [ct.c_int32, ct.c_double, ct.c_double, ct.c_double, I32, I32, I64],
        "sigw_white_noise": [P, ct.c_uint64, P],
        "sigw_generate_field": [P, ct.c_int32, ct.c_uint64, ct.POINTER(Lognormal), ct.POINTER(NGMap)],
        "sigw_set_zeta": [P, ct.c_int32, P],
        "sigw_set_phi_hat": [P, ct.c_int32, P],
        "sigw_get_phi_hat": [P, ct.c_int32, P],
        "sigw_source_convolutions": [P, ct.c_int32, ct.c_double, P],
        "sigw_spectrum": [P, ct.c_int32, ct.c_int32, D, D, D, D, I64],
        "sigw_spectrum_batch": [P, ct.c_int32, I32, ct.c_int32, D, D, D, D, I64],
        "sigw_spectrum_enqueue": [P, ct.c_int32, ct.c_int32, D, D, D],
        "sigw_spectrum_poll": [P, D, I64],
        "sigw_synchronize": [P],
        "sigw_set_timing": [P, ct.c_int32],
        "sigw_kernel_time": [P, ct.c_char_p, D, I64],
        "sigw_last_error": [P],
        "sigw_status_string": [ct.c_int],
        "sigw_graph_create": [P, ct.c_int32, I32, ct.c_int32, D, D, D, ct.POINTER(P)],
        "sigw_graph_launch": [P],
        "sigw_graph_results": [P, D, I64],
        "sigw_graph_destroy": [P],
        "sigw_autotune": [P, ct.c_int32],
        "sigw_spectrum_jackknife": [P, ct.c_int32, ct.c_int32, D, D, D, ct.c_int32, D, I64, D, D],
        "sigw_spectrum_adaptive": [P, ct.c_int32, ct.c_uint64, ct.POINTER(Lognormal), ct.POINTER(NGMap),
                                   ct.c_int32, D, ct.c_double, D, I64, D],
        "sigw_plan_schedule": [P, I32, I32, ct.c_char_p, ct.c_size_t],
        "sigw_plan_set_schedule": [P, ct.c_int32],
        "sigw_plan_set_kernel_table": [P, ct.c_int32, D, D, D],
        "sigw_spectrum_noalloc": [ct.POINTER(PlanDesc), P, ct.c_int32, D, D, D, D, I64, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ct.c_int
    L.sigw_last_error.restype = ct.c_char_p
    L.sigw_status_string.restype = ct.c_char_p
    _lib = L
    return L


def check(status: int, plan_handle=None, what: str = "") -> None:
    if status == SIGW_OK:
        return
    L = lib()
    text = L.sigw_status_string(status).decode()
    detail = L.sigw_last_error(plan_handle if plan_handle else None).decode()
    if detail:
        text += f": {detail}"
    raise SigwError(status, f"{what}: {text}" if what else text)
