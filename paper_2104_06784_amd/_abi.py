"""ctypes binding of ``libm2p.so`` (include/m2p.h): argument marshalling only.

Every step of the path runs in the HIP library; if the library is missing the
import of :func:`lib` raises.  No CPU fallback exists.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# M2P_LIBRARY overrides the library path (for example a build with other
# compile-time tile options); the default is the library built in-tree.
LIB_PATH = os.environ.get("M2P_LIBRARY") or os.path.join(HERE, "libm2p.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "m2p.h")

M2P_OK = 0
M2P_EINVAL = -1
M2P_ENOMEM = -2
M2P_EHIP = -3
M2P_ENONFINITE = -4
M2P_ENEGDEPTH = -5
M2P_EDTFLOOR = -6
M2P_EMAXSTEPS = -7
M2P_ESTATE = -8
M2P_EIO = -9
M2P_FP64 = 0
M2P_FP32 = 1
M2P_DEPTH_NORMAL = 0
M2P_DEPTH_VERTICAL = 1
M2P_VARIANT_AUTO = 0
M2P_VARIANT_REFERENCE = 1
M2P_VARIANT_TILED = 2
M2P_VARIANT_TILED_GLOBAL = 3


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("dy", C.c_double)]


class Params(C.Structure):
    _fields_ = [("delta_b_deg", C.c_double), ("c_d", C.c_double), ("inv_n_r", C.c_double),
                ("theta_b", C.c_double), ("rho_s", C.c_double), ("rho_f", C.c_double),
                ("delta_int_deg", C.c_double), ("cfl", C.c_double), ("L", C.c_double), ("H", C.c_double),
                ("chi", C.c_double), ("g", C.c_double), ("m_dry", C.c_double), ("a_min", C.c_double),
                ("bc", C.c_int32 * 4), ("flags", C.c_int32), ("v_eps", C.c_double)]


class Inflow(C.Structure):
    _fields_ = [("side", C.c_int32), ("i0", C.c_int32), ("ncells", C.c_int32), ("nt", C.c_int32),
                ("t", C.POINTER(C.c_double)), ("Q", C.POINTER(C.c_double)), ("phi_s", C.POINTER(C.c_double))]


class InflowState(C.Structure):
    _fields_ = [("side", C.c_int32), ("i0", C.c_int32), ("ncells", C.c_int32), ("nt", C.c_int32),
                ("t", C.POINTER(C.c_double)), ("h", C.POINTER(C.c_double)), ("phi_s", C.POINTER(C.c_double)),
                ("v", C.POINTER(C.c_double))]


class Diag(C.Structure):
    _fields_ = [("t", C.c_double), ("dt_last", C.c_double), ("dt_next", C.c_double),
                ("mass_s", C.c_double), ("mass_f", C.c_double), ("in_s", C.c_double), ("in_f", C.c_double),
                ("out_s", C.c_double), ("out_f", C.c_double), ("steps", C.c_int64),
                ("clamp_count", C.c_int64), ("status", C.c_int32), ("pad", C.c_int32)]


class M2PError(RuntimeError):
    def __init__(self, code, func, detail):
        super().__init__(f"{func} failed with {code}: {detail}")
        self.code = code


_lib = None

_dp = C.POINTER(C.c_double)
_P = C.c_void_p
SIGNATURES = {
    "m2p_version": (C.c_char_p, []),
    "m2p_strerror": (C.c_char_p, [C.c_int]),
    "m2p_last_error": (C.c_char_p, []),
    "m2p_device_count": (C.c_int, [C.POINTER(C.c_int)]),
    "m2p_create": (C.c_int, [C.POINTER(_P), C.POINTER(Grid), C.POINTER(Params), C.c_int32, _dp, _dp, _P]),
    "m2p_destroy": (None, [_P]),
    "m2p_buffer_bytes": (C.c_int, [C.POINTER(Grid), C.c_int32, C.POINTER(C.c_size_t)]),
    "m2p_bind_buffers": (C.c_int, [_P, _P, _P, C.c_size_t]),
    "m2p_set_state": (C.c_int, [_P, C.c_int32, _dp, _dp, _dp, _dp, _dp, _dp]),
    "m2p_set_state_raw": (C.c_int, [_P, _dp]),
    "m2p_get_state_raw": (C.c_int, [_P, _dp]),
    "m2p_set_time": (C.c_int, [_P, C.c_double]),
    "m2p_set_inflow": (C.c_int, [_P, C.POINTER(Inflow), C.c_int32]),
    "m2p_set_inflow_states": (C.c_int, [_P, C.POINTER(InflowState), C.c_int32]),
    "m2p_run_outputs": (C.c_int, [_P, _dp, C.c_int64, C.c_int64, _dp, C.POINTER(C.c_int64)]),
    "m2p_set_graph": (C.c_int, [_P, C.c_int32]),
    "m2p_set_variant": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "m2p_autotune": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32), _dp]),
    "m2p_step": (C.c_int, [_P, _dp]),
    "m2p_run": (C.c_int, [_P, C.c_int64]),
    "m2p_run_to": (C.c_int, [_P, C.c_double, C.c_int64, C.POINTER(C.c_int64)]),
    "m2p_get_fields": (C.c_int, [_P, _dp, _dp, _dp, _dp, _dp, _dp]),
    "m2p_get_diag": (C.c_int, [_P, C.POINTER(Diag)]),
    "m2p_synchronize": (C.c_int, [_P]),
    "m2p_state_device_ptr": (C.c_int, [_P, C.POINTER(_P), C.POINTER(C.c_int64)]),
    "m2p_set_profiling": (C.c_int, [_P, C.c_int32]),
    "m2p_kernel_times": (C.c_int, [_P, _dp, C.POINTER(C.c_int64)]),
    "m2p_stage_flops": (C.c_int, [C.c_int32, C.c_int32, _dp]),
    "m2p_esri_read": (C.c_int, [C.c_char_p, C.POINTER(Grid), _dp, _dp, _dp, _dp, C.c_size_t]),
    "m2p_esri_write": (C.c_int, [C.c_char_p, C.POINTER(Grid), C.c_double, C.c_double, C.c_double, _dp]),
    "m2p_set_friction_field": (C.c_int, [_P, _dp]),
    "m2p_set_dt_schedule": (C.c_int, [_P, _dp, C.c_int64]),
    "m2p_loss": (C.c_int, [_P, _dp, _dp]),
    "m2p_loss_noalloc": (C.c_int, [_P, _P, _P]),
    "m2p_stage_jvp": (C.c_int, [_P, C.c_int32, _dp, _dp, _dp, _dp]),
    "m2p_stage_vjp": (C.c_int, [_P, C.c_int32, _dp, _dp, _dp]),
    "m2p_adjoint_run": (C.c_int, [_P, C.c_int64, C.c_int32, _dp, C.c_double, _dp, _dp, _dp]),
    "m2p_batch_create": (C.c_int, [C.POINTER(_P), C.c_int32, C.POINTER(Grid), C.POINTER(Params),
                                   C.POINTER(_dp), C.POINTER(_dp), C.c_int32, _P]),
    "m2p_batch_destroy": (None, [_P]),
    "m2p_batch_set_state": (C.c_int, [_P, C.c_int32, C.c_int32, _dp, _dp, _dp, _dp, _dp, _dp]),
    "m2p_batch_run": (C.c_int, [_P, C.c_int64]),
    "m2p_batch_synchronize": (C.c_int, [_P]),
    "m2p_batch_get_state_raw": (C.c_int, [_P, C.c_int32, _dp]),
    "m2p_batch_get_fields": (C.c_int, [_P, C.c_int32, _dp, _dp, _dp, _dp, _dp, _dp]),
    "m2p_batch_get_diag": (C.c_int, [_P, C.c_int32, C.POINTER(Diag)]),
    "m2p_batch_set_tile": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "m2p_batch_set_graph": (C.c_int, [_P, C.c_int32]),
    "m2p_batch_autotune": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double)]),
    "m2p_batch_info": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
}


def lib():
    """Load ``libm2p.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built: run __graft_entry__.build() "
                               "or python -m paper_2104_06784_amd.build_lib")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code, func="m2p"):
    if code != M2P_OK:
        detail = lib().m2p_last_error().decode()
        raise M2PError(code, func, detail)
    return code


def dptr(a):
    return None if a is None else a.ctypes.data_as(_dp)
