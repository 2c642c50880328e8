"""ctypes declarations for libfit.so (argument marshalling only).

The library is built in-tree (``python -m paper_1705_08019_amd.build``) and
loaded from this package directory.  There is no fallback: if the library is
missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfit.so")

FIT_OK = 0
FIT_F32, FIT_F64 = 0, 1
FIT_ALLOW_UNSTABLE = 1
FIT_TRACE_COLS = 10
STATUS = {0: "FIT_OK", -1: "FIT_E_INVALID", -2: "FIT_E_OOM", -3: "FIT_E_HIP",
          -4: "FIT_E_UNSTABLE", -5: "FIT_E_DIVERGED", -6: "FIT_E_STATE"}


class FitError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("eps0", C.c_double), ("mu0", C.c_double),
                ("dtype", C.c_int32), ("flags", C.c_uint32)]


_vp, _i, _i64, _d = C.c_void_p, C.c_int, C.c_int64, C.c_double
_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)

# name -> argtypes (all return int status unless listed in _CHAR)
SIGNATURES = {
    "fit_grid_create": [C.POINTER(GridDesc), _vp, C.POINTER(_vp)],
    "fit_grid_destroy": [_vp],
    "fit_set_materials": [_vp, _dp, _dp, _dp],
    "fit_set_spacing": [_vp, _dp, _dp, _dp],
    "fit_set_source": [_vp, _i, _i, _i, _i, _d, _d],
    "fit_cfl_dt": [_vp, _dp],
    "fit_step_dt": [_vp, _d, _dp],
    "fit_bind_fields": [_vp, _vp, _vp, _vp, _vp],
    "fit_bind_materials": [_vp, _vp, _vp, _vp],
    "fit_get_state": [_vp, C.POINTER(_vp), C.POINTER(_vp)],
    "fit_adjoint_bind": [_vp, _vp, _vp, _vp, _vp, _vp],
    "fit_set_fields": [_vp, _vp, _vp, _i64, _i],
    "fit_get_fields": [_vp, _vp, _vp, _i],
    "fit_get_step": [_vp, _i64p],
    "fit_apply_curl": [_vp, _i, _vp, _vp],
    "fit_step": [_vp, _i64, _d],
    "fit_energy": [_vp, _dp],
    "fit_energy_noalloc": [_vp, _vp],
    "fit_trace_config": [_vp, _i64, _i64],
    "fit_trace_read": [_vp, _dp, _i64, _i64p, _i64p],
    "fit_set_probe": [_vp, _i32p, _i32p],
    "fit_probe_value": [_vp, _dp],
    "fit_probe_reset": [_vp],
    "fit_stream_probe": [_i, _vp, _vp, _i64, _i, _vp],
    "fit_profile_begin": [_vp, _i64],
    "fit_profile_end": [_vp, _dp, _i64p],
    "fit_smvp_count": [_vp, _i64p],
    "fit_set_tuning": [_vp, _i, _i, _i, _i],
    "fit_set_pair_tuning": [_vp, C.c_int, C.c_int, C.c_int, C.c_int],
    "fit_get_pair_tuning": [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "fit_get_tuning": [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                       C.POINTER(C.c_int)],
    "fit_gram": [_vp, _vp, _i64, _i, _i, _dp],
    "fit_expm_params": [_d, _d, _d, C.POINTER(C.c_int), _i64p],
    "fit_expm_tolerance": [_d, _d, _d, C.POINTER(C.c_double)],
    "fit_leja_params": [_d, _d, _d, C.POINTER(C.c_int), _i64p],
    "fit_leja_coefficients": [C.c_int, _d, _dp, _dp, _dp, _dp],
    "fit_op_apply": [_vp, _d, _vp, _vp, _vp, _vp],
    "fit_op_norm": [_vp, _i, C.c_uint64, _dp],
    "fit_expm": [_vp, _d, _d, _d, _vp, _vp, _vp, _vp, C.POINTER(C.c_int), _i64p],
    "fit_expm_leja": [_vp, _d, _d, _d, _vp, _vp, _vp, _vp, C.POINTER(C.c_int), _i64p],
    "fit_shift_h": [_vp, _d, _vp, _vp, _vp],
    "fit_axpy": [_vp, _d, _vp, _vp, _vp, _vp],
    "fit_batch_create": [C.POINTER(_vp), _i, _vp, C.POINTER(_vp)],
    "fit_batch_destroy": [_vp],
    "fit_batch_set_tuning": [_vp, _i, _i, _i, _i],
    "fit_batch_set_pair": [_vp, _i, _i],
    "fit_batch_set_persistent": [_vp, _i],
    "fit_batch_get_persistent": [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                 C.POINTER(C.c_int)],
    "fit_batch_get_pair": [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "fit_batch_get_pair_tile": [_vp, _i, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "fit_batch_get_tuning": [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                             C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "fit_batch_autotune": [_vp, _dp, _i, C.POINTER(C.c_int), C.POINTER(C.c_int),
                           C.POINTER(C.c_int), C.POINTER(C.c_float)],
    "fit_batch_step": [_vp, _i64, _dp, _i],
    "fit_step_record": [_vp, _i64, _d, _vp, _vp],
    "fit_adjoint_set_tuning": [_vp, _i, _i, _i],
    "fit_adjoint_get_tuning": [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "fit_adjoint_begin": [_vp, _i64, _d],
    "fit_adjoint_step": [_vp, _i64, _vp, _vp, _vp],
    "fit_adjoint_segment": [_vp, _i64, _i64, _vp, _vp],
    "fit_adjoint_grad": [_vp, _vp, _vp, _i],
    "fit_autotune": [_vp, _d, _i, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                     C.POINTER(C.c_int), C.POINTER(C.c_float)],
}
PROF_KINDS = ("epass", "hpass", "reduce", "step", "adjoint", "other", "pair", "pair_energy")
_CHAR = {"fit_version": [], "fit_last_error": []}

_lib = None


def lib():
    """Load libfit.so once; raise if it is missing (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1705_08019_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        for name, args in _CHAR.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_char_p
        _lib = L
    return _lib


def check(rc: int):
    if rc != FIT_OK:
        raise FitError(rc, lib().fit_last_error().decode())
    return rc


def call(name: str, *args):
    return check(getattr(lib(), name)(*args))


def dptr(arr):
    """Pointer to a contiguous float64 numpy array (or None)."""
    if arr is None:
        return None
    return arr.ctypes.data_as(_dp)
