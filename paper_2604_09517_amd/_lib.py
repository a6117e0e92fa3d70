"""ctypes binding of libmxlu.so (argument marshalling only).

The library is built in-tree by `python -m paper_2604_09517_amd.build`.  There
is no fallback: when the library is missing every call raises.
"""

from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmxlu.so")

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_int = ctypes.c_int
_vp = ctypes.c_void_p
_dbl = ctypes.c_double
_u64 = ctypes.c_uint64
_sz = ctypes.c_size_t


class MxpOpts(ctypes.Structure):
    _fields_ = [
        ("prec", _i32), ("pivot", _i32), ("nb", _i64), ("refine", _i32),
        ("restart", _i32), ("max_outer", _i32), ("max_inner_total", _i32),
        ("inner_tol", _dbl), ("resid_threshold", _dbl), ("scale_tile", _i32),
        ("reuse_factors", _i32), ("trans", _i32), ("x_init", _i32),
        ("factor_steps", _i32),
    ]


class MxpReport(ctypes.Structure):
    _fields_ = [
        ("converged", _i32), ("outer_iters", _i32), ("inner_iters", _i32),
        ("info", _i32), ("scaled_residual", _dbl), ("t_convert_ms", _dbl),
        ("t_factor_ms", _dbl), ("t_refine_ms", _dbl),
    ]


# name -> (restype, argtypes); exactly the functions declared in include/mxlu.h
SIGNATURES = {
    "lu_factor": (_int, [_i64, _i64, _vp, _i64, _vp, _vp]),
    "mxlu_set_lookahead": (_int, [_int]),
    "mxlu_release": (_int, []),
    "mxlu_debug_expire_waits": (_int, [_int]),
    "mxlu_debug_poison_scratch": (_int, [_int]),
    "mxlu_panel_factor_f64": (_int, [_i64, _i64, _vp, _i64, _vp, _vp]),
    "mxlu_plan_panel_cus": (_int, [_int]),
    "mxlu_plan_panel_leaf": (_int, [_i64, _int, _int, _int, _int, _i64, _int,
                                    ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "mxlu_plan_lookahead": (_int, [_i64, _i64, _int, _int, _int, _i64]),
    "lu_solve": (_int, [_i64, _i64, _vp, _i64, _vp, _vp, _i64, _int, _vp]),
    "lu_solve_noalloc": (_int, [_i64, _i64, _vp, _i64, _vp, _vp, _i64, _int, _vp]),
    "mxlu_schur_update_f64": (_int, [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp]),
    "mxlu_outer_update_f64": (_int, [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _int,
                                     _vp]),
    "mxp_default_opts": (None, [ctypes.POINTER(MxpOpts)]),
    "mxp_workspace_bytes": (_sz, [_i64, _i64, ctypes.POINTER(MxpOpts)]),
    "mxp_factor_ld": (_i64, [_i64]),
    "mxp_convert": (_int, [_i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp]),
    "mxp_solve": (_int, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp,
                         ctypes.POINTER(MxpOpts), ctypes.POINTER(MxpReport), _vp]),
    "mxp_solve_seeded": (_int, [_i64, _u64, _u64, _int, _i64, _vp, _i64, _vp, _i64, _vp, _sz,
                                _vp, ctypes.POINTER(MxpOpts), ctypes.POINTER(MxpReport), _vp]),
    "mxlu_fill_uniform": (_int, [_i64, _i64, _vp, _i64, _u64, _u64, _vp]),
    "mxlu_make_diag_dominant": (_int, [_i64, _vp, _i64, _vp]),
    "mxlu_scaled_residual": (_int, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _int,
                                    ctypes.POINTER(_dbl), _vp]),
    "mxlu_profile_enable": (_int, [_int]),
    "mxlu_profile_reset": (_int, []),
    "mxlu_profile_read": (_int, [ctypes.POINTER(_dbl), ctypes.POINTER(_dbl),
                                 ctypes.POINTER(_i64), _int]),
    "mxlu_profile_intervals": (_i64, [_int, ctypes.POINTER(_i64), ctypes.POINTER(_dbl),
                                      ctypes.POINTER(_dbl), _i64]),
    "mxlu_status_string": (ctypes.c_char_p, [_int]),
    "mxlu_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libmxlu.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2604_09517_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class MxluError(RuntimeError):
    def __init__(self, where, code):
        L = lib()
        msg = L.mxlu_status_string(code).decode()
        detail = L.mxlu_last_error().decode()
        super().__init__(f"{where}: {msg} ({code})" + (f": {detail}" if detail else ""))
        self.code = code


def check(where, rc, positive_ok=False):
    if rc == 0 or (positive_ok and rc > 0):
        return rc
    if -1000 < rc < 0:
        raise ValueError(f"{where}: argument {-rc} is invalid")
    raise MxluError(where, rc)
