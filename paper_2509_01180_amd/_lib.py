"""ctypes loader of libbh.so (the C ABI declared in include/bh.h).

The shared library is built in-tree by ``paper_2509_01180_amd.build``.  There
is no fallback: if the library is missing or fails to load, every call
raises.
"""

from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# BH_LIBRARY selects another build of the same library (e.g. a tuning variant).
LIB_PATH = os.environ.get("BH_LIBRARY") or os.path.join(_PKG, "libbh.so")

BH_OK, BH_EINVAL, BH_ENOMEM, BH_EDEVICE, BH_EUNSUPPORTED = 0, -1, -2, -3, -4
BH_EXPAND_FP32, BH_EXPAND_BF16, BH_EXPAND_BF16X3 = 0, 1, 2
BH_EXPAND_BATCH_INVARIANT = 16
BH_TUNE_MARCH, BH_TUNE_EXPAND, BH_TUNE_EXPAND_BF16 = 1, 2, 4
BH_CALIB_COPY_VECTOR, BH_CALIB_READ_SCALAR = 0, 1
BH_CALIB_READ_GROUPS = 2048
BH_MAX_L = 64
BH_MAX_N = 256


class BhError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


class AlignOpts(ctypes.Structure):
    _fields_ = [
        ("bands", ctypes.POINTER(ctypes.c_int32)),
        ("n_bands", ctypes.c_int32),
        ("steps_per_band", ctypes.c_int32),
        ("n_restarts", ctypes.c_int32),
        ("step_init", ctypes.c_double),
        ("step_grow", ctypes.c_double),
        ("step_shrink", ctypes.c_double),
        ("batch_invariant", ctypes.c_int32),
        ("newton_bands", ctypes.c_int32),
        ("newton_steps", ctypes.c_int32),
        ("n_keep", ctypes.c_int32),
        ("keep_min_sep", ctypes.c_double),
    ]


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_pI32 = ctypes.POINTER(ctypes.c_int32)
_pF64 = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes)
SIGNATURES = {
    "bh_last_error": (ctypes.c_char_p, []),
    "bh_index_size": (_I64, [_I]),
    "bh_index_table": (_I, [_I, _pI32, _pI32, _pI32, _pF64]),
    "bh_radial_count": (_I, [_I]),
    "bh_radial_table": (_I, [_I, _pI32, _pI32, _pF64, _pF64]),
    "bh_ball_voxels": (_I64, [_I]),
    "bh_plan_create": (_I, [_I, _I, _I, ctypes.POINTER(_P)]),
    "bh_plan_destroy": (None, [_P]),
    "bh_plan_num_coeffs": (_I64, [_P, _I]),
    "bh_plan_check": (_I, [_P, _P]),
    "bh_expand": (_I, [_P, _P, _I64, _P, _P]),
    "bh_expand_ex": (_I, [_P, _P, _I64, _I, _P, _P, _P]),
    "bh_expand_noalloc": (_I, [_P, _P, _I64, _P, _P]),
    "bh_expand_noalloc_batch": (_I64, [_P]),
    "bh_cross_power": (_I, [_P, _P, _P, _I64, _I, _P, _P]),
    "bh_correlate": (_I, [_P, _P, _P, _I64, _I, _P, _I, _P, _P, _P]),
    "bh_align": (_I, [_P, _P, _P, _I64, ctypes.POINTER(AlignOpts), _P, _P, _P, _P, _P, _P]),
    "bh_correlate_hess": (_I, [_P, _P, _P, _I64, _I, _P, _I, _P, _P, _P, _P]),
    "bh_degree_energy": (_I, [_P, _P, _P, _I64, _I, _P, _P]),
    "bh_select_bands": (_I, [_P, _P, _P, _I, _P, _I64, _I, _pF64, _I, _P, _P, _P, _P]),
    "bh_prune_candidates": (_I, [_P, _P, _P, _I64, _I, _I, ctypes.c_double, _P, _P, _P]),
    "bh_align_shifts": (_I, [_P, _P, _I64, _P, _I, _P, ctypes.POINTER(AlignOpts), _P, _P, _P, _P, _P]),
    "bh_expand_into": (_I, [_P, _P, _I64, _I, _P, _I64, _P, _P]),
    "bh_expand_rows": (_I, [_P, _P, _I64, _P, _I64, _I, _P, _I64, _P, _P]),
    "bh_profile_busy": (_I, [_P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double)]),
    "bh_plan_set_march_streams": (_I, [_P, _I]),
    "bh_align_uneven": (_I, [_P, _P, _I64, _P, _P, _I64, _I, _P, _I64, ctypes.POINTER(AlignOpts),
                             _P, _P, _P, _P, _P, _P]),
    "bh_align_t": (_I, [_P, _P, _P, _I, _P, _I64, ctypes.POINTER(AlignOpts), _P, _P, _P, _P, _P, _P]),
    "bh_plan_autotune": (_I, [_P, _I64, _I, _P, _I, _I, _P]),
    "bh_plan_tuning": (_I, [_P, _I, _I64, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I),
                            ctypes.POINTER(_I)]),
    "bh_plan_set_tuning": (_I, [_P, _I, _I, _I]),
    "bh_calib_copy": (_I, [_P, _P, _I64, _I, _P]),
    "bh_profile_enable": (_I, [_P, _I]),
    "bh_profile_read": (_I, [_P, ctypes.c_char_p, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(_I64)]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2509_01180_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code: int, where: str) -> int:
    if code < 0:
        msg = lib().bh_last_error().decode(errors="replace")
        raise BhError(int(code), where, msg)
    return code
