"""ctypes binding of ``libixpart.so`` (the C ABI declared in include/ixpart.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Loading fails loudly when the library has not been
built -- there is no fallback.
"""
import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library shares with torch)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("IXP_LIB", os.path.join(_HERE, "libixpart.so"))

IXP_OK, IXP_EINVAL, IXP_ENOMEM, IXP_EHIP, IXP_EUNSUPPORTED, IXP_EWORKSPACE, IXP_EDEVICE = \
    0, -1, -2, -3, -4, -5, -6
IXP_ETOOLARGE = -7
NOALLOC_SCRATCH_BYTES = 4325376
NOALLOC_MAX_N = 2180907008
I32, I64, F32, U8 = 0, 1, 2, 3
PRED_MOD_EQ, PRED_LT, PRED_FLAGS, PRED_LT_ROW, PRED_MOD_ROW = 0, 1, 2, 3, 4
MODE_PARTITION, MODE_FILTER = 0, 1
RANGE, MONO, INJ, BIJ, FILTPART = 1, 2, 4, 8, 16
CLASS_MOD, CLASS_THRESH, CLASS_BYTES = 0, 1, 2
MONO_LE, MONO_LT, MONO_GE, MONO_GT = 0, 1, 2, 3
ROW_SYNC_AUTO, ROW_SYNC_COUNT, ROW_SYNC_NOWAIT, ROW_SYNC_WAIT = 0, 1, 2, 3


class ixp_pred(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("d", ctypes.c_int64), ("r", ctypes.c_int64), ("s", ctypes.c_float),
                ("reserved1", ctypes.c_int32), ("flags", ctypes.c_void_p), ("row_s", ctypes.c_void_p)]


class ixp_classes(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("v", ctypes.c_int32), ("s", ctypes.c_float * 3),
                ("reserved", ctypes.c_int32), ("classes", ctypes.c_void_p)]


class ixp_tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("wgs_per_cu", ctypes.c_int32), ("row_sync", ctypes.c_int32)]


class ixp_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class ixp_verdict(ctypes.Structure):
    _fields_ = [("holds", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("first_violation", ctypes.c_int64), ("aux", ctypes.c_int64)]


class ixp_prop_args(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int64), ("hi", ctypes.c_int64),
                ("img_lo", ctypes.c_int64), ("img_hi", ctypes.c_int64),
                ("mono_op", ctypes.c_int32), ("fp_mode", ctypes.c_int32),
                ("fp_src", ctypes.c_void_p), ("fp_dst", ctypes.c_void_p),
                ("fp_key_t", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("fp_pred", ixp_pred), ("fp_split", ctypes.c_void_p)]


# name -> (restype, argtypes)
_P, _I32, _I64, _U32, _SZ, _F = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_uint32, ctypes.c_size_t, ctypes.c_float)
_PP = ctypes.POINTER(ixp_pred)
_PT = ctypes.POINTER(ixp_tuning)
_PC = ctypes.POINTER(ixp_classes)
_PA = ctypes.POINTER(ixp_prop_args)
SIGNATURES = {
    "ixp_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "ixp_device_cus": (ctypes.c_int, []),
    "ixp_read_error": (ctypes.c_int, [_P, _P]),
    "ixp_partition_workspace": (_SZ, [_I64]),
    "ixp_partition": (ctypes.c_int, [_P, _I32, _I64, _PP, _I32, _P, _P, _I32, _P, _P, _SZ, _P]),
    "ixp_partition_noalloc": (ctypes.c_int, [_P, _I32, _I64, _PP, _I32, _P, _P, _I32, _P, _P]),
    "ixp_partition_v_workspace": (_SZ, [_I64]),
    "ixp_mk_ii_workspace": (_SZ, [_I64, _I64]),
    "ixp_sgm_sum_workspace": (_SZ, [_I64]),
    "ixp_sgm_sum": (ctypes.c_int, [_P, _P, _I64, _P, _P, _SZ, _P]),
    "ixp_mk_ii": (ctypes.c_int, [_P, _I64, _I64, _P, _I32, _P, _SZ, _P]),
    "ixp_mk_sgm_descr": (ctypes.c_int, [_P, _I64, _I64, _P, _P, _P, _SZ, _P]),
    "ixp_partition_v": (ctypes.c_int, [_P, _I32, _I64, _PC, _P, _P, _I32, _P, _P, _SZ, _P]),
    "ixp_segmented_workspace": (_SZ, [_I64, _I64, _PT]),
    "ixp_segmented_partition": (ctypes.c_int, [_P, _I32, _I64, _P, _I64, _PP, _I32, _P, _P,
                                               _I32, _P, _P, _PT, _P, _SZ, _P]),
    "ixp_tune_segmented": (ctypes.c_int, [_P, _I32, _I64, _P, _I64, _PP, _I32, _P, _P, _I32,
                                          _P, _P, _P, _SZ, _I32, _PT,
                                          ctypes.POINTER(ctypes.c_float), _P]),
    "ixp_segmented_graph_create": (ctypes.c_int, [ctypes.POINTER(_P), _P, _I32, _I64, _P, _I64,
                                                  _PP, _I32, _P, _P, _I32, _P, _P, _PT, _P, _SZ]),
    "ixp_graph_launch": (ctypes.c_int, [_P, _P]),
    "ixp_graph_destroy": (ctypes.c_int, [_P]),
    "ixp_scatter_inj": (ctypes.c_int, [_P, _I64, _P, _I32, _P, _I64, _I64, _P]),
    "ixp_gather": (ctypes.c_int, [_P, _P, _I64, _P, _I32, _I64, _I64, _P, _P]),
    "ixp_check_props_workspace": (_SZ, [_I64, _U32, _PA]),
    "ixp_check_props": (ctypes.c_int, [_P, _I32, _I64, _U32, _PA, _P, _P, _SZ, _P]),
    "ixp_hist_min": (ctypes.c_int, [_P, _I64, _I64, _P, _I32, _P, _I64, _P]),
    "ixp_match_min": (ctypes.c_int, [_P, _P, _I64, _P, _I32, _P, _I64, _P]),
    "ixp_scatter_checked_workspace": (_SZ, [_I64]),
    "ixp_scatter_checked": (ctypes.c_int, [_P, _I64, _P, _I32, _P, _I64, _I64, _P, _P, _SZ, _P]),
    "ixp_zero": (ctypes.c_int, [_P, _SZ, _P]),
    "ixp_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "ixp_profile_read": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
}

_lib = None


def lib():
    """The loaded library; raises if it is missing (build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_2506_23058_amd.build or __graft_entry__.build())")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


class IxpError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = lib().ixp_status_str(status).decode()
        super().__init__(f"{what}: {msg} (status {status})")
        self.status = status


def check(status: int, what: str):
    if status != IXP_OK:
        if status == IXP_EINVAL:
            raise ValueError(IxpError(status, what))
        raise IxpError(status, what)
