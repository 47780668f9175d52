"""ctypes declarations of libspleaf's C ABI (include/spleaf.h).

Loading fails loudly when the library has not been built: there is no other
implementation of these calls.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libspleaf.so")

# enum values mirror spleaf.h
OK, ERR_ARG, ERR_FORMAT, ERR_SHAPE, ERR_DTYPE, ERR_UNSUPPORTED, ERR_WORKSPACE, \
    ERR_NOMEM, ERR_HIP, ERR_INVALID = range(10)
F64, F32, BF16 = 0, 1, 2
DENSE, COMPRESSED = 0, 1
I32, I64 = 0, 1
SCHED_DEFAULT, ROW, NNZ, MERGE, SCHED_LEARNED, SCHED_AUTOTUNE = 0, 1, 2, 3, 4, 5
OP_SPMV, OP_SPMM, OP_SPADD3, OP_SDDMM, OP_SPTTV, OP_MTTKRP, OP_INNER = range(7)


class SplSparse(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int32),
        ("vtype", ctypes.c_int32),
        ("dims", ctypes.c_int64 * 3),
        ("level", ctypes.c_int32 * 3),
        ("pos", ctypes.c_void_p * 3),
        ("crd", ctypes.c_void_p * 3),
        ("vals", ctypes.c_void_p),
        ("nnz", ctypes.c_int64),
        ("nfibers", ctypes.c_int64),
        ("pos_type", ctypes.c_int32),
    ]


class SplDense(ctypes.Structure):
    _fields_ = [
        ("data", ctypes.c_void_p),
        ("dtype", ctypes.c_int32),
        ("ndim", ctypes.c_int32),
        ("dims", ctypes.c_int64 * 2),
        ("ld", ctypes.c_int64),
    ]


class SplSchedule(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("lanes_per_row", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("items_per_lane", ctypes.c_int32),
        ("col_tile", ctypes.c_int32),
        ("variant", ctypes.c_int32),
    ]


class SplTinOperand(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char_p),
        ("sparse", ctypes.POINTER(SplSparse)),
        ("dense", ctypes.POINTER(SplDense)),
    ]


_P = ctypes.c_void_p
_SP = ctypes.POINTER(SplSparse)
_DP = ctypes.POINTER(SplDense)
_SCH = ctypes.POINTER(SplSchedule)
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t

# name -> (restype, argtypes); every function in spleaf.h appears here
SIGNATURES = {
    "spl_context_create": (_I32, [ctypes.c_int, ctypes.POINTER(_P)]),
    "spl_context_destroy": (_I32, [_P]),
    "spl_last_error": (ctypes.c_char_p, [_P]),
    "spl_status_string": (ctypes.c_char_p, [_I32]),
    "spl_sync": (_I32, [_P, _P]),
    "spl_op_tin": (ctypes.c_char_p, [_I32]),
    "spl_op_parse": (_I32, [ctypes.c_char_p, ctypes.POINTER(_I32)]),
    "spl_workspace_query": (_I32, [_P, _I32, _SP, _I64, _SCH, ctypes.POINTER(_SZ)]),
    "spl_tile_bounds": (_I32, [_P, _SP, _SCH, _P, _P, _I64, ctypes.POINTER(_I64), _P]),
    "spl_csf_tile_bounds": (_I32, [_P, _SP, _I64, _P, _P, _I64, ctypes.POINTER(_I64), _P]),
    "spl_validate": (_I32, [_P, _SP, _P]),
    "spl_timing_enable": (_I32, [_P, ctypes.c_int]),
    "spl_timing_read": (_I32, [_P, _I32, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_double)]),
    "spl_probe": (_I32, [_P, ctypes.c_int, _P, _I64, _I64, _I64, _P, _I64, _P]),
    "spl_spmv": (_I32, [_P, _SP, _DP, _DP, _SCH, _P, _SZ, _P]),
    "spl_spmv_noalloc": (_I32, [_P, _SP, _DP, _DP, _SCH, _P]),
    "spl_coord_partition": (_I32, [_P, _SP, _I32, _P, _P, _P]),
    "spl_spmv_window": (_I32, [_P, _SP, _P, _P, _DP, _DP, _SCH, _P]),
    "spl_spmm": (_I32, [_P, _SP, _DP, _DP, _SCH, _P, _SZ, _P]),
    "spl_spttv": (_I32, [_P, _SP, _DP, _DP, _SCH, _P, _SZ, _P]),
    "spl_mttkrp": (_I32, [_P, _SP, _DP, _DP, _DP, _SCH, _P, _SZ, _P]),
    "spl_inner": (_I32, [_P, _SP, _SP, _P, _SCH, _P, _SZ, _P]),
    "spl_sddmm": (_I32, [_P, _SP, _DP, _DP, _DP, _SCH, _P, _SZ, _P]),
    "spl_spadd3_symbolic": (_I32, [_P, _SP, _SP, _SP, _P, ctypes.POINTER(_I64), _SCH, _P, _SZ,
                                   _P]),
    "spl_spadd3_numeric": (_I32, [_P, _SP, _SP, _SP, _P, _P, _P, _SCH, _P]),
    "spl_features": (_I32, [_P, _SP, _P, _P, _SZ, _P]),
    "spl_mlp_param_count": (_I64, [ctypes.c_int]),
    "spl_mlp_forward": (_I32, [_P, ctypes.c_int, _P, _P, _P, _I64, _P, _P, _P]),
    "spl_mlp_backward": (_I32, [_P, ctypes.c_int, _P, _I64, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "spl_adam_step": (_I32, [_P, _I64, _P, _P, _P, _P, ctypes.c_float, ctypes.c_float,
                             ctypes.c_float, ctypes.c_float, ctypes.c_int, _P]),
    "spl_autotune": (_I32, [_P, _I32, _SP, _DP, _DP, _SCH, ctypes.c_int, ctypes.c_int, _SCH,
                            _P, _P]),
    "spl_mlp_load": (_I32, [_P, _I32, ctypes.c_int, _SCH, _P, _P]),
    "spl_mlp_save": (_I32, [_P, _I32, ctypes.POINTER(ctypes.c_int), ctypes.c_int, _SCH, _P, _P]),
    "spl_mlp_predict": (_I32, [_P, _I32, _SP, _SCH, _P]),
    "spl_mlp_train_step": (_I32, [_P, _I32, _P, _P, _I64, ctypes.c_float, _P, _P]),
    "spl_transpose_workspace_query": (_I32, [_P, _SP, ctypes.POINTER(_SZ)]),
    "spl_transpose": (_I32, [_P, _SP, _P, _P, _P, _P, _SZ, _P]),
    "spl_tin_workspace_query": (_I32, [_P, ctypes.c_char_p, ctypes.c_int,
                                       ctypes.POINTER(SplTinOperand),
                                       ctypes.POINTER(SplTinOperand), ctypes.POINTER(_SZ)]),
    "spl_tin_symbolic": (_I32, [_P, ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(SplTinOperand),
                                ctypes.POINTER(SplTinOperand), _P, ctypes.POINTER(_I64), _P, _SZ,
                                _P]),
    "spl_tin_eval": (_I32, [_P, ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(SplTinOperand),
                            ctypes.POINTER(SplTinOperand), _P, _SZ, _P]),
    "spl_tin_source": (_I32, [_P, ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(SplTinOperand),
                              ctypes.POINTER(SplTinOperand), ctypes.c_char_p, _SZ,
                              ctypes.POINTER(_SZ)]),
}

_lib = None


class SpleafError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{status_name(status)}: {detail}")


def load() -> ctypes.CDLL:
    """Load libspleaf.so (built by ``python -m paper_2207_13901_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2207_13901_amd.build` (hipcc, gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_name(st: int) -> str:
    return load().spl_status_string(st).decode()
