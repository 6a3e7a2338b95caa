"""ctypes declarations of the C ABI in include/blk.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libblk.so")

BLK_MAX_P = 32
BLK_OP_CSR, BLK_OP_DENSE = 0, 1
BLK_FP64, BLK_MIXED = 0, 1
BLK_CONVERGED = BLK_OK = 0
BLK_MAXIT, BLK_BREAKDOWN = 1, 2
BLK_EINVAL, BLK_ENOMEM, BLK_EHIP = -1, -2, -3

STATUS_NAMES = {
    0: "converged",
    1: "maxit",
    2: "breakdown",
    -1: "einval",
    -2: "enomem",
    -3: "ehip",
}


BLK_STRUCT_UNKNOWN, BLK_STRUCT_GENERAL, BLK_STRUCT_GRID = 0, 1, 2


class BlkOp(C.Structure):
    _fields_ = [
        ("kind", C.c_int32),
        ("structure", C.c_int32),
        ("n", C.c_int64),
        ("nnz", C.c_int64),
        ("rowptr", C.c_void_p),
        ("colind", C.c_void_p),
        ("val", C.c_void_p),
        ("dense", C.c_void_p),
        ("ld", C.c_int64),
        ("grid", C.c_int64 * 3),
    ]


class BlkOpts(C.Structure):
    _fields_ = [
        ("rq", C.c_int32),
        ("precision", C.c_int32),
        ("inner_tol", C.c_double),
        ("inner_maxit", C.c_int32),
        ("check_every", C.c_int32),
        ("refine", C.c_int32),
        ("stream", C.c_void_p),
    ]


_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32
_D = C.c_double
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)

# name -> (restype, argtypes); every symbol include/blk.h declares.
SIGNATURES = {
    "blk_cocg_solve": (_I32, [C.POINTER(BlkOp), _I64, _P, _I64, _P, _I64, _D, _I32,
                              C.POINTER(BlkOpts), _P, _I64, _DP, _IP, _DP]),
    "blk_cocr_solve": (_I32, [C.POINTER(BlkOp), _I64, _P, _I64, _P, _I64, _D, _I32,
                              C.POINTER(BlkOpts), _P, _I64, _DP, _IP, _DP]),
    "blk_spmm_z": (_I32, [C.POINTER(BlkOp), _I64, _P, _I64, _P, _I64, _P, _I64, _P, _P]),
    "blk_op_analyze": (_I32, [C.POINTER(BlkOp), _P]),
    "blk_spmm_c": (_I32, [C.POINTER(BlkOp), _P, _I64, _P, _I64, _P, _I64, _P]),
    "blk_gram_z": (_I32, [_I64, _I64, _P, _I64, _P, _I64, _I32, _P, _P]),
    "blk_thin_qr_z": (_I32, [_I64, _I64, _P, _I64, _P, _I64, _P, _P]),
    "blk_last_error": (C.c_char_p, []),
    "blk_version": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libblk.so; raise if it was not built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')"
        )
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
