"""The C ABI library: it loads, exports what include/blk.h declares, and the
header, ctypes declarations and Python names agree.  No compute calls."""
from __future__ import annotations

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "blk.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(blk_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1601_05362_amd import _capi

    if not os.path.exists(_capi.LIB_PATH):
        pytest.fail("libblk.so is not built (run __graft_entry__.build())")
    lib = C.CDLL(_capi.LIB_PATH)
    names = _declared()
    assert names, "no declarations found"
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(_capi.SIGNATURES) == names


def test_python_binding_has_same_names():
    import paper_1601_05362_amd as pkg

    for name in _declared():
        assert callable(getattr(pkg, name)), name


def test_version_and_error_without_gpu():
    import paper_1601_05362_amd as pkg

    assert "gfx950" in pkg.blk_version()
    assert isinstance(pkg.blk_last_error(), str)


def test_argument_validation_rejects_before_device_work():
    """Invalid arguments return BLK_EINVAL before any HIP call."""
    from paper_1601_05362_amd import _capi

    lib = _capi.load()
    fake = 0x1000
    op = _capi.BlkOp(_capi.BLK_OP_CSR, 0, 10, 30, fake, fake, fake, None, 0)
    it = C.c_int32(0)
    # p out of range
    assert lib.blk_cocr_solve(C.byref(op), 0, fake, 1, None, 0, 1e-8, 10, None, fake + 4096, 1,
                              None, C.byref(it), None) == _capi.BLK_EINVAL
    assert lib.blk_cocg_solve(C.byref(op), 33, fake, 33, None, 0, 1e-8, 10, None, fake + 65536, 33,
                              None, C.byref(it), None) == _capi.BLK_EINVAL
    # tol <= 0, NaN, maxit < 0
    for tol, maxit in ((0.0, 10), (float("nan"), 10), (1e-8, -1)):
        assert lib.blk_cocr_solve(C.byref(op), 2, fake, 2, None, 0, tol, maxit, None, fake + 4096, 2,
                                  None, C.byref(it), None) == _capi.BLK_EINVAL
    # X overlapping B
    assert lib.blk_cocr_solve(C.byref(op), 2, fake, 2, None, 0, 1e-8, 10, None, fake + 16, 2, None,
                              C.byref(it), None) == _capi.BLK_EINVAL
    # leading dimension < p
    assert lib.blk_cocr_solve(C.byref(op), 4, fake, 2, None, 0, 1e-8, 10, None, fake + 8192, 4, None,
                              C.byref(it), None) == _capi.BLK_EINVAL
    # NULL operator, unknown kind, bad dense ld
    assert lib.blk_cocr_solve(None, 2, fake, 2, None, 0, 1e-8, 10, None, fake + 4096, 2, None,
                              C.byref(it), None) == _capi.BLK_EINVAL
    bad = _capi.BlkOp(7, 0, 10, 0, None, None, None, None, 0)
    assert lib.blk_cocr_solve(C.byref(bad), 2, fake, 2, None, 0, 1e-8, 10, None, fake + 4096, 2,
                              None, C.byref(it), None) == _capi.BLK_EINVAL
    dense = _capi.BlkOp(_capi.BLK_OP_DENSE, 0, 10, 0, None, None, None, fake, 5)
    assert lib.blk_cocr_solve(C.byref(dense), 2, fake, 2, None, 0, 1e-8, 10, None, fake + 4096, 2,
                              None, C.byref(it), None) == _capi.BLK_EINVAL
    assert "ld" in lib.blk_last_error().decode()
    # kernels entry points
    assert lib.blk_gram_z(10, 0, fake, 1, fake, 1, 0, fake, None) == _capi.BLK_EINVAL
    assert lib.blk_spmm_c(C.byref(op), None, 2, fake, 2, fake + 4096, 2, None) == _capi.BLK_EINVAL
    assert "vals32" in lib.blk_last_error().decode()
    assert lib.blk_spmm_c(C.byref(op), fake, 33, fake, 33, fake + 65536, 33, None) == _capi.BLK_EINVAL
    assert lib.blk_spmm_c(None, fake, 2, fake, 2, fake + 4096, 2, None) == _capi.BLK_EINVAL
    assert lib.blk_thin_qr_z(10, 2, fake, 1, fake, 2, fake, None) == _capi.BLK_EINVAL


def test_structure_validation_rejects_before_device_work():
    """A grid structure whose dimensions do not multiply to n, or an unknown
    structure code, is BLK_EINVAL; blk_op_analyze leaves the operator as it
    was on EINVAL."""
    from paper_1601_05362_amd import _capi

    lib = _capi.load()
    fake = 0x1000
    it = C.c_int32(0)
    grid = (C.c_int64 * 3)(4, 4, 3)  # 48 != 50
    op = _capi.BlkOp(_capi.BLK_OP_CSR, _capi.BLK_STRUCT_GRID, 50, 200, fake, fake, fake, None, 0, grid)
    assert lib.blk_cocr_solve(C.byref(op), 2, fake, 2, None, 0, 1e-8, 10, None, fake + 8192, 2, None,
                              C.byref(it), None) == _capi.BLK_EINVAL
    assert "grid" in lib.blk_last_error().decode()
    assert lib.blk_spmm_z(C.byref(op), 2, fake, 2, None, 0, fake + 8192, 2, None, None) == _capi.BLK_EINVAL
    op.structure = 7
    assert lib.blk_spmm_z(C.byref(op), 2, fake, 2, None, 0, fake + 8192, 2, None, None) == _capi.BLK_EINVAL
    # analysis of an invalid operator: EINVAL, structure untouched
    bad = _capi.BlkOp(_capi.BLK_OP_CSR, _capi.BLK_STRUCT_GENERAL, 0, 0, None, None, None, None, 0,
                      (C.c_int64 * 3)(0, 0, 0))
    assert lib.blk_op_analyze(C.byref(bad), None) == _capi.BLK_EINVAL
    assert bad.structure == _capi.BLK_STRUCT_GENERAL
    assert lib.blk_op_analyze(None, None) == _capi.BLK_EINVAL
