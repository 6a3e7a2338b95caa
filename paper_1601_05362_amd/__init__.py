"""MI355X block COCG / block COCR solvers for complex symmetric A X = B.

Python binding of the C ABI declared in include/blk.h.  The functions named
``blk_*`` marshal torch tensors (device memory, current stream) into the C
calls one to one; every step of a solve runs in the HIP library.  There is no
CPU fallback: without the built library the calls raise.

Method: Gu, Carpentieri, Huang, Meng, arXiv 1601.05362 (block COCG, block
COCR, and their residual-orthonormalized variants, Algorithms 1-3).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _capi
from ._capi import (
    BLK_BREAKDOWN,
    BLK_CONVERGED,
    BLK_EHIP,
    BLK_EINVAL,
    BLK_ENOMEM,
    BLK_FP64,
    BLK_MAX_P,
    BLK_MAXIT,
    BLK_MIXED,
    BLK_OP_CSR,
    BLK_OP_DENSE,
    STATUS_NAMES,
)

__all__ = [
    "CsrOperator",
    "DenseOperator",
    "SolveResult",
    "blk_cocg_solve",
    "blk_cocr_solve",
    "blk_op_analyze",
    "blk_spmm_z",
    "blk_spmm_c",
    "blk_gram_z",
    "blk_thin_qr_z",
    "blk_last_error",
    "blk_version",
    "BLK_MAX_P",
    "BLK_CONVERGED",
    "BLK_MAXIT",
    "BLK_BREAKDOWN",
]


def _lib():
    return _capi.load()


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _block(t: torch.Tensor, name: str, dtype=torch.complex128) -> int:
    """Validate an n x p device block; return its leading dimension."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if t.dim() != 2 or t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} must be a row-major (n, p) block with unit column stride")
    return t.stride(0)


def _raise(code: int, what: str):
    msg = f"{what}: {blk_last_error()}"
    if code == BLK_EINVAL:
        raise ValueError(msg)
    if code == BLK_ENOMEM:
        raise MemoryError(msg)
    raise RuntimeError(msg)


class CsrOperator:
    """Complex symmetric CSR matrix on the GPU (int32 indices)."""

    def __init__(self, rowptr: torch.Tensor, colind: torch.Tensor, val: torch.Tensor):
        if rowptr.dtype != torch.int32 or colind.dtype != torch.int32:
            raise TypeError("rowptr and colind must be int32")
        if val.dtype != torch.complex128:
            raise TypeError("val must be complex128")
        for t in (rowptr, colind, val):
            if t.device.type != "cuda" or not t.is_contiguous():
                raise ValueError("CSR arrays must be contiguous GPU tensors")
        self.rowptr, self.colind, self.val = rowptr, colind, val
        self.n = rowptr.numel() - 1
        self.nnz = colind.numel()
        self.device = val.device
        self._val32 = None
        self.structure = _capi.BLK_STRUCT_UNKNOWN
        self.grid = (0, 0, 0)

    @classmethod
    def from_arrays(cls, rowptr, colind, val, device="cuda"):
        return cls(
            torch.as_tensor(np.asarray(rowptr, dtype=np.int32), device=device),
            torch.as_tensor(np.asarray(colind, dtype=np.int32), device=device),
            torch.as_tensor(np.asarray(val, dtype=np.complex128), device=device),
        )

    @property
    def val32(self) -> torch.Tensor:
        """complex64 copy of the values (made on first use, kept)."""
        if self._val32 is None:
            self._val32 = self.val.to(torch.complex64)
        return self._val32

    def analyze(self) -> "CsrOperator":
        """Check the pattern once (blk_op_analyze); a grid-stencil pattern
        then takes the 2.5D blocked product in every later call."""
        op = self.as_c()
        with torch.cuda.device(self.device):
            rc = _lib().blk_op_analyze(C.byref(op), _stream(self.device))
        if rc != 0:
            _raise(rc, "blk_op_analyze")
        self.structure = op.structure
        self.grid = tuple(op.grid)
        return self

    def as_c(self) -> _capi.BlkOp:
        return _capi.BlkOp(BLK_OP_CSR, self.structure, self.n, self.nnz, self.rowptr.data_ptr(),
                           self.colind.data_ptr(), self.val.data_ptr(), None, 0,
                           (C.c_int64 * 3)(*self.grid))


class DenseOperator:
    """Dense complex symmetric matrix on the GPU, row-major complex128."""

    def __init__(self, a: torch.Tensor):
        if a.dtype != torch.complex128 or a.device.type != "cuda":
            raise TypeError("dense operator must be a complex128 GPU tensor")
        if a.dim() != 2 or a.shape[0] != a.shape[1] or a.stride(1) != 1:
            raise ValueError("dense operator must be square and row-major")
        self.a = a
        self.n = a.shape[0]
        self.device = a.device
        self._val32 = None

    @property
    def val32(self) -> torch.Tensor:
        """complex64 copy of the matrix (made on first use)."""
        if self._val32 is None:
            self._val32 = self.a.to(torch.complex64)
        return self._val32

    def as_c(self) -> _capi.BlkOp:
        return _capi.BlkOp(BLK_OP_DENSE, _capi.BLK_STRUCT_GENERAL, self.n, 0, None, None, None,
                           self.a.data_ptr(), self.a.stride(0), (C.c_int64 * 3)(0, 0, 0))


@dataclass
class SolveResult:
    X: torch.Tensor
    hist: np.ndarray      # monitored relative residual per iteration (iters + 1 entries)
    iters: int
    status: int           # BLK_CONVERGED / BLK_MAXIT / BLK_BREAKDOWN
    true_relres: float    # ||B - A X||_F / ||B||_F in FP64

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))


def _solve(fn_name: str, A, B, X0, tol, maxit, rq, precision, inner_tol, inner_maxit,
           check_every, out, refine=0):
    lib = _lib()
    dev = B.device
    ldb = _block(B, "B")
    n, p = B.shape
    if A.n != n:
        raise ValueError(f"A is {A.n} x {A.n} but B has {n} rows")
    ldx0 = _block(X0, "X0") if X0 is not None else 0
    X = out if out is not None else torch.empty((n, p), dtype=torch.complex128, device=dev)
    ldx = _block(X, "out")
    prec = {"fp64": BLK_FP64, "mixed": BLK_MIXED}[precision]
    hist = np.zeros(maxit + 1, dtype=np.float64)
    iters = C.c_int32(0)
    trr = C.c_double(0.0)
    op = A.as_c()
    with torch.cuda.device(dev):
        opts = _capi.BlkOpts(1 if rq else 0, prec, float(inner_tol), int(inner_maxit),
                             int(check_every), int(refine), _stream(dev))
        rc = getattr(lib, fn_name)(
            C.byref(op), p, _ptr(B), ldb, _ptr(X0), ldx0, float(tol), int(maxit), C.byref(opts),
            _ptr(X), ldx, hist.ctypes.data_as(C.POINTER(C.c_double)), C.byref(iters),
            C.byref(trr))
    if rc < 0:
        _raise(rc, fn_name)
    k = iters.value
    return SolveResult(X=X, hist=hist[: k + 1].copy(), iters=k, status=rc,
                       true_relres=trr.value)


def blk_cocg_solve(A, B, X0=None, tol=1e-8, maxit=1000, *, rq=True, precision="fp64",
                   inner_tol=1e-3, inner_maxit=0, check_every=16, refine=0,
                   out=None) -> SolveResult:
    """Block COCG (rq=False) or block COCG with residual orthonormalization
    (rq=True, Algorithm 2) for A X = B."""
    return _solve("blk_cocg_solve", A, B, X0, tol, maxit, rq, precision, inner_tol,
                  inner_maxit, check_every, out, refine)


def blk_cocr_solve(A, B, X0=None, tol=1e-8, maxit=1000, *, rq=True, precision="fp64",
                   inner_tol=1e-3, inner_maxit=0, check_every=16, refine=0,
                   out=None) -> SolveResult:
    """Block COCR (rq=False, Algorithm 1) or block COCR with residual
    orthonormalization (rq=True, Algorithm 3) for A X = B."""
    return _solve("blk_cocr_solve", A, B, X0, tol, maxit, rq, precision, inner_tol,
                  inner_maxit, check_every, out, refine)


def blk_op_analyze(A):
    """Pattern analysis of a CSR operator (grid-stencil detection); returns A
    with its `structure` and `grid` set.  Dense operators need none."""
    if isinstance(A, CsrOperator):
        return A.analyze()
    return A


def blk_spmm_z(A, Z: torch.Tensor, C_: torch.Tensor | None = None, out=None, gram=False):
    """Y = A Z (or C - A Z); with gram=True also returns Z^T Y (numpy p x p)."""
    lib = _lib()
    ldz = _block(Z, "Z")
    n, p = Z.shape
    ldc = _block(C_, "C") if C_ is not None else 0
    Y = out if out is not None else torch.empty((n, p), dtype=torch.complex128, device=Z.device)
    ldy = _block(Y, "out")
    G = np.zeros((p, p), dtype=np.complex128) if gram else None
    op = A.as_c()
    with torch.cuda.device(Z.device):
        rc = lib.blk_spmm_z(C.byref(op), p, _ptr(Z), ldz, _ptr(C_), ldc, _ptr(Y), ldy,
                            G.ctypes.data if gram else None, _stream(Z.device))
    if rc != 0:
        _raise(rc, "blk_spmm_z")
    return (Y, G) if gram else Y


def blk_spmm_c(A, Z: torch.Tensor, out=None):
    """complex64 Y = A Z with FP32 accumulation, for a CsrOperator (its
    complex64 values, grid structure if analysed) or a DenseOperator (its
    complex64 copy)."""
    lib = _lib()
    ldz = _block(Z, "Z", torch.complex64)
    n, p = Z.shape
    Y = out if out is not None else torch.empty((n, p), dtype=torch.complex64, device=Z.device)
    ldy = _block(Y, "out", torch.complex64)
    v = A.val32
    op = A.as_c()
    if isinstance(A, DenseOperator):
        op.ld = v.stride(0)
    with torch.cuda.device(Z.device):
        rc = lib.blk_spmm_c(C.byref(op), v.data_ptr(), p, _ptr(Z), ldz, _ptr(Y), ldy,
                            _stream(Z.device))
    if rc != 0:
        _raise(rc, "blk_spmm_c")
    return Y


def blk_gram_z(Y: torch.Tensor, Z: torch.Tensor, conj: bool = False) -> np.ndarray:
    """p x p form Y^T Z (conj=False) or Y^H Z (conj=True), returned on the host."""
    lib = _lib()
    ldy = _block(Y, "Y")
    ldz = _block(Z, "Z")
    if Y.shape != Z.shape:
        raise ValueError("Y and Z must have the same shape")
    n, p = Y.shape
    G = np.zeros((p, p), dtype=np.complex128)
    with torch.cuda.device(Y.device):
        rc = lib.blk_gram_z(n, p, _ptr(Y), ldy, _ptr(Z), ldz, 1 if conj else 0, G.ctypes.data,
                            _stream(Y.device))
    if rc != 0:
        _raise(rc, "blk_gram_z")
    return G


def blk_thin_qr_z(W: torch.Tensor, out=None):
    """Thin QR W = Q R (Cholesky QR twice); returns (Q, R) with R on the host.

    Raises ArithmeticError when W is numerically rank deficient."""
    lib = _lib()
    ldw = _block(W, "W")
    n, p = W.shape
    Q = out if out is not None else torch.empty_like(W)
    ldq = _block(Q, "out")
    R = np.zeros((p, p), dtype=np.complex128)
    with torch.cuda.device(W.device):
        rc = lib.blk_thin_qr_z(n, p, _ptr(W), ldw, _ptr(Q), ldq, R.ctypes.data, _stream(W.device))
    if rc == BLK_BREAKDOWN:
        raise ArithmeticError(blk_last_error())
    if rc != 0:
        _raise(rc, "blk_thin_qr_z")
    return Q, R


def blk_last_error() -> str:
    return _lib().blk_last_error().decode()


def blk_version() -> str:
    return _lib().blk_version().decode()
