"""Independent checks that pin the oracle to the paper's definitions.

Nothing here calls the oracle's recurrences: these are closed forms and
textbook routines written separately, against which the oracle's iterates are
compared.
"""
from __future__ import annotations

import numpy as np


def krylov_basis(A, R0: np.ndarray, m: int) -> np.ndarray:
    """Orthonormal basis (Hermitian sense) of span{R0, A R0, ..., A^{m-1} R0}.

    Block Arnoldi with two passes of classical Gram-Schmidt; the span equals
    the block Krylov space of eq. (1.3) as long as nothing deflates.
    """
    Q, _ = np.linalg.qr(R0)
    blocks = [Q]
    cur = Q
    for _ in range(1, m):
        W = A @ cur
        for _ in range(2):
            for Bk in blocks:
                W = W - Bk @ (Bk.conj().T @ W)
        cur, _ = np.linalg.qr(W)
        blocks.append(cur)
    return np.hstack(blocks)


def petrov_galerkin_iterate(A, B: np.ndarray, X0: np.ndarray, m: int, method: str) -> np.ndarray:
    """The m-th iterate defined by the constraints of Table 1.

    X_m = X_0 + K Y with K a basis of K_m(A; R_0).  COCG imposes
    K^T R_m = 0 (R_m orthogonal to conj(K) in the Hermitian sense), COCR
    imposes (A K)^T R_m = 0.  Both are unconjugated bilinear forms.
    """
    R0 = B - A @ X0
    if m == 0:
        return X0.copy()
    K = krylov_basis(A, R0, m)
    AK = A @ K
    if method.startswith("cocg"):
        Y = np.linalg.solve(K.T @ AK, K.T @ R0)
    elif method.startswith("cocr"):
        Y = np.linalg.solve(AK.T @ AK, AK.T @ R0)
    else:
        raise ValueError(method)
    return X0 + K @ Y


def scalar_cocg(A, b: np.ndarray, iters: int) -> list:
    """Textbook COCG (one right-hand side, x0 = 0); returns x_0..x_iters."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r  # unconjugated
    xs = [x.copy()]
    for _ in range(iters):
        Ap = A @ p
        a = rr / (p @ Ap)
        x = x + a * p
        r = r - a * Ap
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
        xs.append(x.copy())
    return xs


def scalar_cocr(A, b: np.ndarray, iters: int) -> list:
    """Textbook COCR (one right-hand side, x0 = 0); returns x_0..x_iters."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    Ar = A @ r
    Ap = Ar.copy()
    rAr = r @ Ar
    xs = [x.copy()]
    for _ in range(iters):
        a = rAr / (Ap @ Ap)
        x = x + a * p
        r = r - a * Ap
        Ar = A @ r
        rAr_new = r @ Ar
        b_ = rAr_new / rAr
        p = r + b_ * p
        Ap = Ar + b_ * Ap
        rAr = rAr_new
        xs.append(x.copy())
    return xs


def well_conditioned_cs(n: int, seed: int) -> np.ndarray:
    """Complex symmetric, non-Hermitian, well-conditioned dense matrix."""
    rng = np.random.default_rng(seed)
    G = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    return 0.5 * (G + G.T) + (2.0 + 1.0j) * np.eye(n)


def rel(a, b) -> float:
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
