"""CPU FP64 oracle for the block COCG / block COCR solvers (arXiv 1601.05362).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow reference that the
GPU path is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.

Everything runs in complex128.  Library primitives serve as single steps: a
sparse or dense matrix product (scipy / numpy), a dense LU solve with partial
pivoting (scipy.linalg.lu_factor / lu_solve, i.e. LAPACK zgetrf / zgetrs) and a Householder thin QR
(numpy.linalg.qr, i.e. LAPACK zgeqrf).  There is no blocking, fusion or
reordering beyond what the paper's recurrences state.

Notation follows the paper: X, R, P, Q, S, U, V are n x p blocks, alpha,
beta, xi, tau are p x p.  ``Y^T`` is the transpose WITHOUT conjugation (the
constraint spaces in Table 1 are built from conj(A) and conj(R_0), so their
orthogonality conditions are unconjugated bilinear forms).

Readings where the paper is silent or garbled (each also listed in the
design notes):
  * Block COCG is not printed; its coefficients come from the recurrences of
    section 2.1 with the COCG conditions of Table 1 (alpha from the Galerkin
    condition on R, beta from the one on A P).
  * In section 2.2 the superscript -1 is rendered as a subscript: read
    tau_{m+1} = xi_{m+1} xi_m^{-1}, S_m = P_m xi_m^{-1},
    alpha'_m = xi_m alpha_m xi_m^{-1}, beta'_m = xi_m beta_m xi_{m+1}^{-1}.
  * Algorithm 3 updates X with an undefined P; the oracle uses
    X += S alpha' xi as Algorithm 2 does (equal after the substitution above).
  * Algorithm 3 solves for beta' with the printed right-hand side
    tau^T Q_{m+1}^T V_{m+1}; its alpha' right-hand side is taken as
    Q_m^T V_m (the form Algorithm 1 gives) rather than the printed Q_m^T U_m,
    which is equal in exact arithmetic but unstable (see bl_cocr_rq).
  * Every variant stops on ||R_m||_F / ||B||_F <= tol, tested at the top of
    the loop (section 3 protocol).  Iters = completed loop bodies.
  * The thin QR is normalized so that diag(xi) is real and positive, which
    makes it unique for a full-rank block.
  * A block is treated as rank deficient (breakdown) when some |R_kk| of its
    Householder QR is <= RANK_TOL times its largest column norm.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import warnings

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

CONVERGED = 0
MAXIT = 1
BREAKDOWN = 2

# Relative rank threshold for the thin QR (see module docstring).
RANK_TOL = 1e-7
# Relative pivot threshold for the p x p LU solves.
PIVOT_TOL = 1e-13


class Breakdown(Exception):
    """A p x p system or a thin QR could not be completed."""


@dataclass
class Result:
    X: np.ndarray
    hist: list
    iters: int
    status: int
    # Optional per-iteration records (record=True): X_m, R_m, P_m, A P_m.
    Xs: list = field(default_factory=list)
    Rs: list = field(default_factory=list)
    Ps: list = field(default_factory=list)


# ---------------------------------------------------------------------------
# Primitives
# ---------------------------------------------------------------------------

def as_operator(A):
    """Wrap a dense ndarray or a CSR triple (workloads.Csr) as a linear map."""
    if isinstance(A, np.ndarray):
        return A
    if sp.issparse(A):
        return A.tocsr()
    # workloads.Csr or anything with rowptr/colind/val
    return sp.csr_matrix(
        (np.asarray(A.val, dtype=np.complex128), np.asarray(A.colind), np.asarray(A.rowptr)),
        shape=(A.n, A.n),
    )


def apply(A, Z: np.ndarray) -> np.ndarray:
    """Block product A Z (the single operator application of eq. 1.1)."""
    return np.asarray(A @ Z)


def gram_t(Y: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """Unconjugated p x p bilinear form Y^T Z."""
    return Y.T @ Z


def solve(M: np.ndarray, Rhs: np.ndarray) -> np.ndarray:
    """Solve M C = Rhs for the p x p coefficient C (LU, partial pivoting).

    The paper does not say how the p x p systems are solved; LU with partial
    pivoting is the general-matrix choice.  The system counts as singular
    (breakdown) when a pivot is <= PIVOT_TOL times the largest |M_ij|.
    """
    if not (np.all(np.isfinite(M)) and np.all(np.isfinite(Rhs))):
        raise Breakdown("non-finite p x p system")
    scale = np.max(np.abs(M)) if M.size else 0.0
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        lu, piv = sla.lu_factor(M, check_finite=False)
    if scale == 0.0 or np.min(np.abs(np.diag(lu))) <= PIVOT_TOL * scale:
        raise Breakdown("singular p x p system")
    C = sla.lu_solve((lu, piv), Rhs, check_finite=False)
    if not np.all(np.isfinite(C)):
        raise Breakdown("non-finite p x p solution")
    return C


def thin_qr_pos(W: np.ndarray):
    """Thin QR W = Q R with Q^H Q = I and diag(R) real positive (section 2.2).

    Raises Breakdown when W is numerically rank deficient.
    """
    if not np.all(np.isfinite(W)):
        raise Breakdown("non-finite block")
    Q, R = np.linalg.qr(W, mode="reduced")
    d = np.diag(R).copy()
    colnorm = np.sqrt(np.max(np.sum(np.abs(W) ** 2, axis=0))) if W.size else 0.0
    if colnorm == 0.0 or np.min(np.abs(d)) <= RANK_TOL * colnorm:
        raise Breakdown("rank-deficient block in thin QR")
    ph = d / np.abs(d)
    Q = Q * ph[None, :]
    R = R / ph[:, None]
    return Q, R


def fro(M: np.ndarray) -> float:
    return float(np.sqrt(np.sum(np.abs(M) ** 2)))


def true_relres(A, B: np.ndarray, X: np.ndarray) -> float:
    """||B - A X||_F / ||B||_F, the TRR quantity of section 3 (before log10)."""
    A = as_operator(A)
    nb = fro(B)
    return fro(B - apply(A, X)) / nb if nb > 0 else 0.0


def _late_breakdown(res: Result, r_next: float, tol: float) -> None:
    """The beta solve of iteration m failed after X_{m+1} was formed.

    X_{m+1} is a valid iterate; its residual decides the status.
    """
    res.hist.append(r_next)
    res.status = CONVERGED if r_next <= tol else BREAKDOWN


def _start(A, B, X0):
    A = as_operator(A)
    B = np.asarray(B, dtype=np.complex128)
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=np.complex128, copy=True)
    R = B.copy() if X0 is None else B - apply(A, X)
    return A, B, X, R


# ---------------------------------------------------------------------------
# Plain variants
# ---------------------------------------------------------------------------

def bl_cocg(A, B, X0=None, tol=1e-8, maxit=1000, record=False) -> Result:
    """Block COCG (section 2.1 recurrences, COCG conditions of Table 1).

    R_0 = P_0 = B - A X_0;  alpha_m solves (P^T A P) alpha = R^T R;
    X += P alpha;  R -= A P alpha;  beta_m solves (R_m^T R_m) beta =
    R_{m+1}^T R_{m+1};  P = R + P beta.
    """
    A, B, X, R = _start(A, B, X0)
    nb = fro(B)
    res = Result(X=X, hist=[], iters=0, status=CONVERGED)
    if nb == 0.0:
        res.X = np.zeros_like(B)
        res.hist = [0.0]
        return res
    P = R.copy()
    rho = gram_t(R, R)
    m = 0
    while True:
        res.hist.append(fro(R) / nb)
        if record:
            res.Xs.append(X.copy()); res.Rs.append(R.copy()); res.Ps.append(P.copy())
        if res.hist[m] <= tol:
            res.status = CONVERGED
            break
        if m == maxit:
            res.status = MAXIT
            break
        try:
            Z = apply(A, P)
            alpha = solve(gram_t(P, Z), rho)
        except Breakdown:
            res.status = BREAKDOWN
            break
        X = X + P @ alpha
        R = R - Z @ alpha
        rho_n = gram_t(R, R)
        try:
            beta = solve(rho, rho_n)
        except Breakdown:
            _late_breakdown(res, fro(R) / nb, tol)
            m += 1
            break
        P = R + P @ beta
        rho = rho_n
        m += 1
    res.X, res.iters = X, m
    return res


def bl_cocr(A, B, X0=None, tol=1e-8, maxit=1000, record=False) -> Result:
    """Block COCR, Algorithm 1.

    R_0 = P_0 = B - A X_0, U_0 = V_0 = A R_0;  alpha solves (U^T U) alpha =
    R^T V;  X += P alpha;  R_{m+1} = R - U alpha;  V_{m+1} = A R_{m+1};
    beta solves (R_m^T V_m) beta = R_{m+1}^T V_{m+1};  P = R + P beta;
    U = V + U beta.
    """
    A, B, X, R = _start(A, B, X0)
    nb = fro(B)
    res = Result(X=X, hist=[], iters=0, status=CONVERGED)
    if nb == 0.0:
        res.X = np.zeros_like(B)
        res.hist = [0.0]
        return res
    P = R.copy()
    V = apply(A, R)
    U = V.copy()
    m = 0
    while True:
        res.hist.append(fro(R) / nb)
        if record:
            res.Xs.append(X.copy()); res.Rs.append(R.copy()); res.Ps.append(P.copy())
        if res.hist[m] <= tol:
            res.status = CONVERGED
            break
        if m == maxit:
            res.status = MAXIT
            break
        rv = gram_t(R, V)
        try:
            alpha = solve(gram_t(U, U), rv)
        except Breakdown:
            res.status = BREAKDOWN
            break
        X = X + P @ alpha
        Rn = R - U @ alpha
        Vn = apply(A, Rn)
        try:
            beta = solve(rv, gram_t(Rn, Vn))
        except Breakdown:
            _late_breakdown(res, fro(Rn) / nb, tol)
            m += 1
            break
        P = Rn + P @ beta
        U = Vn + U @ beta
        R, V = Rn, Vn
        m += 1
    res.X, res.iters = X, m
    return res


# ---------------------------------------------------------------------------
# Residual-orthonormalized variants (section 2.2)
# ---------------------------------------------------------------------------

def _rq_next(W, xi, nb, X, res, m, tol):
    """Orthonormalize W = Q_{m+1} tau_{m+1}; xi_{m+1} = tau xi_m.

    If W is rank deficient, the residual R_{m+1} = W xi_m decides between
    convergence and breakdown.  Returns (Qn, tau, xi_n) or None when stopping.
    """
    try:
        Qn, tau = thin_qr_pos(W)
    except Breakdown:
        r = fro(W @ xi) / nb if np.all(np.isfinite(W)) else float("nan")
        res.hist.append(r)
        res.iters = m + 1
        res.status = CONVERGED if r <= tol else BREAKDOWN
        return None
    return Qn, tau, tau @ xi


def bl_cocg_rq(A, B, X0=None, tol=1e-8, maxit=1000, record=False) -> Result:
    """Block COCG with residual orthonormalization, Algorithm 2.

    Q_0 xi_0 = B - A X_0, S_0 = Q_0;  alpha' solves (S^T A S) alpha' = Q^T Q;
    X += S alpha' xi;  Q_{m+1} tau_{m+1} = Q - A S alpha';  xi = tau xi;
    beta' solves (Q_m^T Q_m) beta' = tau^T Q_{m+1}^T Q_{m+1};
    S = Q_{m+1} + S beta'.
    """
    A, B, X, R = _start(A, B, X0)
    nb = fro(B)
    res = Result(X=X, hist=[], iters=0, status=CONVERGED)
    if nb == 0.0:
        res.X = np.zeros_like(B)
        res.hist = [0.0]
        return res
    try:
        Q, xi = thin_qr_pos(R)
    except Breakdown:
        res.hist = [fro(R) / nb]
        res.status = CONVERGED if res.hist[0] <= tol else BREAKDOWN
        return res
    S = Q.copy()
    gqq = gram_t(Q, Q)
    m = 0
    while True:
        res.hist.append(fro(xi) / nb)
        if record:
            res.Xs.append(X.copy()); res.Rs.append(Q @ xi); res.Ps.append(S @ xi)
        if res.hist[m] <= tol:
            res.status = CONVERGED
            break
        if m == maxit:
            res.status = MAXIT
            break
        try:
            Z = apply(A, S)
            alpha = solve(gram_t(S, Z), gqq)
        except Breakdown:
            res.status = BREAKDOWN
            break
        X = X + S @ (alpha @ xi)
        W = Q - Z @ alpha
        nxt = _rq_next(W, xi, nb, X, res, m, tol)
        if nxt is None:
            res.X = X
            if record:
                res.Xs.append(X.copy())
            return res
        Qn, tau, xi = nxt
        gn = gram_t(Qn, Qn)
        try:
            beta = solve(gqq, tau.T @ gn)
        except Breakdown:
            _late_breakdown(res, fro(xi) / nb, tol)
            m += 1
            break
        S = Qn + S @ beta
        Q, gqq = Qn, gn
        m += 1
    res.X, res.iters = X, m
    return res


def bl_cocr_rq(A, B, X0=None, tol=1e-8, maxit=1000, record=False, alpha_rhs="QtV") -> Result:
    """Block COCR with residual orthonormalization, Algorithm 3.

    Q_0 xi_0 = B - A X_0, S_0 = Q_0, U_0 = V_0 = A Q_0;
    alpha' solves (U^T U) alpha' = Q_m^T V_m;  X += S alpha' xi;
    Q_{m+1} tau_{m+1} = Q - U alpha';  xi = tau xi;  V_{m+1} = A Q_{m+1};
    beta' solves (Q_m^T V_m) beta' = tau^T Q_{m+1}^T V_{m+1};
    S = Q_{m+1} + S beta';  U = V_{m+1} + U beta'.

    The alpha' right-hand side is Q_m^T V_m, which is what substituting
    R = Q xi, P = S xi into Algorithm 1 (whose right-hand side is R^T V)
    yields.  Algorithm 3 prints Q_m^T U_m instead; the two agree in exact
    arithmetic because the COCR condition of Table 1 makes Q_m^T U_{m-1}
    vanish, but in floating point the printed form loses that orthogonality
    and diverges on the 2D Helmholtz workload.  alpha_rhs="QtU" selects the
    printed form (for the tests that compare the two).
    """
    A, B, X, R = _start(A, B, X0)
    nb = fro(B)
    res = Result(X=X, hist=[], iters=0, status=CONVERGED)
    if nb == 0.0:
        res.X = np.zeros_like(B)
        res.hist = [0.0]
        return res
    try:
        Q, xi = thin_qr_pos(R)
    except Breakdown:
        res.hist = [fro(R) / nb]
        res.status = CONVERGED if res.hist[0] <= tol else BREAKDOWN
        return res
    S = Q.copy()
    V = apply(A, Q)
    U = V.copy()
    gqv = gram_t(Q, V)
    m = 0
    while True:
        res.hist.append(fro(xi) / nb)
        if record:
            res.Xs.append(X.copy()); res.Rs.append(Q @ xi); res.Ps.append(S @ xi)
        if res.hist[m] <= tol:
            res.status = CONVERGED
            break
        if m == maxit:
            res.status = MAXIT
            break
        try:
            rhs = gqv if alpha_rhs == "QtV" else gram_t(Q, U)
            alpha = solve(gram_t(U, U), rhs)
        except Breakdown:
            res.status = BREAKDOWN
            break
        X = X + S @ (alpha @ xi)
        W = Q - U @ alpha
        nxt = _rq_next(W, xi, nb, X, res, m, tol)
        if nxt is None:
            res.X = X
            if record:
                res.Xs.append(X.copy())
            return res
        Qn, tau, xi = nxt
        Vn = apply(A, Qn)
        gn = gram_t(Qn, Vn)
        try:
            beta = solve(gqv, tau.T @ gn)
        except Breakdown:
            _late_breakdown(res, fro(xi) / nb, tol)
            m += 1
            break
        S = Qn + S @ beta
        U = Vn + U @ beta
        Q, V, gqv = Qn, Vn, gn
        m += 1
    res.X, res.iters = X, m
    return res


METHODS = {
    "cocg": bl_cocg,
    "cocr": bl_cocr,
    "cocg_rq": bl_cocg_rq,
    "cocr_rq": bl_cocr_rq,
}


def solve_block(method: str, A, B, X0=None, tol=1e-8, maxit=1000, record=False, **kw) -> Result:
    """Dispatch by name: 'cocg', 'cocr', 'cocg_rq', 'cocr_rq'."""
    return METHODS[method](A, B, X0=X0, tol=tol, maxit=maxit, record=record, **kw)
