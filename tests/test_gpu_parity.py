"""GPU path vs the CPU oracle, element by element, through the C ABI.

Tolerances: FP64 kernels match the oracle's primitives to a few ulps of the
operands' scale (1e-13 relative).  FP64 solves of the 2D Helmholtz workload
with residual orthonormalization match the residual history to 1e-9 relative
over the first 50 iterations, the final X to 1e-7 relative Frobenius and the
iteration count within 2%.  Where rounding alone moves the oracle further
(the plain variants, whose late convergence is chaotic, and operators with
near-singular unconjugated p x p forms), the bounds are the oracle's own
spread under a 1e-15 perturbation of B, measured in the test.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import blk_oracle as O
from tests import pins

pytestmark = pytest.mark.gpu

VARIANTS = [("cocg", False), ("cocr", False), ("cocg", True), ("cocr", True)]
ORACLE_NAME = {("cocg", False): "cocg", ("cocr", False): "cocr", ("cocg", True): "cocg_rq",
               ("cocr", True): "cocr_rq"}


@pytest.fixture(scope="module")
def pkg():
    import paper_1601_05362_amd as p

    p._capi.load()
    return p


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def cfg1(pkg, dev):
    A, B = W.config1()
    return A, B, pkg.CsrOperator.from_arrays(A.rowptr, A.colind, A.val, device=dev), torch.as_tensor(B, device=dev)


def _solve(pkg, method, rq, Ad, Bd, **kw):
    fn = pkg.blk_cocg_solve if method == "cocg" else pkg.blk_cocr_solve
    return fn(Ad, Bd, rq=rq, **kw)


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ---------------------------------------------------------------------------
# Kernels
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p", [1, 3, 4, 8, 13, 16, 32])
def test_spmm_matches_oracle(pkg, dev, cfg1, p):
    A, _, Ad, _ = cfg1
    Z = W.cgauss(A.n, p, seed=p)
    C = W.cgauss(A.n, p, seed=100 + p)
    Zd, Cd = torch.as_tensor(Z, device=dev), torch.as_tensor(C, device=dev)
    Aop = O.as_operator(A)
    Y_ref = O.apply(Aop, Z)
    Y, G = pkg.blk_spmm_z(Ad, Zd, gram=True)
    scale = np.abs(A.val).max() * np.abs(Z).max()
    assert np.max(np.abs(Y.cpu().numpy() - Y_ref)) <= 1e-13 * scale * 7
    G_ref = O.gram_t(Z, Y_ref)
    assert _relerr(G, G_ref) < 1e-12
    Y2 = pkg.blk_spmm_z(Ad, Zd, C_=Cd)
    assert np.max(np.abs(Y2.cpu().numpy() - (C - Y_ref))) <= 1e-13 * scale * 7


def test_spmm_ragged_rows_and_ld(pkg, dev):
    """n not a multiple of any tile, empty rows, unsorted columns, ld > p."""
    rng = np.random.default_rng(5)
    n, p = 1237, 5
    D = np.zeros((n, n), complex)
    for i in range(n):
        if i % 97 == 13:
            continue  # empty row
        cols = rng.choice(n, size=rng.integers(1, 9), replace=False)
        D[i, cols] = rng.standard_normal(len(cols)) + 1j * rng.standard_normal(len(cols))
    rows, cols = np.nonzero(D)
    order = rng.permutation(len(rows))  # unsorted within rows after stable sort by row
    order = order[np.argsort(rows[order], kind="stable")]
    rowptr = np.zeros(n + 1, np.int32)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    Ad = pkg.CsrOperator.from_arrays(rowptr, cols[order], D[rows[order], cols[order]], device=dev)
    Zbig = torch.as_tensor(W.cgauss(n, 8, seed=6), device=dev)
    Z = Zbig[:, :p]  # ld = 8
    Y = pkg.blk_spmm_z(Ad, Z)
    torch.cuda.synchronize()
    ref = D @ Zbig[:, :p].cpu().numpy()
    assert _relerr(Y.cpu().numpy(), ref) < 1e-14


@pytest.mark.parametrize("p", [1, 4, 32])
def test_spmm_c64_matches_oracle(pkg, dev, cfg1, p):
    A, _, Ad, _ = cfg1
    Z = W.cgauss(A.n, p, seed=7).astype(np.complex64)
    Y = pkg.blk_spmm_c(Ad, torch.as_tensor(Z, device=dev)).cpu().numpy()
    ref = O.apply(O.as_operator(A), Z.astype(np.complex128))
    # FP32 storage of A and Z plus FP32 accumulation: a few ulps of |A||Z|
    scale = np.abs(A.val).max() * np.abs(Z).max()
    assert np.max(np.abs(Y - ref)) <= 5 * 6e-8 * scale * 5


@pytest.mark.parametrize("dims", [(13, 11, 9), (37, 29, 1), (16, 16, 33)])
@pytest.mark.parametrize("p", [5, 8, 16, 17, 32])
def test_spmm_c64_grid_within_fp32_bound(pkg, dev, dims, p):
    """The complex64 product through the 2.5D stencil kernel (an analysed
    operator) and the general kernel, against the FP64 product of the same
    complex64 values: each part of an entry is a sum of at most 14 real
    products in FP32, so its modulus error is at most sqrt(2) gamma_14
    (|A| |Z|)_ij, u = 2^-24."""
    A = W.grid_stencil_random(*dims, seed=5)
    A.val = A.val.astype(np.complex64).astype(np.complex128)
    Z = W.cgauss(A.n, p, seed=6).astype(np.complex64)
    ref = O.apply(O.as_operator(A), Z.astype(np.complex128))
    absA = O.as_operator(A).copy()
    absA.data = np.abs(absA.data)
    bound = math.sqrt(2) * (14 * 2.0 ** -24 / (1 - 14 * 2.0 ** -24)) * (absA @ np.abs(Z).astype(np.float64))
    grd = pkg.CsrOperator.from_arrays(A.rowptr, A.colind, A.val, device=dev).analyze()
    assert grd.structure == pkg._capi.BLK_STRUCT_GRID
    gen = pkg.CsrOperator.from_arrays(A.rowptr, A.colind, A.val, device=dev)
    gen.structure = pkg._capi.BLK_STRUCT_GENERAL
    Zd = torch.as_tensor(Z, device=dev)
    for op in (grd, gen):
        Y = pkg.blk_spmm_c(op, Zd).cpu().numpy().astype(np.complex128)
        assert np.all(np.abs(Y - ref) <= bound), float(np.max(np.abs(Y - ref) / np.maximum(bound, 1e-300)))


@pytest.mark.parametrize("p", [1, 2, 7, 16, 32])
@pytest.mark.parametrize("conj", [False, True])
def test_gram_matches_oracle(pkg, dev, p, conj):
    n = 100003
    Y = W.cgauss(n, p, seed=1)
    Z = W.cgauss(n, p, seed=2)
    G = pkg.blk_gram_z(torch.as_tensor(Y, device=dev), torch.as_tensor(Z, device=dev), conj=conj)
    ref = (Y.conj().T if conj else Y.T) @ Z
    assert _relerr(G, ref) < 1e-13


@pytest.mark.parametrize("n,p", [(4096, 4), (50001, 32), (777, 9)])
def test_thin_qr_matches_oracle(pkg, dev, n, p):
    Wb = W.cgauss(n, p, seed=n) @ (np.eye(p) + 0.3 * W.cgauss(p, p, seed=1))
    Q, R = pkg.blk_thin_qr_z(torch.as_tensor(Wb, device=dev))
    Q = Q.cpu().numpy()
    Qr, Rr = O.thin_qr_pos(Wb)
    assert _relerr(R, Rr) < 1e-12
    assert _relerr(Q, Qr) < 1e-12
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(p))) < 1e-13


def test_thin_qr_rank_deficient(pkg, dev):
    Wb = W.cgauss(1000, 3, seed=3)
    Wb[:, 2] = Wb[:, 0]
    with pytest.raises(ArithmeticError):
        pkg.blk_thin_qr_z(torch.as_tensor(Wb, device=dev))


# ---------------------------------------------------------------------------
# Solvers
# ---------------------------------------------------------------------------

def _check_parity(r, ref, horizon=50, iters_tol=None, x_tol=1e-7, iters_range=None):
    """History to 1e-9 relative over the first `horizon` iterations, X to
    x_tol relative Frobenius, iteration count within iters_tol (default 2%)
    of the oracle's, or of the range of counts the oracle itself gives under
    rounding-level perturbations of B (iters_range)."""
    k = min(horizon + 1, len(ref.hist), len(r.hist))
    h_gpu, h_ref = np.asarray(r.hist[:k]), np.asarray(ref.hist[:k])
    herr = np.max(np.abs(h_gpu - h_ref) / h_ref)
    xerr = _relerr(r.X.cpu().numpy(), ref.X)
    assert herr < 1e-9, (herr, k)
    assert xerr < x_tol, (xerr, x_tol)
    if iters_tol is None:
        iters_tol = max(1, math.floor(0.02 * ref.iters))
    lo, hi = iters_range if iters_range is not None else (ref.iters, ref.iters)
    assert lo - iters_tol <= r.iters <= hi + iters_tol, (r.iters, ref.iters, (lo, hi), iters_tol)
    assert r.status == ref.status


def _oracle_with_spread(name, A, B, X0=None, tol=1e-8, maxit=1000, runs=10):
    """The oracle's result plus how far rounding alone moves it: rerun on B
    perturbed at 1e-15 relative.  Returns (ref, horizon, iters_tol, x_tol):
    the history horizon over which the perturbed runs still agree to 1e-11
    (capped at 50), and tolerances of three times the observed spread (at
    least 2% of the count and 1e-7 in X).  The plain variants' counts scatter with
    occasional outliers far beyond a few samples' spread (e.g. 47 -> 62 at
    p = 16 on the 3D Helmholtz operator), so for them the count bound is at
    least 25%."""
    ref = O.solve_block(name, A, B, X0=X0, tol=tol, maxit=maxit)
    rng = np.random.default_rng(123)
    horizon, it_spread, x_spread = 50, 0, 0.0
    for _ in range(runs):
        Bp = B * (1 + 1e-15 * rng.standard_normal(B.shape))
        r = O.solve_block(name, A, Bp, X0=X0, tol=tol, maxit=maxit)
        k = min(51, len(r.hist), len(ref.hist))
        d = np.abs(np.array(r.hist[:k]) - np.array(ref.hist[:k])) / np.array(ref.hist[:k])
        bad = np.nonzero(d > 1e-11)[0]
        if len(bad):
            horizon = min(horizon, int(bad[0]) - 1)
        it_spread = max(it_spread, abs(r.iters - ref.iters))
        x_spread = max(x_spread, _relerr(r.X, ref.X))
    frac = 0.02 if name.endswith("_rq") else 0.25
    iters_tol = max(2, math.ceil(frac * ref.iters), 3 * it_spread)
    return ref, max(horizon, 1), iters_tol, max(1e-7, 3 * x_spread)


def _count_range(name, A, B, X0=None, tol=1e-8, maxit=2000, runs=10):
    """Iteration counts of the oracle on B and on B perturbed at 1e-15 (the
    spread rounding alone produces when the residual hovers near tol)."""
    rng = np.random.default_rng(100)
    counts = [O.solve_block(name, A, B, X0=X0, tol=tol, maxit=maxit).iters]
    for _ in range(runs):
        Bp = B * (1 + 1e-15 * (rng.standard_normal(B.shape) + 1j * rng.standard_normal(B.shape)))
        counts.append(O.solve_block(name, A, Bp, X0=X0, tol=tol, maxit=maxit).iters)
    return min(counts), max(counts)


@pytest.mark.parametrize("method,rq", VARIANTS)
def test_config1_solver_parity(pkg, cfg1, method, rq):
    A, B, Ad, Bd = cfg1
    name = ORACLE_NAME[(method, rq)]
    r = _solve(pkg, method, rq, Ad, Bd, tol=1e-8, maxit=2000)
    if rq:
        # the named parity configuration: 50 iterations, 2%, 1e-7.  Near
        # 1e-8 the residual hovers within a factor of 3 of the tolerance for
        # about ten iterations, so the crossing itself moves with rounding:
        # B perturbed at 1e-15 gives counts 234..239 (COCG) and 226..231
        # (COCR) in the oracle.  The count is held to 2% of that range.
        ref = O.solve_block(name, A, B, tol=1e-8, maxit=2000)
        _check_parity(r, ref, iters_range=_count_range(name, A, B))
        # the monitored norm is the true residual (section 2.2)
        assert r.true_relres == pytest.approx(r.hist[-1], rel=1e-3)
    else:
        ref, H, it_tol, x_tol = _oracle_with_spread(name, A, B, tol=1e-8, maxit=2000)
        _check_parity(r, ref, H, it_tol, x_tol)
    assert r.true_relres < 3e-8


@pytest.mark.parametrize("method,rq", VARIANTS)
def test_solver_repeatable(pkg, cfg1, method, rq):
    _, _, Ad, Bd = cfg1
    a = _solve(pkg, method, rq, Ad, Bd, tol=1e-8, maxit=60)
    b = _solve(pkg, method, rq, Ad, Bd, tol=1e-8, maxit=60)
    assert np.array_equal(a.hist, b.hist)
    assert torch.equal(a.X, b.X)


@pytest.mark.parametrize("method,rq", VARIANTS)
@pytest.mark.parametrize("p", [1, 3, 8])
def test_small_dense_like_parity(pkg, dev, method, rq, p):
    """Well-conditioned complex symmetric matrix stored as CSR, several p."""
    n = 300
    D = pins.well_conditioned_cs(n, 40 + p)
    rows, cols = np.nonzero(np.ones((n, n)))
    rowptr = np.arange(0, n * n + 1, n, dtype=np.int32)
    Ad = pkg.CsrOperator.from_arrays(rowptr, cols, D.reshape(-1), device=dev)
    B = W.cgauss(n, p, seed=p)
    ref, H, it_tol, x_tol = _oracle_with_spread(ORACLE_NAME[(method, rq)], D, B, tol=1e-10, maxit=500)
    r = _solve(pkg, method, rq, Ad, torch.as_tensor(B, device=dev), tol=1e-10, maxit=500)
    _check_parity(r, ref, H, it_tol, x_tol)


@pytest.mark.parametrize("method,rq", VARIANTS)
def test_x0_and_in_place(pkg, dev, method, rq):
    """A nonzero initial guess, with X aliasing X0 (in place)."""
    n, p = 300, 3
    D = pins.well_conditioned_cs(n, 77)
    rowptr = np.arange(0, n * n + 1, n, dtype=np.int32)
    cols = np.tile(np.arange(n), n)
    Ad = pkg.CsrOperator.from_arrays(rowptr, cols, D.reshape(-1), device=dev)
    B = W.cgauss(n, p, seed=78)
    X0 = 0.3 * W.cgauss(n, p, seed=79)
    name = ORACLE_NAME[(method, rq)]
    ref, H, it_tol, x_tol = _oracle_with_spread(name, D, B, X0=X0, tol=1e-10, maxit=500)
    X = torch.as_tensor(X0, device=dev).clone()
    r = _solve(pkg, method, rq, Ad, torch.as_tensor(B, device=dev), X0=X, out=X, tol=1e-10, maxit=500)
    assert r.X.data_ptr() == X.data_ptr()
    _check_parity(r, ref, H, it_tol, x_tol)


@pytest.mark.parametrize("method", ["cocg", "cocr"])
def test_warm_start_config1(pkg, dev, cfg1, method):
    """Config 1 restarted from the oracle's 40th iterate (the oracle's own
    count there spreads over 242..252 for COCG under 1e-15 perturbations)."""
    A, B, Ad, Bd = cfg1
    name = method + "_rq"
    X0 = O.solve_block(name, A, B, tol=1e-30, maxit=40).X
    ref = O.solve_block(name, A, B, X0=X0, tol=1e-8, maxit=2000)
    r = _solve(pkg, method, True, Ad, Bd, X0=torch.as_tensor(X0, device=dev), tol=1e-8, maxit=2000)
    _check_parity(r, ref, 50, iters_range=_count_range(name, A, B, X0=X0))


@pytest.mark.parametrize("method,rq", VARIANTS)
def test_status_paths(pkg, dev, cfg1, method, rq):
    A, B, Ad, Bd = cfg1
    # maxit
    r = _solve(pkg, method, rq, Ad, Bd, tol=1e-8, maxit=3)
    assert r.status == pkg.BLK_MAXIT and r.iters == 3 and len(r.hist) == 4
    ref = O.solve_block(ORACLE_NAME[(method, rq)], A, B, tol=1e-8, maxit=3)
    assert np.allclose(r.hist, ref.hist, rtol=1e-12)
    # zero right-hand side
    r = _solve(pkg, method, rq, Ad, torch.zeros_like(Bd), tol=1e-8, maxit=10)
    assert r.status == pkg.BLK_CONVERGED and r.iters == 0 and torch.count_nonzero(r.X) == 0
    # maxit = 0
    r = _solve(pkg, method, rq, Ad, Bd, tol=1e-8, maxit=0)
    assert r.status == pkg.BLK_MAXIT and r.iters == 0
    # duplicate columns: rank-deficient block
    B2 = B.copy()
    B2[:, 3] = B2[:, 1]
    r = _solve(pkg, method, rq, Ad, torch.as_tensor(B2, device=dev), tol=1e-8, maxit=50)
    ref = O.solve_block(ORACLE_NAME[(method, rq)], A, B2, tol=1e-8, maxit=50)
    assert r.status == pkg.BLK_BREAKDOWN == ref.status
    assert r.iters == ref.iters


def test_einval(pkg, dev, cfg1):
    A, B, Ad, Bd = cfg1
    with pytest.raises(ValueError):
        pkg.blk_cocr_solve(Ad, Bd, tol=0.0)
    with pytest.raises(ValueError):
        pkg.blk_cocr_solve(Ad, Bd, maxit=-1)
    big = torch.zeros((A.n, 33), dtype=torch.complex128, device=dev)
    with pytest.raises(ValueError):
        pkg.blk_cocr_solve(Ad, big)
    with pytest.raises(ValueError):
        pkg.blk_cocr_solve(Ad, Bd, out=Bd)  # X aliases B


# ---------------------------------------------------------------------------
# Dense operator and mixed precision
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def greens_small(pkg, dev):
    n, p = 1024, 4
    k = 2 * math.pi * 1.5
    A = W.greens_sphere(n, k)
    B = W.plane_waves3d(W.fibonacci_sphere(n), k, p)
    return A, B, pkg.DenseOperator(torch.as_tensor(A, device=dev)), torch.as_tensor(B, device=dev)


def test_dense_apply_matches_oracle(pkg, greens_small):
    A, B, Ad, Bd = greens_small
    Y, G = pkg.blk_spmm_z(Ad, Bd, gram=True)
    ref = A @ B
    assert _relerr(Y.cpu().numpy(), ref) < 1e-13
    assert _relerr(G, B.T @ ref) < 1e-12


@pytest.mark.parametrize("method", ["cocg", "cocr"])
def test_dense_solver_parity(pkg, greens_small, method):
    A, B, Ad, Bd = greens_small
    ref, H, it_tol, x_tol = _oracle_with_spread(method + "_rq", A, B, tol=1e-8, maxit=1000)
    r = _solve(pkg, method, True, Ad, Bd, tol=1e-8, maxit=1000)
    _check_parity(r, ref, H, it_tol, x_tol)


@pytest.mark.parametrize("method", ["cocg", "cocr"])
def test_mixed_precision_config1(pkg, cfg1, method):
    A, B, Ad, Bd = cfg1
    ref = O.solve_block(method + "_rq", A, B, tol=1e-12, maxit=4000)
    r = _solve(pkg, method, True, Ad, Bd, tol=1e-10, maxit=4000, precision="mixed")
    assert r.status == pkg.BLK_CONVERGED, r.status_name
    assert r.true_relres <= 1e-10
    assert O.true_relres(A, B, r.X.cpu().numpy()) <= 1.01e-10
    # error against the FP64 oracle solution: both residuals are ~1e-10..1e-12
    err = _relerr(r.X.cpu().numpy(), ref.X)
    print(f"mixed {method}: iters={r.iters} trr={r.true_relres:.2e} |X-X_oracle|/|X_oracle|={err:.2e}")
    assert err < 1e-6


def test_mixed_precision_dense(pkg, greens_small):
    A, B, Ad, Bd = greens_small
    ref = O.bl_cocr_rq(A, B, tol=1e-12, maxit=2000)
    r = pkg.blk_cocr_solve(Ad, Bd, tol=1e-8, maxit=2000, precision="mixed")
    assert r.status == pkg.BLK_CONVERGED
    assert r.true_relres <= 1e-8
    assert _relerr(r.X.cpu().numpy(), ref.X) < 1e-5


WIDE_CASES = [(m, rq, p) for (m, rq) in VARIANTS for p in (12, 16, 32) if rq or p <= 16]


@pytest.mark.parametrize("method,rq,p", WIDE_CASES)
def test_wide_block_parity(pkg, dev, method, rq, p):
    """p > 8 runs the block updates and Grams on the FP64 matrix cores.

    The plain variants are run up to p = 16 only: at p = 32 their p x p forms
    go near-singular at rounding-dependent iterations (the oracle itself
    breaks down or converges depending on a 1e-15 perturbation of B), which is
    the loss of independence that residual orthonormalization removes."""
    A = W.config2_operator(12)  # 3D Helmholtz, n = 1728, k h = 0.25
    B = W.cgauss(A.n, p, seed=p)
    Ad = pkg.CsrOperator.from_arrays(A.rowptr, A.colind, A.val, device=dev)
    # 1e-9 is crossed on the steep part of the convergence curve; near 1e-10
    # the p = 32 histories plateau at the attainable accuracy, where the
    # crossing iteration is set by rounding.
    ref, H, it_tol, x_tol = _oracle_with_spread(ORACLE_NAME[(method, rq)], A, B, tol=1e-9, maxit=400)
    r = _solve(pkg, method, rq, Ad, torch.as_tensor(B, device=dev), tol=1e-9, maxit=400)
    _check_parity(r, ref, H, it_tol, x_tol)


@pytest.mark.parametrize("p", [16, 24, 32])
def test_wide_block_kernels(pkg, dev, p):
    """Gram and thin QR at tile-ragged n for the matrix-core kernels."""
    n = 1000 + 7
    Y = W.cgauss(n, p, seed=1)
    Z = W.cgauss(n, p, seed=2)
    Yd, Zd = torch.as_tensor(Y, device=dev), torch.as_tensor(Z, device=dev)
    assert _relerr(pkg.blk_gram_z(Yd, Zd, conj=False), Y.T @ Z) < 1e-13
    assert _relerr(pkg.blk_gram_z(Yd, Zd, conj=True), Y.conj().T @ Z) < 1e-13
    Q, R = pkg.blk_thin_qr_z(Yd)
    Qr, Rr = O.thin_qr_pos(Y)
    assert _relerr(R, Rr) < 1e-12
    assert _relerr(Q.cpu().numpy(), Qr) < 1e-12


@pytest.mark.parametrize("method", ["cocg", "cocr"])
def test_refine_restarts(pkg, cfg1, method):
    """refine > 0 restarts from X only while the true residual lags the
    monitored one; the restarted run continues the first run's history."""
    A, B, Ad, Bd = cfg1
    base = _solve(pkg, method, True, Ad, Bd, tol=1e-8, maxit=2000)
    same = _solve(pkg, method, True, Ad, Bd, tol=1e-8, maxit=2000, refine=2)
    assert base.true_relres <= 1e-8
    assert same.iters == base.iters and np.array_equal(same.hist, base.hist)
    assert torch.equal(same.X, base.X)
    # a tolerance near the attainable accuracy
    tol = 1e-13
    t0 = _solve(pkg, method, True, Ad, Bd, tol=tol, maxit=3000)
    t2 = _solve(pkg, method, True, Ad, Bd, tol=tol, maxit=3000, refine=2)
    print(f"{method}: refine=0 iters={t0.iters} {t0.status_name} trr={t0.true_relres:.2e}; "
          f"refine=2 iters={t2.iters} {t2.status_name} trr={t2.true_relres:.2e}")
    assert t2.iters >= t0.iters
    assert np.array_equal(t2.hist[: t0.iters + 1], t0.hist)
    if t0.status == pkg.BLK_CONVERGED and t0.true_relres > tol:
        assert t2.iters > t0.iters
        assert t2.true_relres < t0.true_relres
    # the reported true residual is the residual of the returned X; forming
    # B - A X in FP64 is itself accurate to about eps |A| |X| / |B|
    trr = O.true_relres(A, B, t2.X.cpu().numpy())
    assert abs(trr - t2.true_relres) <= 1e-6 * trr + 1e-14


# ---------------------------------------------------------------------------
# Grid-stencil operators: pattern analysis and the 2.5D blocked product
# ---------------------------------------------------------------------------

# Small grids walk one plane per unit (few x-y tiles: many z chunks fill the
# CUs); 64 x 64 x 47 walks multi-plane chunks with a shorter last one (12,
# 6 and 3 planes at p = 32, 16 and 8 on a 256-CU device).
GRID_SHAPES = [(13, 11, 9), (8, 4, 70), (37, 29, 1), (16, 16, 33), (64, 64, 47)]


@pytest.mark.parametrize("dims", GRID_SHAPES)
def test_grid_analyze_detects(pkg, dev, dims):
    A = W.grid_stencil_random(*dims, seed=3)
    Ad = pkg.CsrOperator.from_arrays(A.rowptr, A.colind, A.val, device=dev).analyze()
    assert Ad.structure == pkg._capi.BLK_STRUCT_GRID
    assert Ad.grid == dims


def test_grid_analyze_rejects(pkg, dev):
    A = W.grid_stencil_random(9, 7, 5, seed=4)
    # one row with a missing entry
    r = 100
    k0, k1 = A.rowptr[r], A.rowptr[r + 1]
    colind = np.delete(A.colind, k0 + 1)
    val = np.delete(A.val, k0 + 1)
    rowptr = A.rowptr.copy()
    rowptr[r + 1:] -= 1
    Ad = pkg.CsrOperator.from_arrays(rowptr, colind, val, device=dev).analyze()
    assert Ad.structure == pkg._capi.BLK_STRUCT_GENERAL
    # one row with its columns out of order
    colind = A.colind.copy()
    colind[k0], colind[k0 + 1] = colind[k0 + 1], colind[k0]
    Ad = pkg.CsrOperator.from_arrays(A.rowptr, colind, A.val, device=dev).analyze()
    assert Ad.structure == pkg._capi.BLK_STRUCT_GENERAL
    # not a grid at all
    B = W.random_complex_symmetric(60, seed=1)
    rows, cols = np.nonzero(np.abs(B) > 0.8)
    rowptr = np.searchsorted(rows, np.arange(61)).astype(np.int32)
    Bd = pkg.CsrOperator.from_arrays(rowptr, cols.astype(np.int32), B[rows, cols], device=dev)
    assert Bd.analyze().structure == pkg._capi.BLK_STRUCT_GENERAL


@pytest.mark.parametrize("dims", GRID_SHAPES)
@pytest.mark.parametrize("p", [5, 8, 13, 16, 17, 32])
def test_grid_spmm_matches_oracle(pkg, dev, dims, p):
    """The 2.5D product against the oracle's CSR product, element by element:
    tiles and z-chunks that do not divide the grid, 2D grids, padded columns."""
    A = W.grid_stencil_random(*dims, seed=5)
    Ad = pkg.CsrOperator.from_arrays(A.rowptr, A.colind, A.val, device=dev).analyze()
    assert Ad.structure == pkg._capi.BLK_STRUCT_GRID
    Z = W.cgauss(A.n, p, seed=6)
    Cm = W.cgauss(A.n, p, seed=7)
    Zd, Cd = torch.as_tensor(Z, device=dev), torch.as_tensor(Cm, device=dev)
    ref = O.apply(O.as_operator(A), Z)
    Y = pkg.blk_spmm_z(Ad, Zd).cpu().numpy()
    assert np.max(np.abs(Y - ref)) <= 1e-13 * np.max(np.abs(ref))
    Y2, G = pkg.blk_spmm_z(Ad, Zd, gram=True)
    assert np.array_equal(Y2.cpu().numpy(), Y)
    assert _relerr(G, O.gram_t(Z, ref)) < 1e-13
    Y3 = pkg.blk_spmm_z(Ad, Zd, Cd).cpu().numpy()
    assert np.max(np.abs(Y3 - (Cm - ref))) <= 1e-13 * np.max(np.abs(ref))


def test_grid_and_general_paths_agree(pkg, dev):
    A = W.helmholtz3d(20, 5.0, 0.02)
    Z = torch.as_tensor(W.cgauss(A.n, 32, seed=8), device=dev)
    gen = pkg.CsrOperator.from_arrays(A.rowptr, A.colind, A.val, device=dev)
    gen.structure = pkg._capi.BLK_STRUCT_GENERAL
    grd = pkg.CsrOperator.from_arrays(A.rowptr, A.colind, A.val, device=dev).analyze()
    assert grd.grid == (20, 20, 20)
    a = pkg.blk_spmm_z(gen, Z).cpu().numpy()
    b = pkg.blk_spmm_z(grd, Z).cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))
    # solves: the pattern is analysed inside the call unless told not to
    B = torch.as_tensor(W.cgauss(A.n, 32, seed=9), device=dev)
    r1 = pkg.blk_cocr_solve(gen, B, tol=1e-8, maxit=500)
    r2 = pkg.blk_cocr_solve(pkg.CsrOperator.from_arrays(A.rowptr, A.colind, A.val, device=dev), B,
                            tol=1e-8, maxit=500)
    assert r1.status == r2.status == pkg.BLK_CONVERGED
    # the two products sum in different orders; the recurrences amplify that
    # (to ~1e-5 relative in the history by iteration 40 on this operator), so
    # the histories are compared early and the answers by their residuals
    k = min(20, r1.iters, r2.iters)
    assert np.max(np.abs(r1.hist[:k] - r2.hist[:k]) / r1.hist[:k]) < 1e-9
    assert max(r1.true_relres, r2.true_relres) < 1.5e-8
    assert _relerr(r2.X.cpu().numpy(), r1.X.cpu().numpy()) < 1e-5


def test_grid_multiplane_chunks_solver(pkg, dev):
    """A 64^3 grid, where the fused product-and-Gram walks chunks of 16
    planes (on a 256-CU device): block COCR_rq through it tracks the run
    through the general CSR kernel.  The two products sum in different
    orders and the recurrences amplify the difference (1e-15 at the first
    iteration, ~1e-9 by the 17th on this operator), so the history is held
    to 1e-9 over 12 iterations and the iterate after 20 by its residual."""
    A = W.helmholtz3d(64, 5.0, 0.02)
    B = torch.as_tensor(W.cgauss(A.n, 32, seed=11), device=dev)
    gen = pkg.CsrOperator.from_arrays(A.rowptr, A.colind, A.val, device=dev)
    gen.structure = pkg._capi.BLK_STRUCT_GENERAL
    grd = pkg.CsrOperator.from_arrays(A.rowptr, A.colind, A.val, device=dev).analyze()
    assert grd.grid == (64, 64, 64)
    r1 = pkg.blk_cocr_solve(gen, B, tol=1e-30, maxit=20)
    r2 = pkg.blk_cocr_solve(grd, B, tol=1e-30, maxit=20)
    assert r1.iters == r2.iters == 20
    assert np.max(np.abs(r1.hist[:13] - r2.hist[:13]) / r1.hist[:13]) < 1e-9
    assert abs(r1.true_relres - r2.true_relres) < 1e-6 * r1.true_relres
    assert _relerr(r2.X.cpu().numpy(), r1.X.cpu().numpy()) < 1e-6


def test_grid_mixed_precision(pkg, dev):
    """complex64 inner solves through the 2.5D product (p = 32)."""
    A = W.config2_operator(12)
    B = W.cgauss(A.n, 32, seed=10)
    Ad = pkg.CsrOperator.from_arrays(A.rowptr, A.colind, A.val, device=dev)
    r = pkg.blk_cocr_solve(Ad, torch.as_tensor(B, device=dev), tol=1e-9, maxit=2000,
                           precision="mixed")
    assert r.status == pkg.BLK_CONVERGED, r.status_name
    assert r.true_relres <= 1e-9
    assert O.true_relres(A, B, r.X.cpu().numpy()) <= 1.01e-9


# ---------------------------------------------------------------------------
# Dense operators at p > 16: the matrix-core product with split-K partials
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,p", [(1000, 32), (1024, 20), (77, 17)])
def test_dense_mfma_apply_matches_oracle(pkg, dev, n, p):
    """Element-wise against the oracle's product: ragged row blocks and K
    ranges (n not a multiple of 64 or 32), padded columns, C - A Z, the Gram."""
    k = 2 * math.pi * 1.5
    A = W.greens_sphere(n, k)
    Z = W.cgauss(n, p, seed=11)
    Cm = W.cgauss(n, p, seed=12)
    Ad = pkg.DenseOperator(torch.as_tensor(A, device=dev))
    Zd, Cd = torch.as_tensor(Z, device=dev), torch.as_tensor(Cm, device=dev)
    ref = O.apply(A, Z)
    Y = pkg.blk_spmm_z(Ad, Zd).cpu().numpy()
    assert np.max(np.abs(Y - ref)) <= 1e-13 * np.max(np.abs(ref))
    Y2, G = pkg.blk_spmm_z(Ad, Zd, gram=True)
    assert np.max(np.abs(Y2.cpu().numpy() - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert _relerr(G, O.gram_t(Z, ref)) < 1e-12
    Y3 = pkg.blk_spmm_z(Ad, Zd, Cd).cpu().numpy()
    assert np.max(np.abs(Y3 - (Cm - ref))) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,p", [(1000, 32), (1024, 20), (77, 17), (333, 8)])
def test_dense_c64_product_within_fp32_bound(pkg, dev, n, p):
    """The complex64 dense product (FP32 matrix cores at p > 16, the vector
    kernel below) against the oracle's FP64 product of the same complex64
    inputs.  The real (imaginary) part of an entry is a sum of 2n real
    products taken in FP32 in some order (split K, matrix-core blocks), so its
    error is at most gamma_{2n} sum_k |a_ik| |z_kj| (|ar zr| + |ai zi| <=
    |a| |z|), gamma_m = m u / (1 - m u), u = 2^-24; the modulus error is at
    most sqrt(2) times that.  The test asserts this bound, and that the
    typical error is near sqrt(n) u, far below it.  Ragged row blocks and K
    ranges (n = 77, 333, 1000), odd lda, padded columns."""
    k = 2 * math.pi * 1.5
    A = W.greens_sphere(n, k).astype(np.complex64)
    Z = W.cgauss(n, p, seed=14).astype(np.complex64)
    ref = O.apply(A.astype(np.complex128), Z.astype(np.complex128))
    # the operator's complex64 copy of these complex64-representable values is exact
    Ad = pkg.DenseOperator(torch.as_tensor(A.astype(np.complex128), device=dev))
    Y = pkg.blk_spmm_c(Ad, torch.as_tensor(Z, device=dev)).cpu().numpy()
    u = 2.0 ** -24
    m = 2 * n
    gamma = m * u / (1 - m * u)
    absprod = np.abs(A).astype(np.float64) @ np.abs(Z).astype(np.float64)
    err = np.abs(Y.astype(np.complex128) - ref)
    assert np.all(err <= math.sqrt(2) * gamma * absprod), float(np.max(err / (gamma * absprod)))
    rel = np.linalg.norm(Y.astype(np.complex128) - ref) / np.linalg.norm(ref)
    assert rel < 50 * math.sqrt(n) * u, rel


def test_dense_mfma_solver_parity(pkg, dev):
    """Block COCR_rq on a dense Green's operator at p = 32 against the oracle."""
    n, p = 1024, 32
    k = 2 * math.pi * 1.5
    A = W.greens_sphere(n, k)
    B = W.plane_waves3d(W.fibonacci_sphere(n), k, p) + 1e-3 * W.cgauss(n, p, seed=13)
    Ad = pkg.DenseOperator(torch.as_tensor(A, device=dev))
    ref, H, it_tol, x_tol = _oracle_with_spread("cocr_rq", A, B, tol=1e-8, maxit=500, runs=4)
    r = pkg.blk_cocr_solve(Ad, torch.as_tensor(B, device=dev), tol=1e-8, maxit=500)
    _check_parity(r, ref, H, it_tol, x_tol)


def test_mixed_precision_dense_p32(pkg, dev):
    """The mixed form on a dense Green's operator at p = 32, whose complex64
    inner products run on the FP32 matrix cores: it reaches the tolerance in
    the true FP64 residual (the driver falls back to FP64 when an inner run
    diverges), and its X is the oracle's within the tolerance's reach."""
    n, p = 1024, 32
    k = 2 * math.pi * 1.5
    A = W.greens_sphere(n, k)
    B = W.plane_waves3d(W.fibonacci_sphere(n), k, p) + 1e-3 * W.cgauss(n, p, seed=13)
    ref = O.bl_cocr_rq(A, B, tol=1e-12, maxit=1000)
    Ad = pkg.DenseOperator(torch.as_tensor(A, device=dev))
    r = pkg.blk_cocr_solve(Ad, torch.as_tensor(B, device=dev), tol=1e-8, maxit=1000, precision="mixed")
    assert r.status == pkg.BLK_CONVERGED, r.status_name
    assert r.true_relres <= 1e-8
    assert O.true_relres(A, B, r.X.cpu().numpy()) <= 1.01e-8
    err = _relerr(r.X.cpu().numpy(), ref.X)
    print(f"mixed dense p=32: iters={r.iters} trr={r.true_relres:.2e} |X-X_oracle|/|X_oracle|={err:.2e}")
    assert err < 1e-5
