"""Seeded synthetic operators and right-hand sides.

This module only builds inputs: complex-symmetric Helmholtz operators on
finite-difference grids, dense Green's-function operators on a sphere, and
block right-hand sides.  It holds none of the solver arithmetic, so both the
CPU oracle and the GPU path can consume the same arrays.

The paper (section 3) solves acoustic-scattering matrices and dense
radar-cross-section matrices that are not available here; the operators below
stand in for them with the same structure: complex symmetric (A = A^T,
A != A^H), sparse with a few nonzeros per row, or dense with an oscillatory
kernel.

Conventions
-----------
* Grids have N interior nodes per axis, spacing h = 1/(N+1), homogeneous
  Dirichlet boundary.  Node (ix, iy[, iz]) with 0-based indices sits at
  ((ix+1)h, (iy+1)h[, (iz+1)h]) and has row index ix + N*iy [+ N*N*iz]
  (x fastest).
* The operator is the unscaled A = -Laplacian_h - k^2 (1 + i*delta) I, where
  delta may be a scalar or a per-node array.
* CSR uses 0-based int32 row pointers and column indices, columns sorted
  ascending inside each row, complex128 values.
* Complex Gaussian blocks are (g0 + i*g1)/sqrt(2) with g drawn as
  numpy.random.default_rng(seed).standard_normal((n, p, 2)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Csr",
    "helmholtz2d",
    "helmholtz3d",
    "grid_coords2d",
    "cgauss",
    "plane_waves2d",
    "fibonacci_sphere",
    "greens_sphere",
    "plane_waves3d",
    "smooth_field2d",
    "config1",
    "config2_operator",
    "config2_rhs",
    "config3b",
    "random_complex_symmetric",
]


@dataclass
class Csr:
    """Square complex matrix in CSR form (0-based, int32 indices)."""

    n: int
    rowptr: np.ndarray  # int32[n+1]
    colind: np.ndarray  # int32[nnz]
    val: np.ndarray  # complex128[nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def todense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n), dtype=self.val.dtype)
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        d[rows, self.colind] = self.val
        return d


def _stencil_csr(dims: tuple[int, ...], h: float, k: float, delta) -> Csr:
    """Assemble -Laplacian_h - k^2(1+i delta) on a tensor grid with Dirichlet BC."""
    nd = len(dims)
    N = dims[0]
    assert all(d == N for d in dims)
    n = N**nd
    idx = np.arange(n, dtype=np.int64)
    # per-axis coordinate index of every node (x fastest)
    coord = [(idx // (N**a)) % N for a in range(nd)]
    inv_h2 = 1.0 / (h * h)
    delta_arr = np.broadcast_to(np.asarray(delta, dtype=np.float64), (n,))
    diag = 2.0 * nd * inv_h2 - (k * k) * (1.0 + 1j * delta_arr)
    # candidate neighbours in ascending column order: -z, -y, -x, self, +x, +y, +z
    offs = []
    for a in reversed(range(nd)):
        offs.append((a, -1))
    offs.append((None, 0))
    for a in range(nd):
        offs.append((a, +1))
    cols = np.empty((n, len(offs)), dtype=np.int64)
    vals = np.empty((n, len(offs)), dtype=np.complex128)
    mask = np.empty((n, len(offs)), dtype=bool)
    for c, (a, s) in enumerate(offs):
        if a is None:
            cols[:, c] = idx
            vals[:, c] = diag
            mask[:, c] = True
        else:
            stride = N**a
            cols[:, c] = idx + s * stride
            vals[:, c] = -inv_h2
            if s < 0:
                mask[:, c] = coord[a] > 0
            else:
                mask[:, c] = coord[a] < N - 1
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = cols[mask].astype(np.int32)
    val = vals[mask]
    return Csr(n=n, rowptr=rowptr.astype(np.int32), colind=colind, val=val)


def grid_stencil_random(nx: int, ny: int, nz: int, seed: int) -> Csr:
    """The 7-point pattern (5-point when nz == 1) of a lexicographic
    nx x ny x nz grid (x fastest, columns ascending in each row) with complex
    Gaussian entries (seed): an input for pattern and product tests."""
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    sxy = nx * ny
    cand = [(z > 0, -sxy), (y > 0, -nx), (x > 0, -1), (np.ones(n, bool), 0),
            (x < nx - 1, 1), (y < ny - 1, nx), (z < nz - 1, sxy)]
    mask = np.stack([m for m, _ in cand], axis=1)
    cols = np.stack([idx + o for _, o in cand], axis=1)
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(counts)
    colind = cols[mask].astype(np.int32)
    g = np.random.default_rng(seed).standard_normal((len(colind), 2))
    val = (g[:, 0] + 1j * g[:, 1]) / math.sqrt(2.0)
    return Csr(n, rowptr, colind, val)


def helmholtz2d(N: int, k: float, delta) -> Csr:
    """5-point -Laplacian_h - k^2(1+i delta) I on an N x N interior grid."""
    return _stencil_csr((N, N), 1.0 / (N + 1), k, delta)


def helmholtz3d(N: int, k: float, delta) -> Csr:
    """7-point -Laplacian_h - k^2(1+i delta) I on an N^3 interior grid."""
    return _stencil_csr((N, N, N), 1.0 / (N + 1), k, delta)


def grid_coords2d(N: int) -> tuple[np.ndarray, np.ndarray]:
    """(x, y) coordinates of the N*N interior nodes in row order."""
    h = 1.0 / (N + 1)
    idx = np.arange(N * N)
    return (idx % N + 1) * h, (idx // N + 1) * h


def cgauss(n: int, p: int, seed: int) -> np.ndarray:
    """Unit-variance complex Gaussian block (n, p), complex128, C-contiguous."""
    g = np.random.default_rng(seed).standard_normal((n, p, 2))
    return np.ascontiguousarray((g[..., 0] + 1j * g[..., 1]) / math.sqrt(2.0))


def plane_waves2d(N: int, k: float, p: int) -> np.ndarray:
    """Columns exp(i k (x cos t_j + y sin t_j)) with t_j = 2 pi j / p."""
    x, y = grid_coords2d(N)
    th = 2.0 * math.pi * np.arange(p) / p
    phase = k * (np.outer(x, np.cos(th)) + np.outer(y, np.sin(th)))
    return np.ascontiguousarray(np.exp(1j * phase))


def fibonacci_sphere(n: int) -> np.ndarray:
    """n points of the Fibonacci lattice on the unit sphere, float64 (n, 3).

    z_i = 1 - (2i+1)/n, azimuth i * pi * (3 - sqrt 5).
    """
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def greens_sphere(n: int, k: float, diag: complex = 1.0 + 0.5j, row_block: int = 1024) -> np.ndarray:
    """Dense Helmholtz Green's matrix exp(i k r_ij)/(4 pi r_ij), A_ii = diag.

    Points are the Fibonacci lattice on the unit sphere.  Row-major complex128.
    """
    pts = fibonacci_sphere(n)
    A = np.empty((n, n), dtype=np.complex128)
    for r0 in range(0, n, row_block):
        r1 = min(n, r0 + row_block)
        d = pts[r0:r1, None, :] - pts[None, :, :]
        r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
        rows = np.arange(r0, r1)
        r[rows - r0, rows] = 1.0  # placeholder, overwritten below
        blk = np.exp(1j * k * r) / (4.0 * math.pi * r)
        blk[rows - r0, rows] = diag
        A[r0:r1] = blk
    return A


def plane_waves3d(points: np.ndarray, k: float, p: int) -> np.ndarray:
    """Columns exp(i k d_j . x) for p Fibonacci directions d_j."""
    dirs = fibonacci_sphere(p)
    return np.ascontiguousarray(np.exp(1j * k * (points @ dirs.T)))


def smooth_field2d(N: int, lo: float, hi: float, seed: int, modes: int = 6) -> np.ndarray:
    """Smooth random field on the N x N grid mapped into [lo, hi] (row order)."""
    rng = np.random.default_rng(seed)
    x, y = grid_coords2d(N)
    f = np.zeros(N * N)
    for a in range(1, modes + 1):
        for b in range(1, modes + 1):
            c = rng.standard_normal() / (a * a + b * b)
            f += c * np.sin(a * math.pi * x) * np.sin(b * math.pi * y)
    f = (f - f.min()) / max(f.max() - f.min(), 1e-300)
    return lo + (hi - lo) * f


def random_complex_symmetric(n: int, seed: int, shift: complex = 0.0, scale: float = 1.0) -> np.ndarray:
    """Dense random complex symmetric matrix (A = A^T), complex128.

    M = scale * (G + G^T)/2 + shift * I with G a complex Gaussian matrix.
    """
    g = np.random.default_rng(seed).standard_normal((n, n, 2))
    G = (g[..., 0] + 1j * g[..., 1]) / math.sqrt(2.0)
    return np.ascontiguousarray(scale * 0.5 * (G + G.T) + shift * np.eye(n))


# ---------------------------------------------------------------------------
# The workloads the measurements and parity tests use.
# ---------------------------------------------------------------------------

def config1():
    """2D Helmholtz, 64x64 interior grid (n=4096), k=20, 5% damping; p=4.

    Right-hand sides are plane waves at angles 2 pi j/4 plus 1e-3 complex
    Gaussian noise (seed 0).  Returns (Csr, B).
    """
    N, k, delta, p = 64, 20.0, 0.05, 4
    A = helmholtz2d(N, k, delta)
    B = plane_waves2d(N, k, p) + 1e-3 * cgauss(N * N, p, seed=0)
    return A, np.ascontiguousarray(B)


def config2_operator(N: int = 128) -> Csr:
    """3D Helmholtz, N^3 interior grid, k h = 0.25, 2% damping."""
    h = 1.0 / (N + 1)
    return helmholtz3d(N, 0.25 / h, 0.02)


def config2_rhs(n: int, p: int) -> np.ndarray:
    """Complex Gaussian right-hand sides (seed 1)."""
    return cgauss(n, p, seed=1)


def config3b(n: int = 16384, p: int = 32, k: float = 2.0 * math.pi * 8.0):
    """Dense Green's-function operator on a Fibonacci sphere, plane-wave RHS."""
    A = greens_sphere(n, k)
    B = plane_waves3d(fibonacci_sphere(n), k, p)
    return A, B
