// Shared device-side types for the block COCG / COCR kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace blk {

// Threads per block of every row-pass kernel: four wave64s.
constexpr int NT = 256;
// Largest number of right-hand sides a kernel is instantiated for.
constexpr int PMAX = 32;
// Stride (in complex entries) between p x p coefficient slots.
constexpr int SLOT = PMAX * PMAX;

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};
using z64 = cx<double>;
using c32 = cx<float>;

template <typename T>
__host__ __device__ inline cx<T> czero() {
  return cx<T>{T(0), T(0)};
}

template <typename D, typename S>
__host__ __device__ inline cx<D> ccast(cx<S> a) {
  return cx<D>{D(a.re), D(a.im)};
}

template <typename T>
__device__ inline cx<T> cadd(cx<T> a, cx<T> b) {
  return cx<T>{a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ inline cx<T> csub(cx<T> a, cx<T> b) {
  return cx<T>{a.re - b.re, a.im - b.im};
}
template <typename T>
__device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
  return cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ inline cx<T> cconj(cx<T> a) {
  return cx<T>{a.re, -a.im};
}
// acc += a * b
template <typename T>
__device__ inline void cfma(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename T>
__device__ inline void cfma_conj(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
// acc -= a * b
template <typename T>
__device__ inline void cfms(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.re = fma(-a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(-a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
// Streaming (nontemporal) store of a block entry: n x p blocks are written
// once per pass and read again only by a later launch, so they need not
// occupy L2, which then keeps the rows a pass still reads.
template <typename T>
__device__ inline void st_nt(cx<T>* dst, cx<T> v) {
  __builtin_nontemporal_store(v.re, &dst->re);
  __builtin_nontemporal_store(v.im, &dst->im);
}

// Streaming (nontemporal) load of an entry read once per pass.
template <typename T>
__device__ inline cx<T> ld_nt(const cx<T>* src) {
  return cx<T>{__builtin_nontemporal_load(&src->re), __builtin_nontemporal_load(&src->im)};
}

template <typename T>
__device__ inline T cabs2(cx<T> a) {
  return a.re * a.re + a.im * a.im;
}

// Solver status shared by every kernel of one solve.  Kernels of iteration m
// do nothing once m >= stop_iter, so work queued past convergence is inert.
struct DevState {
  int stop_iter;  // first iteration index that must not run (INT_MAX while running)
  int status;     // 0 converged / running, 1 maxit, 2 breakdown
  int maxit;
  int p;
  double normB;      // ||B||_F
  double tol;
  double div_limit;  // a monitored relative residual above this stops the run (breakdown)
};

enum : int { ST_CONVERGED = 0, ST_MAXIT = 1, ST_BREAKDOWN = 2 };

// Rank threshold of the Cholesky QR: a pivot <= CHOL_TOL * max_j G_jj fails.
constexpr double CHOL_TOL = 1e-14;
// Pivot threshold of the p x p LU: |u_kk| <= PIVOT_TOL * max |M_ij| fails.
constexpr double PIVOT_TOL = 1e-13;

// Where a reduced Gram lives: rows [0, nrows) of `base` with row stride `ld`
// doubles; entry block starts at double offset `off`.
struct Red {
  const double* base;
  int nrows;
  int ld;
  int off;
};

}  // namespace blk
