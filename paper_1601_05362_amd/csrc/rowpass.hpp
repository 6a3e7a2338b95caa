// Row-pass kernels: every n x p block update of one iteration, each fused
// with the p x p bilinear forms that the next p x p step needs.
//
// Layout: blocks are row-major n x p (leading dimension ld >= p), complex
// values interleaved.  A block of NT = 256 threads works on tiles of
// RPB = NT/PP rows; thread t owns column c = t % PP of tile row t / PP, so a
// row's p values are read and written by PP consecutive lanes (coalesced
// 16-byte accesses for complex128).  PP is the power of two >= p; lanes with
// c >= p hold zeros.
//
// Gram partials: each block accumulates its rows' contribution to a p x p
// form in registers and writes it to part[block * E + off]; a fixed-order
// second stage sums the blocks (no atomics, so results are bitwise
// repeatable).
#pragma once

#include "common.hpp"

namespace blk {

// Contiguous range of row tiles owned by this block.  Blocks are dealt to
// the eight XCDs round-robin, so logical block numbers are remapped to give
// each XCD one contiguous slab of rows (neighbour rows of a stencil then hit
// the same L2).
__device__ inline void tile_range(int64_t ntiles, int64_t& t0, int64_t& t1, bool remap = true) {
  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int lb = (remap && (G & 7) == 0) ? (b & 7) * (G >> 3) + (b >> 3) : b;
  const int64_t per = (ntiles + G - 1) / G;
  t0 = (int64_t)lb * per;
  t1 = t0 + per < ntiles ? t0 + per : ntiles;
}

// Deterministic block sum of one double per thread; result valid in thread 0.
__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) s += sh[w];
  return s;
}

// Per-block accumulator of G = Y^T Z (CONJ = false) or Y^H Z (CONJ = true)
// over rows staged in LDS tiles ys/zs of RPB x PP entries.  Accumulates in A.
// PP >= 16: thread t owns entries t, t + NT, ... and sums every row of a
// tile.  PP < 16 (fewer entries than threads): the tile's rows are split into
// NG = NT / PP^2 groups of PP rows, thread t owns entry t % PP^2 of group
// t / PP^2, and store() adds the groups in group order.
template <typename T, typename A, int PP, bool CONJ>
struct GramAcc {
  static constexpr int RPB = NT / PP;
  static constexpr int NE = (PP * PP + NT - 1) / NT;
  static constexpr int NG = PP * PP >= NT ? 1 : NT / (PP * PP);
  static_assert(NG == 1 || RPB == NG * PP, "row groups tile the rows");
  cx<A> acc[NE];

  __device__ void zero() {
#pragma unroll
    for (int q = 0; q < NE; ++q) acc[q] = czero<A>();
  }
  __device__ void add(const cx<T>* ys, const cx<T>* zs) {
    if constexpr (NG > 1) {
      const int e = threadIdx.x % (PP * PP), r0 = (threadIdx.x / (PP * PP)) * PP;
      const int i = e / PP, j = e % PP;
#pragma unroll
      for (int r = r0; r < r0 + PP; ++r) {
        const cx<A> a = ccast<A>(ys[r * PP + i]);
        const cx<A> b = ccast<A>(zs[r * PP + j]);
        if (CONJ)
          cfma_conj(acc[0], a, b);
        else
          cfma(acc[0], a, b);
      }
    } else {
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = threadIdx.x + q * NT;
        if (e < PP * PP) {
          const int i = e / PP, j = e % PP;
#pragma unroll
          for (int r = 0; r < RPB; ++r) {
            const cx<A> a = ccast<A>(ys[r * PP + i]);
            const cx<A> b = ccast<A>(zs[r * PP + j]);
            if (CONJ)
              cfma_conj(acc[q], a, b);
            else
              cfma(acc[q], a, b);
          }
        }
      }
    }
  }
  // Write the p x p block partial (row-major, ld p) as doubles at dst.
  // Every thread must call it.
  __device__ void store(double* dst, int p) const {
    if constexpr (NG > 1) {
      __shared__ cx<A> gs[NT];
      gs[threadIdx.x] = acc[0];
      __syncthreads();
      const int e = threadIdx.x;
      if (e < PP * PP) {
        cx<A> v = gs[e];
        for (int g = 1; g < NG; ++g) {
          v.re += gs[g * PP * PP + e].re;
          v.im += gs[g * PP * PP + e].im;
        }
        const int i = e / PP, j = e % PP;
        if (i < p && j < p) {
          dst[2 * (i * p + j)] = (double)v.re;
          dst[2 * (i * p + j) + 1] = (double)v.im;
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = threadIdx.x + q * NT;
        if (e < PP * PP) {
          const int i = e / PP, j = e % PP;
          if (i < p && j < p) {
            dst[2 * (i * p + j)] = (double)acc[q].re;
            dst[2 * (i * p + j) + 1] = (double)acc[q].im;
          }
        }
      }
    }
  }
};

// Stage a p x p FP64 coefficient (row-major, ld p) into LDS as PP x PP of T.
template <typename T, int PP>
__device__ inline void load_coef(cx<T>* cs, const z64* C, int p) {
  for (int e = threadIdx.x; e < PP * PP; e += NT) {
    const int k = e / PP, j = e % PP;
    cs[e] = (k < p && j < p) ? ccast<T>(C[k * p + j]) : czero<T>();
  }
}

// sum_k row[k] * cs[k][c] over the padded width (padding holds zeros).
template <typename T, int PP>
__device__ inline cx<T> rowmul(const cx<T>* row, const cx<T>* cs, int c, cx<T> acc) {
#pragma unroll
  for (int k = 0; k < PP; ++k) cfma(acc, row[k], cs[k * PP + c]);
  return acc;
}
template <typename T, int PP>
__device__ inline cx<T> rowmul_sub(const cx<T>* row, const cx<T>* cs, int c, cx<T> acc) {
#pragma unroll
  for (int k = 0; k < PP; ++k) cfms(acc, row[k], cs[k * PP + c]);
  return acc;
}

enum : int { G_NONE = 0, G_CONJ = 1, G_UNCONJ = 2 };

// Out = Ain - Bin * C (the residual-type update W = Q - U alpha', or
// R = R - Z alpha), plus the Gram of Out (GM = G_CONJ: Out^H Out for the
// first Cholesky-QR pass; G_UNCONJ: Out^T Out) and ||Out||_F^2 (NORM) into
// part[E-1].  Out may alias Ain.
template <typename T, typename A, int PP, int GM, bool NORM>
__global__ __launch_bounds__(NT) void k_axpy(int64_t n, int p, const cx<T>* Ain, int lda,
                                             const cx<T>* __restrict__ Bin, int ldb, const z64* C,
                                             cx<T>* Out, int ldo, double* part, int E,
                                             const DevState* st, int gate) {
  if (gate >= st->stop_iter) return;
  constexpr int RPB = NT / PP;
  __shared__ cx<T> cs[PP * PP];
  __shared__ cx<T> bs[2 * NT];
  __shared__ cx<T> os[GM != G_NONE ? 2 * NT : 1];
  __shared__ double sh[NT / 64];
  load_coef<T, PP>(cs, C, p);
  GramAcc<T, A, PP, GM == G_CONJ> g;
  g.zero();
  double nrm = 0.0;
  const int lr = threadIdx.x / PP, c = threadIdx.x % PP;
  const bool cok = c < p;
  int64_t t0, t1;
  tile_range((n + RPB - 1) / RPB, t0, t1);
  // two tiles per step: twice the loads in flight per barrier
  for (int64_t t = t0; t < t1; t += 2) {
    const int64_t row0 = t * RPB + lr, row1 = row0 + RPB;
    const bool ok0 = cok && row0 < n, ok1 = cok && t + 1 < t1 && row1 < n;
    cx<T> a0 = ok0 ? Ain[row0 * lda + c] : czero<T>();
    cx<T> a1 = ok1 ? Ain[row1 * lda + c] : czero<T>();
    const cx<T> b0 = ok0 ? Bin[row0 * ldb + c] : czero<T>();
    const cx<T> b1 = ok1 ? Bin[row1 * ldb + c] : czero<T>();
    __syncthreads();
    bs[threadIdx.x] = b0;
    bs[NT + threadIdx.x] = b1;
    __syncthreads();
    a0 = rowmul_sub<T, PP>(&bs[lr * PP], cs, c, a0);
    a1 = rowmul_sub<T, PP>(&bs[NT + lr * PP], cs, c, a1);
    if (ok0)
      st_nt(&Out[row0 * ldo + c], a0);
    else
      a0 = czero<T>();
    if (ok1)
      st_nt(&Out[row1 * ldo + c], a1);
    else
      a1 = czero<T>();
    if (NORM) {
      nrm += (double)cabs2(a0);
      nrm += (double)cabs2(a1);
    }
    if (GM != G_NONE) {
      os[threadIdx.x] = a0;
      os[NT + threadIdx.x] = a1;
      __syncthreads();
      g.add(os, os);
      g.add(os + NT, os + NT);
    }
  }
  double* dst = part + (size_t)blockIdx.x * E;
  if (GM != G_NONE) g.store(dst, p);
  if (NORM) {
    const double s = block_sum(nrm, sh);
    if (threadIdx.x == 0) dst[E - 1] = s;
  }
}

// Second Cholesky-QR pass: Gram (W M)^H (W M) with M = R1^{-1}, formed row
// by row without storing W M.
template <typename T, int PP>
__global__ __launch_bounds__(NT) void k_cholqr_pass2(int64_t n, int p, const cx<T>* __restrict__ Win,
                                                     int ldw, const z64* M, double* part, int E,
                                                     const DevState* st, int gate) {
  if (gate >= st->stop_iter) return;
  constexpr int RPB = NT / PP;
  __shared__ cx<T> cs[PP * PP];
  __shared__ cx<T> ws[2 * NT];
  __shared__ cx<T> os[2 * NT];
  load_coef<T, PP>(cs, M, p);
  GramAcc<T, double, PP, true> g;
  g.zero();
  const int lr = threadIdx.x / PP, c = threadIdx.x % PP;
  const bool cok = c < p;
  int64_t t0, t1;
  tile_range((n + RPB - 1) / RPB, t0, t1);
  // two tiles per step: twice the loads in flight per barrier
  for (int64_t t = t0; t < t1; t += 2) {
    const int64_t row0 = t * RPB + lr, row1 = row0 + RPB;
    const bool ok0 = cok && row0 < n, ok1 = cok && t + 1 < t1 && row1 < n;
    const cx<T> w0 = ok0 ? Win[row0 * ldw + c] : czero<T>();
    const cx<T> w1 = ok1 ? Win[row1 * ldw + c] : czero<T>();
    __syncthreads();
    ws[threadIdx.x] = w0;
    ws[NT + threadIdx.x] = w1;
    __syncthreads();
    cx<T> y0 = rowmul<T, PP>(&ws[lr * PP], cs, c, czero<T>());
    cx<T> y1 = rowmul<T, PP>(&ws[NT + lr * PP], cs, c, czero<T>());
    if (!ok0) y0 = czero<T>();
    if (!ok1) y1 = czero<T>();
    os[threadIdx.x] = y0;
    os[NT + threadIdx.x] = y1;
    __syncthreads();
    g.add(os, os);
    g.add(os + NT, os + NT);
  }
  g.store(part + (size_t)blockIdx.x * E, p);
}

// Third Cholesky-QR pass: Q = W M with M = tau^{-1}; optionally the
// unconjugated Q^T Q (block COCG with residual orthonormalization needs it).
// Q may alias W.
template <typename T, typename A, int PP, bool GRAM>
__global__ __launch_bounds__(NT) void k_cholqr_pass3(int64_t n, int p, const cx<T>* Win, int ldw,
                                                     const z64* M, cx<T>* Q, int ldq, double* part,
                                                     int E, const DevState* st, int gate) {
  if (gate >= st->stop_iter) return;
  constexpr int RPB = NT / PP;
  __shared__ cx<T> cs[PP * PP];
  __shared__ cx<T> ws[NT];
  __shared__ cx<T> os[GRAM ? NT : 1];
  load_coef<T, PP>(cs, M, p);
  GramAcc<T, A, PP, false> g;
  g.zero();
  const int lr = threadIdx.x / PP, c = threadIdx.x % PP;
  const bool cok = c < p;
  int64_t t0, t1;
  tile_range((n + RPB - 1) / RPB, t0, t1);
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t row = t * RPB + lr;
    const bool ok = cok && row < n;
    const cx<T> w = ok ? Win[row * ldw + c] : czero<T>();
    __syncthreads();
    ws[threadIdx.x] = w;
    __syncthreads();
    cx<T> q = rowmul<T, PP>(&ws[lr * PP], cs, c, czero<T>());
    if (ok)
      st_nt(&Q[row * ldq + c], q);
    else
      q = czero<T>();
    if (GRAM) {
      os[threadIdx.x] = q;
      __syncthreads();
      g.add(os, os);
    }
  }
  if (GRAM) g.store(part + (size_t)blockIdx.x * E, p);
}

// Fused block update at the end of an iteration:
//   X += S C1;  S = Q + S C2;  and with WITH_U:  U = V + U C2, plus U^T U.
// (rq variants: C1 = alpha' xi, C2 = beta'; plain variants: P in place of S,
// R in place of Q, C1 = alpha, C2 = beta.)
template <typename T, typename A, int PP, bool WITH_U>
__global__ __launch_bounds__(NT) void k_update(int64_t n, int p, cx<T>* X, int ldx, cx<T>* S, int lds,
                                               const cx<T>* __restrict__ Q, int ldq, cx<T>* U, int ldu,
                                               const cx<T>* __restrict__ V, int ldv, const z64* C1,
                                               const z64* C2, double* part, int E,
                                               const DevState* st, int gate) {
  if (gate >= st->stop_iter) return;
  constexpr int RPB = NT / PP;
  __shared__ cx<T> cs1[PP * PP];
  __shared__ cx<T> cs2[PP * PP];
  __shared__ cx<T> ss[NT];
  __shared__ cx<T> us[WITH_U ? NT : 1];
  __shared__ cx<T> os[WITH_U ? NT : 1];
  load_coef<T, PP>(cs1, C1, p);
  load_coef<T, PP>(cs2, C2, p);
  GramAcc<T, A, PP, false> g;
  g.zero();
  const int lr = threadIdx.x / PP, c = threadIdx.x % PP;
  const bool cok = c < p;
  int64_t t0, t1;
  tile_range((n + RPB - 1) / RPB, t0, t1);
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t row = t * RPB + lr;
    const bool ok = cok && row < n;
    const cx<T> s = ok ? S[row * lds + c] : czero<T>();
    cx<T> x = ok ? X[row * ldx + c] : czero<T>();
    cx<T> q = ok ? Q[row * ldq + c] : czero<T>();
    cx<T> u = czero<T>(), v = czero<T>();
    if (WITH_U) {
      u = ok ? U[row * ldu + c] : czero<T>();
      v = ok ? V[row * ldv + c] : czero<T>();
    }
    __syncthreads();
    ss[threadIdx.x] = s;
    if (WITH_U) us[threadIdx.x] = u;
    __syncthreads();
    x = rowmul<T, PP>(&ss[lr * PP], cs1, c, x);
    q = rowmul<T, PP>(&ss[lr * PP], cs2, c, q);
    if (WITH_U) v = rowmul<T, PP>(&us[lr * PP], cs2, c, v);
    if (ok) {
      st_nt(&X[row * ldx + c], x);
      st_nt(&S[row * lds + c], q);
      if (WITH_U) st_nt(&U[row * ldu + c], v);
    } else {
      v = czero<T>();
    }
    if (WITH_U) {
      os[threadIdx.x] = v;
      __syncthreads();
      g.add(os, os);
    }
  }
  if (WITH_U) g.store(part + (size_t)blockIdx.x * E, p);
}

// Gram of two blocks: G = Y^T Z (GM = G_UNCONJ) or Y^H Z (G_CONJ), or none;
// NORM adds ||Y||_F^2 at part[E-1].
template <typename T, typename A, int PP, int GM, bool NORM>
__global__ __launch_bounds__(NT) void k_gram(int64_t n, int p, const cx<T>* __restrict__ Y, int ldy,
                                             const cx<T>* __restrict__ Z, int ldz, double* part,
                                             int E, const DevState* st, int gate) {
  if (st && gate >= st->stop_iter) return;
  constexpr int RPB = NT / PP;
  __shared__ cx<T> ys[GM != G_NONE ? NT : 1];
  __shared__ cx<T> zs[GM != G_NONE ? NT : 1];
  __shared__ double sh[NT / 64];
  GramAcc<T, A, PP, GM == G_CONJ> g;
  g.zero();
  double nrm = 0.0;
  const int lr = threadIdx.x / PP, c = threadIdx.x % PP;
  const bool cok = c < p;
  int64_t t0, t1;
  tile_range((n + RPB - 1) / RPB, t0, t1);
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t row = t * RPB + lr;
    const bool ok = cok && row < n;
    const cx<T> y = ok ? Y[row * ldy + c] : czero<T>();
    if (NORM) nrm += (double)cabs2(y);
    if (GM != G_NONE) {
      const cx<T> z = ok ? Z[row * ldz + c] : czero<T>();
      __syncthreads();
      ys[threadIdx.x] = y;
      zs[threadIdx.x] = z;
      __syncthreads();
      g.add(ys, zs);
    }
  }
  double* dst = part + (size_t)blockIdx.x * E;
  if (GM != G_NONE) g.store(dst, p);
  if (NORM) {
    const double s = block_sum(nrm, sh);
    if (threadIdx.x == 0) dst[E - 1] = s;
  }
}

// Fixed-order first reduction stage: red[s][e] = sum of part[g][e] over the
// s-th of S contiguous ranges of the G block partials.
__global__ __launch_bounds__(NT) void k_reduce(const double* __restrict__ part, int G, int E,
                                               double* __restrict__ red, int S, const DevState* st,
                                               int gate) {
  if (st && gate >= st->stop_iter) return;
  const int e = blockIdx.x * NT + threadIdx.x;
  const int s = blockIdx.y;
  if (e >= E) return;
  const int g0 = (int)((int64_t)G * s / S), g1 = (int)((int64_t)G * (s + 1) / S);
  double acc = 0.0;
  int g = g0;
  for (; g + 8 <= g1; g += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(g + u) * E + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; g < g1; ++g) acc += part[(size_t)g * E + e];
  red[(size_t)s * E + e] = acc;
}

// Y = X (with leading dimensions), optionally converting precision.
template <typename TD, typename TS>
__global__ __launch_bounds__(NT) void k_copy(int64_t n, int p, const cx<TS>* __restrict__ Xs, int ldx,
                                             cx<TD>* __restrict__ Yd, int ldy, double scale,
                                             const DevState* st, int gate) {
  if (st && gate >= st->stop_iter) return;
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= n * p) return;
  const int64_t r = e / p;
  const int c = (int)(e % p);
  const cx<TS> v = Xs[r * ldx + c];
  Yd[r * ldy + c] = cx<TD>{(TD)((double)v.re * scale), (TD)((double)v.im * scale)};
}

// Y = 0.
template <typename T>
__global__ __launch_bounds__(NT) void k_zero(int64_t n, int p, cx<T>* Y, int ldy) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= n * p) return;
  Y[(e / p) * ldy + (e % p)] = czero<T>();
}

// X += scale * D with X complex128 and D of type TS (iterative refinement).
template <typename TS>
__global__ __launch_bounds__(NT) void k_axpy_up(int64_t n, int p, z64* X, int ldx,
                                                const cx<TS>* __restrict__ D, int ldd, double scale) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= n * p) return;
  const int64_t r = e / p;
  const int c = (int)(e % p);
  const cx<TS> d = D[r * ldd + c];
  z64 x = X[r * ldx + c];
  x.re = fma(scale, (double)d.re, x.re);
  x.im = fma(scale, (double)d.im, x.im);
  X[r * ldx + c] = x;
}

}  // namespace blk
