// Operator application Y = A Z for a complex symmetric CSR matrix and an
// n x p block with interleaved complex columns (the one block product per
// iteration of section 2.1).
//
// Each row of A is read once for all p columns: the PP lanes that own a row
// (one lane per column) walk the row's nonzeros together, every lane reading
// the same (colind, val) entry and its own column of the neighbour row of Z.
// Accumulation is in the storage precision (FP64 for complex128, FP32 for
// complex64).  Optional fused epilogues: Y = C - A Z (initial / true residual), the
// unconjugated Gram Z^T Y (the Z row of Y's own index is the diagonal
// neighbour), and ||Y||_F^2.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "rowpass.hpp"
#include "rowpass_mfma.hpp"

namespace blk {

// Gram Z^T Y of a 16-row x 32-column group staged in LDS (row-major,
// ld 32), on the FP64 matrix cores: wave w accumulates the 16 x 16 block
// (w / 2, w % 2) over four 4-row k-steps.
__device__ inline void spmm_gram16(const z64* zs, const z64* ys, d4& gr, d4& gi) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ib = w >> 1, jb = w & 1;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int r = 4 * s + (l >> 4);
    const z64 a = zs[r * 32 + 16 * ib + (l & 15)];
    const z64 b = ys[r * 32 + 16 * jb + (l & 15)];
    gr = mfma64(a.re, b.re, gr);
    gr = mfma64(-a.im, b.im, gr);
    gi = mfma64(a.re, b.im, gi);
    gi = mfma64(a.im, b.re, gi);
  }
}

template <typename T, int PP, bool SUB, bool STORE, bool GRAM, bool NORM>
__global__ __launch_bounds__(NT) void k_spmm(int64_t n, const int32_t* __restrict__ rowptr,
                                             const int32_t* __restrict__ colind,
                                             const cx<T>* __restrict__ val,
                                             const cx<T>* __restrict__ Z, int ldz,
                                             const cx<T>* __restrict__ Cm, int ldc,
                                             cx<T>* __restrict__ Y, int ldy, int p, double* part,
                                             int E, const DevState* st, int gate, int remap) {
  if (st && gate >= st->stop_iter) return;
  constexpr int RPB = NT / PP;
  // complex128 at p <= 32: the Gram runs on the matrix cores over 16-row groups
  constexpr bool MFG = GRAM && std::is_same<T, double>::value && PP == 32;
  __shared__ cx<T> zs[GRAM ? (MFG ? 2 * NT : NT) : 1];
  __shared__ cx<T> ys[GRAM ? (MFG ? 2 * NT : NT) : 1];
  __shared__ double sh[NT / 64];
  GramAcc<T, double, PP, false> g;
  if (GRAM && !MFG) g.zero();
  d4 mgr = d4{0.0, 0.0, 0.0, 0.0}, mgi = d4{0.0, 0.0, 0.0, 0.0};
  int half = 0;
  double nrm = 0.0;
  const int lr = threadIdx.x / PP, c = threadIdx.x % PP;
  const bool cok = c < p;
  int64_t t0, t1;
  tile_range((n + RPB - 1) / RPB, t0, t1, remap != 0);
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t row = t * RPB + lr;
    cx<T> y = czero<T>();
    cx<T> zr = czero<T>();
    if (row < n) {
      const int k0 = rowptr[row], k1 = rowptr[row + 1];
      cx<T> acc = czero<T>();
      // Entries in batches of 8: all index/value loads of a batch are issued
      // together, then all gathers of Z, so each lane keeps up to 8
      // independent loads in flight instead of one dependent chain per entry.
      for (int kb = k0; kb < k1; kb += 8) {
        int jj[8];
        cx<T> a[8], z[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const bool ok = kb + u < k1;
          jj[u] = ok ? colind[kb + u] : 0;
          a[u] = ok ? val[kb + u] : czero<T>();
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) z[u] = (cok && kb + u < k1) ? Z[(int64_t)jj[u] * ldz + c] : czero<T>();
#pragma unroll
        for (int u = 0; u < 8; ++u) cfma(acc, a[u], z[u]);
      }
      if (SUB) {
        y = cok ? Cm[row * ldc + c] : czero<T>();
        y = csub(y, acc);
      } else {
        y = acc;
      }
      if (!cok) y = czero<T>();
      if (STORE && cok) st_nt(&Y[row * ldy + c], y);
      if (GRAM && cok) zr = Z[row * ldz + c];
    }
    if (NORM) nrm += (double)cabs2(y);
    if constexpr (MFG) {
      // rows of this tile fill half of the 16-row group (half is block-uniform)
      zs[half * NT + threadIdx.x] = zr;
      ys[half * NT + threadIdx.x] = y;
      half ^= 1;
      if (half == 0) {
        __syncthreads();
        spmm_gram16(reinterpret_cast<const z64*>(zs), reinterpret_cast<const z64*>(ys), mgr, mgi);
        __syncthreads();
      }
    } else if (GRAM) {
      __syncthreads();
      zs[threadIdx.x] = zr;
      ys[threadIdx.x] = y;
      __syncthreads();
      g.add(zs, ys);
    }
  }
  if constexpr (MFG) {
    if (half == 1) {  // an odd tile count: the group's second half is zero
      zs[NT + threadIdx.x] = czero<T>();
      ys[NT + threadIdx.x] = czero<T>();
      __syncthreads();
      spmm_gram16(reinterpret_cast<const z64*>(zs), reinterpret_cast<const z64*>(ys), mgr, mgi);
    }
  }
  if (GRAM || NORM) {
    double* dst = part + (size_t)blockIdx.x * E;
    if constexpr (MFG) {
      // D layout: register v of lane l holds G[16 ib + 4 v + l / 16][16 jb + l % 16]
      const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
      const int j = 16 * (w & 1) + (l & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * (w >> 1) + 4 * v + (l >> 4);
        if (i < p && j < p) {
          dst[2 * (i * p + j)] = mgr[v];
          dst[2 * (i * p + j) + 1] = mgi[v];
        }
      }
    } else if (GRAM) {
      g.store(dst, p);
    }
    if (NORM) {
      const double s = block_sum(nrm, sh);
      if (threadIdx.x == 0) dst[E - 1] = s;
    }
  }
}

// Dense operator: Y = A Z (or C - A Z) with A row-major n x n (leading
// dimension lda).  A tile of RPB rows x 32 columns of A is staged in LDS so
// each row of A is read once, coalesced, for all p columns.
template <typename T, int PP, bool SUB, bool STORE, bool GRAM, bool NORM>
__global__ __launch_bounds__(NT) void k_dense(int64_t n, const cx<T>* __restrict__ Am, int64_t lda,
                                              const cx<T>* __restrict__ Z, int ldz,
                                              const cx<T>* __restrict__ Cm, int ldc,
                                              cx<T>* __restrict__ Y, int ldy, int p, double* part,
                                              int E, const DevState* st, int gate) {
  if (st && gate >= st->stop_iter) return;
  constexpr int RPB = NT / PP;
  constexpr int KC = 32;  // columns of A per stage
  __shared__ cx<T> as[RPB * KC];
  __shared__ cx<T> zt[KC * PP];
  __shared__ cx<T> zs[GRAM ? NT : 1];
  __shared__ cx<T> ys[GRAM ? NT : 1];
  __shared__ double sh[NT / 64];
  GramAcc<T, double, PP, false> g;
  if (GRAM) g.zero();
  double nrm = 0.0;
  const int lr = threadIdx.x / PP, c = threadIdx.x % PP;
  const bool cok = c < p;
  int64_t t0, t1;
  tile_range((n + RPB - 1) / RPB, t0, t1);
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t row = t * RPB + lr;
    cx<T> acc = czero<T>();
    for (int64_t k0 = 0; k0 < n; k0 += KC) {
      __syncthreads();
      for (int e = threadIdx.x; e < RPB * KC; e += NT) {
        const int rr = e / KC, kk = e % KC;
        const int64_t gr = t * RPB + rr, gk = k0 + kk;
        as[e] = (gr < n && gk < n) ? Am[gr * lda + gk] : czero<T>();
      }
      for (int e = threadIdx.x; e < KC * PP; e += NT) {
        const int kk = e / PP, cc = e % PP;
        const int64_t gk = k0 + kk;
        zt[e] = (gk < n && cc < p) ? Z[gk * ldz + cc] : czero<T>();
      }
      __syncthreads();
#pragma unroll 8
      for (int kk = 0; kk < KC; ++kk) cfma(acc, as[lr * KC + kk], zt[kk * PP + c]);
    }
    cx<T> y = czero<T>(), zr = czero<T>();
    if (row < n && cok) {
      y = SUB ? csub(Cm[row * ldc + c], acc) : acc;
      if (STORE) st_nt(&Y[row * ldy + c], y);
      if (GRAM) zr = Z[row * ldz + c];
    }
    if (NORM) nrm += (double)cabs2(y);
    if (GRAM) {
      __syncthreads();
      zs[threadIdx.x] = zr;
      ys[threadIdx.x] = y;
      __syncthreads();
      g.add(zs, ys);
    }
  }
  if (GRAM || NORM) {
    double* dst = part + (size_t)blockIdx.x * E;
    if (GRAM) g.store(dst, p);
    if (NORM) {
      const double s = block_sum(nrm, sh);
      if (threadIdx.x == 0) dst[E - 1] = s;
    }
  }
}

}  // namespace blk
