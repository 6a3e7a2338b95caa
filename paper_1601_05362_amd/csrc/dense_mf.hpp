// Dense operator application Y = A Z (the Green's-function matrices of the
// paper's second experiment) on the matrix cores, p <= 32: complex128 on the
// FP64 instruction (k_dense_mf), complex64 on the FP32 one (k_dense_mf32).
//
// A is row-major n x n.  A workgroup of four waves owns 64 rows (16 per wave)
// and one of DSPLIT contiguous ranges of the columns of A (split K); it
// streams its range in chunks of 32: the 32 x 32 chunk of Z is staged in LDS
// (shared by the four waves) and each wave loads its 16 x 32 block of A in
// the matrix-core operand layout.  Complex products as four real products:
//   Yr += Ar Zr + Ai (-Zi),  Yi += Ar Zi + Ai Zr.
// The DSPLIT partial products go to a workspace and k_dense_fin sums them in
// a fixed order (bitwise repeatable), with the optional Y = C - A Z and
// ||Y||_F^2 epilogues.
#pragma once

#include "common.hpp"
#include "rowpass.hpp"
#include "rowpass_mfma.hpp"

namespace blk {

constexpr int DSPLIT = 4;   // K ranges per 64-row block
constexpr int DKC = 32;     // K chunk staged per step
constexpr int DROWS = 64;   // rows per workgroup

__host__ __device__ inline int64_t dense_blocks(int64_t n) { return ((n + DROWS - 1) / DROWS) * DSPLIT; }

// part: DSPLIT x n x 32 complex partial products (columns >= p are zero).
__global__ __launch_bounds__(NT, 2) void k_dense_mf(int64_t n, const z64* __restrict__ A, int64_t lda,
                                                    const z64* __restrict__ Z, int ldz, int p,
                                                    z64* __restrict__ part, const DevState* st,
                                                    int gate) {
  if (st && gate >= st->stop_iter) return;
  __shared__ z64 zs[DKC * 32];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t rb = blockIdx.x / DSPLIT;
  const int sp = blockIdx.x % DSPLIT;
  const int64_t kper = ((n + DSPLIT - 1) / DSPLIT + DKC - 1) / DKC * DKC;
  const int64_t kb = sp * kper, ke = kb + kper < n ? kb + kper : n;
  const int64_t row = rb * DROWS + 16 * w + (l & 15);  // A-layout row of this lane
  const bool rok = row < n;
  d4 cr[2], ci[2];
#pragma unroll
  for (int jb = 0; jb < 2; ++jb) cr[jb] = ci[jb] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = kb; k0 < ke; k0 += DKC) {
    // stage Z[k0 : k0 + 32][0 : 32]
    __syncthreads();
#pragma unroll
    for (int u = 0; u < DKC * 32 / NT; ++u) {
      const int e = threadIdx.x + u * NT;
      const int64_t k = k0 + e / 32;
      const int col = e % 32;
      zs[e] = (k < ke && col < p) ? Z[k * ldz + col] : czero<double>();
    }
    // this wave's 16 x 32 block of A in the A layout: A[row][k0 + 4 s + l / 16]
    double ar[DKC / 4], ai[DKC / 4];
#pragma unroll
    for (int s = 0; s < DKC / 4; ++s) {
      const int64_t k = k0 + 4 * s + (l >> 4);
      const z64 a = (rok && k < ke) ? A[row * lda + k] : czero<double>();
      ar[s] = a.re;
      ai[s] = a.im;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < DKC / 4; ++s) {
      const int kk = 4 * s + (l >> 4);
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) {
        const z64 b = zs[kk * 32 + 16 * jb + (l & 15)];
        cr[jb] = mfma64(ar[s], b.re, cr[jb]);
        cr[jb] = mfma64(ai[s], -b.im, cr[jb]);
        ci[jb] = mfma64(ar[s], b.im, ci[jb]);
        ci[jb] = mfma64(ai[s], b.re, ci[jb]);
      }
    }
  }
  // D layout: register v of lane l holds rows 16 w + 4 v + l / 16, column 16 jb + l % 16
  z64* dst = part + (size_t)sp * n * 32;
#pragma unroll
  for (int jb = 0; jb < 2; ++jb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = rb * DROWS + 16 * w + 4 * v + (l >> 4);
      if (r < n) dst[r * 32 + 16 * jb + (l & 15)] = z64{cr[jb][v], ci[jb][v]};
    }
}

// The complex64 product (the inner solves of the mixed-precision form) on the
// FP32 matrix cores, v_mfma_f32_16x16x4f32 with FP32 accumulation, in the
// same tiling as k_dense_mf.  Its D layout differs from the FP64
// instruction's: register v of lane l holds row 4 (l / 16) + v.  Each lane
// loads two consecutive complex entries of A (16 bytes) per pair of k-steps,
// so the k index of step s for lane group m = l / 16 is
// 8 (s / 2) + 2 m + s % 2, and the staged Z is read with the same index.
typedef float f4 __attribute__((ext_vector_type(4)));
__device__ inline f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
struct __attribute__((aligned(8))) c32x2 {
  float r0, i0, r1, i1;
};

// part: DSPLIT x n x 32 complex64 partial products (columns >= p are zero).
__global__ __launch_bounds__(NT, 2) void k_dense_mf32(int64_t n, const c32* __restrict__ A, int64_t lda,
                                                      const c32* __restrict__ Z, int ldz, int p,
                                                      c32* __restrict__ part, const DevState* st,
                                                      int gate) {
  if (st && gate >= st->stop_iter) return;
  __shared__ c32 zs[DKC * 32];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6, m = l >> 4;
  const int64_t rb = blockIdx.x / DSPLIT;
  const int sp = blockIdx.x % DSPLIT;
  const int64_t kper = ((n + DSPLIT - 1) / DSPLIT + DKC - 1) / DKC * DKC;
  const int64_t kb = sp * kper, ke = kb + kper < n ? kb + kper : n;
  const int64_t row = rb * DROWS + 16 * w + (l & 15);  // A-layout row of this lane
  const bool rok = row < n;
  f4 cr[2], ci[2];
#pragma unroll
  for (int jb = 0; jb < 2; ++jb) cr[jb] = ci[jb] = f4{0.f, 0.f, 0.f, 0.f};
  for (int64_t k0 = kb; k0 < ke; k0 += DKC) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < DKC * 32 / NT; ++u) {
      const int e = threadIdx.x + u * NT;
      const int64_t k = k0 + e / 32;
      const int col = e % 32;
      zs[e] = (k < ke && col < p) ? Z[k * ldz + col] : czero<float>();
    }
    float ar[DKC / 4], ai[DKC / 4];
#pragma unroll
    for (int t = 0; t < DKC / 8; ++t) {
      const int64_t k = k0 + 8 * t + 2 * m;
      if (rok && k + 1 < ke) {
        const c32x2 a = *reinterpret_cast<const c32x2*>(A + row * lda + k);
        ar[2 * t] = a.r0;
        ai[2 * t] = a.i0;
        ar[2 * t + 1] = a.r1;
        ai[2 * t + 1] = a.i1;
      } else {
        const c32 a0 = (rok && k < ke) ? A[row * lda + k] : czero<float>();
        ar[2 * t] = a0.re;
        ai[2 * t] = a0.im;
        ar[2 * t + 1] = 0.f;
        ai[2 * t + 1] = 0.f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < DKC / 4; ++s) {
      const int kk = 8 * (s >> 1) + 2 * m + (s & 1);
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) {
        const c32 b = zs[kk * 32 + 16 * jb + (l & 15)];
        cr[jb] = mfma32(ar[s], b.re, cr[jb]);
        cr[jb] = mfma32(-ai[s], b.im, cr[jb]);
        ci[jb] = mfma32(ar[s], b.im, ci[jb]);
        ci[jb] = mfma32(ai[s], b.re, ci[jb]);
      }
    }
  }
  c32* dst = part + (size_t)sp * n * 32;
#pragma unroll
  for (int jb = 0; jb < 2; ++jb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = rb * DROWS + 16 * w + 4 * m + v;
      if (r < n) dst[r * 32 + 16 * jb + (l & 15)] = c32{cr[jb][v], ci[jb][v]};
    }
}

// Y = sum of the DSPLIT partials in split order (SUB: Y = C - sum), stored
// if STORE; NORM: ||Y||_F^2 partial of this block at part[blockIdx.x * E + E - 1].
template <typename T, bool SUB, bool STORE, bool NORM>
__global__ __launch_bounds__(NT) void k_dense_fin(int64_t n, int p, const cx<T>* __restrict__ ws,
                                                  const cx<T>* __restrict__ Cm, int ldc,
                                                  cx<T>* __restrict__ Y, int ldy, double* part, int E,
                                                  const DevState* st, int gate) {
  if (st && gate >= st->stop_iter) return;
  __shared__ double sh[NT / 64];
  double nrm = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n * 32; e += (int64_t)gridDim.x * NT) {
    const int64_t r = e / 32;
    const int col = (int)(e % 32);
    if (col >= p) continue;
    cx<T> y = ws[e];
#pragma unroll
    for (int sp = 1; sp < DSPLIT; ++sp) {
      const cx<T> v = ws[(size_t)sp * n * 32 + e];
      y.re += v.re;
      y.im += v.im;
    }
    if (SUB) y = csub(Cm[r * ldc + col], y);
    if (STORE) st_nt(&Y[r * ldy + col], y);
    if (NORM) nrm += (double)cabs2(y);
  }
  if (NORM) {
    const double s = block_sum(nrm, sh);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * E + E - 1] = s;
  }
}

}  // namespace blk
