// Row-pass kernels for p in (8, 32] on the FP64 matrix cores (complex128).
//
// A wave owns 16-row tiles.  Block products Y = Z C (C p x p) run as
// v_mfma_f64_16x16x4f64 on the real and imaginary planes:
//   Yr += Zr Cr + Zi (-Ci),   Yi += Zr Ci + Zi Cr.
// Operand layouts of the instruction (lane l of a wave64):
//   A (16 x 4):  A[l % 16][l / 16]
//   B (4 x 16):  B[l / 16][l % 16]
//   D (16 x 16): register v of lane l holds D[4 v + l / 16][l % 16]
// So Z enters row-gathered ("A layout": row r0 + l%16, column 4 s + l/16 for
// k-step s), while the addends and results of an update live in the D
// layout (row r0 + 4 v + l/16, column 16 jb + l%16), which is also exactly
// the operand layout a Gram Y^T Y needs when the reduction index is the row:
// for each v the 4 rows {4v + l/16} form one k-step.  The Grams of the
// freshly updated block are therefore formed from registers, with no extra
// memory traffic.  Coefficients sit in LDS as two real planes (Re, Im).
#pragma once

#include "common.hpp"
#include "rowpass.hpp"

namespace blk {

typedef double d4 __attribute__((ext_vector_type(4)));

#ifndef MF_WAVES
#define MF_WAVES 2
#endif


__device__ inline d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int JB>
struct MfCoef {
  static constexpr int PP = 16 * JB;
  static constexpr int LD = PP + 1;  // padded row
  double re[PP * LD];
  double im[PP * LD];
};

// Load the p x p FP64 coefficient (row-major, ld p) into LDS planes, scaled
// by `sign` (+1 or -1), zero-padded to PP x PP.
template <int JB>
__device__ inline void mf_load_coef(MfCoef<JB>* C, const z64* src, int p, double sign) {
  constexpr int PP = 16 * JB, LD = PP + 1;
  for (int e = threadIdx.x; e < PP * PP; e += NT) {
    const int k = e / PP, j = e % PP;
    z64 v = (k < p && j < p) ? src[k * p + j] : czero<double>();
    C->re[k * LD + j] = sign * v.re;
    C->im[k * LD + j] = sign * v.im;
  }
}

// Hide a coefficient pointer from loop-invariant code motion: re-reading
// the B operands from LDS per tile keeps them out of registers (hoisted
// operands would cost ~100 VGPRs per coefficient and halve occupancy).
template <typename P>
__device__ inline P* mf_opaque(P* ptr) {
  asm volatile("" : "+v"(ptr));
  return ptr;
}

// A layout: ar[s], ai[s] = Z[r0 + l%16][4 s + l/16].
template <int JB>
__device__ inline void mf_load_A(const z64* __restrict__ Z, int ld, int64_t r0, int64_t n, int p,
                                 double (&ar)[4 * JB], double (&ai)[4 * JB]) {
  const int l = threadIdx.x & 63;
  const int64_t row = r0 + (l & 15);
#pragma unroll
  for (int s = 0; s < 4 * JB; ++s) {
    const int col = 4 * s + (l >> 4);
    z64 v = (row < n && col < p) ? Z[row * ld + col] : czero<double>();
    ar[s] = v.re;
    ai[s] = v.im;
  }
}

// D layout: xr[jb][v], xi[jb][v] = X[r0 + 4 v + l/16][16 jb + l%16].
template <int JB>
__device__ inline void mf_load_D(const z64* X, int ld, int64_t r0, int64_t n, int p, d4 (&xr)[JB],
                                 d4 (&xi)[JB]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int jb = 0; jb < JB; ++jb) {
    const int col = 16 * jb + (l & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 4 * v + (l >> 4);
      // streaming load: each D-layout instruction reads whole lines that no
      // other load of the pass touches (A-layout reads of a row share lines
      // between consecutive k-steps and stay cached)
      z64 x = czero<double>();
      if (row < n && col < p) {
        x.re = __builtin_nontemporal_load(&X[row * ld + col].re);
        x.im = __builtin_nontemporal_load(&X[row * ld + col].im);
      }
      xr[jb][v] = x.re;
      xi[jb][v] = x.im;
    }
  }
}

template <int JB>
__device__ inline void mf_zero_D(d4 (&xr)[JB], d4 (&xi)[JB]) {
#pragma unroll
  for (int jb = 0; jb < JB; ++jb) {
    xr[jb] = d4{0.0, 0.0, 0.0, 0.0};
    xi[jb] = d4{0.0, 0.0, 0.0, 0.0};
  }
}

// acc += d elementwise (D layout).
template <int JB>
__device__ inline void mf_add_D(d4 (&ar)[JB], d4 (&ai)[JB], const d4 (&dr)[JB], const d4 (&di)[JB]) {
#pragma unroll
  for (int jb = 0; jb < JB; ++jb) {
    ar[jb] += dr[jb];
    ai[jb] += di[jb];
  }
}

template <int JB>
__device__ inline void mf_store_D(z64* X, int ld, int64_t r0, int64_t n, int p, const d4 (&xr)[JB],
                                  const d4 (&xi)[JB]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int jb = 0; jb < JB; ++jb) {
    const int col = 16 * jb + (l & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 4 * v + (l >> 4);
      if (row < n && col < p) st_nt(&X[row * ld + col], z64{xr[jb][v], xi[jb][v]});
    }
  }
}

// acc += Z C with Z in the A layout and C in LDS:
//   Re += Zr Cr + Zi (-Ci),  Im += Zr Ci + Zi Cr.
// (Three-product complex forms ran no faster here: these passes are bound by
// memory and latency more than by the matrix cores.)
// UPPER: C is upper triangular, so the k-steps below a column block vanish.
template <int JB, bool UPPER>
__device__ inline void mf_mma(d4 (&cr)[JB], d4 (&ci)[JB], const double (&ar)[4 * JB],
                              const double (&ai)[4 * JB], const MfCoef<JB>* C) {
  constexpr int LD = 16 * JB + 1;
  const int l = threadIdx.x & 63;
  const int kr = l >> 4, jc = l & 15;
#pragma unroll
  for (int jb = 0; jb < JB; ++jb) {
#pragma unroll
    for (int s = 0; s < 4 * JB; ++s) {
      if (UPPER && 4 * s > 16 * jb + 15) continue;
      const int k = 4 * s + kr, j = 16 * jb + jc;
      const double br = C->re[k * LD + j], bi = C->im[k * LD + j];
      cr[jb] = mfma64(ar[s], br, cr[jb]);
      cr[jb] = mfma64(ai[s], -bi, cr[jb]);
      ci[jb] = mfma64(ar[s], bi, ci[jb]);
      ci[jb] = mfma64(ai[s], br, ci[jb]);
    }
  }
}

// Gram accumulation from D-layout values: blocks (ib <= jb) of G = Y^T Y
// (CONJ = false) or Y^H Y (CONJ = true).  Block index b(ib, jb) enumerates
// the upper block triangle row by row.
template <int JB>
struct MfGram {
  static constexpr int NB = JB * (JB + 1) / 2;
  d4 gr[NB], gi[NB];
  __device__ void zero() {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      gr[b] = d4{0.0, 0.0, 0.0, 0.0};
      gi[b] = d4{0.0, 0.0, 0.0, 0.0};
    }
  }
  template <bool CONJ>
  __device__ void add(const d4 (&yr)[JB], const d4 (&yi)[JB]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int b = 0;
#pragma unroll
      for (int ib = 0; ib < JB; ++ib) {
        const double ar = yr[ib][v], ai = yi[ib][v], nai = -ai;
#pragma unroll
        for (int jb = ib; jb < JB; ++jb, ++b) {
          const double br = yr[jb][v], bi = yi[jb][v];
          gr[b] = mfma64(ar, br, gr[b]);
          gr[b] = mfma64(CONJ ? ai : nai, bi, gr[b]);
          gi[b] = mfma64(ar, bi, gi[b]);
          gi[b] = mfma64(CONJ ? nai : ai, br, gi[b]);
        }
      }
    }
  }
  // Sum the block's waves in fixed order (wave 0, 1, ...) and write the
  // p x p partial (row-major, ld p) to dst; the lower block triangle is the
  // transpose (CONJ: conjugate transpose) of the upper one.  scratch holds
  // NB * 2 * 256 doubles and may alias LDS the kernel no longer reads.
  // Must be called by every thread.
  template <bool CONJ>
  __device__ void store(double* dst, int p, double* scratch) const {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int NW = NT / 64;
    for (int ww = 0; ww < NW; ++ww) {
      __syncthreads();
      if (w == ww) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double* r = &scratch[((b * 2 + 0) * 4 + v) * 64 + l];
            double* i = &scratch[((b * 2 + 1) * 4 + v) * 64 + l];
            *r = (ww == 0) ? gr[b][v] : *r + gr[b][v];
            *i = (ww == 0) ? gi[b][v] : *i + gi[b][v];
          }
      }
    }
    __syncthreads();
    for (int item = threadIdx.x; item < NB * 4 * 64; item += NT) {
      const int b = item / 256, v = (item / 64) % 4, ll = item % 64;
      const double re = scratch[((b * 2 + 0) * 4 + v) * 64 + ll];
      const double im = scratch[((b * 2 + 1) * 4 + v) * 64 + ll];
      int ib = 0, jb = 0, bb = b;
      for (ib = 0; ib < JB; ++ib) {
        if (bb < JB - ib) {
          jb = ib + bb;
          break;
        }
        bb -= JB - ib;
      }
      const int i = 16 * ib + 4 * v + ll / 16, j = 16 * jb + ll % 16;
      if (i < p && j < p) {
        dst[2 * (i * p + j)] = re;
        dst[2 * (i * p + j) + 1] = im;
        if (ib != jb) {
          dst[2 * (j * p + i)] = re;
          dst[2 * (j * p + i) + 1] = CONJ ? -im : im;
        }
      }
    }
  }
};

template <int JB>
__device__ inline double mf_norm2(const d4 (&xr)[JB], const d4 (&xi)[JB]) {
  double s = 0.0;
#pragma unroll
  for (int jb = 0; jb < JB; ++jb)
#pragma unroll
    for (int v = 0; v < 4; ++v) s += xr[jb][v] * xr[jb][v] + xi[jb][v] * xi[jb][v];
  return s;
}

// Tiles of 16 rows owned by this block; its waves take them in turn.
__device__ inline void mf_tiles(int64_t n, int64_t& t0, int64_t& t1) {
  tile_range((n + 15) / 16, t0, t1);
}

// LDS of a kernel: coefficient planes, later reused as the Gram scratch.
template <int JB>
constexpr int mf_coef_doubles() {
  return 2 * (16 * JB) * (16 * JB + 1);
}
template <int JB>
constexpr int mf_scratch_doubles() {
  return (JB * (JB + 1) / 2) * 2 * 256;
}
template <int JB, int NCOEF>
constexpr int mf_smem_doubles() {
  return NCOEF * mf_coef_doubles<JB>() > mf_scratch_doubles<JB>() ? NCOEF * mf_coef_doubles<JB>()
                                                                   : mf_scratch_doubles<JB>();
}

// Out = Ain + sign Bin C, Gram of Out (GM), ||Out||^2 (NORM).  Out may alias
// Ain or Bin (each wave reads its whole tile before writing it).
template <int JB, int GM, bool NORM>
__global__ __launch_bounds__(NT, MF_WAVES) void k_axpy_mf(int64_t n, int p, const z64* Ain, int lda,
                                                const z64* Bin, int ldb, const z64* C, double sign,
                                                z64* Out, int ldo, double* part, int E,
                                                const DevState* st, int gate) {
  if (gate >= st->stop_iter) return;
  __shared__ double smem[mf_smem_doubles<JB, 1>()];
  __shared__ double sh[NT / 64];
  MfCoef<JB>& cf = *reinterpret_cast<MfCoef<JB>*>(smem);
  double* scratch = smem;
  mf_load_coef<JB>(&cf, C, p, sign);
  __syncthreads();
  MfGram<JB> g;
  g.zero();
  double nrm = 0.0;
  const int w = threadIdx.x >> 6;
  int64_t t0, t1;
  mf_tiles(n, t0, t1);
  for (int64_t t = t0 + w; t < t1; t += NT / 64) {
    const int64_t r0 = t * 16;
    // all loads first; the products accumulate from zero and the addend
    // (whose loads complete under the products) joins at the end
    double ar[4 * JB], ai[4 * JB];
    d4 dr[JB], di[JB], cr[JB], ci[JB];
    mf_load_A<JB>(Bin, ldb, r0, n, p, ar, ai);
    mf_load_D<JB>(Ain, lda, r0, n, p, dr, di);
    mf_zero_D<JB>(cr, ci);
    mf_mma<JB, false>(cr, ci, ar, ai, mf_opaque(&cf));
    mf_add_D<JB>(cr, ci, dr, di);
    mf_store_D<JB>(Out, ldo, r0, n, p, cr, ci);
    if (GM == G_CONJ) g.template add<true>(cr, ci);
    if (GM == G_UNCONJ) g.template add<false>(cr, ci);
    if (NORM) nrm += mf_norm2<JB>(cr, ci);
  }
  double* dst = part + (size_t)blockIdx.x * E;
  if (GM != G_NONE) g.template store<GM == G_CONJ>(dst, p, scratch);
  if (NORM) {
    const double s = block_sum(nrm, sh);
    if (threadIdx.x == 0) dst[E - 1] = s;
  }
}

// Second Cholesky-QR pass: Gram (W M)^H (W M), M upper triangular.
template <int JB>
__global__ __launch_bounds__(NT, MF_WAVES) void k_cholqr_pass2_mf(int64_t n, int p, const z64* __restrict__ Win,
                                                        int ldw, const z64* M, double* part, int E,
                                                        const DevState* st, int gate) {
  if (gate >= st->stop_iter) return;
  __shared__ double smem[mf_smem_doubles<JB, 1>()];
  MfCoef<JB>& cf = *reinterpret_cast<MfCoef<JB>*>(smem);
  double* scratch = smem;
  mf_load_coef<JB>(&cf, M, p, 1.0);
  __syncthreads();
  MfGram<JB> g;
  g.zero();
  const int w = threadIdx.x >> 6;
  int64_t t0, t1;
  mf_tiles(n, t0, t1);
  for (int64_t t = t0 + w; t < t1; t += NT / 64) {
    const int64_t r0 = t * 16;
    double ar[4 * JB], ai[4 * JB];
    d4 cr[JB], ci[JB];
    mf_load_A<JB>(Win, ldw, r0, n, p, ar, ai);
    mf_zero_D<JB>(cr, ci);
    mf_mma<JB, true>(cr, ci, ar, ai, mf_opaque(&cf));
    g.template add<true>(cr, ci);
  }
  g.template store<true>(part + (size_t)blockIdx.x * E, p, scratch);
}

// Third Cholesky-QR pass: Q = W M (M upper triangular), optional Q^T Q.
template <int JB, bool GRAM>
__global__ __launch_bounds__(NT, MF_WAVES) void k_cholqr_pass3_mf(int64_t n, int p, const z64* Win, int ldw,
                                                        const z64* M, z64* Q, int ldq, double* part,
                                                        int E, const DevState* st, int gate) {
  if (gate >= st->stop_iter) return;
  __shared__ double smem[mf_smem_doubles<JB, 1>()];
  MfCoef<JB>& cf = *reinterpret_cast<MfCoef<JB>*>(smem);
  double* scratch = smem;
  mf_load_coef<JB>(&cf, M, p, 1.0);
  __syncthreads();
  MfGram<JB> g;
  g.zero();
  const int w = threadIdx.x >> 6;
  int64_t t0, t1;
  mf_tiles(n, t0, t1);
  for (int64_t t = t0 + w; t < t1; t += NT / 64) {
    const int64_t r0 = t * 16;
    double ar[4 * JB], ai[4 * JB];
    d4 cr[JB], ci[JB];
    mf_load_A<JB>(Win, ldw, r0, n, p, ar, ai);
    mf_zero_D<JB>(cr, ci);
    mf_mma<JB, true>(cr, ci, ar, ai, mf_opaque(&cf));
    mf_store_D<JB>(Q, ldq, r0, n, p, cr, ci);
    if (GRAM) g.template add<false>(cr, ci);
  }
  if (GRAM) g.template store<false>(part + (size_t)blockIdx.x * E, p, scratch);
}

// X += S C1;  S = Q + S C2.
template <int JB>
__global__ __launch_bounds__(NT, MF_WAVES) void k_update_mf(int64_t n, int p, z64* X, int ldx, z64* S,
                                                         int lds, const z64* __restrict__ Q, int ldq,
                                                         const z64* C1, const z64* C2,
                                                         const DevState* st, int gate) {
  if (gate >= st->stop_iter) return;
  __shared__ double smem[mf_smem_doubles<JB, 2>()];
  MfCoef<JB>& cf1 = *reinterpret_cast<MfCoef<JB>*>(smem);
  MfCoef<JB>& cf2 = *reinterpret_cast<MfCoef<JB>*>(smem + mf_coef_doubles<JB>());
  mf_load_coef<JB>(&cf1, C1, p, 1.0);
  mf_load_coef<JB>(&cf2, C2, p, 1.0);
  __syncthreads();
  const int w = threadIdx.x >> 6;
  int64_t t0, t1;
  mf_tiles(n, t0, t1);
  for (int64_t t = t0 + w; t < t1; t += NT / 64) {
    const int64_t r0 = t * 16;
    // all loads first; the products accumulate from zero and the addends,
    // whose loads complete under the products, join last
    double sr[4 * JB], si[4 * JB];
    d4 xr[JB], xi[JB], qr[JB], qi[JB], ar[JB], ai[JB], br[JB], bi[JB];
    mf_load_A<JB>(S, lds, r0, n, p, sr, si);
    mf_load_D<JB>(X, ldx, r0, n, p, xr, xi);
    mf_load_D<JB>(Q, ldq, r0, n, p, qr, qi);
    mf_zero_D<JB>(ar, ai);
    mf_zero_D<JB>(br, bi);
    mf_mma<JB, false>(ar, ai, sr, si, mf_opaque(&cf1));
    mf_mma<JB, false>(br, bi, sr, si, mf_opaque(&cf2));
    mf_add_D<JB>(ar, ai, xr, xi);
    mf_add_D<JB>(br, bi, qr, qi);
    mf_store_D<JB>(X, ldx, r0, n, p, ar, ai);
    mf_store_D<JB>(S, lds, r0, n, p, br, bi);
  }
}

// Gram of two blocks G = Y^T Z (GM = G_UNCONJ) or Y^H Z (G_CONJ) from D-layout
// loads, plus ||Y||^2 (NORM).  General (non-symmetric) form: all JB x JB blocks.
template <int JB, int GM, bool NORM>
__global__ __launch_bounds__(NT, MF_WAVES) void k_gram_mf(int64_t n, int p, const z64* __restrict__ Y, int ldy,
                                                const z64* __restrict__ Z, int ldz, double* part, int E,
                                                const DevState* st, int gate) {
  if (st && gate >= st->stop_iter) return;
  __shared__ double scratch[JB * JB * 2 * 256];
  __shared__ double sh[NT / 64];
  d4 gr[JB * JB], gi[JB * JB];
#pragma unroll
  for (int b = 0; b < JB * JB; ++b) {
    gr[b] = d4{0.0, 0.0, 0.0, 0.0};
    gi[b] = d4{0.0, 0.0, 0.0, 0.0};
  }
  double nrm = 0.0;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t t0, t1;
  mf_tiles(n, t0, t1);
  for (int64_t t = t0 + w; t < t1; t += NT / 64) {
    const int64_t r0 = t * 16;
    d4 yr[JB], yi[JB], zr[JB], zi[JB];
    mf_load_D<JB>(Y, ldy, r0, n, p, yr, yi);
    if (NORM) nrm += mf_norm2<JB>(yr, yi);
    if (GM != G_NONE) {
      mf_load_D<JB>(Z, ldz, r0, n, p, zr, zi);
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int ib = 0; ib < JB; ++ib)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb) {
            const int b = ib * JB + jb;
            const double ar = yr[ib][v], ai = yi[ib][v];
            gr[b] = mfma64(ar, zr[jb][v], gr[b]);
            gr[b] = mfma64(GM == G_CONJ ? ai : -ai, zi[jb][v], gr[b]);
            gi[b] = mfma64(ar, zi[jb][v], gi[b]);
            gi[b] = mfma64(GM == G_CONJ ? -ai : ai, zr[jb][v], gi[b]);
          }
    }
  }
  double* dst = part + (size_t)blockIdx.x * E;
  if (GM != G_NONE) {
    constexpr int NW = NT / 64;
    for (int ww = 0; ww < NW; ++ww) {
      __syncthreads();
      if (w == ww) {
#pragma unroll
        for (int b = 0; b < JB * JB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double* r = &scratch[((b * 2 + 0) * 4 + v) * 64 + l];
            double* i = &scratch[((b * 2 + 1) * 4 + v) * 64 + l];
            *r = (ww == 0) ? gr[b][v] : *r + gr[b][v];
            *i = (ww == 0) ? gi[b][v] : *i + gi[b][v];
          }
      }
    }
    __syncthreads();
    for (int item = threadIdx.x; item < JB * JB * 256; item += NT) {
      const int b = item / 256, v = (item / 64) % 4, ll = item % 64;
      const double re = scratch[((b * 2 + 0) * 4 + v) * 64 + ll];
      const double im = scratch[((b * 2 + 1) * 4 + v) * 64 + ll];
      const int ib = b / JB, jb = b % JB;
      const int i = 16 * ib + 4 * v + ll / 16, j = 16 * jb + ll % 16;
      if (i < p && j < p) {
        dst[2 * (i * p + j)] = re;
        dst[2 * (i * p + j) + 1] = im;
      }
    }
  }
  if (NORM) {
    const double s = block_sum(nrm, sh);
    if (threadIdx.x == 0) dst[E - 1] = s;
  }
}

}  // namespace blk
