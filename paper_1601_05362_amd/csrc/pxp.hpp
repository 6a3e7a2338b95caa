// p x p steps of an iteration, always in FP64 on one workgroup:
//   * the coefficient solves ("solve ... for alpha / beta" of Algorithms 1-3
//     and the block COCG recurrences) by LU with partial pivoting;
//   * the Cholesky factors of the two Cholesky-QR passes that orthonormalize
//     the residual block (section 2.2), tau = R2 R1, xi_{m+1} = tau xi_m,
//     and the monitored norm ||xi_{m+1}||_F / ||B||_F;
//   * convergence, iteration-cap and breakdown decisions (DevState).
// Each kernel first sums the fixed-order partials of the Gram it consumes.
#pragma once

#include "common.hpp"
#include "rowpass.hpp"

namespace blk {

// Coefficient slots (each SLOT complex entries, p x p row-major, ld p).
enum : int {
  S_ALPHA = 0,   // alpha' (rq) or alpha
  S_ALPHAXI,     // alpha' xi_m, the X-update coefficient of the rq variants
  S_BETA,        // beta' or beta
  S_XI,          // xi_m
  S_TAU,         // tau_{m+1}
  S_TAUINV,      // tau_{m+1}^{-1}
  S_R1,          // first Cholesky-QR factor
  S_R1INV,       // its inverse
  S_GOLD,        // the previous iteration's Gram that the next solves reuse
  S_NSLOTS
};

__device__ inline z64 cdiv(z64 a, z64 b) {
  // Smith's algorithm avoids overflow in |b|^2.
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return z64{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  } else {
    const double r = b.re / b.im, d = b.re * r + b.im;
    return z64{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
  }
}

// The p x p kernels run one workgroup of m^2 threads, m = 8, 16 or 32 the
// smallest that holds p (px_threads); thread t owns entry (i, j) =
// (t / m, t % m) of a p x p matrix (row-major, ld p), so every elimination
// step updates all of its entries at once.  Small blocks get one wave and
// barriers that cost next to nothing.
constexpr int PXT = PMAX * PMAX;  // largest workgroup
constexpr int PXW = PXT / 64;     // its waves

__host__ __device__ inline int px_threads(int p) { return p <= 4 ? 64 : (p <= 16 ? 256 : PXT); }
__device__ inline int px_m() { return blockDim.x == 64 ? 8 : (blockDim.x == 256 ? 16 : PMAX); }
__device__ inline int px_i() { return threadIdx.x / px_m(); }
__device__ inline int px_j() { return threadIdx.x % px_m(); }
__device__ inline int px_waves() { return blockDim.x / 64; }

// Sum of rows [s0, s1) of column c of a reduced Gram (ascending, loads
// issued up to 16 rows at a time).
__device__ inline z64 red_rows(const Red r, int c, int s0, int s1) {
  const double* src = r.base + r.off + 2 * c;
  double re = 0.0, im = 0.0;
  int s = s0;
  for (; s + 16 <= s1; s += 16) {
    double vr[16], vi[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      vr[u] = src[(size_t)(s + u) * r.ld];
      vi[u] = src[(size_t)(s + u) * r.ld + 1];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      re += vr[u];
      im += vi[u];
    }
  }
  for (; s < s1; ++s) {
    re += src[(size_t)s * r.ld];
    im += src[(size_t)s * r.ld + 1];
  }
  return z64{re, im};
}

// dst[p x p] = sum of the rows of a reduced Gram.  The workgroup's threads
// split each entry's rows into nseg contiguous segments (nseg = threads per
// entry); each segment is summed in ascending order and the segment sums are
// added in segment order, so the result depends only on p and the row count.
// seg is LDS scratch of blockDim.x entries that must not alias dst.  Every
// thread must call it.
__device__ inline void red_load(const Red r, z64* dst, int p, z64* seg) {
  const int E = p * p, t = threadIdx.x;
  const int nseg = max(1, min((int)blockDim.x / E, r.nrows));
  const int chunk = (r.nrows + nseg - 1) / nseg;
  const int sg = t / E, e = t % E;
  if (nseg == 1) {
    if (t < E) dst[e] = red_rows(r, e, 0, r.nrows);
    return;
  }
  if (sg < nseg) seg[sg * E + e] = red_rows(r, e, min(r.nrows, sg * chunk), min(r.nrows, (sg + 1) * chunk));
  __syncthreads();
  if (t < E) {
    z64 acc = seg[e];
    for (int k = 1; k < nseg; ++k) {
      acc.re += seg[k * E + e].re;
      acc.im += seg[k * E + e].im;
    }
    dst[e] = acc;
  }
  __syncthreads();  // seg may be reused
}

// Sum of one column of a reduced scalar, computed by a whole wave: lane l
// sums a contiguous range of rows in ascending order, then the lanes combine
// by a butterfly (every lane ends with the same value).  Every lane of the
// calling wave must call it.
__device__ inline double red_scalar(const Red r) {
  const int l = threadIdx.x & 63;
  const int chunk = (r.nrows + 63) / 64;
  const int s0 = min(r.nrows, l * chunk), s1 = min(r.nrows, s0 + chunk);
  double s = 0.0;
  for (int k = s0; k < s1; ++k) s += r.base[(size_t)k * r.ld + r.off];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  return s;
}

// C = A for p x p blocks (global or LDS).
__device__ inline void copy_pp(const z64* A, z64* C, int p) {
  const int e = threadIdx.x;
  if (e < p * p) C[e] = A[e];
}

// C = A B for p x p row-major operands in LDS (C may be global; it must not
// alias A or B).  TA: use A^T.
template <bool TA>
__device__ inline void mm(const z64* A, const z64* B, z64* C, int p) {
  const int i = px_i(), j = px_j();
  if (i >= p || j >= p) return;
  z64 acc = czero<double>();
  for (int k = 0; k < p; ++k) cfma(acc, TA ? A[k * p + i] : A[i * p + k], B[k * p + j]);
  C[i * p + j] = acc;
}

// Upper Cholesky factor in place: a = R with R^H R = G (upper triangle of a
// holds G on entry).  Fails (uniformly across the block) on a pivot <= thr.
__device__ inline bool chol_upper(z64* a, int p, double thr) {
  const int i = px_i(), j = px_j();
  for (int k = 0; k < p; ++k) {
    __syncthreads();
    const double d = a[k * p + k].re;
    if (!(d > thr)) return false;
    const double rk = sqrt(d);
    __syncthreads();
    if (i == k && j >= k && j < p)
      a[k * p + j] = (j == k) ? z64{rk, 0.0} : z64{a[k * p + j].re / rk, a[k * p + j].im / rk};
    __syncthreads();
    if (i > k && j >= i && j < p) {
      // a[i][j] -= conj(a[k][i]) * a[k][j]
      const z64 ki = a[k * p + i], kj = a[k * p + j];
      z64 v = a[i * p + j];
      v.re -= ki.re * kj.re + ki.im * kj.im;
      v.im -= ki.re * kj.im - ki.im * kj.re;
      a[i * p + j] = v;
    }
  }
  __syncthreads();
  if (i < p && j < i) a[i * p + j] = czero<double>();
  __syncthreads();
  return true;
}

// Solve U X = B in place (B -> X) for upper-triangular U, p columns,
// eliminating one row at a time from the bottom.
__device__ inline void back_subst(const z64* U, z64* B, int p) {
  const int i = px_i(), j = px_j();
  for (int k = p - 1; k >= 0; --k) {
    __syncthreads();
    if (i == k && j < p) B[k * p + j] = cdiv(B[k * p + j], U[k * p + k]);
    __syncthreads();
    if (i < k && j < p) cfms(B[i * p + j], U[i * p + k], B[k * p + j]);
  }
  __syncthreads();
}

// ri = r^{-1} for upper-triangular r.
__device__ inline void tri_inv_upper(const z64* r, z64* ri, int p) {
  const int i = px_i(), j = px_j();
  if (i < p && j < p) ri[i * p + j] = (i == j) ? z64{1.0, 0.0} : czero<double>();
  back_subst(r, ri, p);
}

// Largest |M_ij| (every thread gets the value).
__device__ inline double max_abs(const z64* M, int p, double* sh) {
  double v = threadIdx.x < p * p ? sqrt(cabs2(M[threadIdx.x])) : 0.0;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
  for (int w = 1; w < px_waves(); ++w) r = fmax(r, sh[w]);
  __syncthreads();
  return r;
}

// Sum over the block (every thread gets the value; waves in fixed order).
__device__ inline double sum_all(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < px_waves(); ++w) r += sh[w];
  __syncthreads();
  return r;
}

// Solve M C = Rh (p x p each, LDS) by LU with partial pivoting: pivot = the
// largest |re| + |im| in the column, lowest row on ties.  On success Rh holds
// C.  Fails (uniformly) on a pivot of modulus <= thr or a non-finite one.
__device__ inline bool lu_solve(z64* M, z64* Rh, int p, double thr, int* piv) {
  const int i = px_i(), j = px_j();
  for (int k = 0; k < p; ++k) {
    __syncthreads();
    if (threadIdx.x < 64) {
      double v = -1.0;
      int idx = p;
      const int r = k + threadIdx.x;
      if (r < p) {
        v = fabs(M[r * p + k].re) + fabs(M[r * p + k].im);
        idx = r;
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double v2 = __shfl_xor(v, o);
        const int i2 = __shfl_xor(idx, o);
        if (v2 > v || (v2 == v && i2 < idx)) {
          v = v2;
          idx = i2;
        }
      }
      if (threadIdx.x == 0) *piv = idx;
    }
    __syncthreads();
    const int pv = *piv;
    if (pv >= p) return false;
    if (!(sqrt(cabs2(M[pv * p + k])) > thr)) return false;
    if (pv != k && j < p) {
      // thread row 0 swaps rows k and pv of M, thread row 1 those of Rh
      if (i == 0) {
        const z64 t = M[k * p + j];
        M[k * p + j] = M[pv * p + j];
        M[pv * p + j] = t;
      } else if (i == 1) {
        const z64 t = Rh[k * p + j];
        Rh[k * p + j] = Rh[pv * p + j];
        Rh[pv * p + j] = t;
      }
    }
    __syncthreads();
    if (i > k && i < p && j < p) {
      const z64 l = cdiv(M[i * p + k], M[k * p + k]);
      if (j > k) cfms(M[i * p + j], l, M[k * p + j]);
      cfms(Rh[i * p + j], l, Rh[k * p + j]);
    }
  }
  back_subst(M, Rh, p);
  return true;
}

struct CholArgs {
  Red g;         // Hermitian Gram to factor
  int mode;      // 1: first Cholesky-QR pass, 2: second pass
  int gate;      // runs iff gate < stop_iter
  int idx;       // index m+1 of the xi being produced (0 at start-up)
  int init;      // xi_prev = I (start-up)
  z64* slots;
  double* hist;
  DevState* st;
};

// Cholesky of a Cholesky-QR Gram.  Mode 1 stores R1 and R1^{-1}.  Mode 2
// forms tau = R2 R1, tau^{-1}, xi_{m+1} = tau xi_m and records
// ||xi_{m+1}||_F / ||B||_F, then decides convergence / iteration cap.
// A failed factorization means the residual block lost rank: its norm
// ||W xi_m||_F (from the Gram) decides between converged and breakdown.
__global__ __launch_bounds__(PXT) void k_chol(CholArgs a) {
  DevState* st = a.st;
  if (a.gate >= st->stop_iter) return;
  __shared__ z64 G[SLOT];
  __shared__ z64 R[SLOT];
  __shared__ z64 Ri[SLOT];
  __shared__ z64 T1[SLOT];
  __shared__ z64 T2[SLOT];
  __shared__ double sh[PXW];
  const int p = st->p;
  z64* slots = a.slots;
  red_load(a.g, G, p, T1);
  __syncthreads();
  double dmax = 0.0;
  for (int i = 0; i < p; ++i) dmax = fmax(dmax, G[i * p + i].re);
  copy_pp(G, R, p);
  __syncthreads();
  const bool ok = (dmax > 0.0) && chol_upper(R, p, CHOL_TOL * dmax);
  if (!ok) {
    // residual estimate r^2 = ||W xi||_F^2
    __syncthreads();
    const z64* xi = slots + S_XI * SLOT;
    double r2 = 0.0;
    if (a.mode == 1) {
      // tr(xi^H G xi) = sum_ij conj(xi_ij) (G xi)_ij  (xi = I at start-up)
      for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
        const int i = e / p, j = e % p;
        if (a.init) {
          if (i == j) r2 += G[e].re;
        } else {
          z64 t = czero<double>();
          for (int k = 0; k < p; ++k) cfma(t, G[i * p + k], xi[k * p + j]);
          r2 += xi[e].re * t.re + xi[e].im * t.im;
        }
      }
    } else {
      const z64* R1 = slots + S_R1 * SLOT;
      for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
        const int i = e / p, j = e % p;
        z64 t = czero<double>();
        for (int k = 0; k < p; ++k) cfma(t, R1[i * p + k], a.init ? (k == j ? z64{1, 0} : z64{0, 0}) : xi[k * p + j]);
        r2 += cabs2(t);
      }
    }
    r2 = sum_all(r2, sh);
    if (threadIdx.x == 0) {
      const double r = sqrt(fmax(r2, 0.0)) / st->normB;
      a.hist[a.idx] = r;
      st->stop_iter = a.idx;
      st->status = (r <= st->tol) ? ST_CONVERGED : ST_BREAKDOWN;
    }
    return;
  }
  tri_inv_upper(R, Ri, p);
  if (a.mode == 1) {
    copy_pp(R, slots + S_R1 * SLOT, p);
    copy_pp(Ri, slots + S_R1INV * SLOT, p);
    return;
  }
  // stage R1, R1^{-1} and xi_m (G is free once R holds the factor)
  copy_pp(slots + S_R1 * SLOT, T1, p);
  copy_pp(slots + S_R1INV * SLOT, T2, p);
  if (!a.init) copy_pp(slots + S_XI * SLOT, G, p);
  __syncthreads();
  // tau^{-1} = R1^{-1} R2^{-1}, then tau = R2 R1 (into T2)
  mm<false>(T2, Ri, slots + S_TAUINV * SLOT, p);
  __syncthreads();
  mm<false>(R, T1, T2, p);
  __syncthreads();
  copy_pp(T2, slots + S_TAU * SLOT, p);
  // xi_{m+1} = tau xi_m (into R)
  if (a.init)
    copy_pp(T2, R, p);
  else
    mm<false>(T2, G, R, p);
  __syncthreads();
  double n2 = 0.0;
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) n2 += cabs2(R[e]);
  n2 = sum_all(n2, sh);
  copy_pp(R, slots + S_XI * SLOT, p);
  if (threadIdx.x == 0) {
    const double r = sqrt(n2) / st->normB;
    a.hist[a.idx] = r;
    if (!(r == r) || isinf(r) || r > st->div_limit) {
      st->stop_iter = a.idx;
      st->status = ST_BREAKDOWN;
    } else if (r <= st->tol) {
      st->stop_iter = a.idx;
      st->status = ST_CONVERGED;
    } else if (a.idx >= st->maxit) {
      st->stop_iter = a.idx;
      st->status = ST_MAXIT;
    }
  }
}

struct SolveArgs {
  Red mred;       // M from a reduced Gram (mred.base != nullptr) ...
  int mslot;      // ... or from this slot
  Red rred;       // right-hand side from a reduced Gram ...
  int rslot;      // ... or from this slot
  int rhs_tauT;   // right-hand side <- tau^T * (right-hand side)
  int save_slot;  // >= 0: store the raw right-hand side source here
  int out_slot;   // solution C
  int outxi_slot; // >= 0: also store C xi_m here
  Red nred;       // >= 0 rows: squared residual norm -> hist[hist_idx] + stop test
  int hist_idx;
  int gate;       // runs iff gate < stop_iter
  int fail_idx;   // on failure stop_iter = fail_idx ...
  int late;       // ... unless the solve is late and the run already stops there
  z64* slots;
  double* hist;
  DevState* st;
};

__global__ __launch_bounds__(PXT) void k_solve(SolveArgs a) {
  DevState* st = a.st;
  if (a.gate >= st->stop_iter) return;
  __shared__ z64 M[SLOT];
  __shared__ z64 Rh[SLOT];
  __shared__ z64 T[SLOT];
  __shared__ z64 X[SLOT];
  __shared__ int piv;
  __shared__ double sh[PXW];
  const int p = st->p;
  z64* slots = a.slots;
  const double nsum = (a.nred.base != nullptr) ? red_scalar(a.nred) : 0.0;
  if (a.nred.base != nullptr && threadIdx.x == 0) {
    const double r = sqrt(fmax(nsum, 0.0)) / st->normB;
    a.hist[a.hist_idx] = r;
    if (!(r == r) || isinf(r) || r > st->div_limit) {
      st->stop_iter = a.hist_idx;
      st->status = ST_BREAKDOWN;
    } else if (r <= st->tol) {
      st->stop_iter = a.hist_idx;
      st->status = ST_CONVERGED;
    } else if (a.hist_idx >= st->maxit) {
      st->stop_iter = a.hist_idx;
      st->status = ST_MAXIT;
    }
  }
  // every slot is read before save_slot (which may be mslot) is written
  if (a.mred.base != nullptr)
    red_load(a.mred, M, p, X);
  else
    copy_pp(slots + a.mslot * SLOT, M, p);
  if (a.rred.base != nullptr)
    red_load(a.rred, Rh, p, X);
  else
    copy_pp(slots + a.rslot * SLOT, Rh, p);
  if (a.rhs_tauT) copy_pp(slots + S_TAU * SLOT, T, p);
  __syncthreads();
  if (a.save_slot >= 0) copy_pp(Rh, slots + a.save_slot * SLOT, p);
  if (a.rhs_tauT) {
    mm<true>(T, Rh, X, p);
    __syncthreads();
    copy_pp(X, Rh, p);
  }
  if (a.outxi_slot >= 0) copy_pp(slots + S_XI * SLOT, T, p);
  __syncthreads();
  const double thr = PIVOT_TOL * max_abs(M, p, sh);
  const bool ok = thr > 0.0 && lu_solve(M, Rh, p, thr, &piv);
  bool finite = ok;
  if (ok) {
    double chk = 0.0;
    for (int e = threadIdx.x; e < p * p; e += blockDim.x) chk += Rh[e].re + Rh[e].im;
    chk = sum_all(chk * 0.0, sh);  // NaN/Inf anywhere propagates
    finite = (chk == 0.0);
  }
  if (!finite) {
    if (threadIdx.x == 0) {
      if (!(a.late && st->stop_iter <= a.fail_idx)) {
        st->stop_iter = a.fail_idx;
        st->status = ST_BREAKDOWN;
      }
    }
    return;
  }
  copy_pp(Rh, slots + a.out_slot * SLOT, p);
  if (a.outxi_slot >= 0) mm<false>(Rh, T, slots + a.outxi_slot * SLOT, p);
}

// Start-up: slot <- a reduced Gram (if gred is given) and, for the plain
// variants, hist[0] = sqrt(sum nred) / ||B|| with the stop test (if nred is).
__global__ __launch_bounds__(PXT) void k_start(Red nred, Red gred, int slot, z64* slots, double* hist,
                                              DevState* st) {
  __shared__ z64 seg[SLOT];
  const int p = st->p;
  if (gred.base != nullptr) red_load(gred, slots + slot * SLOT, p, seg);
  const double nsum = (nred.base != nullptr) ? red_scalar(nred) : 0.0;
  if (nred.base != nullptr && threadIdx.x == 0) {
    const double r = sqrt(fmax(nsum, 0.0)) / st->normB;
    hist[0] = r;
    if (!(r == r) || isinf(r)) {
      st->stop_iter = 0;
      st->status = ST_BREAKDOWN;
    } else if (r <= st->tol) {
      st->stop_iter = 0;
      st->status = ST_CONVERGED;
    } else if (st->maxit <= 0) {
      st->stop_iter = 0;
      st->status = ST_MAXIT;
    }
  }
}

// DevState <- running with ||B||_F = 1 (set the true norm with k_set_norm).
// Must precede every other kernel of a solve: their gates read stop_iter.
__global__ void k_state_init(DevState* st, int p, int maxit, double tol, double div_limit) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->stop_iter = 0x7fffffff;
    st->status = ST_CONVERGED;
    st->maxit = maxit;
    st->p = p;
    st->tol = tol;
    st->normB = 1.0;
    st->div_limit = div_limit;
  }
}

// normB = sqrt(sum nred).
__global__ void k_set_norm(DevState* st, Red nred) {
  const double s = red_scalar(nred);  // launched as one wave
  if (threadIdx.x == 0 && blockIdx.x == 0) st->normB = sqrt(fmax(s, 0.0));
}

}  // namespace blk
