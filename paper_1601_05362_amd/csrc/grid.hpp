// Operator application Y = A Z for a CSR matrix whose pattern is the
// 7-point stencil of a lexicographic nx x ny x nz grid (5-point when nz = 1):
// row r = x + nx (y + ny z) holds, in ascending column order, the existing
// ones of r - nx ny, r - nx, r - 1, r, r + 1, r + nx, r + nx ny.  The values
// are read from the CSR (any coefficients); the column indices are not
// read, since the pattern has been verified (k_grid_check).
//
// 2.5D blocking: a workgroup owns an x-y tile of a plane (8 x 4 points at
// p = 32) and walks zc consecutive planes (several tile columns per
// workgroup when the grid is bounded by the reduction partials).  The host
// picks zc so that the (tile, z chunk) units about fill the resident
// workgroup slots once: longer chunks re-read fewer boundary planes, too few
// units leave CUs idle.  Each thread row owns one grid point and PP lanes its
// columns.  The current plane plus a one-point halo sits in LDS (the +-x,
// +-y neighbours); the -z and +z neighbours stay in registers as the walk
// advances, so each Z row is fetched about once per plane instead of once
// per stored entry.  Epilogues: Y = C - A Z and ||Y||_F^2 (k_spmm_grid), and
// the Gram Z^T Y on the FP64 matrix cores (k_spmm_grid_walk, p = 32).  Y is
// written with streaming stores.
#pragma once

#include "common.hpp"
#include "rowpass_mfma.hpp"

namespace blk {

constexpr int GT = 1024;  // threads: 32 grid points x 32 columns
constexpr int GTX = 8, GTY = 4;
constexpr int GRID_WG_PER_CU = 2;  // resident 1024-thread workgroups per CU
static_assert(GTX * GTY * 32 == GT, "one thread row per tile point");

// x-y tile of the pipelined product for PP lanes per grid point: GT / PP
// points, as square as the width 2..32 points per x-run allows.
template <int PP>
struct GridTile;
template <>
struct GridTile<32> {
  static constexpr int X = 8, Y = 4;
};
template <>
struct GridTile<16> {
  static constexpr int X = 8, Y = 8;
};
template <>
struct GridTile<8> {
  static constexpr int X = 16, Y = 8;
};

template <int PP>
__host__ __device__ inline int64_t grid_tiles_pp(int nx, int ny) {
  constexpr int TX = GridTile<PP>::X, TY = GridTile<PP>::Y;
  return (int64_t)((nx + TX - 1) / TX) * ((ny + TY - 1) / TY);
}

// Units of a launch: (x-y tile, z chunk of zc planes) pairs.
template <int PP>
__host__ __device__ inline int64_t grid_units_pp(int nx, int ny, int nz, int zc) {
  return grid_tiles_pp<PP>(nx, ny) * ((nz + zc - 1) / zc);
}

// Chunk length: the fewest chunks per tile column that give every resident
// workgroup slot a unit.  At 128^3 (two slots on each of 256 CUs): 128
// planes for p = 32 (512 tiles), 64 for p = 16, 32 for p = 8.
template <int PP>
inline int grid_zchunk(int nx, int ny, int nz, int slots) {
  const int64_t tiles = grid_tiles_pp<PP>(nx, ny);
  const int64_t chunks = (slots + tiles - 1) / tiles;
  const int64_t zc = (nz + chunks - 1) / chunks;
  return (int)(zc < 1 ? 1 : zc);
}

// Verify the stencil pattern: any mismatching row stores 1 to *bad.
__global__ __launch_bounds__(NT) void k_grid_check(int64_t n, const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ colind, int nx, int ny,
                                                   int nz, int* bad) {
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (r >= n) return;
  const int64_t sxy = (int64_t)nx * ny;
  const int x = (int)(r % nx), y = (int)((r / nx) % ny), z = (int)(r / sxy);
  int64_t want[7];
  int cnt = 0;
  if (z > 0) want[cnt++] = r - sxy;
  if (y > 0) want[cnt++] = r - nx;
  if (x > 0) want[cnt++] = r - 1;
  want[cnt++] = r;
  if (x < nx - 1) want[cnt++] = r + 1;
  if (y < ny - 1) want[cnt++] = r + nx;
  if (z < nz - 1) want[cnt++] = r + sxy;
  const int k0 = rowptr[r], k1 = rowptr[r + 1];
  bool ok = (k1 - k0 == cnt);
  for (int i = 0; ok && i < cnt; ++i) ok = (colind[k0 + i] == want[i]);
  if (!ok) *bad = 1;
}

// Gram block (ib, jb) of a 16-row group staged in LDS (row-major, ld 32).
__device__ inline void grid_gram16(const z64* zs, const z64* ys, int ib, int jb, d4& gr, d4& gi) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int r = 4 * s + (l >> 4);
    const z64 a = zs[r * 32 + 16 * ib + (l & 15)];
    const z64 b = ys[r * 32 + 16 * jb + (l & 15)];
    gr = mfma64(a.re, b.re, gr);
    gr = mfma64(-a.im, b.im, gr);
    gi = mfma64(a.re, b.im, gi);
    gi = mfma64(a.im, b.re, gi);
    // one k-step's operands at a time: batching the LDS reads of all steps
    // would raise the kernel's register count and halve its occupancy
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The walk is software-pipelined one plane ahead: while plane z is computed,
// plane z+2's interior rows and row offsets, plane z+1's halo and plane z+1's
// coefficients are in flight, and loads are issued in the order they are
// consumed (the vector-memory counter retires them in order).  The
// coefficients of a plane arrive as whole x-runs: the rows of one tile line
// are consecutive, so their stored entries are contiguous in the CSR and one
// group of loader threads per line fetches them once into LDS.  PP lanes own
// a grid point's columns (PP = 8, 16, 32 with 128, 64, 32 points per tile);
// the fused Gram is left to k_spmm_grid_walk.
template <typename T, int PP, bool SUB, bool STORE, bool NORM>
__global__ __launch_bounds__(GT) __attribute__((amdgpu_waves_per_eu(8))) void k_spmm_grid(
    int nx, int ny, int nz, const int32_t* __restrict__ rowptr, const cx<T>* __restrict__ val,
    const cx<T>* __restrict__ Z, int ldz, const cx<T>* __restrict__ Cm, int ldc,
    cx<T>* __restrict__ Y, int ldy, int p, int zc, double* part, int E, const DevState* st,
    int gate) {
  if (st && gate >= st->stop_iter) return;
  constexpr int GTX = GridTile<PP>::X, GTY = GridTile<PP>::Y;
  static_assert(GTX * GTY * PP == GT, "one thread row per tile point");
  constexpr int W = GTX + 2, H = GTY + 2, NH = 2 * (GTX + GTY);
  static_assert(NH <= GTX * GTY, "one halo point per thread row");
  constexpr int PL = W * H * PP;                   // plane + halo, in cx<T>
  constexpr int RS = (GTX * 7 + 31) / 32 * 32;     // coefficient slots per x-run
  static_assert(GTY * RS <= GT, "one coefficient per loader thread");
  // two plane buffers, used alternately: one barrier per plane separates the
  // writes of a buffer from the reads of the plane before the last
  __shared__ __align__(16) cx<T> pls[2][PL];
  __shared__ __align__(16) cx<T> coefs[2][GTY * RS];
  __shared__ double sh[GT / 64];
  const int t = threadIdx.x, c = t % PP, q = t / PP, w = t >> 6;
  int it = 0;  // planes walked by this block (buffer parity)
  const bool cok = c < p;
  const int tilesx = (nx + GTX - 1) / GTX, tilesy = (ny + GTY - 1) / GTY;
  const int64_t units = grid_units_pp<PP>(nx, ny, nz, zc);
  const int sxy = nx * ny;  // rows fit int32 (n < 2^31 is checked by the caller)
  // halo point owned by thread row q (q < NH): ring of the (W x H) frame
  int hx = 0, hy = 0;
  if (q < GTX) {
    hx = q + 1;
  } else if (q < 2 * GTX) {
    hx = q - GTX + 1;
    hy = H - 1;
  } else if (q < 2 * GTX + GTY) {
    hy = q - 2 * GTX + 1;
  } else {
    hx = W - 1;
    hy = q - 2 * GTX - GTY + 1;
  }
  const int lx = q % GTX + 1, ly = q / GTX + 1;  // this point's frame position
  const int qrun = q / GTX;                     // its x-run (tile line)
  const bool loader = t < GTY * RS;             // coefficient loader: run lj, slot le
  const int lj = t / RS, le = t % RS;
  double nrm = 0.0;
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const int bx = (int)(u % tilesx), by = (int)((u / tilesx) % tilesy);
    const int bz = (int)(u / ((int64_t)tilesx * tilesy));
    const int x = bx * GTX + q % GTX, y = by * GTY + q / GTX;
    const int z0 = bz * zc, z1 = min(nz, z0 + zc);
    const bool in = x < nx && y < ny;
    const int r0 = in ? x + nx * y : 0;
    const int ors = in ? bx * GTX + nx * y : 0;  // start of this point's run
    const int ex = bx * GTX + hx - 1, ey = by * GTY + hy - 1;
    const bool hok = q < NH && ex >= 0 && ex < nx && ey >= 0 && ey < ny && cok;
    const int hr0 = hok ? ex + nx * ey : 0;
    const int runlen = min(GTX, nx - bx * GTX);
    const bool lrun = loader && by * GTY + lj < ny;
    const int lrs = lrun ? bx * GTX + nx * (by * GTY + lj) : 0;
    // prologue: plane z0 in registers, offsets of planes z0 and z0 + 1
    cx<T> prev = (in && cok && z0 > 0) ? Z[(int64_t)(r0 + sxy * (z0 - 1)) * ldz + c] : czero<T>();
    cx<T> cur = (in && cok) ? Z[(int64_t)(r0 + sxy * z0) * ldz + c] : czero<T>();
    cx<T> nxt = (in && cok && z0 + 1 < nz) ? Z[(int64_t)(r0 + sxy * (z0 + 1)) * ldz + c] : czero<T>();
    cx<T> hcur = hok ? Z[(int64_t)(hr0 + sxy * z0) * ldz + c] : czero<T>();
    int off0 = 0, lb0 = 0, lc0 = 0, off1 = 0, lb1 = 0, lc1 = 0;
    if (in) off0 = rowptr[r0 + sxy * z0] - rowptr[ors + sxy * z0];
    if (lrun) {
      lb0 = rowptr[lrs + sxy * z0];
      lc0 = rowptr[lrs + sxy * z0 + runlen] - lb0;
    }
    if (z0 + 1 < z1) {
      if (in) off1 = rowptr[r0 + sxy * (z0 + 1)] - rowptr[ors + sxy * (z0 + 1)];
      if (lrun) {
        lb1 = rowptr[lrs + sxy * (z0 + 1)];
        lc1 = rowptr[lrs + sxy * (z0 + 1) + runlen] - lb1;
      }
    }
    cx<T> cv = (lrun && le < lc0) ? ld_nt(&val[lb0 + le]) : czero<T>();
    for (int z = z0; z < z1; ++z) {
      // plane z+1's coefficients (their offsets arrived one plane ago)
      const cx<T> cvn = (lrun && z + 1 < z1 && le < lc1) ? ld_nt(&val[lb1 + le]) : czero<T>();
      // plane z+2's offsets and interior rows, plane z+1's halo
      int off2 = 0, lb2 = 0, lc2 = 0;
      if (z + 2 < z1) {
        if (in) off2 = rowptr[r0 + sxy * (z + 2)] - rowptr[ors + sxy * (z + 2)];
        if (lrun) {
          lb2 = rowptr[lrs + sxy * (z + 2)];
          lc2 = rowptr[lrs + sxy * (z + 2) + runlen] - lb2;
        }
      }
      const cx<T> nn = (in && cok && z + 2 < nz) ? Z[(int64_t)(r0 + sxy * (z + 2)) * ldz + c] : czero<T>();
      const cx<T> hn = (hok && z + 1 < z1) ? Z[(int64_t)(hr0 + sxy * (z + 1)) * ldz + c] : czero<T>();
      // plane z into LDS
      cx<T>* pl = pls[it & 1];
      cx<T>* coef = coefs[it & 1];
      ++it;
      if (q < NH) pl[(hy * W + hx) * PP + c] = hcur;
      pl[(ly * W + lx) * PP + c] = cur;
      if (loader) coef[t] = cv;
      __syncthreads();
      cx<T> yv = czero<T>();
      if (in) {
        // CSR slots of the existing neighbours, in column order
        const bool h0 = z > 0, h1 = y > 0, h2 = x > 0, h4 = x < nx - 1, h5 = y < ny - 1, h6 = z < nz - 1;
        const int s1 = h0, s2 = s1 + h1, s3 = s2 + h2, s4 = s3 + 1, s5 = s4 + h4, s6 = s5 + h5;
        const cx<T>* v = coef + qrun * RS + off0;
        cx<T> acc = czero<T>();
        if (h0) cfma(acc, v[0], prev);
        if (h1) cfma(acc, v[s1], pl[((ly - 1) * W + lx) * PP + c]);
        if (h2) cfma(acc, v[s2], pl[(ly * W + lx - 1) * PP + c]);
        cfma(acc, v[s3], cur);
        if (h4) cfma(acc, v[s4], pl[(ly * W + lx + 1) * PP + c]);
        if (h5) cfma(acc, v[s5], pl[((ly + 1) * W + lx) * PP + c]);
        if (h6) cfma(acc, v[s6], nxt);
        if (cok) {
          yv = SUB ? csub(Cm[(int64_t)(r0 + sxy * z) * ldc + c], acc) : acc;
          // streaming store: Y is not read again here, and keeping it out
          // of L2 leaves room for the Z rows neighbouring tiles still need
          if (STORE) st_nt(&Y[(int64_t)(r0 + sxy * z) * ldy + c], yv);
        }
      }
      if (NORM) nrm += (double)cabs2(yv);
      prev = cur;
      cur = nxt;
      nxt = nn;
      hcur = hn;
      cv = cvn;
      off0 = off1;
      off1 = off2;
      lb1 = lb2;
      lc1 = lc2;
    }
  }
  if (NORM) {
    for (int o = 32; o > 0; o >>= 1) nrm += __shfl_xor(nrm, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int k = 0; k < GT / 64; ++k) s += sh[k];
      part[(size_t)blockIdx.x * E + E - 1] = s;
    }
  }
}

// The same product, not pipelined, for launches with the fused Gram: the
// Gram's extra staging and barriers leave no registers for the one-plane
// lookahead (with it the kernel spills and runs slower).
template <typename T, bool SUB, bool STORE, bool GRAM, bool NORM>
__global__ __launch_bounds__(GT) __attribute__((amdgpu_waves_per_eu(8))) void k_spmm_grid_walk(int nx, int ny, int nz,
                                                  const int32_t* __restrict__ rowptr,
                                                  const cx<T>* __restrict__ val,
                                                  const cx<T>* __restrict__ Z, int ldz,
                                                  const cx<T>* __restrict__ Cm, int ldc,
                                                  cx<T>* __restrict__ Y, int ldy, int p, int zc,
                                                  double* part, int E, const DevState* st, int gate) {
  if (st && gate >= st->stop_iter) return;
  constexpr int W = GTX + 2, H = GTY + 2, NH = 2 * (GTX + GTY);
  constexpr int PL = W * H * 32;  // plane + halo, in cx<T>
  // with GRAM the plane buffer also stages the 32 Z and Y rows (as z64)
  constexpr int PB = (int)sizeof(cx<T>) * PL, GB = GRAM ? 2 * 32 * 32 * 16 : 0;
  __shared__ __align__(16) char lds_buf[PB > GB ? PB : GB];
  // Gram accumulators of waves 0-3 (block (w >> 1, w & 1)) between planes,
  // kept in LDS so that no registers stay live across the walk
  __shared__ __align__(16) double gacc[GRAM ? 4 * 2 * 4 * 64 : 1];
  __shared__ double sh[GT / 64];
  cx<T>* pl = reinterpret_cast<cx<T>*>(lds_buf);
  z64* gs = reinterpret_cast<z64*>(lds_buf);
  const int c = threadIdx.x & 31, q = threadIdx.x >> 5, w = threadIdx.x >> 6;
  const bool cok = c < p;
  const int tilesx = (nx + GTX - 1) / GTX, tilesy = (ny + GTY - 1) / GTY;
  const int64_t units = grid_units_pp<32>(nx, ny, nz, zc);
  const int64_t sxy = (int64_t)nx * ny;
  // halo point owned by thread row q (q < NH): ring of the (W x H) frame
  int hx = 0, hy = 0;
  if (q < GTX) {
    hx = q + 1;
  } else if (q < 2 * GTX) {
    hx = q - GTX + 1;
    hy = H - 1;
  } else if (q < 2 * GTX + GTY) {
    hy = q - 2 * GTX + 1;
  } else {
    hx = W - 1;
    hy = q - 2 * GTX - GTY + 1;
  }
  const int lx = q % GTX + 1, ly = q / GTX + 1;  // this point's frame position
  const int l = threadIdx.x & 63;
  if (GRAM && w < 4)
    for (int k = 0; k < 8; ++k) gacc[(w * 8 + k) * 64 + l] = 0.0;
  double nrm = 0.0;
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const int bx = (int)(u % tilesx), by = (int)((u / tilesx) % tilesy), bz = (int)(u / ((int64_t)tilesx * tilesy));
    const int x = bx * GTX + q % GTX, y = by * GTY + q / GTX;
    const int z0 = bz * zc, z1 = min(nz, z0 + zc);
    const bool in = x < nx && y < ny;
    const int64_t r0 = in ? x + (int64_t)nx * y : 0;
    const int ex = bx * GTX + hx - 1, ey = by * GTY + hy - 1;
    const bool hok = q < NH && ex >= 0 && ex < nx && ey >= 0 && ey < ny && cok;
    const int64_t hr0 = hok ? ex + (int64_t)nx * ey : 0;
    cx<T> prev = (in && cok && z0 > 0) ? Z[(r0 + sxy * (z0 - 1)) * ldz + c] : czero<T>();
    cx<T> cur = (in && cok) ? Z[(r0 + sxy * z0) * ldz + c] : czero<T>();
    for (int z = z0; z < z1; ++z) {
      const int64_t r = r0 + sxy * z;
      const cx<T> nxt = (in && cok && z + 1 < nz) ? Z[(r + sxy) * ldz + c] : czero<T>();
      const int rp = in ? rowptr[r] : 0;
      if (q < NH) pl[(hy * W + hx) * 32 + c] = hok ? Z[(hr0 + sxy * z) * ldz + c] : czero<T>();
      pl[(ly * W + lx) * 32 + c] = cur;
      __syncthreads();
      cx<T> yv = czero<T>();
      if (in) {
        // CSR slots of the existing neighbours, in column order
        const bool h0 = z > 0, h1 = y > 0, h2 = x > 0, h4 = x < nx - 1, h5 = y < ny - 1, h6 = z < nz - 1;
        const int s1 = h0, s2 = s1 + h1, s3 = s2 + h2, s4 = s3 + 1, s5 = s4 + h4, s6 = s5 + h5;
        const cx<T>* v = val + rp;
        cx<T> acc = czero<T>();
        if (h0) cfma(acc, v[0], prev);
        if (h1) cfma(acc, v[s1], pl[((ly - 1) * W + lx) * 32 + c]);
        if (h2) cfma(acc, v[s2], pl[(ly * W + lx - 1) * 32 + c]);
        cfma(acc, v[s3], cur);
        if (h4) cfma(acc, v[s4], pl[(ly * W + lx + 1) * 32 + c]);
        if (h5) cfma(acc, v[s5], pl[((ly + 1) * W + lx) * 32 + c]);
        if (h6) cfma(acc, v[s6], nxt);
        if (cok) {
          yv = SUB ? csub(Cm[r * ldc + c], acc) : acc;
          if (STORE) st_nt(&Y[r * ldy + c], yv);
        }
      }
      if (NORM) nrm += (double)cabs2(yv);
      if (GRAM) {
        __syncthreads();  // the plane has been read; stage the rows over it
        gs[q * 32 + c] = z64{(double)cur.re, (double)cur.im};
        gs[32 * 32 + q * 32 + c] = z64{(double)yv.re, (double)yv.im};
        __syncthreads();
        if (w < 4) {
          d4 gr, gi;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            gr[v] = gacc[(w * 8 + v) * 64 + l];
            gi[v] = gacc[(w * 8 + 4 + v) * 64 + l];
          }
          // rows 0-15, then rows 16-31
          grid_gram16(gs, gs + 32 * 32, (w >> 1) & 1, w & 1, gr, gi);
          grid_gram16(gs + 16 * 32, gs + 32 * 32 + 16 * 32, (w >> 1) & 1, w & 1, gr, gi);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            gacc[(w * 8 + v) * 64 + l] = gr[v];
            gacc[(w * 8 + 4 + v) * 64 + l] = gi[v];
          }
        }
      }
      __syncthreads();  // the buffer is free for the next plane
      prev = cur;
      cur = nxt;
    }
  }
  if (GRAM || NORM) {
    double* dst = part + (size_t)blockIdx.x * E;
    if (GRAM) {
      __syncthreads();
      if (w < 4) {
        const int ib = (w >> 1) & 1, jb = w & 1;
        const int j = 16 * jb + (l & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * ib + 4 * v + (l >> 4);
          if (i < p && j < p) {
            dst[2 * (i * p + j)] = gacc[(w * 8 + v) * 64 + l];
            dst[2 * (i * p + j) + 1] = gacc[(w * 8 + 4 + v) * 64 + l];
          }
        }
      }
    }
    if (NORM) {
      for (int o = 32; o > 0; o >>= 1) nrm += __shfl_xor(nrm, o);
      __syncthreads();
      if ((threadIdx.x & 63) == 0) sh[w] = nrm;
      __syncthreads();
      if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < GT / 64; ++k) s += sh[k];
        dst[E - 1] = s;
      }
    }
  }
}

}  // namespace blk
