// Host driver and C ABI of the block COCG / block COCR solvers.
//
// One solve = a start-up (initial residual, residual orthonormalization or
// first Grams) followed by iterations, each a fixed sequence of kernel
// launches on the caller's stream:
//
//   block COCR + residual orthonormalization (Algorithm 3), iteration m:
//     solve (U^T U) alpha' = Q^T V            [k_solve]
//     W = Q - U alpha', Gram W^H W            [k_axpy + k_reduce]
//     Q tau = W by two Cholesky-QR passes     [k_chol, k_cholqr_pass2, k_chol, k_cholqr_pass3]
//     V = A Q, Gram Q^T V                     [k_spmm + k_reduce]
//     solve (Q_m^T V_m) beta' = tau^T Q^T V   [k_solve]
//     X += S alpha' xi, S = Q + S beta', U = V + U beta', Gram U^T U [k_update]
//
// Every kernel of iteration m is a no-op once the device state says the run
// stopped before m, so the host only synchronizes every `check_every`
// iterations to read the 4-byte stop index.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/blk.h"
#include "common.hpp"
#include "pxp.hpp"
#include "rowpass.hpp"
#include "rowpass_mfma.hpp"
#include "grid.hpp"
#include "dense_mf.hpp"
#include "spmm.hpp"

namespace blk {

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

struct HipError {
  hipError_t e;
  const char* what;
};

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) throw HipError{e_, #x};   \
  } while (0)

#define LAUNCH_CHECK() HIPCHK(hipGetLastError())

template <int V>
using IC = std::integral_constant<int, V>;

// Call f with the padded column count PP (power of two >= p).
template <typename F>
static void with_pp(int p, F&& f) {
  if (p <= 1)
    f(IC<1>{});
  else if (p <= 2)
    f(IC<2>{});
  else if (p <= 4)
    f(IC<4>{});
  else if (p <= 8)
    f(IC<8>{});
  else if (p <= 16)
    f(IC<16>{});
  else
    f(IC<32>{});
}

// FP64 blocks wider than 8 columns run on the matrix cores
// (rowpass_mfma.hpp), everything else on the vector units.
template <typename T>
static constexpr bool use_mfma(int PP) {
  return std::is_same<T, double>::value && PP >= 16;
}

static int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return (v && *v) ? atoi(v) : dflt;
}

// Device memory owned by one call.
struct Pool {
  std::vector<void*> ptrs;
  template <typename P>
  P* get(size_t bytes) {
    void* q = nullptr;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) throw HipError{e, "hipMalloc"};
    ptrs.push_back(q);
    return static_cast<P*>(q);
  }
  ~Pool() {
    for (void* q : ptrs) (void)hipFree(q);
  }
};

enum Role { RO_A = 0, RO_P2, RO_P3, RO_S, RO_B, RO_N, RO_COUNT };

// Launch geometry and reduction buffers shared by every pass of a solve.
struct Ctx {
  hipStream_t s = nullptr;
  int64_t n = 0;
  int p = 0;
  int G = 1;     // blocks of a row pass
  int Gs = 1;    // blocks of an operator application that reduces a Gram or norm
  int S = 0;     // first-stage reduction segments (0: p x p kernels read the partials)
  int cus = 256; // compute units of the current device
  int Emax = 0;  // doubles per block partial
  int nblk[RO_COUNT] = {};  // blocks that wrote the partials of each role
  double* part[RO_COUNT] = {};
  double* red[RO_COUNT] = {};
  z64* slots = nullptr;
  DevState* st = nullptr;
  double* hist = nullptr;  // device, maxit + 2 entries
  int hist_cap = 0;
  z64* dws = nullptr;      // split-K partials of the dense product (DSPLIT x n x 32)
};

// Compute units of the current device (256 if the query fails).
static int device_cus() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1)
    return 256;
  return v;
}

// Launch geometry of a row pass over n rows of p columns.
static void ctx_geometry(Ctx& c, int64_t n, int p, hipStream_t s) {
  c.s = s;
  c.cus = device_cus();
  c.n = n;
  c.p = p;
  int PP = 1;
  while (PP < p) PP <<= 1;
  const int64_t ntiles = (n + (NT / PP) - 1) / (NT / PP);
  // row passes: the vector-unit kernels (p < 16) gain from more resident
  // workgroups; the matrix-core ones (two waves per SIMD) do not
  const int gmax = std::max(8, env_int("BLK_GRID", PP < 16 ? 2048 : 1024));
  c.G = (int)std::min<int64_t>(gmax, ntiles);
  if (c.G >= 64) c.G &= ~7;  // multiple of 8 for the XCD remap
  c.Gs = (int)std::min<int64_t>(std::max(8, env_int("BLK_GRID_SPMM", 4096)), ntiles);
  if (c.Gs >= 64) c.Gs &= ~7;
  c.S = (std::max(c.G, c.Gs) > 64) ? 32 : 0;
  for (int r = 0; r < RO_COUNT; ++r) c.nblk[r] = c.G;
}

static void ctx_alloc(Ctx& c, Pool& pool, int64_t n, int p, int maxit, hipStream_t s) {
  ctx_geometry(c, n, p, s);
  c.Emax = 2 * p * p + 1;
  for (int r = 0; r < RO_COUNT; ++r) {
    c.part[r] = pool.get<double>(sizeof(double) * (size_t)std::max(c.G, c.Gs) * c.Emax);
    if (c.S) c.red[r] = pool.get<double>(sizeof(double) * (size_t)c.S * c.Emax);
  }
  c.slots = pool.get<z64>(sizeof(z64) * (size_t)SLOT * S_NSLOTS);
  c.st = pool.get<DevState>(sizeof(DevState));
  c.hist_cap = maxit + 2;
  c.hist = pool.get<double>(sizeof(double) * (size_t)c.hist_cap);
}

// Reduce the partials of `role` (E doubles per block) and describe the result.
static Red finish(Ctx& c, int role, int E, int off, int gate) {
  const int G = c.nblk[role];
  if (c.S == 0) return Red{c.part[role], G, E, off};
  dim3 grid((E + NT - 1) / NT, c.S);
  k_reduce<<<grid, NT, 0, c.s>>>(c.part[role], G, E, c.red[role], c.S, c.st, gate);
  LAUNCH_CHECK();
  return Red{c.red[role], c.S, E, off};
}

static Red no_red() { return Red{nullptr, 0, 0, 0}; }

template <typename T>
struct DevOp {
  int kind = BLK_OP_CSR;
  int64_t n = 0;
  const int32_t* rowptr = nullptr;
  const int32_t* colind = nullptr;
  const cx<T>* val = nullptr;
  const cx<T>* dense = nullptr;
  int64_t ld = 0;
  int gnx = 0, gny = 0, gnz = 0;  // gnx > 0: verified grid-stencil pattern
};

// Y = A Z (SUB: Y = C - A Z), optional store / Gram Z^T Y / ||Y||^2.
template <typename T, bool SUB, bool STORE, bool GRAM, bool NORM>
static void apply_op(Ctx& c, const DevOp<T>& A, const cx<T>* Z, int ldz, const cx<T>* C, int ldc,
                     cx<T>* Y, int ldy, int role, int E, int gate) {
  with_pp(c.p, [&](auto ppc) {
    constexpr int PP = decltype(ppc)::value;
    double* part = (GRAM || NORM) ? c.part[role] : nullptr;
    const DevState* st = c.st;
    if constexpr (PP == 32 || PP == 16 || PP == 8) {
      if (A.kind == BLK_OP_CSR && A.gnx > 0 && (PP == 32 || !GRAM)) {
        // grid-stencil pattern: 2.5D blocked product; with a reduction the
        // grid is bounded by the partial buffers (blocks loop over units)
        const int cap = std::max(c.G, c.Gs);
        const int zc = grid_zchunk<PP>(A.gnx, A.gny, A.gnz, GRID_WG_PER_CU * c.cus);
        const int64_t units = grid_units_pp<PP>(A.gnx, A.gny, A.gnz, zc);
        if constexpr (GRAM) {
          const int64_t G = std::min<int64_t>(units, cap);
          c.nblk[role] = (int)G;
          k_spmm_grid_walk<T, SUB, STORE, GRAM, NORM><<<(unsigned)G, GT, 0, c.s>>>(
              A.gnx, A.gny, A.gnz, A.rowptr, A.val, Z, ldz, C, ldc, Y, ldy, c.p, zc, part, E, st,
              gate);
        } else {
          const int64_t G = NORM ? std::min<int64_t>(units, cap) : units;
          if (NORM) c.nblk[role] = (int)G;
          k_spmm_grid<T, PP, SUB, STORE, NORM><<<(unsigned)G, GT, 0, c.s>>>(
              A.gnx, A.gny, A.gnz, A.rowptr, A.val, Z, ldz, C, ldc, Y, ldy, c.p, zc, part, E, st,
              gate);
        }
        LAUNCH_CHECK();
        return;
      }
      if constexpr ((PP == 16 || PP == 8) && GRAM && STORE && !NORM) {
        if (A.kind == BLK_OP_CSR && A.gnx > 0) {
          // grid-stencil pattern, p <= 16 with the Gram: the 2.5D product, then
          // the Gram Z^T Y (FP64 accumulation) as a pass over the stored Y --
          // fused, its staging and registers cost more than the pass
          const int zc = grid_zchunk<PP>(A.gnx, A.gny, A.gnz, GRID_WG_PER_CU * c.cus);
          const int64_t units = grid_units_pp<PP>(A.gnx, A.gny, A.gnz, zc);
          k_spmm_grid<T, PP, SUB, STORE, false><<<(unsigned)units, GT, 0, c.s>>>(
              A.gnx, A.gny, A.gnz, A.rowptr, A.val, Z, ldz, C, ldc, Y, ldy, c.p, zc, nullptr, 0, st,
              gate);
          LAUNCH_CHECK();
          c.nblk[role] = c.G;
          k_gram<T, double, PP, G_UNCONJ, false><<<c.G, NT, 0, c.s>>>(c.n, c.p, Z, ldz, Y, ldy, part, E,
                                                                      st, gate);
          LAUNCH_CHECK();
          return;
        }
      }
    }
    if (A.kind == BLK_OP_CSR) {
      // Without a reduction every tile of RPB rows is its own block, which
      // keeps the most waves in flight; with one, the grid is bounded by
      // the partials it writes.
      const int64_t ntiles = (c.n + NT / PP - 1) / (NT / PP);
      const int64_t G = (GRAM || NORM) ? c.Gs : ntiles;
      if (GRAM || NORM) c.nblk[role] = c.Gs;
      // one tile per block: natural block order (consecutive tiles on
      // different XCDs); bounded grids: one contiguous slab per XCD
      const int remap = (GRAM || NORM) ? 1 : 0;
      k_spmm<T, PP, SUB, STORE, GRAM, NORM><<<(unsigned)G, NT, 0, c.s>>>(
          c.n, A.rowptr, A.colind, A.val, Z, ldz, C, ldc, Y, ldy, c.p, part, E, st, gate, remap);
    } else {
      if (GRAM || NORM) c.nblk[role] = c.G;
      if constexpr (std::is_same<T, double>::value && PP == 32) {
        if (c.dws) {
          // matrix-core product into split-K partials, then their fixed-order
          // sum with the epilogues; the Gram Z^T Y reads the stored Y
          // (the casts only name T = double; this branch exists for it alone)
          const z64* Ad = reinterpret_cast<const z64*>(A.dense);
          const z64* Zd = reinterpret_cast<const z64*>(Z);
          const z64* Cd = reinterpret_cast<const z64*>(C);
          z64* Yd = reinterpret_cast<z64*>(Y);
          k_dense_mf<<<(unsigned)dense_blocks(c.n), NT, 0, c.s>>>(c.n, Ad, A.ld, Zd, ldz, c.p, c.dws,
                                                                  st, gate);
          LAUNCH_CHECK();
          k_dense_fin<double, SUB, STORE, NORM><<<c.G, NT, 0, c.s>>>(c.n, c.p, c.dws, Cd, ldc, Yd, ldy,
                                                                     part, E, st, gate);
          LAUNCH_CHECK();
          if (GRAM) {
            static_assert(!GRAM || STORE, "the Gram of a dense product reads the stored Y");
            k_gram_mf<2, G_UNCONJ, false><<<c.G, NT, 0, c.s>>>(c.n, c.p, Zd, ldz, Yd, ldy, part, E, st,
                                                               gate);
          }
          LAUNCH_CHECK();
          return;
        }
      }
      if constexpr (std::is_same<T, float>::value && PP == 32) {
        if (c.dws) {
          // complex64 (the mixed form's inner solves): FP32 matrix cores into
          // split-K partials held in the same workspace, their fixed-order sum
          // with the epilogues, then the Gram Z^T Y with FP64 accumulation
          // from the stored Y (the casts only name T = float)
          const c32* Af = reinterpret_cast<const c32*>(A.dense);
          const c32* Zf = reinterpret_cast<const c32*>(Z);
          const c32* Cf = reinterpret_cast<const c32*>(C);
          c32* Yf = reinterpret_cast<c32*>(Y);
          c32* ws = reinterpret_cast<c32*>(c.dws);
          k_dense_mf32<<<(unsigned)dense_blocks(c.n), NT, 0, c.s>>>(c.n, Af, A.ld, Zf, ldz, c.p, ws, st,
                                                                    gate);
          LAUNCH_CHECK();
          k_dense_fin<float, SUB, STORE, NORM><<<c.G, NT, 0, c.s>>>(c.n, c.p, ws, Cf, ldc, Yf, ldy, part,
                                                                    E, st, gate);
          LAUNCH_CHECK();
          if (GRAM) {
            static_assert(!GRAM || STORE, "the Gram of a dense product reads the stored Y");
            k_gram<float, double, 32, G_UNCONJ, false><<<c.G, NT, 0, c.s>>>(c.n, c.p, Zf, ldz, Yf, ldy,
                                                                            part, E, st, gate);
          }
          LAUNCH_CHECK();
          return;
        }
      }
      k_dense<T, PP, SUB, STORE, GRAM, NORM><<<c.G, NT, 0, c.s>>>(
          c.n, A.dense, A.ld, Z, ldz, C, ldc, Y, ldy, c.p, part, E, st, gate);
    }
    LAUNCH_CHECK();
  });
}

template <typename TD, typename TS>
static void copy_block(Ctx& c, const cx<TS>* X, int ldx, cx<TD>* Y, int ldy, double scale, int gate,
                       int64_t rows = -1, int cols = -1) {
  const int64_t r = rows < 0 ? c.n : rows;
  const int q = cols < 0 ? c.p : cols;
  const int64_t tot = r * q;
  if (tot == 0) return;
  k_copy<TD, TS><<<(unsigned)((tot + NT - 1) / NT), NT, 0, c.s>>>(r, q, X, ldx, Y, ldy, scale, c.st,
                                                                  gate);
  LAUNCH_CHECK();
}

template <typename T>
static void zero_block(Ctx& c, cx<T>* Y, int ldy) {
  const int64_t tot = c.n * c.p;
  k_zero<T><<<(unsigned)((tot + NT - 1) / NT), NT, 0, c.s>>>(c.n, c.p, Y, ldy);
  LAUNCH_CHECK();
}

template <typename T, typename A, int GM, bool NORM>
static Red gram(Ctx& c, const cx<T>* Y, int ldy, const cx<T>* Z, int ldz, int role, int gate) {
  const int E = (GM != G_NONE ? 2 * c.p * c.p : 0) + (NORM ? 1 : 0);
  c.nblk[role] = c.G;
  with_pp(c.p, [&](auto ppc) {
    constexpr int PP = decltype(ppc)::value;
    if constexpr (use_mfma<T>(PP)) {
      k_gram_mf<PP / 16, GM, NORM><<<c.G, NT, 0, c.s>>>(c.n, c.p, Y, ldy, Z, ldz, c.part[role], E,
                                                        c.st, gate);
    } else {
      k_gram<T, A, PP, GM, NORM><<<c.G, NT, 0, c.s>>>(c.n, c.p, Y, ldy, Z, ldz, c.part[role], E,
                                                      c.st, gate);
    }
    LAUNCH_CHECK();
  });
  return finish(c, role, E, 0, gate);
}

template <typename T, typename A, int GM, bool NORM>
static void launch_axpy(Ctx& c, const cx<T>* Ain, int lda, const cx<T>* Bin, int ldb, const z64* C,
                        cx<T>* Out, int ldo, int role, int E, int gate) {
  c.nblk[role] = c.G;
  with_pp(c.p, [&](auto ppc) {
    constexpr int PP = decltype(ppc)::value;
    if constexpr (use_mfma<T>(PP)) {
      k_axpy_mf<PP / 16, GM, NORM><<<c.G, NT, 0, c.s>>>(c.n, c.p, Ain, lda, Bin, ldb, C, -1.0, Out,
                                                        ldo, c.part[role], E, c.st, gate);
    } else {
      k_axpy<T, A, PP, GM, NORM><<<c.G, NT, 0, c.s>>>(c.n, c.p, Ain, lda, Bin, ldb, C, Out, ldo,
                                                      c.part[role], E, c.st, gate);
    }
    LAUNCH_CHECK();
  });
}

template <typename T, typename A, bool WITH_U>
static void launch_update(Ctx& c, cx<T>* X, int ldx, cx<T>* S, int lds, const cx<T>* Q, int ldq,
                          cx<T>* U, int ldu, const cx<T>* V, int ldv, const z64* C1, const z64* C2,
                          int role, int E, int gate) {
  c.nblk[role] = c.G;
  with_pp(c.p, [&](auto ppc) {
    constexpr int PP = decltype(ppc)::value;
    double* part = WITH_U ? c.part[role] : nullptr;
    if constexpr (use_mfma<T>(PP)) {
      // U = V + U C2 with U^T U, then X += S C1, S = Q + S C2: two launches
      // over disjoint data keep each kernel within two waves' registers
      if (WITH_U)
        k_axpy_mf<PP / 16, G_UNCONJ, false><<<c.G, NT, 0, c.s>>>(c.n, c.p, V, ldv, U, ldu, C2, 1.0, U,
                                                                 ldu, part, E, c.st, gate);
      k_update_mf<PP / 16><<<c.G, NT, 0, c.s>>>(c.n, c.p, X, ldx, S, lds, Q, ldq, C1, C2, c.st, gate);
    } else {
      k_update<T, A, PP, WITH_U><<<c.G, NT, 0, c.s>>>(c.n, c.p, X, ldx, S, lds, Q, ldq, U, ldu, V,
                                                      ldv, C1, C2, part, E, c.st, gate);
    }
    LAUNCH_CHECK();
  });
}

static void solve_pp(Ctx& c, SolveArgs a) {
  a.slots = c.slots;
  a.hist = c.hist;
  a.st = c.st;
  k_solve<<<1, px_threads(c.p), 0, c.s>>>(a);
  LAUNCH_CHECK();
}

static void chol_pp(Ctx& c, Red g, int mode, int gate, int idx, int init) {
  CholArgs a{g, mode, gate, idx, init, c.slots, c.hist, c.st};
  k_chol<<<1, px_threads(c.p), 0, c.s>>>(a);
  LAUNCH_CHECK();
}

static SolveArgs solve_args() {
  SolveArgs a;
  memset(&a, 0, sizeof a);
  a.mslot = a.rslot = -1;
  a.save_slot = a.outxi_slot = -1;
  return a;
}

// Thin QR of W (in place -> Q = W tau^{-1}) by Cholesky QR twice; the first
// Gram W^H W must already be reduced in g1.  Produces xi (see k_chol).
template <typename T, typename A, bool GRAM_QQ>
static Red cholqr(Ctx& c, Red g1, cx<T>* W, int ldw, cx<T>* Q, int ldq, int gate1, int gate2, int idx,
                  int init) {
  chol_pp(c, g1, 1, gate1, idx, init);
  const int E2 = 2 * c.p * c.p;
  c.nblk[RO_P2] = c.nblk[RO_P3] = c.G;
  Red out = no_red();
  with_pp(c.p, [&](auto ppc) {
    constexpr int PP = decltype(ppc)::value;
    if constexpr (use_mfma<T>(PP)) {
      k_cholqr_pass2_mf<PP / 16><<<c.G, NT, 0, c.s>>>(c.n, c.p, W, ldw, c.slots + S_R1INV * SLOT,
                                                      c.part[RO_P2], E2, c.st, gate2);
    } else {
      k_cholqr_pass2<T, PP><<<c.G, NT, 0, c.s>>>(c.n, c.p, W, ldw, c.slots + S_R1INV * SLOT,
                                                c.part[RO_P2], E2, c.st, gate2);
    }
    LAUNCH_CHECK();
    Red g2 = finish(c, RO_P2, E2, 0, gate2);
    chol_pp(c, g2, 2, gate2, idx, init);
    if constexpr (use_mfma<T>(PP)) {
      k_cholqr_pass3_mf<PP / 16, GRAM_QQ><<<c.G, NT, 0, c.s>>>(
          c.n, c.p, W, ldw, c.slots + S_TAUINV * SLOT, Q, ldq, c.part[RO_P3], E2, c.st, gate2);
    } else {
      k_cholqr_pass3<T, A, PP, GRAM_QQ><<<c.G, NT, 0, c.s>>>(
          c.n, c.p, W, ldw, c.slots + S_TAUINV * SLOT, Q, ldq, c.part[RO_P3], E2, c.st, gate2);
    }
    LAUNCH_CHECK();
    if (GRAM_QQ) out = finish(c, RO_P3, E2, 0, gate2);
  });
  return out;
}

static DevState read_state(Ctx& c) {
  DevState h;
  HIPCHK(hipMemcpyAsync(&h, c.st, sizeof h, hipMemcpyDeviceToHost, c.s));
  HIPCHK(hipStreamSynchronize(c.s));
  return h;
}

static double read_scalar(Ctx& c, Red r) {
  std::vector<double> h((size_t)r.nrows * r.ld);
  HIPCHK(hipMemcpyAsync(h.data(), r.base, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c.s));
  HIPCHK(hipStreamSynchronize(c.s));
  double s = 0.0;
  for (int k = 0; k < r.nrows; ++k) s += h[(size_t)k * r.ld + r.off];
  return s;
}

struct SolveOut {
  int status = ST_CONVERGED;
  int iters = 0;
  std::vector<double> hist;
};

// Working blocks of a solve (n x p, ld p).
template <typename T>
struct Blocks {
  cx<T>* b[5] = {};
};

// One block solve in arithmetic T on right-hand side B (n x p) starting from
// X0 (NULL = 0), writing X.  The device state is (re)initialized here.
template <typename T, typename A>
static SolveOut run_solve(Ctx& c, const DevOp<T>& Aop, bool cocr, bool rq, const cx<T>* B, int ldb,
                          const cx<T>* X0, int ldx0, cx<T>* X, int ldx, double tol, int maxit,
                          int check_every, Blocks<T>& bk, double div_limit = INFINITY) {
  SolveOut out;
  const int p = c.p;
  const int E2 = 2 * p * p;
  // the device state, then ||B||_F
  {
    k_state_init<<<1, 64, 0, c.s>>>(c.st, p, maxit, tol, div_limit);
    LAUNCH_CHECK();
    Red nb = gram<T, double, G_NONE, true>(c, B, ldb, B, ldb, RO_N, -1);
    k_set_norm<<<1, 64, 0, c.s>>>(c.st, nb);
    LAUNCH_CHECK();
  }
  DevState h = read_state(c);
  if (!(h.normB > 0.0)) {
    if (h.normB == 0.0) {
      zero_block<T>(c, X, ldx);
      out.hist.assign(1, 0.0);
      HIPCHK(hipStreamSynchronize(c.s));
      return out;
    }
    out.status = ST_BREAKDOWN;  // non-finite B
    out.hist.assign(1, h.normB);
    return out;
  }
  // R_0 = B - A X_0 into the first working block, X = X_0
  cx<T>* R0 = bk.b[0];
  if (X0) {
    apply_op<T, true, true, false, false>(c, Aop, X0, ldx0, B, ldb, R0, p, RO_N, 0, -1);
    if ((const void*)X0 != (const void*)X) copy_block<T, T>(c, X0, ldx0, X, ldx, 1.0, -1);
  } else {
    copy_block<T, T>(c, B, ldb, R0, p, 1.0, -1);
    zero_block<T>(c, X, ldx);
  }

  if (rq) {
    // Q_0 xi_0 = R_0; S_0 = Q_0 (Algorithms 2 and 3, start-up)
    cx<T>* W = bk.b[0];
    cx<T>* Q = bk.b[1];
    cx<T>* S = bk.b[2];
    cx<T>* V = bk.b[3];  // V (COCR) or Z = A S (COCG)
    cx<T>* U = bk.b[4];
    Red g1 = gram<T, double, G_CONJ, false>(c, W, p, W, p, RO_A, -1);
    Red gqq = cholqr<T, A, true>(c, g1, W, p, Q, p, -1, 0, 0, 1);
    copy_block<T, T>(c, Q, p, S, p, 1.0, 0);
    if (cocr) {
      // U_0 = V_0 = A Q_0, G_old = Q_0^T V_0, U_0^T U_0
      apply_op<T, false, true, true, false>(c, Aop, Q, p, nullptr, 0, V, p, RO_S, E2, 0);
      Red gqv = finish(c, RO_S, E2, 0, 0);
      copy_block<T, T>(c, V, p, U, p, 1.0, 0);
      gram<T, A, G_UNCONJ, false>(c, U, p, U, p, RO_B, 0);
      k_start<<<1, px_threads(c.p), 0, c.s>>>(no_red(), gqv, S_GOLD, c.slots, c.hist, c.st);
      LAUNCH_CHECK();
    } else {
      k_start<<<1, px_threads(c.p), 0, c.s>>>(no_red(), gqq, S_GOLD, c.slots, c.hist, c.st);
      LAUNCH_CHECK();
    }
    h = read_state(c);
    Red guu_prev = (c.S == 0) ? Red{c.part[RO_B], c.G, E2, 0} : Red{c.red[RO_B], c.S, E2, 0};
    int m = 0;
    if (h.stop_iter > 0) {
      for (m = 0; m < maxit; ++m) {
        if (cocr) {
          SolveArgs al = solve_args();
          al.mred = guu_prev;
          al.rslot = S_GOLD;
          al.out_slot = S_ALPHA;
          al.outxi_slot = S_ALPHAXI;
          al.gate = m;
          al.fail_idx = m;
          solve_pp(c, al);
          Red g1m = no_red();
          launch_axpy<T, double, G_CONJ, false>(c, Q, p, U, p, c.slots + S_ALPHA * SLOT, W, p, RO_A,
                                             E2, m);
          g1m = finish(c, RO_A, E2, 0, m);
          cholqr<T, A, false>(c, g1m, W, p, Q, p, m, m, m + 1, 0);
          apply_op<T, false, true, true, false>(c, Aop, Q, p, nullptr, 0, V, p, RO_S, E2, m);
          Red gqv = finish(c, RO_S, E2, 0, m);
          SolveArgs be = solve_args();
          be.mslot = S_GOLD;
          be.rred = gqv;
          be.rhs_tauT = 1;
          be.save_slot = S_GOLD;
          be.out_slot = S_BETA;
          be.gate = m;
          be.fail_idx = m + 1;
          be.late = 1;
          solve_pp(c, be);
          launch_update<T, A, true>(c, X, ldx, S, p, Q, p, U, p, V, p, c.slots + S_ALPHAXI * SLOT,
                                    c.slots + S_BETA * SLOT, RO_B, E2, m);
          guu_prev = finish(c, RO_B, E2, 0, m);
        } else {
          apply_op<T, false, true, true, false>(c, Aop, S, p, nullptr, 0, V, p, RO_S, E2, m);
          Red gsz = finish(c, RO_S, E2, 0, m);
          SolveArgs al = solve_args();
          al.mred = gsz;
          al.rslot = S_GOLD;
          al.out_slot = S_ALPHA;
          al.outxi_slot = S_ALPHAXI;
          al.gate = m;
          al.fail_idx = m;
          solve_pp(c, al);
          launch_axpy<T, double, G_CONJ, false>(c, Q, p, V, p, c.slots + S_ALPHA * SLOT, W, p, RO_A,
                                             E2, m);
          Red g1m = finish(c, RO_A, E2, 0, m);
          Red gq = cholqr<T, A, true>(c, g1m, W, p, Q, p, m, m, m + 1, 0);
          SolveArgs be = solve_args();
          be.mslot = S_GOLD;
          be.rred = gq;
          be.rhs_tauT = 1;
          be.save_slot = S_GOLD;
          be.out_slot = S_BETA;
          be.gate = m;
          be.fail_idx = m + 1;
          be.late = 1;
          solve_pp(c, be);
          launch_update<T, A, false>(c, X, ldx, S, p, Q, p, nullptr, 0, nullptr, 0,
                                    c.slots + S_ALPHAXI * SLOT, c.slots + S_BETA * SLOT, RO_B, 0, m);
        }
        if ((m + 1) % check_every == 0 || m + 1 == maxit) {
          h = read_state(c);
          if (h.stop_iter <= m + 1) break;
        }
      }
    }
  } else {
    // plain variants: R, P (= S), V/Z, U
    cx<T>* R = bk.b[0];
    cx<T>* P = bk.b[1];
    cx<T>* V = bk.b[3];
    cx<T>* U = bk.b[4];
    copy_block<T, T>(c, R, p, P, p, 1.0, -1);
    const int EA = E2 + 1;  // Gram + norm
    if (cocr) {
      Red nr = gram<T, A, G_NONE, true>(c, R, p, R, p, RO_A, -1);
      apply_op<T, false, true, true, false>(c, Aop, R, p, nullptr, 0, V, p, RO_S, E2, -1);
      Red grv = finish(c, RO_S, E2, 0, -1);
      copy_block<T, T>(c, V, p, U, p, 1.0, -1);
      gram<T, A, G_UNCONJ, false>(c, U, p, U, p, RO_B, -1);
      k_start<<<1, px_threads(c.p), 0, c.s>>>(nr, grv, S_GOLD, c.slots, c.hist, c.st);
      LAUNCH_CHECK();
    } else {
      Red gr = gram<T, A, G_UNCONJ, true>(c, R, p, R, p, RO_A, -1);
      Red nr = gr;
      nr.off = E2;
      k_start<<<1, px_threads(c.p), 0, c.s>>>(nr, gr, S_GOLD, c.slots, c.hist, c.st);
      LAUNCH_CHECK();
    }
    h = read_state(c);
    Red guu_prev = (c.S == 0) ? Red{c.part[RO_B], c.G, E2, 0} : Red{c.red[RO_B], c.S, E2, 0};
    if (h.stop_iter > 0) {
      for (int m = 0; m < maxit; ++m) {
        if (cocr) {
          SolveArgs al = solve_args();
          al.mred = guu_prev;
          al.rslot = S_GOLD;
          al.out_slot = S_ALPHA;
          al.gate = m;
          al.fail_idx = m;
          solve_pp(c, al);
          launch_axpy<T, A, G_NONE, true>(c, R, p, U, p, c.slots + S_ALPHA * SLOT, R, p, RO_A,
                                             1, m);
          Red nr = finish(c, RO_A, 1, 0, m);
          apply_op<T, false, true, true, false>(c, Aop, R, p, nullptr, 0, V, p, RO_S, E2, m);
          Red grv = finish(c, RO_S, E2, 0, m);
          SolveArgs be = solve_args();
          be.mslot = S_GOLD;
          be.rred = grv;
          be.save_slot = S_GOLD;
          be.out_slot = S_BETA;
          be.nred = nr;
          be.hist_idx = m + 1;
          be.gate = m;
          be.fail_idx = m + 1;
          be.late = 1;
          solve_pp(c, be);
          launch_update<T, A, true>(c, X, ldx, P, p, R, p, U, p, V, p, c.slots + S_ALPHA * SLOT,
                                    c.slots + S_BETA * SLOT, RO_B, E2, m);
          guu_prev = finish(c, RO_B, E2, 0, m);
        } else {
          apply_op<T, false, true, true, false>(c, Aop, P, p, nullptr, 0, V, p, RO_S, E2, m);
          Red gpz = finish(c, RO_S, E2, 0, m);
          SolveArgs al = solve_args();
          al.mred = gpz;
          al.rslot = S_GOLD;
          al.out_slot = S_ALPHA;
          al.gate = m;
          al.fail_idx = m;
          solve_pp(c, al);
          launch_axpy<T, A, G_UNCONJ, true>(c, R, p, V, p, c.slots + S_ALPHA * SLOT, R, p, RO_A,
                                             EA, m);
          Red grr = finish(c, RO_A, EA, 0, m);
          Red nr = grr;
          nr.off = E2;
          SolveArgs be = solve_args();
          be.mslot = S_GOLD;
          be.rred = grr;
          be.save_slot = S_GOLD;
          be.out_slot = S_BETA;
          be.nred = nr;
          be.hist_idx = m + 1;
          be.gate = m;
          be.fail_idx = m + 1;
          be.late = 1;
          solve_pp(c, be);
          launch_update<T, A, false>(c, X, ldx, P, p, R, p, nullptr, 0, nullptr, 0,
                                    c.slots + S_ALPHA * SLOT, c.slots + S_BETA * SLOT, RO_B, 0, m);
        }
        if ((m + 1) % check_every == 0 || m + 1 == maxit) {
          h = read_state(c);
          if (h.stop_iter <= m + 1) break;
        }
      }
    }
  }
  h = read_state(c);
  out.status = h.status;
  out.iters = (h.stop_iter == 0x7fffffff) ? maxit : h.stop_iter;
  out.hist.resize((size_t)out.iters + 1);
  HIPCHK(hipMemcpyAsync(out.hist.data(), c.hist, sizeof(double) * out.hist.size(),
                        hipMemcpyDeviceToHost, c.s));
  HIPCHK(hipStreamSynchronize(c.s));
  return out;
}

// ||B - A X||_F / ||B||_F in FP64.
static double true_relres(Ctx& c, const DevOp<double>& A, const z64* B, int ldb, const z64* X,
                          int ldx, double normB) {
  apply_op<double, true, false, false, true>(c, A, X, ldx, B, ldb, nullptr, 0, RO_N, 1, -1);
  Red r = finish(c, RO_N, 1, 0, -1);
  const double s = read_scalar(c, r);
  return std::sqrt(std::max(s, 0.0)) / normB;
}

static bool blk_log() {
  static const bool on = env_int("BLK_LOG", 0) != 0;
  return on;
}

// Restart from X while the monitored residual says converged but the true
// FP64 residual does not (at most `refine` times, within maxit in total).
static void refine_fp64(Ctx& c, const DevOp<double>& A64, bool cocr, bool rq, const z64* Bz, int ldb,
                        z64* Xz, int ldx, double tol, int maxit, int check_every, int refine,
                        double normB, Blocks<double>& bk, SolveOut& so) {
  for (int k = 0; k < refine && so.status == ST_CONVERGED && so.iters < maxit; ++k) {
    const double trr = true_relres(c, A64, Bz, ldb, Xz, ldx, normB);
    if (blk_log()) fprintf(stderr, "[blk] refine check after %d iterations: true rel. residual %.3e\n", so.iters, trr);
    if (!(trr > tol)) break;
    SolveOut r = run_solve<double, double>(c, A64, cocr, rq, Bz, ldb, Xz, ldx, Xz, ldx, tol,
                                           maxit - so.iters, check_every, bk);
    for (int m = 1; m <= r.iters; ++m) so.hist.push_back(r.hist[m]);
    so.iters += r.iters;
    so.status = r.status;
  }
}

// Mixed precision: FP64 residual B - A X and FP64 X, complex64 inner solves
// of A D = R / ||R|| (iterative refinement).  A correction that makes the
// FP64 residual grow is undone; when refinement stops paying (a worse or
// barely better residual, or an inner solve that cannot start), the solve
// finishes in FP64 from the best X so far.
static SolveOut run_mixed(Ctx& c, Pool& pool, const blk_op* A, const DevOp<double>& A64, bool cocr,
                          const blk_opts& o, const z64* Bz, int ldb, const z64* X0z, int ldx0, z64* Xz,
                          int ldx, double tol, int maxit, double& normB) {
  SolveOut so;
  const int64_t n = c.n;
  const int pi = c.p;
  const int hist_len = maxit + 1;
  Blocks<float> bk;
  for (int i = 0; i < 5; ++i) bk.b[i] = pool.get<c32>(sizeof(c32) * (size_t)n * pi);
  c32* Rf = pool.get<c32>(sizeof(c32) * (size_t)n * pi);
  c32* D = pool.get<c32>(sizeof(c32) * (size_t)n * pi);
  z64* R = pool.get<z64>(sizeof(z64) * (size_t)n * pi);
  DevOp<float> A32;
  A32.kind = A->kind;
  A32.n = n;
  A32.rowptr = A->rowptr;
  A32.colind = A->colind;
  A32.ld = A->kind == BLK_OP_DENSE ? n : 0;
  A32.gnx = A64.gnx;
  A32.gny = A64.gny;
  A32.gnz = A64.gnz;
  k_state_init<<<1, 64, 0, c.s>>>(c.st, pi, maxit, tol, INFINITY);
  LAUNCH_CHECK();
  if (A->kind == BLK_OP_CSR) {
    c32* v = pool.get<c32>(sizeof(c32) * (size_t)std::max<int64_t>(A->nnz, 1));
    copy_block<float, double>(c, A64.val, 1, v, 1, 1.0, -1, A->nnz, 1);
    A32.val = v;
  } else {
    c32* d = pool.get<c32>(sizeof(c32) * (size_t)n * n);
    for (int64_t r0 = 0; r0 < n; r0 += 4096) {
      const int64_t rows = std::min<int64_t>(4096, n - r0);
      copy_block<float, double>(c, A64.dense + r0 * A->ld, (int)A->ld, d + r0 * n, (int)n, 1.0, -1,
                                rows, (int)n);
    }
    A32.dense = d;
  }
  Red nb = gram<double, double, G_NONE, true>(c, Bz, ldb, Bz, ldb, RO_N, -1);
  normB = std::sqrt(std::max(read_scalar(c, nb), 0.0));
  if (normB == 0.0) {
    zero_block<double>(c, Xz, ldx);
    so.hist.assign(1, 0.0);
    return so;
  }
  if (!std::isfinite(normB)) {
    so.status = ST_BREAKDOWN;
    so.hist.assign(1, normB);
    return so;
  }
  if (X0z) {
    if (X0z != Xz) copy_block<double, double>(c, X0z, ldx0, Xz, ldx, 1.0, -1);
  } else {
    zero_block<double>(c, Xz, ldx);
  }
  const int inner_cap = o.inner_maxit > 0 ? o.inner_maxit : std::max(maxit, 1);
  const int64_t tot = n * pi;
  const unsigned gridx = (unsigned)((tot + NT - 1) / NT);
  int total = 0;
  double prev = INFINITY, prev_rho = 0.0;
  bool fallback = false;
  so.status = ST_MAXIT;
  for (int cyc = 0;; ++cyc) {
    k_state_init<<<1, 64, 0, c.s>>>(c.st, pi, maxit, tol, INFINITY);
    LAUNCH_CHECK();
    apply_op<double, true, true, false, true>(c, A64, Xz, ldx, Bz, ldb, R, pi, RO_N, 1, -1);
    const double rho = std::sqrt(std::max(read_scalar(c, finish(c, RO_N, 1, 0, -1)), 0.0));
    double rel = rho / normB;
    if (cyc == 0) so.hist.push_back(rel);
    if (blk_log()) fprintf(stderr, "[blk mixed] cycle %d: true rel. residual %.3e, inner its %d\n", cyc, rel, total);
    if (!std::isfinite(rel) || rel > prev) {
      if (cyc == 0) {
        so.status = ST_BREAKDOWN;
        break;
      }
      // undo the last correction
      k_axpy_up<float><<<gridx, NT, 0, c.s>>>(n, pi, Xz, ldx, D, pi, -prev_rho);
      LAUNCH_CHECK();
      rel = prev;
      fallback = true;
      break;
    }
    if (rel <= tol) {
      so.status = ST_CONVERGED;
      break;
    }
    if (total >= maxit) {
      so.status = ST_MAXIT;
      break;
    }
    if (rel > 0.5 * prev) {
      fallback = true;
      break;
    }
    prev = rel;
    prev_rho = rho;
    copy_block<float, double>(c, R, pi, Rf, pi, 1.0 / rho, -1);
    const int cap = std::min(inner_cap, maxit - total);
    // the inner tolerance never asks for more than the outer target needs
    const double itol = std::max(o.inner_tol, 0.5 * tol / rel);
    // complex64 storage, FP64 accumulation of every Gram: the unconjugated
    // forms cancel heavily and FP32 sums lose the recurrences' coefficients.
    // An inner run whose monitored residual grows tenfold has diverged (the
    // FP64 iteration's early plateau stays below twice its start).
    SolveOut in = run_solve<float, double>(c, A32, cocr, o.rq != 0, Rf, pi, nullptr, 0, D, pi, itol,
                                           cap, o.check_every, bk, 10.0);
    for (int k = 1; k <= in.iters && (int)so.hist.size() < hist_len; ++k)
      so.hist.push_back(rel * in.hist[k]);
    total += in.iters;
    if (in.iters == 0) {
      fallback = true;
      break;
    }
    k_axpy_up<float><<<gridx, NT, 0, c.s>>>(n, pi, Xz, ldx, D, pi, rho);
    LAUNCH_CHECK();
  }
  if (fallback && total < maxit) {
    if (blk_log()) fprintf(stderr, "[blk mixed] finishing in FP64 after %d inner iterations\n", total);
    Blocks<double> bk64;
    for (int i = 0; i < 5; ++i) bk64.b[i] = pool.get<z64>(sizeof(z64) * (size_t)n * pi);
    SolveOut f = run_solve<double, double>(c, A64, cocr, o.rq != 0, Bz, ldb, Xz, ldx, Xz, ldx, tol,
                                           maxit - total, o.check_every, bk64);
    refine_fp64(c, A64, cocr, o.rq != 0, Bz, ldb, Xz, ldx, tol, maxit - total, o.check_every,
                std::max(0, o.refine), normB, bk64, f);
    for (int k = 1; k <= f.iters && (int)so.hist.size() < hist_len; ++k) so.hist.push_back(f.hist[k]);
    total += f.iters;
    so.status = f.status;
  } else if (fallback) {
    so.status = ST_MAXIT;
  }
  so.iters = total;
  return so;
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + nb && y < x + na;
}

// values = false: the complex128 values (val / dense) are not needed.
static int check_op(const blk_op* A, bool values = true) {
  if (!A) return fail(BLK_EINVAL, "A is NULL");
  if (A->n < 1) return fail(BLK_EINVAL, "n = %lld < 1", (long long)A->n);
  if (A->n > (int64_t)0x7fffffff) return fail(BLK_EINVAL, "n too large for int32 indices");
  if (A->kind == BLK_OP_CSR) {
    if (!A->rowptr || !A->colind || (values && !A->val)) return fail(BLK_EINVAL, "CSR pointer is NULL");
    if (A->nnz < 0 || A->nnz > (int64_t)0x7fffffff) return fail(BLK_EINVAL, "bad nnz");
    if (A->structure < BLK_STRUCT_UNKNOWN || A->structure > BLK_STRUCT_GRID)
      return fail(BLK_EINVAL, "unknown structure %d", (int)A->structure);
    if (A->structure == BLK_STRUCT_GRID &&
        (A->grid[0] < 2 || A->grid[1] < 2 || A->grid[2] < 1 || A->grid[0] > A->n ||
         A->grid[1] > A->n || A->grid[2] > A->n || A->grid[0] * A->grid[1] * A->grid[2] != A->n))
      return fail(BLK_EINVAL, "grid dimensions do not match n");
  } else if (A->kind == BLK_OP_DENSE) {
    if (values && !A->dense) return fail(BLK_EINVAL, "dense pointer is NULL");
    if (A->ld < A->n) return fail(BLK_EINVAL, "dense ld < n");
  } else {
    return fail(BLK_EINVAL, "unknown operator kind %d", (int)A->kind);
  }
  return BLK_OK;
}

static DevOp<double> op64(const blk_op* A) {
  DevOp<double> o;
  o.kind = A->kind;
  o.n = A->n;
  o.rowptr = A->rowptr;
  o.colind = A->colind;
  o.val = reinterpret_cast<const z64*>(A->val);
  o.dense = reinterpret_cast<const z64*>(A->dense);
  o.ld = A->ld;
  if (A->kind == BLK_OP_CSR && A->structure == BLK_STRUCT_GRID) {
    o.gnx = (int)A->grid[0];
    o.gny = (int)A->grid[1];
    o.gnz = (int)A->grid[2];
  }
  return o;
}

// Grid-stencil detection: the dimensions come from row 0 (its columns are
// 0, 1, nx and, in 3D, nx ny); every row is then checked on the device.
// Returns true with (nx, ny, nz) when the whole pattern matches.
static bool analyze_grid(const blk_op* A, hipStream_t s, int64_t dims[3]) {
  if (A->kind != BLK_OP_CSR || A->n < 4) return false;
  int32_t rp[2];
  HIPCHK(hipMemcpyAsync(rp, A->rowptr, sizeof rp, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int len = rp[1] - rp[0];
  if (rp[0] < 0 || (len != 3 && len != 4) || (int64_t)rp[1] > A->nnz) return false;
  int32_t col[4];
  HIPCHK(hipMemcpyAsync(col, A->colind + rp[0], sizeof(int32_t) * len, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int64_t n = A->n;
  if (col[0] != 0 || col[1] != 1) return false;
  const int64_t nx = col[2];
  if (nx < 2 || nx > n) return false;
  int64_t ny, nz;
  if (len == 4) {
    const int64_t nxy = col[3];
    if (nxy % nx != 0 || n % nxy != 0) return false;
    ny = nxy / nx;
    nz = n / nxy;
    if (nz < 2) return false;
  } else {
    if (n % nx != 0) return false;
    ny = n / nx;
    nz = 1;
  }
  if (ny < 2) return false;
  int* bad = nullptr;
  HIPCHK(hipMalloc(&bad, sizeof(int)));
  int h = 1;
  try {
    HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), s));
    k_grid_check<<<(unsigned)((n + NT - 1) / NT), NT, 0, s>>>(n, A->rowptr, A->colind, (int)nx, (int)ny,
                                                            (int)nz, bad);
    LAUNCH_CHECK();
    HIPCHK(hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipFree(bad);
    throw;
  }
  HIPCHK(hipFree(bad));
  if (h != 0) return false;
  dims[0] = nx;
  dims[1] = ny;
  dims[2] = nz;
  return true;
}

static int solve_entry(bool cocr, const blk_op* A, int64_t p, const blk_z* B, int64_t ldb,
                       const blk_z* X0, int64_t ldx0, double tol, int32_t maxit, const blk_opts* opts,
                       blk_z* X, int64_t ldx, double* res_hist, int32_t* iters, double* trr) {
  g_err.clear();
  int rc = check_op(A);
  if (rc) return rc;
  const int64_t n = A->n;
  if (p < 1 || p > BLK_MAX_P) return fail(BLK_EINVAL, "p = %lld outside 1..%d", (long long)p, BLK_MAX_P);
  if (!B || !X) return fail(BLK_EINVAL, "B or X is NULL");
  if (ldb < p || ldx < p || (X0 && ldx0 < p)) return fail(BLK_EINVAL, "leading dimension < p");
  if (!(tol > 0.0) || std::isinf(tol)) return fail(BLK_EINVAL, "tol must be finite and > 0");
  if (maxit < 0) return fail(BLK_EINVAL, "maxit < 0");
  if (overlaps(X, sizeof(blk_z) * ((n - 1) * ldx + p), B, sizeof(blk_z) * ((n - 1) * ldb + p)))
    return fail(BLK_EINVAL, "X overlaps B");
  if (X0 && X0 != X &&
      overlaps(X, sizeof(blk_z) * ((n - 1) * ldx + p), X0, sizeof(blk_z) * ((n - 1) * ldx0 + p)))
    return fail(BLK_EINVAL, "X partially overlaps X0");
  if (X0 == X && ldx0 != ldx) return fail(BLK_EINVAL, "X aliases X0 with a different ld");
  blk_opts o;
  memset(&o, 0, sizeof o);
  o.rq = 1;
  o.precision = BLK_FP64;
  o.inner_tol = 1e-3;
  o.inner_maxit = 0;
  o.check_every = 16;
  if (opts) {
    o = *opts;
    if (o.check_every <= 0) o.check_every = 16;
    if (!(o.inner_tol > 0.0)) o.inner_tol = 1e-3;
  }
  if (o.precision != BLK_FP64 && o.precision != BLK_MIXED)
    return fail(BLK_EINVAL, "unknown precision %d", (int)o.precision);
  if (o.rq != 0 && o.rq != 1) return fail(BLK_EINVAL, "rq must be 0 or 1");
  hipStream_t s = (hipStream_t)o.stream;
  const int pi = (int)p;
  try {
    Pool pool;
    Ctx c;
    const int hist_len = maxit + 1;
    ctx_alloc(c, pool, n, pi, maxit, s);
    if (A->kind == BLK_OP_DENSE && pi > 16)
      c.dws = pool.get<z64>(sizeof(z64) * (size_t)DSPLIT * n * 32);
    DevOp<double> A64 = op64(A);
    if (A->kind == BLK_OP_CSR && A->structure == BLK_STRUCT_UNKNOWN) {
      int64_t d[3];
      if (analyze_grid(A, s, d)) {
        A64.gnx = (int)d[0];
        A64.gny = (int)d[1];
        A64.gnz = (int)d[2];
      }
    }
    const z64* Bz = reinterpret_cast<const z64*>(B);
    const z64* X0z = reinterpret_cast<const z64*>(X0);
    z64* Xz = reinterpret_cast<z64*>(X);
    SolveOut so;
    double normB = 0.0;
    if (o.precision == BLK_FP64) {
      Blocks<double> bk;
      for (int i = 0; i < 5; ++i) bk.b[i] = pool.get<z64>(sizeof(z64) * (size_t)n * pi);
      so = run_solve<double, double>(c, A64, cocr, o.rq != 0, Bz, (int)ldb, X0z, (int)ldx0, Xz,
                                     (int)ldx, tol, maxit, o.check_every, bk);
      normB = read_state(c).normB;
      if (normB > 0.0 && std::isfinite(normB))
        refine_fp64(c, A64, cocr, o.rq != 0, Bz, (int)ldb, Xz, (int)ldx, tol, maxit, o.check_every,
                    std::max(0, o.refine), normB, bk, so);
    } else {
      so = run_mixed(c, pool, A, A64, cocr, o, Bz, (int)ldb, X0z, (int)ldx0, Xz, (int)ldx, tol,
                     maxit, normB);
    }
    if (res_hist) {
      const size_t k = std::min<size_t>(so.hist.size(), (size_t)hist_len);
      memcpy(res_hist, so.hist.data(), sizeof(double) * k);
    }
    if (iters) *iters = so.iters;
    if (trr) *trr = (normB > 0.0 && std::isfinite(normB)) ? true_relres(c, A64, Bz, (int)ldb, Xz, (int)ldx, normB) : 0.0;
    HIPCHK(hipStreamSynchronize(s));
    if (so.status == ST_MAXIT) {
      fail(BLK_MAXIT, "no convergence within %d iterations", maxit);
      return BLK_MAXIT;
    }
    if (so.status == ST_BREAKDOWN) {
      if (g_err.empty()) fail(BLK_BREAKDOWN, "breakdown after %d iterations", so.iters);
      return BLK_BREAKDOWN;
    }
    return BLK_CONVERGED;
  } catch (const HipError& e) {
    if (e.e == hipErrorOutOfMemory) return fail(BLK_ENOMEM, "%s: %s", e.what, hipGetErrorString(e.e));
    return fail(BLK_EHIP, "%s: %s", e.what, hipGetErrorString(e.e));
  }
}

}  // namespace blk

using namespace blk;

extern "C" {

int32_t blk_cocg_solve(const blk_op* A, int64_t p, const blk_z* B, int64_t ldb, const blk_z* X0,
                       int64_t ldx0, double tol, int32_t maxit, const blk_opts* opts, blk_z* X,
                       int64_t ldx, double* res_hist, int32_t* iters, double* true_relres) {
  return solve_entry(false, A, p, B, ldb, X0, ldx0, tol, maxit, opts, X, ldx, res_hist, iters,
                     true_relres);
}

int32_t blk_cocr_solve(const blk_op* A, int64_t p, const blk_z* B, int64_t ldb, const blk_z* X0,
                       int64_t ldx0, double tol, int32_t maxit, const blk_opts* opts, blk_z* X,
                       int64_t ldx, double* res_hist, int32_t* iters, double* true_relres) {
  return solve_entry(true, A, p, B, ldb, X0, ldx0, tol, maxit, opts, X, ldx, res_hist, iters,
                     true_relres);
}

int32_t blk_op_analyze(blk_op* A, void* stream) {
  g_err.clear();
  if (!A) return fail(BLK_EINVAL, "A is NULL");
  const int32_t saved = A->structure;
  A->structure = BLK_STRUCT_UNKNOWN;
  int rc = check_op(A);
  if (rc) {
    A->structure = saved;
    return rc;
  }
  try {
    int64_t d[3] = {0, 0, 0};
    if (analyze_grid(A, (hipStream_t)stream, d)) {
      A->structure = BLK_STRUCT_GRID;
      for (int k = 0; k < 3; ++k) A->grid[k] = d[k];
    } else {
      A->structure = BLK_STRUCT_GENERAL;
      for (int k = 0; k < 3; ++k) A->grid[k] = 0;
    }
    return BLK_OK;
  } catch (const HipError& e) {
    A->structure = saved;
    if (e.e == hipErrorOutOfMemory) return fail(BLK_ENOMEM, "%s: %s", e.what, hipGetErrorString(e.e));
    return fail(BLK_EHIP, "%s: %s", e.what, hipGetErrorString(e.e));
  }
}

int32_t blk_spmm_z(const blk_op* A, int64_t p, const blk_z* Z, int64_t ldz, const blk_z* C,
                   int64_t ldc, blk_z* Y, int64_t ldy, blk_z* gram, void* stream) {
  g_err.clear();
  int rc = check_op(A);
  if (rc) return rc;
  if (p < 1 || p > BLK_MAX_P) return fail(BLK_EINVAL, "p outside 1..%d", BLK_MAX_P);
  if (!Z || !Y) return fail(BLK_EINVAL, "Z or Y is NULL");
  if (ldz < p || ldy < p || (C && ldc < p)) return fail(BLK_EINVAL, "leading dimension < p");
  const int64_t n = A->n;
  if (overlaps(Y, sizeof(blk_z) * ((n - 1) * ldy + p), Z, sizeof(blk_z) * ((n - 1) * ldz + p)))
    return fail(BLK_EINVAL, "Y overlaps Z");
  hipStream_t s = (hipStream_t)stream;
  try {
    Pool pool;
    Ctx c;
    DevOp<double> A64 = op64(A);
    const int E2 = 2 * (int)(p * p);
    const z64* Zz = reinterpret_cast<const z64*>(Z);
    const z64* Cz = reinterpret_cast<const z64*>(C);
    z64* Yz = reinterpret_cast<z64*>(Y);
    if (gram) {
      ctx_alloc(c, pool, n, (int)p, 0, s);
      // gate -1 with a fresh running state
      k_state_init<<<1, 64, 0, s>>>(c.st, (int)p, 0, 1.0, INFINITY);
      LAUNCH_CHECK();
    } else {
      // no workspace (CSR): the product alone, asynchronous on `stream`
      ctx_geometry(c, n, (int)p, s);
    }
    // a dense operator at p > 16 needs the split-K partials
    if (A->kind == BLK_OP_DENSE && p > 16) c.dws = pool.get<z64>(sizeof(z64) * (size_t)DSPLIT * n * 32);
    if (gram) {
      if (C)
        apply_op<double, true, true, true, false>(c, A64, Zz, (int)ldz, Cz, (int)ldc, Yz, (int)ldy,
                                                  RO_S, E2, -1);
      else
        apply_op<double, false, true, true, false>(c, A64, Zz, (int)ldz, nullptr, 0, Yz, (int)ldy,
                                                   RO_S, E2, -1);
      Red g = finish(c, RO_S, E2, 0, -1);
      std::vector<double> h((size_t)g.nrows * g.ld);
      HIPCHK(hipMemcpyAsync(h.data(), g.base, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int e = 0; e < (int)(p * p); ++e) {
        double re = 0, im = 0;
        for (int k = 0; k < g.nrows; ++k) {
          re += h[(size_t)k * g.ld + 2 * e];
          im += h[(size_t)k * g.ld + 2 * e + 1];
        }
        gram[e].re = re;
        gram[e].im = im;
      }
    } else {
      if (C)
        apply_op<double, true, true, false, false>(c, A64, Zz, (int)ldz, Cz, (int)ldc, Yz, (int)ldy,
                                                   RO_S, 0, -1);
      else
        apply_op<double, false, true, false, false>(c, A64, Zz, (int)ldz, nullptr, 0, Yz, (int)ldy,
                                                    RO_S, 0, -1);
    }
    if (gram || c.dws) HIPCHK(hipStreamSynchronize(s));  // before the workspace is freed
    return BLK_OK;
  } catch (const HipError& e) {
    if (e.e == hipErrorOutOfMemory) return fail(BLK_ENOMEM, "%s: %s", e.what, hipGetErrorString(e.e));
    return fail(BLK_EHIP, "%s: %s", e.what, hipGetErrorString(e.e));
  }
}

int32_t blk_spmm_c(const blk_op* A, const blk_c* vals32, int64_t p, const blk_c* Z, int64_t ldz,
                   blk_c* Y, int64_t ldy, void* stream) {
  g_err.clear();
  int rc = check_op(A, false);
  if (rc) return rc;
  if (!vals32) return fail(BLK_EINVAL, "vals32 is NULL");
  if (p < 1 || p > BLK_MAX_P) return fail(BLK_EINVAL, "p outside 1..%d", BLK_MAX_P);
  if (!Z || !Y) return fail(BLK_EINVAL, "Z or Y is NULL");
  if (ldz < p || ldy < p) return fail(BLK_EINVAL, "leading dimension < p");
  const int64_t n = A->n;
  if (overlaps(Y, sizeof(blk_c) * ((n - 1) * ldy + p), Z, sizeof(blk_c) * ((n - 1) * ldz + p)))
    return fail(BLK_EINVAL, "Y overlaps Z");
  hipStream_t s = (hipStream_t)stream;
  try {
    Pool pool;
    Ctx c;
    ctx_geometry(c, n, (int)p, s);
    DevOp<float> A32;
    A32.kind = A->kind;
    A32.n = n;
    if (A->kind == BLK_OP_CSR) {
      A32.rowptr = A->rowptr;
      A32.colind = A->colind;
      A32.val = reinterpret_cast<const c32*>(vals32);
      if (A->structure == BLK_STRUCT_GRID) {
        A32.gnx = (int)A->grid[0];
        A32.gny = (int)A->grid[1];
        A32.gnz = (int)A->grid[2];
      }
    } else {
      A32.dense = reinterpret_cast<const c32*>(vals32);
      A32.ld = A->ld;
      // p > 16: the matrix-core product needs the split-K partials
      if (p > 16) c.dws = pool.get<z64>(sizeof(z64) * (size_t)DSPLIT * n * 32);
    }
    apply_op<float, false, true, false, false>(c, A32, reinterpret_cast<const c32*>(Z), (int)ldz,
                                               nullptr, 0, reinterpret_cast<c32*>(Y), (int)ldy,
                                               RO_S, 0, -1);
    if (c.dws) HIPCHK(hipStreamSynchronize(s));  // before the workspace is freed
    return BLK_OK;
  } catch (const HipError& e) {
    if (e.e == hipErrorOutOfMemory) return fail(BLK_ENOMEM, "%s: %s", e.what, hipGetErrorString(e.e));
    return fail(BLK_EHIP, "%s: %s", e.what, hipGetErrorString(e.e));
  }
}

int32_t blk_gram_z(int64_t n, int64_t p, const blk_z* Y, int64_t ldy, const blk_z* Z, int64_t ldz,
                   int32_t conj, blk_z* Gout, void* stream) {
  g_err.clear();
  if (n < 1 || n > (int64_t)0x7fffffff) return fail(BLK_EINVAL, "bad n");
  if (p < 1 || p > BLK_MAX_P) return fail(BLK_EINVAL, "p outside 1..%d", BLK_MAX_P);
  if (!Y || !Z || !Gout) return fail(BLK_EINVAL, "NULL pointer");
  if (ldy < p || ldz < p) return fail(BLK_EINVAL, "leading dimension < p");
  hipStream_t s = (hipStream_t)stream;
  try {
    Pool pool;
    Ctx c;
    ctx_alloc(c, pool, n, (int)p, 0, s);
    k_state_init<<<1, 64, 0, s>>>(c.st, (int)p, 0, 1.0, INFINITY);
    LAUNCH_CHECK();
    const z64* Yz = reinterpret_cast<const z64*>(Y);
    const z64* Zz = reinterpret_cast<const z64*>(Z);
    Red g = conj ? gram<double, double, G_CONJ, false>(c, Yz, (int)ldy, Zz, (int)ldz, RO_A, -1)
                 : gram<double, double, G_UNCONJ, false>(c, Yz, (int)ldy, Zz, (int)ldz, RO_A, -1);
    std::vector<double> h((size_t)g.nrows * g.ld);
    HIPCHK(hipMemcpyAsync(h.data(), g.base, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int e = 0; e < (int)(p * p); ++e) {
      double re = 0, im = 0;
      for (int k = 0; k < g.nrows; ++k) {
        re += h[(size_t)k * g.ld + 2 * e];
        im += h[(size_t)k * g.ld + 2 * e + 1];
      }
      Gout[e].re = re;
      Gout[e].im = im;
    }
    return BLK_OK;
  } catch (const HipError& e) {
    if (e.e == hipErrorOutOfMemory) return fail(BLK_ENOMEM, "%s: %s", e.what, hipGetErrorString(e.e));
    return fail(BLK_EHIP, "%s: %s", e.what, hipGetErrorString(e.e));
  }
}

int32_t blk_thin_qr_z(int64_t n, int64_t p, const blk_z* W, int64_t ldw, blk_z* Q, int64_t ldq,
                      blk_z* Rout, void* stream) {
  g_err.clear();
  if (n < 1 || n > (int64_t)0x7fffffff) return fail(BLK_EINVAL, "bad n");
  if (p < 1 || p > BLK_MAX_P) return fail(BLK_EINVAL, "p outside 1..%d", BLK_MAX_P);
  if (!W || !Q || !Rout) return fail(BLK_EINVAL, "NULL pointer");
  if (ldw < p || ldq < p) return fail(BLK_EINVAL, "leading dimension < p");
  if (W != Q &&
      overlaps(W, sizeof(blk_z) * ((n - 1) * ldw + p), Q, sizeof(blk_z) * ((n - 1) * ldq + p)))
    return fail(BLK_EINVAL, "Q partially overlaps W");
  if (W == Q && ldw != ldq) return fail(BLK_EINVAL, "Q aliases W with a different ld");
  hipStream_t s = (hipStream_t)stream;
  try {
    Pool pool;
    Ctx c;
    ctx_alloc(c, pool, n, (int)p, 0, s);
    k_state_init<<<1, 64, 0, s>>>(c.st, (int)p, 1, 0.0, INFINITY);
    LAUNCH_CHECK();
    const z64* Wz = reinterpret_cast<const z64*>(W);
    z64* Qz = reinterpret_cast<z64*>(Q);
    Red g1 = gram<double, double, G_CONJ, false>(c, Wz, (int)ldw, Wz, (int)ldw, RO_A, -1);
    // The state's tol is 0, so only a failed factorization stops the run.
    cholqr<double, double, false>(c, g1, const_cast<z64*>(Wz), (int)ldw, Qz, (int)ldq, -1, 0, 0, 1);
    DevState h = read_state(c);
    if (h.stop_iter == 0) return fail(BLK_BREAKDOWN, "block is numerically rank deficient");
    HIPCHK(hipMemcpyAsync(Rout, c.slots + S_XI * SLOT, sizeof(z64) * (size_t)(p * p),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return BLK_OK;
  } catch (const HipError& e) {
    if (e.e == hipErrorOutOfMemory) return fail(BLK_ENOMEM, "%s: %s", e.what, hipGetErrorString(e.e));
    return fail(BLK_EHIP, "%s: %s", e.what, hipGetErrorString(e.e));
  }
}

const char* blk_last_error(void) { return g_err.c_str(); }

const char* blk_version(void) { return "blk-mi355x 0.1 (gfx950)"; }

}  // extern "C"
