/*
 * blk.h -- C ABI of the MI355X block COCG / block COCR solver library.
 *
 * Method: Gu, Carpentieri, Huang, Meng, "Block variants of the COCG and COCR
 * methods for solving complex symmetric linear systems with multiple
 * right-hand sides" (arXiv 1601.05362).  The problem is eq. (1.1):
 * A X = B with A complex symmetric (A = A^T, A != A^H), X, B of size n x p,
 * p << n.
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer (memory of the current HIP
 *     device) unless its comment says [host].
 *   - Complex values are interleaved (re, im) pairs: blk_z is complex128 and
 *     blk_c is complex64, bit-compatible with torch.complex128/complex64 and
 *     hipDoubleComplex/hipFloatComplex.
 *   - Blocks of p right-hand sides are row-major n x p with a leading
 *     dimension ld >= p (element (i, j) at ptr[i*ld + j]); a contiguous
 *     torch tensor of shape (n, p) has ld = p.
 *   - The caller owns every pointer it passes.  The library allocates its
 *     own device workspace for the duration of a call, frees it before
 *     returning and keeps no caller pointer.
 *   - Calls are ordered on `stream` (a hipStream_t; NULL = the legacy
 *     default stream) after work already queued there.  The solvers, the
 *     Gram, the thin QR and blk_spmm_z with a gram output return only when
 *     their outputs are final (host-blocking); the plain products are queued
 *     and return at once.
 *   - The return value is a blk_status.  On BLK_EINVAL nothing was launched
 *     and outputs are untouched; blk_last_error() describes any status other
 *     than BLK_CONVERGED (BLK_OK for the non-iterative calls).
 *   - p must satisfy 1 <= p <= BLK_MAX_P.
 */
#ifndef BLK_H
#define BLK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BLK_MAX_P 32

typedef struct { double re, im; } blk_z; /* complex128 */
typedef struct { float re, im; } blk_c;  /* complex64 */

/* Operator kinds. */
enum { BLK_OP_CSR = 0, BLK_OP_DENSE = 1 };

/* Pattern knowledge of a CSR operator (blk_op.structure). */
enum {
  BLK_STRUCT_UNKNOWN = 0, /* the solvers analyse the pattern once per call
                             (blk_op_analyze); single products use the
                             general CSR kernel */
  BLK_STRUCT_GENERAL = 1, /* never analyse: always the general CSR kernel */
  BLK_STRUCT_GRID = 2     /* the pattern is the 7-point stencil of the
                             lexicographic grid[0] x grid[1] x grid[2] grid
                             (x fastest; 5-point when grid[2] == 1), columns
                             ascending within each row.  Set by
                             blk_op_analyze after checking every row; a
                             caller that sets it guarantees the pattern. */
};

/* The matrix A of eq. (1.1).  Symmetry (A = A^T) is the caller's promise and
 * is not checked on the device.
 *   CSR:   0-based int32 rowptr[n+1], colind[nnz], complex128 val[nnz];
 *          column indices need not be sorted; a row may be empty.
 *   DENSE: row-major complex128 `dense` with leading dimension ld >= n.
 * structure / grid: see BLK_STRUCT_*; ignored for DENSE.  With
 * BLK_STRUCT_GRID the CSR values are still read (any coefficients); the
 * column indices are not. */
typedef struct {
  int32_t kind;
  int32_t structure;
  int64_t n;
  int64_t nnz;
  const int32_t *rowptr;
  const int32_t *colind;
  const blk_z *val;
  const blk_z *dense;
  int64_t ld;
  int64_t grid[3];
} blk_op;

/* Arithmetic of a solve. */
enum {
  BLK_FP64 = 0,  /* every step in complex128 / FP64 */
  BLK_MIXED = 1  /* complex64 inner solver under FP64 iterative refinement */
};

/* Options; pass NULL for all defaults. */
typedef struct {
  int32_t rq;          /* 1 (default): residual orthonormalization (Algorithms 2-3);
                          0: plain block COCG / block COCR (Algorithm 1). */
  int32_t precision;   /* BLK_FP64 (default) or BLK_MIXED. */
  double inner_tol;    /* BLK_MIXED: relative tolerance of each inner solve
                          (default 1e-3). */
  int32_t inner_maxit; /* BLK_MIXED: iteration cap of one inner solve
                          (default: maxit). */
  int32_t check_every; /* iterations between host convergence checks
                          (default 16); does not change results. */
  int32_t refine;      /* restarts allowed when the monitored residual has
                          reached tol but the true FP64 residual ||B - A X||_F
                          / ||B||_F has not (rounding drift of the recurrences);
                          each restart solves again from the current X.
                          0 (default): stop on the monitored residual as the
                          algorithms do. */
  void *stream;        /* hipStream_t, NULL = legacy default stream. */
} blk_opts;

typedef enum {
  BLK_CONVERGED = 0,  /* ||R_m||_F / ||B||_F <= tol */
  BLK_OK = 0,         /* success of a non-iterative call */
  BLK_MAXIT = 1,      /* maxit iterations done without reaching tol */
  BLK_BREAKDOWN = 2,  /* singular p x p system or rank-deficient residual block */
  BLK_EINVAL = -1,    /* invalid argument; nothing was launched */
  BLK_ENOMEM = -2,    /* device workspace allocation failed */
  BLK_EHIP = -3       /* a HIP runtime call failed */
} blk_status;

/*
 * Block COCG (rq = 0: recurrences of section 2.1 with the COCG conditions of
 * Table 1) or block COCG with residual orthonormalization (rq = 1,
 * Algorithm 2): solve A X = B for X.
 *
 *   A          operator (see blk_op).
 *   p          number of right-hand sides, 1..BLK_MAX_P.
 *   B, ldb     right-hand sides, n x p.
 *   X0, ldx0   initial guess, n x p; NULL means X0 = 0.
 *   tol        stop when ||R_m||_F / ||B||_F <= tol (> 0), tested before each
 *              iteration; with rq = 1 the norm is monitored as ||xi_m||_F
 *              (section 2.2).
 *   maxit      iteration cap (>= 0).  One iteration is one loop body of the
 *              algorithm (one operator application).
 *   opts       options or NULL.
 *   X, ldx     output n x p; may alias X0 (same pointer and ld), must not
 *              overlap B.
 *   res_hist   [host] double[maxit + 1] or NULL: res_hist[m] is the monitored
 *              relative residual of iterate m, m = 0..*iters.  BLK_MIXED
 *              writes the inner estimates scaled to ||B||_F, one per inner
 *              iteration, so it then needs room for maxit + 1 entries too.
 *              After a refine restart the entries continue with the
 *              restarted run's monitored residuals (relative to ||B||_F).
 *   iters      [host] number of iterations done (total inner iterations
 *              for BLK_MIXED), or NULL.
 *   true_relres [host] ||B - A X||_F / ||B||_F of the returned X computed in
 *              FP64 (the paper's TRR before log10), or NULL.
 *
 * Returns BLK_CONVERGED, BLK_MAXIT (X is the last iterate), BLK_BREAKDOWN
 * (X is the last valid iterate) or an error.  ||B||_F = 0 gives X = 0,
 * *iters = 0 and BLK_CONVERGED.
 */
int32_t blk_cocg_solve(const blk_op *A, int64_t p, const blk_z *B, int64_t ldb, const blk_z *X0,
                       int64_t ldx0, double tol, int32_t maxit, const blk_opts *opts, blk_z *X,
                       int64_t ldx, double *res_hist, int32_t *iters, double *true_relres);

/*
 * Block COCR (rq = 0, Algorithm 1) or block COCR with residual
 * orthonormalization (rq = 1, Algorithm 3).  Arguments, outputs and status as
 * for blk_cocg_solve.
 */
int32_t blk_cocr_solve(const blk_op *A, int64_t p, const blk_z *B, int64_t ldb, const blk_z *X0,
                       int64_t ldx0, double tol, int32_t maxit, const blk_opts *opts, blk_z *X,
                       int64_t ldx, double *res_hist, int32_t *iters, double *true_relres);

/*
 * The operator application A Z of every iteration (the block product the
 * paper counts as the cost of one step, section 1), complex128:
 * Y = A Z, or Y = C - A Z when C is not NULL.  If gram is not NULL it receives
 * [host] the unconjugated p x p form Z^T Y, row-major complex128.
 * Y must not overlap Z.  Returns BLK_OK or an error.  Without gram the call
 * allocates nothing and does not wait: the product is queued on `stream` --
 * except for a DENSE operator with p > 16, whose matrix-core product needs a
 * split-K workspace (4 n 32 complex128): that call allocates it and returns
 * when the product is done.
 */
int32_t blk_spmm_z(const blk_op *A, int64_t p, const blk_z *Z, int64_t ldz, const blk_z *C,
                   int64_t ldc, blk_z *Y, int64_t ldy, blk_z *gram, void *stream);

/*
 * Pattern analysis of A (section 3's operators are grid stencils): sets
 * A->structure to BLK_STRUCT_GRID and A->grid to (nx, ny, nz) when every row
 * of the CSR pattern is that of the 7-point (nz > 1) or 5-point (nz == 1)
 * stencil of a lexicographic grid with nx, ny >= 2, else to
 * BLK_STRUCT_GENERAL (always for DENSE).  Reads rowptr and colind once on
 * the device; host-blocking; allocates a 4-byte flag.  The result stays
 * valid while the pattern (not the values) is unchanged.
 */
int32_t blk_op_analyze(blk_op *A, void *stream);

/*
 * The block product of section 1 in complex64, as the mixed-precision form's
 * inner solves use it: Y = A Z with A's pattern, kind and structure from *A and its
 * values in complex64 from vals32 -- for CSR, vals32[nnz] in the order of
 * colind; for DENSE, the row-major n x n matrix with leading dimension
 * A->ld (A->val / A->dense are not read and may be NULL).  FP32
 * accumulation; a DENSE operator at p > 16 runs on the FP32 matrix cores, a
 * CSR operator marked BLK_STRUCT_GRID on the 2.5D stencil kernel (nothing is
 * analysed here: BLK_STRUCT_UNKNOWN takes the general kernel).  Y must not
 * overlap Z.  Allocates nothing and does not wait -- except for a DENSE
 * operator with p > 16, whose product needs a split-K workspace (4 n 32
 * complex128-sized entries): that call allocates it and returns when the
 * product is done.  Returns BLK_OK or an error.
 */
int32_t blk_spmm_c(const blk_op *A, const blk_c *vals32, int64_t p, const blk_c *Z, int64_t ldz,
                   blk_c *Y, int64_t ldy, void *stream);

/*
 * p x p bilinear form of two n x p blocks, complex128, written [host]
 * row-major to G: G = Y^T Z (conj = 0, the unconjugated form of Table 1)
 * or G = Y^H Z (conj = 1).
 */
int32_t blk_gram_z(int64_t n, int64_t p, const blk_z *Y, int64_t ldy, const blk_z *Z,
                   int64_t ldz, int32_t conj, blk_z *G, void *stream);

/*
 * Thin QR W = Q R of an n x p block (the residual orthonormalization of
 * section 2.2) by two passes of Cholesky QR, complex128.  R [host] is p x p
 * upper triangular with a real positive diagonal, Q^H Q = I.  Q may alias W.
 * Returns BLK_BREAKDOWN when W is numerically rank deficient (a Cholesky
 * pivot <= 1e-14 times the largest squared column norm).
 */
int32_t blk_thin_qr_z(int64_t n, int64_t p, const blk_z *W, int64_t ldw, blk_z *Q, int64_t ldq,
                      blk_z *R, void *stream);

/* Message for the last status other than BLK_OK/BLK_CONVERGED on this
 * thread ("" if none).  The pointer stays valid until the next call on the
 * same thread. */
const char *blk_last_error(void);

/* Library version string. */
const char *blk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BLK_H */
