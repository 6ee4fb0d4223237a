/*
 * blrqr — Householder QR of Block Low-Rank (BLR) matrices on AMD MI355X (gfx950).
 *
 * C ABI of libblrqr.so.  All entry points return a blr_status and never throw
 * or abort; blr_last_error() gives a thread-local description of the last
 * failure.  Method: Apriansyah & Yokota, "Parallel QR Factorization of Block
 * Low-Rank Matrices" (arXiv 2208.06194).
 *
 * Storage model.  A BLR matrix A~ (m x n, m >= n) has p x q tiles of size
 * b x b (p = ceil(m/b), q = ceil(n/b)).  Tile (i,j) is dense or low-rank
 * U V^T with U orthonormal (Section 3.1, eq. blr_matrix_def).  When b does
 * not divide m or n (the rectangular edge blocks Section 3.1 allows), the
 * last tile row and column hold fewer rows and columns of A~, and the
 * library factors the embedding [A~ 0; 0 E] of m_pad x n_pad (blr_info):
 * zero rows and columns fill the edge tiles to b x b, and E is an identity
 * block in the padded columns on padded rows (with one more tile row when
 * the padded rows are too few).  Its R is diag(R, -I) up to row signs, its
 * thin factor is [Q1; 0], and its least-squares solution for [b; 0] is
 * [x; 0]: the solve, products and R solves take and return the caller's m-
 * and n-row blocks; Q^T B (blr_apply_qt) acts on m_pad rows.  The
 * handle owns every device buffer (tiles, reflectors, T factors, workspace).
 * Device pointers passed in are borrowed until the work enqueued on the
 * given stream completes; the library copies what it keeps.  Calls on one
 * handle must be serialised by the caller; different handles are independent.
 *
 * Synchronisation and workspace.  Each handle keeps a grow-only device
 * workspace for its plans and temporaries, reused by every later call (a
 * call that repeats an earlier call's shapes allocates nothing), and records
 * an event on the caller's stream at the end of each call's work.  A call
 * that reuses the workspace, or reads results back, first waits on the host
 * for that event: for this handle's previous work only.  No entry point
 * waits for the whole device.  Where a declaration below says "synchronises
 * the stream", the call returns after its own work on hip_stream is done.
 *
 * Errors.  Argument errors are detected synchronously before any work is
 * enqueued.  A device fault surfaces as BLR_ERR_DEVICE at the next call that
 * synchronises.  Truncation at the rank cap is not an error: it is counted in
 * blr_info.
 */
#ifndef BLRQR_H
#define BLRQR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum blr_status {
  BLR_OK = 0,
  BLR_ERR_INVALID = 1,   /* bad argument (null, m < n, tol <= 0, ...) */
  BLR_ERR_STATE = 2,     /* call not valid in the handle's state (e.g. factor twice) */
  BLR_ERR_OOM = 3,       /* device allocation failed */
  BLR_ERR_DEVICE = 4,    /* HIP runtime or kernel error (text in blr_last_error) */
  BLR_ERR_NONFINITE = 5, /* NaN or Inf in the input matrix */
  BLR_ERR_SINGULAR = 6   /* least squares: some |R_jj| <= n * u * ||R||_F */
} blr_status;

typedef struct blr_matrix_s* blr_matrix;

/* Source of the matrix for blr_compress. */
enum { BLR_SRC_KERNEL = 0, BLR_SRC_DENSE = 1 };
/* Kernel functions: A_ij = f(|x_i - y_j|). */
enum { BLR_KERNEL_LOG2D = 0 /* -log(d + reg) */, BLR_KERNEL_INV_R = 1 /* 1/(d + reg) */ };
/* Admissibility rules (Section 3.1).  Diagonal tiles (k,k), k < q, are always dense.
 * ADJACENT:      dense iff the cluster boxes touch (Euclidean gap 0).
 * DIST_GT_DIAM:  low-rank iff gap > max(diameter of the two boxes).
 * WEAK:          every off-diagonal tile is low-rank.
 * MASK:          caller-supplied p x q mask. */
enum { BLR_ADM_ADJACENT = 0, BLR_ADM_DIST_GT_DIAM = 1, BLR_ADM_WEAK = 2, BLR_ADM_MASK = 3 };
/* What compression does with a tile whose eps-rank exceeds max_rank. */
enum { BLR_OVERFLOW_DENSE = 0, BLR_OVERFLOW_TRUNCATE = 1 };
/* Factorization variants: tiled (Alg. 4, Section 3.4) and block-column (Alg. 2, Section 3.3). */
enum { BLR_TILED = 0, BLR_BLOCK_COLUMN = 1 };
/* Precision: all FP64, or reflector-apply products in FP32 on the matrix
 * cores (FP32 inputs, FP32 accumulation) with reflector generation, the R
 * diagonal and every recompression in FP64. */
enum { BLR_FP64 = 0, BLR_MIXED_FP32 = 1 };
/* Handle states. */
enum { BLR_STATE_COMPRESSED = 0, BLR_STATE_FACTORED = 1 };

typedef struct blr_source {
  int32_t kind;             /* BLR_SRC_KERNEL or BLR_SRC_DENSE */
  /* KERNEL: device pointers to row points x (m x dim) and column points
   * y (n x dim), row-major FP64, used in the order given (callers sort them,
   * e.g. in Morton order, so that consecutive points are close). */
  const double* x;
  const double* y;
  int32_t dim;              /* 2 or 3 */
  int32_t kernel;           /* BLR_KERNEL_* */
  double reg;               /* regularisation added to the distance (1e-3) */
  /* DENSE: device pointer to A, column-major, leading dimension lda >= m. */
  const double* A;
  int64_t lda;
  /* Admissibility (BLR_ADM_*).  ADJACENT and DIST_GT_DIAM need KERNEL. */
  int32_t admissibility;
  /* MASK: host array p*q, element i*q + j, nonzero = low-rank. */
  const int8_t* mask;
} blr_source;

typedef struct blr_compress_opts {
  int64_t m, n;             /* matrix size, m >= n >= 1 */
  int32_t tile;             /* b: 16 <= b <= 1024, multiple of 16 (need not divide m or n) */
  double tol;               /* eps > 0: per-tile ||A~_ij - A_ij||_F <= eps ||A_ij||_F */
  int32_t max_rank;         /* rank cap, 1 <= max_rank <= min(b, 128) */
  int32_t overflow;         /* BLR_OVERFLOW_* */
  uint64_t seed;            /* seed of the random test matrix of the range finder */
} blr_compress_opts;

typedef struct blr_factor_opts {
  int32_t variant;          /* BLR_TILED or BLR_BLOCK_COLUMN */
  int32_t precision;        /* BLR_FP64 or BLR_MIXED_FP32 */
  int32_t ib;               /* widest inner block of reflector generation: 16 or 32 (0 = 32);
                               panels taller than 512 rows use 16 whatever is asked */
  int32_t stop_after_k;     /* debug: factor only block columns 0..K-1 (-1 = all) */
  int32_t keep_a;           /* 1: keep a device copy of A~ (doubles the tile memory) so that
                               blr_matmul with A~ and refined least squares work after the
                               in-place factorization; 0: no copy */
} blr_factor_opts;

typedef struct blr_info {
  int64_t m, n;
  int32_t tile, p, q;
  int32_t max_rank;         /* truncation cap */
  int32_t rank_capacity;    /* columns of a low-rank slot (max_rank rounded up to 16) */
  int32_t state;            /* BLR_STATE_* */
  int32_t variant, precision, ib;
  int64_t n_dense, n_lowrank;     /* current tile formats */
  int64_t n_fill_in;              /* low-rank tiles turned dense by the factorization */
  int64_t device_bytes;           /* device memory owned by the handle */
  int64_t compress_overflow;      /* tiles whose eps-rank exceeded max_rank at compression */
  int64_t factor_overflow;        /* recompressions truncated at the cap during the factor */
  double max_dropped_rel;         /* largest dropped relative singular-value tail */
  double flops_factor;            /* algorithmic flops of the last factorization */
  int64_t kernel_launches;        /* kernels enqueued by the last factorization */
  /* The matrix the kernels factor: m_pad x n_pad in p_pad x q tiles.  It
   * equals m x n when b divides both; otherwise it is the embedding
   * [A 0; 0 E] (zero rows and columns up to whole tiles, E an identity block
   * in the padded columns on padded rows, one more tile row if the padded
   * rows are too few), whose R is diag(R_A, -I) and whose least-squares
   * solution for [b; 0] is [x; 0]. */
  int64_t m_pad, n_pad;
  int32_t p_pad;
  int32_t pad_;
} blr_info;

/* Host copies of the tile data (blr_import / blr_export).  Every array is
 * caller-owned and sized for all p*q tiles of A~ (p = ceil(m/b) tile rows:
 * a tile row that only the embedding adds is neither read nor written),
 * tile t = i*q + j; an edge tile holds A~'s entries in its leading rows and
 * columns (the rest is ignored on import, and holds the embedding's
 * entries on export):
 *   fmt   [p*q]          0 = dense, 1 = low-rank
 *   rank  [p*q]          rank of low-rank tiles (ignored for dense tiles)
 *   dense [p*q*b*b]      tile t at t*b*b, column-major b x b
 *   U     [p*q*b*rc]     tile t at t*b*rc, column-major b x rc (first rank columns used)
 *   V     [p*q*b*rc]     tile t at t*b*rc, column-major b x rc, so A_ij = U V^T
 * rc = blr_info.rank_capacity.  After the factorization, export also fills
 *   Y     [p*q*rc*b]     for low-rank tiles below the diagonal: the reflector rows
 *                        Y_ik (rc x b, column-major), with Ytilde_ik = U_ik Y_ik
 *   T     [p*q*b*b]      tiled: T of tile (i,k), i >= k;  block column: T_k at tile (k,k)
 * and dense holds R (upper part of diagonal tiles, tiles right of the
 * diagonal) and the dense reflector blocks Y (strict lower part of diagonal
 * tiles, dense tiles below the diagonal).  Pointers may be NULL to skip. */
typedef struct blr_tiles_host {
  int8_t* fmt;
  int32_t* rank;
  double* dense;
  double* U;
  double* V;
  double* Y;
  double* T;
} blr_tiles_host;

/* The explicit orthogonal factor Q~ of a factored handle as a new BLR handle
 * (Section 3.3: Q~ is a BLR matrix with the structure of A~, its admissible
 * blocks approximated at the same threshold).  The thin Q [I_n; 0] (m x n)
 * is formed on the device, a block of 4096 columns at a time, then
 * compressed with the tile formats A~ had when the factor started as the
 * mask, tolerance and rank cap of A~ (a block whose rank exceeds the cap is
 * stored dense).  Needs m*n*8 bytes of temporary device memory, stream-ordered
 * (allocated and freed on hip_stream).  *q_out is a new handle in state
 * COMPRESSED (its products and export work as for A~).  Synchronises the
 * stream.  Errors: BLR_ERR_STATE if not (fully) factored; BLR_ERR_INVALID
 * when b does not divide m or n. */
blr_status blr_form_q(blr_matrix h, void* hip_stream, blr_matrix* q_out);

/* Blocked modified Gram-Schmidt QR of the BLR matrix: the method the paper
 * compares its Householder algorithms with (Section 2.1 Alg. 1, Section
 * 3.2).  For each block column j: the right factors of its tiles (dense:
 * the tile; low-rank U V^T: V^T) are stacked over every block row and
 * orthogonalized by column-by-column MGS, Q_ij = U_ij Q^B_ij keeps the
 * tile's U, and R_jk = Q_j^T A_k, A_k -= Q_j R_jk (k > j) run in BLR
 * arithmetic (a low-rank tile receiving a dense update becomes dense).
 * h must be COMPRESSED with b dividing m and n.  On return h holds the
 * explicit Q~ (state COMPRESSED: products and export work as for A~) and
 * *r_out is a new n x n handle holding R~ (dense upper triangular diagonal
 * tiles, R_jk dense or low-rank, zero tiles below the diagonal).  The
 * stack QR runs in one workgroup per block column: an accuracy comparison
 * path, not a fast one.  Synchronises the stream.  Errors: BLR_ERR_STATE if
 * h is not COMPRESSED, BLR_ERR_INVALID if b does not divide m or n. */
blr_status blr_mgs_qr(blr_matrix h, void* hip_stream, blr_matrix* r_out);

/* X <- R^{-1} X (trans = 0) or X <- R^{-T} X (trans = 1) with the R factor of
 * a factored handle (Section 3.3 / 3.4: R has the tile structure of A~), for
 * X n x nrhs, column-major, device, ld ldx >= n, overwritten.  The blocked
 * back- or forward substitution of the least-squares solve.  Asynchronous on
 * hip_stream.  Errors: BLR_ERR_STATE if not (fully) factored. */
blr_status blr_rsolve(blr_matrix h, int32_t trans, double* X, int64_t ldx, int32_t nrhs, void* hip_stream);

/* Adjoint of the least-squares solve X = argmin ||A~ X - B||_F (full column
 * rank; the use of the QR factorization that motivates the paper).  Given B
 * (m x nrhs), the solution X (n x nrhs) and Xbar = dL/dX (n x nrhs) for a
 * scalar loss L, computes Z = R^{-1} R^{-T} Xbar, the residual Rs = B - A~ X,
 *   Bbar = dL/dB = A~ Z                                (m x nrhs, ld ldbb)
 * and dL/dA~ = Rs Z^T - Bbar X^T restricted to the stored tiles of A~ (the
 * matrix as compressed, kept by a factor made with keep_a):
 *   dD: dense tile (i,j) gets its b x b block, column-major at offset
 *       (i*q + j)*b*b;
 *   dU, dV: low-rank tile U V^T (U, V b x rc as in blr_tiles_host) gets
 *       dU = dA_ij V and dV = dA_ij^T U, b x rc column-major at offset
 *       (i*q + j)*b*rc (columns past the rank are zero).
 * All pointers are device memory; dD, dU and dV may be NULL to skip, and
 * only the slots of tiles of the matching format are written.  Asynchronous
 * on hip_stream.  Errors: BLR_ERR_STATE if not factored or A~ was not kept;
 * BLR_ERR_INVALID when b does not divide m or n. */
blr_status blr_lstsq_adjoint(blr_matrix h, const double* B, int64_t ldb, const double* X, int64_t ldx,
                             const double* Xbar, int64_t ldxb, int32_t nrhs, double* Bbar, int64_t ldbb,
                             double* dD, double* dU, double* dV, void* hip_stream);

/* Morton (Z-order) ordering of n points (dim 1..3, row-major FP64, device
 * pointer pts), the input preparation of a kernel-matrix workload: tiles of
 * consecutive points in this order are spatially compact, so the
 * admissibility test of Section 3.1 finds far-field tiles.  Each coordinate
 * is quantised to 2^21 levels (floor(x * 2^21), clamped to [0, 2^21 - 1];
 * coordinates are expected in [0, 1)), the bits are interleaved most
 * significant first in coordinate order, and the points are sorted by key,
 * ties by original index.  perm (device, n int64, required) receives the
 * original index of the r-th point in that order; sorted (device, n x dim
 * row-major, may be NULL) receives the points in that order.  Its scratch is
 * stream-ordered device memory (allocated and freed on hip_stream), and the
 * call is asynchronous on hip_stream.  Errors:
 * BLR_ERR_INVALID for NULL pts/perm, n < 0 or dim outside 1..3. */
blr_status blr_morton_sort(const double* pts, int64_t n, int32_t dim, int64_t* perm, double* sorted,
                           void* hip_stream);

/* Compress a kernel or dense matrix into a new BLR handle (Section 3.1:
 * admissibility, then a truncated SVD of each admissible tile to the
 * smallest rank meeting the tolerance; U orthonormal, V = W Sigma).
 * Synchronises the stream (the tile formats are read back to plan the
 * factorization).  On success *out is a new handle in state COMPRESSED. */
blr_status blr_compress(const blr_source* src, const blr_compress_opts* opts,
                        void* hip_stream, blr_matrix* out);

/* Build a handle from host tiles (fmt, rank, dense, U, V of blr_tiles_host).
 * Only m, n, tile, tol, max_rank of opts are used.  Low-rank U must have
 * orthonormal columns (the factorization relies on it, Section 3.3.1).
 * Synchronises the stream. */
blr_status blr_import(const blr_compress_opts* opts, const blr_tiles_host* tiles,
                      void* hip_stream, blr_matrix* out);

/* Copy the handle's tiles to host arrays (see blr_tiles_host).  Waits for the
 * handle's previous work first. */
blr_status blr_export(blr_matrix h, blr_tiles_host* tiles);

/* Householder QR of the BLR matrix, in place (tiled: Alg. 4 with the
 * operations of Section 3.4; block column: Alg. 2 with Section 3.3).
 * The handle goes from COMPRESSED to FACTORED; a second call returns
 * BLR_ERR_STATE.  Enqueued on hip_stream (asynchronous). */
blr_status blr_qr_factor(blr_matrix h, const blr_factor_opts* opts, void* hip_stream);

/* Householder QR of count independent BLR matrices of any sizes, as one
 * batch (the block-column algorithm, Alg. 2 with Section 3.3, on each; the
 * task graph of Section 4.3 taken over the batch).  hs (host array) holds
 * count distinct handles in state COMPRESSED that share tile size, rank cap
 * and tolerance; opts->variant must be BLR_BLOCK_COLUMN, and precision,
 * keep_a and stop_after_k apply to every matrix.  The steps of all matrices
 * are merged so that one kernel launch serves the same step of many
 * matrices; each matrix ends exactly as blr_qr_factor with the same opts
 * leaves it (bit-identical factors, FACTORED state, own overflow counters;
 * blr_query reports the batch's launch count).  The matrices run in two
 * groups of about equal work, each group's merged launches on a stream of
 * hs[0] joined to hip_stream before and after.  Enqueued on hip_stream
 * (asynchronous); a group's merged launch list lives in the workspace of its
 * first member until that handle's next factorization or destruction (both
 * wait for the handle's previous work).  Errors: BLR_ERR_INVALID for NULL
 * arguments, count < 1, a repeated or NULL handle, unequal tile size, cap or
 * tolerance, or another variant; BLR_ERR_STATE if a handle is not
 * COMPRESSED.  If the call fails after validation, the handles stay
 * COMPRESSED but may hold fill-in slots and workspace. */
blr_status blr_qr_factor_batch(blr_matrix* hs, int32_t count, const blr_factor_opts* opts,
                               void* hip_stream);

/* B <- Q^T B (trans = 0) or B <- Q B (trans = 1), replaying the stored
 * reflectors (Alg. 3 / Alg. 5).  B: device, column-major m_pad x nrhs
 * (blr_info.m_pad, which is m when b divides m and n), ldb >= m_pad,
 * overwritten; for a ragged matrix rows m.. of B are the embedding's
 * (zero for a block of R^m, whose leading n rows of Q^T B are then Q1^T B).
 * Requires FACTORED.  Asynchronous. */
blr_status blr_apply_qt(blr_matrix h, int32_t trans, double* B, int64_t ldb,
                        int32_t nrhs, void* hip_stream);

/* blr_apply_qt for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, result and state rules as blr_apply_qt, and the same
 * kernels; it calls no hipMalloc, hipFree or allocating library routine.
 * Its temporaries and launch descriptors live in one static device array of
 * BLR_NOALLOC_SCRATCH_BYTES per GPU (held from the first call on that GPU
 * until the process ends).  A call whose matrix and nrhs need more returns
 * BLR_ERR_INVALID before enqueuing anything (the message states the bytes
 * needed); the need grows with nrhs (block column: about 64 b + p rc
 * doubles per right-hand side; tiled: about 6 b + rc per right-hand side
 * for each of up to 64 merged step chains, at most 16 MiB in all, at least
 * one chain) plus the launch descriptors (a few MiB at 128 x 64 tiles).
 * Every
 * call on one GPU shares the array: calls on the same stream are ordered,
 * calls that overlap on one GPU (other streams or threads) race. */
#define BLR_NOALLOC_SCRATCH_BYTES (64LL * 1024 * 1024)
blr_status blr_apply_qt_noalloc(blr_matrix h, int32_t trans, double* B, int64_t ldb,
                                int32_t nrhs, void* hip_stream);

/* Products with the stored BLR matrix, for residual and orthogonality
 * checks and refinement (eq. blr_matrix_def, eq. qr_fact):
 *   BLR_MATMUL_A   Y = A~ X     requires COMPRESSED, or a factor made with keep_a;
 *                               X n x nrhs, Y m x nrhs
 *   BLR_MATMUL_AT  Y = A~^T X   same requirement; X m x nrhs, Y n x nrhs
 *   BLR_MATMUL_R   Y = R X      requires a complete factor; X, Y n x nrhs
 * X and Y: device, column-major (ldx, ldy at least their row counts), must
 * not overlap; Y is overwritten.  Dense tiles multiply directly, low-rank
 * tiles as U (V^T X) (or V (U^T X)); R uses the upper triangle of the
 * diagonal tiles and the stored R_kj tiles.  Asynchronous on hip_stream. */
typedef enum { BLR_MATMUL_A = 0, BLR_MATMUL_AT = 1, BLR_MATMUL_R = 2 } blr_matmul_op;
blr_status blr_matmul(blr_matrix h, int32_t op, const double* X, int64_t ldx, double* Y, int64_t ldy,
                      int32_t nrhs, void* hip_stream);

/* Least squares X = argmin ||A~ X - B||_F column by column, the problem the
 * QR factorization serves (Section 1: with A = QR, the solution of an
 * overdetermined system is R^{-1} (Q^T b)[0:n]): X = R^{-1} (Q^T B)[0:n]
 * with tile back-substitution through the BLR factor R (Sections 3.3, 3.4).
 * B: device m x nrhs (ldb >= m), not modified.  X: device n x nrhs
 * (ldx >= n).  max_refine > 0 (needs a factor made with keep_a): up to that
 * many steps of iterative refinement of the augmented system
 * [I A~; A~^T 0][r; x] = [b; 0] with FP64 residuals f = b - r - A~ x and
 * g = -A~^T r and corrections from the stored factor, d = Q^T f,
 * h = R^{-T} g, dx = R^{-1}(d_1 - h), dr = Q [h; d_2].  Per column, a step's
 * correction is taken only while it is at most half the previous one taken;
 * a larger one is dropped and the column stops with its current iterate
 * (the residuals have reached their rounding noise, or the iteration
 * diverges); a column also stops after taking a correction with
 * ||dx|| <= 2 u ||x||.  The loop ends when no column is refining.  It
 * recovers FP64 accuracy for a BLR_MIXED_FP32 factor.  resid_norms: optional
 * device array of nrhs doubles receiving the squared least-squares residual
 * norm per column (||(Q^T B)[n:m]||^2, or ||r||^2 of the refined residual).
 * Requires a complete factor.
 * Synchronises the stream (the singularity check reads the diagonal of R). */
blr_status blr_lstsq_solve(blr_matrix h, const double* B, int64_t ldb, double* X,
                           int64_t ldx, int32_t nrhs, int32_t max_refine,
                           double* resid_norms, void* hip_stream);

/* Least squares for count independent factored matrices as one batch: for
 * each i, X[i] = argmin ||A~_i X - B[i]||_F exactly as blr_lstsq_solve(hs[i],
 * B[i], ldb[i], X[i], ldx[i], nrhs, max_refine, NULL, stream) computes it
 * (bit-identical results), with the launches of all members merged as in
 * blr_qr_factor_batch.  hs, B, ldb, X, ldx are host arrays of count entries;
 * B[i] (device, m_i x nrhs, ldb[i] >= m_i) is not modified, X[i] (device,
 * n_i x nrhs, ldx[i] >= n_i) is overwritten.  Members may differ in size,
 * tile size and variant.  max_refine > 0 needs every factor made with keep_a;
 * each member stops refining when its own test is met.  No residual norms.
 * Synchronises the stream.  Errors: BLR_ERR_INVALID (NULL pointers, count <
 * 1, a repeated handle, bad shapes), BLR_ERR_STATE (a member not fully
 * factored, or refinement without keep_a), BLR_ERR_SINGULAR (the message
 * names the first singular member; no X is written then). */
blr_status blr_lstsq_solve_batch(blr_matrix* hs, int32_t count, const double* const* B, const int64_t* ldb,
                                 double* const* X, const int64_t* ldx, int32_t nrhs, int32_t max_refine,
                                 void* hip_stream);

/* Shape, formats, state, memory and counters of a handle.  Waits for the
 * handle's previous work first. */
blr_status blr_query(blr_matrix h, blr_info* info);

/* Release the handle and all its device memory (waits for the handle's
 * previous work first). */
void blr_destroy(blr_matrix h);

const char* blr_status_string(blr_status s);
const char* blr_last_error(void);

/* Kernel-level timing of the dominant kernel, the untransposed 128 x 128
 * matrix-core product (k_gemm_fast<double|float, false, false>: trailing
 * updates and block-reflector applications).  While enabled, HIP events
 * bracket every launch of it on this handle, on the stream it runs on
 * (blr_qr_factor clears the record first).  blr_profile_read returns, for
 * kernel 0 (FP64 operands) or 1 (FP32 operands), the number of launches,
 * their total device time in milliseconds and their total algorithmic flops.
 * blr_profile_read waits for the handle's previous work first. */
blr_status blr_profile_enable(blr_matrix h, int32_t on);
blr_status blr_profile_read(blr_matrix h, int32_t kernel, int64_t* launches, double* total_ms,
                            double* total_flops);

#ifdef __cplusplus
}
#endif

#endif /* BLRQR_H */
