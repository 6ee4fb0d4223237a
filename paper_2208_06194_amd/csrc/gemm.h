// Batched, heterogeneous matrix-core GEMM used for every product of the
// factorization (reflector applications, basis products, Gram matrices).
//
//   C = alpha * sum_s op(A_s) op(B_s) + beta * Cin        (D2 = raw sum, optional)
//
// One launch executes a list of descriptors; each descriptor has its own
// M, N, pointers and a list of K segments (so a block-column product
// sum_i Y_ik^T A_ij is one descriptor).  Column-major storage throughout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

enum GemmSegFlags {
  SEG_TRANS_A = 1,       // op(A) = A^T (A stored K x M)
  SEG_TRANS_B = 2,       // op(B) = B^T (B stored N x K)
  SEG_A_UNIT_LOWER = 4,  // stored A read as unit lower triangular (diag 1, upper 0)
  SEG_A_UPPER = 8,       // stored A is upper triangular (zeros stored): K range pruned
  SEG_B_UNIT_LOWER = 16, // stored B read as unit lower triangular
};
enum GemmDescFlags {
  DESC_LOWER_ONLY = 1,   // only output tiles touching the lower triangle are written
};

struct GemmSeg {
  const double* A;
  const double* B;
  int64_t lda, ldb;
  int32_t K;
  int32_t flags;
};

struct GemmDesc {
  double* C;
  const double* Cin;   // may equal C; nullptr = zero
  double* D2;          // optional copy of the raw product
  int64_t ldc, ldcin, ldd2;
  int32_t M, N;
  double alpha, beta;
  int32_t seg_begin, nseg;
  int32_t tile_begin;  // prefix sum of tiles over the launch's descriptors
  int32_t tilesM;
  int32_t flags;
  int32_t pad_;
};

// Kernel variants: generic 64x64 and 128x128 tiles (any shape, masks, several
// K segments) and the fast 128x128 path (full tiles, every K segment a multiple
// of the K step, one transpose pattern per launch, 16-byte aligned operands and
// even leading dimensions, no unit-lower masks), specialised on the two
// transposes.  K step of the fast path: 16.
constexpr int kFastKStep64 = 16;
constexpr int kFastKStep32 = 16;
enum GemmMode {
  GEMM_SMALL = 0, GEMM_BIG = 1,
  GEMM_FAST_NN = 2, GEMM_FAST_TN = 3, GEMM_FAST_NT = 4, GEMM_FAST_TT = 5,
  GEMM_SKINNY_N = 6, GEMM_SKINNY_T = 7,   // FP64, N <= 16, B not transposed: 64-row tiles
};

// Launch host wrapper: descs / segs are device arrays; ntiles = total WG tiles
// (tiles of 64 x 64 for GEMM_SMALL, 64 x 16 for the skinny modes, 128 x 128
// otherwise).  fp32 = 1 computes in FP32 on
// the matrix cores (operands rounded to FP32, FP32 accumulation); fp32 = 2
// (fast modes) also rounds operands to FP32 but adds the FP32 partial sums
// into FP64 accumulators every 1024 of K and at every segment end.
hipError_t launch_gemm(const GemmDesc* d_descs, int ndesc, const GemmSeg* d_segs, int ntiles,
                       int mode, int fp32, hipStream_t stream);
