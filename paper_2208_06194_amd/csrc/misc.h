// Element-wise / reduction kernels used by compression and the solve.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

struct TileFillDesc {
  double* dst;   // b x b tile, ld b
  int32_t ti, tj;
};
struct TileFillParams {
  int b;
  int src_dense;        // 1: copy from A; 0: evaluate the kernel from points
  const double* A;
  int64_t lda;
  const double* x;
  const double* y;
  int dim;
  int kernel;           // 0 log2d, 1 inv_r
  double reg;
  // rows mu and columns nu of the matrix itself; the tiles cover the
  // embedding [A 0; 0 E] (E: identity rows m..m+pc-1 in the padded columns
  // n..n+pc-1, zero elsewhere)
  int64_t mu, nu;
};
struct Frob2Desc {
  const double* M;
  int64_t ld;
  int32_t rows, cols;
  double* out;
};
struct DiagDesc {
  const double* R;      // diagonal tile, b x b, ld b
  int ncols;            // columns taken into account (the rest are padding)
};

hipError_t launch_fill_tiles(const TileFillDesc* d, int n, const TileFillParams& p, hipStream_t s);
hipError_t launch_boxes(const double* pts, int npts, int dim, int b, double* lo, double* hi,
                        hipStream_t s);
hipError_t launch_gaussian(double* out, int64_t n, unsigned long long seed, unsigned long long stream,
                           hipStream_t s);
hipError_t launch_nonfinite(const double* a, int64_t rows, int64_t cols, int64_t ld, int* flag,
                            hipStream_t s);
hipError_t launch_frob2(const Frob2Desc* d, int n, hipStream_t s);
hipError_t launch_trsm_upper(const double* R, int64_t ldr, int n, double* X, int64_t ldx, int nrhs,
                             hipStream_t s);
// R^T X = B in place (R upper triangular n x n): forward substitution.
hipError_t launch_trsm_upper_t(const double* R, int64_t ldr, int n, double* X, int64_t ldx, int nrhs,
                               hipStream_t s);
// out = a x + b y + c z (rows x cols, column-major; y and z may be null).
hipError_t launch_lincomb(double* out, int64_t ldo, const double* x, int64_t ldx, const double* y, int64_t ldy,
                          const double* z, int64_t ldz, double a, double b, double c, int rows, int cols,
                          hipStream_t s);
hipError_t launch_diag_absmin(const DiagDesc* d, int n, int b, double* out, hipStream_t s);

// One triangular solve of a batched launch (op(R) X = C in place, R upper
// triangular n x n): the arguments of launch_trsm_upper(_t).  Device array.
struct TrsmJob {
  const double* R;
  int64_t ldr;
  double* X;
  int64_t ldx;
  int32_t n, nrhs;
};
hipError_t launch_trsm_batch(const TrsmJob* d, int count, int trans, int max_nrhs, hipStream_t s);
// out = a x + b y + c z for each descriptor (device array; y, z may be null).
struct LincombDesc {
  double* out;
  int64_t ldo;
  const double* x;
  int64_t ldx;
  const double* y;
  int64_t ldy;
  const double* z;
  int64_t ldz;
  double a, b, c;
  int32_t rows, cols;
};
hipError_t launch_lincomb_batch(const LincombDesc* d, int count, int64_t max_elems, hipStream_t s);
