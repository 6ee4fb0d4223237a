/*
 * Kernel-level test hook of libblrqr (not part of the factorization API).
 *
 * blr_selftest_gemm runs the library's matrix-core GEMM kernel on one
 * problem, C = alpha * op(A) op(B) + beta * C, so that tests can check it
 * against a plain reference.  Column-major device pointers; flags are the
 * kernel's segment flags (1 = A transposed, 2 = B transposed, 4 = A read as
 * unit lower triangular, 8 = A upper triangular, 16 = B read as unit lower
 * triangular).  fp32 = 1 rounds the operands to FP32 and accumulates in FP32
 * on the matrix cores.  Callers: the test suite.  Asynchronous on stream.
 */
#ifndef BLRQR_SELFTEST_H
#define BLRQR_SELFTEST_H
#include <stdint.h>
#include "blrqr.h"
#ifdef __cplusplus
extern "C" {
#endif
blr_status blr_selftest_gemm(int32_t flags, int32_t M, int32_t N, int32_t K, double alpha,
                             const double* A, int64_t lda, const double* B, int64_t ldb,
                             double beta, double* C, int64_t ldc, int32_t fp32, void* hip_stream);
#ifdef __cplusplus
}
#endif
#endif
