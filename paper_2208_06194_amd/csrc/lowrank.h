// Low-rank kernels: rounded addition (Alg. 6 of arXiv 2208.06194) and the
// truncated-SVD compression of admissible tiles (Section 3.1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// One term sign * U[:, :r] * Vt[:r, :] of a sum of low-rank matrices.
// U is b x r stored column-major (ldu >= b) or, with transU, stored as the
// r x b matrix U^T (U(i,l) at U[l + i*ldu]).  Vt is r x b column-major.
struct RcTerm {
  const double* U;
  const double* Vt;
  const int* rank_ptr;   // device rank, or nullptr to use `rank`
  int64_t ldu, ldvt;
  int32_t rank;
  int32_t transU;
  double sign;
};

struct RcDesc {
  RcTerm t[3];
  int32_t nterm;
  int32_t pad_;
  double* Uout;          // b x rc (ld b); columns >= rank are zeroed
  double* Vtout;         // rc x b (ld rc); rows >= rank are zeroed
  int* rank_out;
  double* work;          // per-problem workspace (rc_work_doubles)
  unsigned long long* counters;  // own [overflow count, max dropped bits], or nullptr: the launch's
};

struct RcParams {
  int b, rc;             // tile size, slot capacity
  int cap;               // truncation cap (<= rc)
  double eps;            // relative truncation tolerance
  unsigned long long* overflow_count;   // device counter
  unsigned long long* max_dropped_bits; // device: bit pattern of max dropped relative tail
};

size_t rc_work_doubles(int b, int rc);
hipError_t launch_recompress(const RcDesc* d_descs, int n, const RcParams& p, hipStream_t stream);

// ---- compression -----------------------------------------------------------
struct CompDesc {
  const double* A;       // tile, b x b (ld b)
  double* Y;             // b x l sample A*Omega (overwritten by reflectors)
  double* Q;             // b x l explicit orthonormal basis (output of range finder)
  double* B;             // l x b = Q^T A
  double* Uout;          // b x rc
  double* Vtout;         // rc x b
  int* rank_out;
  int* status_out;       // 0 = low-rank, 1 = exceeds the cap
  double* work;          // comp_work_doubles
  double* enorm2;        // ||A - Q B||_F^2 (precomputed)
  double* anorm2;        // ||A||_F^2 (precomputed)
};

struct CompParams {
  int b, rc, l, cap;
  double eps;
  int truncate;          // 1: overflow truncates to the cap instead of reporting
};

size_t comp_work_doubles(int b, int l);
hipError_t launch_rangefinder(const CompDesc* d, int n, int b, int l, hipStream_t stream);
hipError_t launch_comp_svd(const CompDesc* d, int n, const CompParams& p, hipStream_t stream);
