// Reflector generation kernels (panel factorization, T factor).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

enum { PANEL_GEQRT = 0, PANEL_TPQRT = 1 };

struct PanelArgs {
  int mode;        // PANEL_GEQRT / PANEL_TPQRT
  int h;           // rows of the panel (GEQRT: from the pivot row down; TPQRT: rows of B)
  int ib;          // panel width (16 or 32)
  double* X;       // panel start (GEQRT: element (c0,c0); TPQRT: B column c0)
  int64_t ldx;
  double* R;       // TPQRT: R element (c0,c0)
  int64_t ldr;
  double* T;       // T element (c0,c0): receives the IB x IB diagonal block
  int64_t ldt;
  double* tau;     // tau[c0 .. c0+ib)
};

struct TBackArgs {
  int n;           // order of T
  int ib;          // diagonal blocks of this size are already filled
  const double* G; // Gram matrix, lower triangle valid (G[t + r*ldg], t > r)
  int64_t ldg;
  const double* tau;
  double* T;
  int64_t ldt;
};

struct TallArgs {
  double* X;       // panel pivot (c0, c0) of the stack
  int64_t ldx;
  int h;           // rows from the pivot down
  int ib;          // panel width (<= 32)
  int jj;          // column of the panel being factored
  double* part;    // partials: 2 x (G + 1) x 2*ib doubles
  double* T;       // T element (c0, c0)
  int64_t ldt;
  double* tau;     // tau[c0 ..]
};

struct CopyDesc {
  const double* src;
  double* dst;
  int64_t lds, ldd;
  int32_t rows, cols;
  int32_t unit_lower;   // 1: write the unit lower triangular part of src (diag 1, upper 0);
                        // 2: write the upper triangular part (zeros below the diagonal);
                        // 3: src and dst point to one int32 (a tile rank), copied as is
  int32_t nsum;         // > 1: dst = sum of nsum blocks of src, sstride doubles apart (split-K)
  int64_t sstride;
};

hipError_t launch_panel(const PanelArgs& a, hipStream_t stream);
// One launch per column of a tall panel (two for its first column), over
// groups row groups (1 .. kTallMaxGroups); ib must be 16 or 32.
constexpr int kTallMaxGroups = 512;
constexpr int kTallThreads = 256;   // threads per row group (two rows each for 512-row groups)
hipError_t launch_tall_column(const TallArgs& a, int groups, hipStream_t stream);
// Split-K trailing update of a tall panel over 1 .. kTallApplySlices row
// slices; part: slices * ceil(nt/32) * ib * 32 doubles.
constexpr int kTallApplySlices = 256;
hipError_t launch_tall_apply(const PanelArgs& a, int nt, int slices, double* part, hipStream_t stream);
hipError_t launch_copy_blocks(const CopyDesc* d, int n, int64_t max_elems, hipStream_t stream);
// Modified Gram-Schmidt QR of an h x w column-major block X (ld ldx) in one
// workgroup: X is overwritten by Q, R (w x w, ld ldr) receives R (zeros
// below the diagonal).  Full column rank is assumed (a zero column divides
// by zero).
hipError_t launch_mgs_stack(double* X, int64_t ldx, int h, int w, double* R, int64_t ldr, hipStream_t stream);
hipError_t launch_t_backsolve(const TBackArgs& a, hipStream_t stream);
// Fused trailing update of the nt columns right of panel a (same PanelArgs:
// X points at the panel's first column / first row, T at its diagonal block).
hipError_t launch_panel_apply(const PanelArgs& a, int nt, hipStream_t stream);

// One job of a batched launch of the kernels above (one per independent
// matrix of a batched factorization): the single-problem arguments and the
// job's own extent.  Each job is computed exactly as by its single-problem
// launch.  Job arrays are device memory.
struct PanelJob {
  PanelArgs a;     // panel, panel update, tall update
  TallArgs t;      // tall column
  TBackArgs tb;    // T back-substitution (order tb.n > tb.ib)
  int nt;          // panel update / tall update: trailing columns (> 0)
  int groups;      // tall column: row groups; tall update: row slices
  double* part;    // tall update: partial sums
};
// max_rows selects the register-tile template: every job's h must fall in
// the same bucket as max_rows (1, 2, 4, 8, 16 chunks of 64 rows).
hipError_t launch_panel_batch(const PanelJob* d, int n, int ib, int max_rows, hipStream_t stream);
hipError_t launch_panel_apply_batch(const PanelJob* d, int n, int ib, int max_nt, hipStream_t stream);
hipError_t launch_t_backsolve_batch(const PanelJob* d, int n, int max_n, hipStream_t stream);
// first = 1: the jobs are the first column of their panels (jj = 0)
hipError_t launch_tall_column_batch(const PanelJob* d, int n, int ib, int first, int max_groups,
                                    hipStream_t stream);
hipError_t launch_tall_apply_batch(const PanelJob* d, int n, int ib, int max_nt, int max_slices,
                                   hipStream_t stream);
