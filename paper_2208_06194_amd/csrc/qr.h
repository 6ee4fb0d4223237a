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
// Split-K trailing update of a tall panel over 1 .. kTallApplySlices row
// slices; part: slices * ceil(nt/32) * ib * 32 doubles.
constexpr int kTallApplySlices = 256;
hipError_t launch_tall_apply(const PanelArgs& a, int nt, int slices, double* part, hipStream_t stream);

// Tall panels as a tree (TSQR) with Householder reconstruction.  A tall
// panel of h rows and kTsqrIB columns is cut into count[0] leaves of at most
// kTsqrRows rows (balanced: the first h % count[0] leaves get one row more);
// every leaf is factored, the leaves' R factors are stacked in S[1] (leaf g
// in rows 16 g .. 16 g + 15) and factored in groups of at most 16 (count[1]
// nodes, balanced like the leaves), and so on up to the single root
// (count[levels] == 1).  Every factor is a Householder QR with LAPACK's
// larfg convention, its reflectors left in place and its T in Tn[level]
// (16 x 16 per node, ld 16); each leaf also keeps a unit-lower copy of its
// top 16 x 16 reflector block in Y1.  The final step forms each leaf's rows
// of the explicit Q and turns them into the Householder vectors, T and tau
// of the whole panel (an LU factorization of Q's top block with the sign
// choice that avoids cancellation), with R = D R_root written on the top
// rows of the panel: the same reflectors, T, tau and R (up to rounding) as
// the column-by-column Householder QR.  levels == 0: the single leaf's QR is
// the panel's.
constexpr int kTsqrIB = 16;
constexpr int kTsqrRows = 256;
constexpr int kTsqrFan = 16;
constexpr int kTsqrMaxLevels = 6;
struct TsqrTree {
  double* X;      // panel pivot (c0, c0)
  int64_t ldx;
  int h;          // rows from the pivot down
  int levels;
  double* T;      // output: 16 x 16 upper triangular block (ld ldt)
  int64_t ldt;
  double* tau;    // output: 16 values
  double* Y1;     // count[0] x 256
  int count[kTsqrMaxLevels + 1];
  double* S[kTsqrMaxLevels + 1];    // S[l], l >= 1: 16 count[l-1] rows x 16, column-major
  double* Tn[kTsqrMaxLevels + 1];   // Tn[l]: count[l] x 256
};
// One tree level (QR launch: every node of that level; final launch: every
// leaf) of a batched launch; wg_begin is the first workgroup of the item.
struct TsqrItem {
  int tree;
  int level;
  int wg_begin;
  int pad;
};
hipError_t launch_tsqr_qr(const TsqrTree* trees, const TsqrItem* items, int n, int total_wg, hipStream_t stream);
hipError_t launch_tsqr_final(const TsqrTree* trees, const TsqrItem* items, int n, int total_wg,
                             hipStream_t stream);

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
  TBackArgs tb;    // T back-substitution (order tb.n > tb.ib)
  int nt;          // panel update / tall update: trailing columns (> 0)
  int groups;      // tall update: row slices
  double* part;    // tall update: partial sums
};
// max_rows selects the register-tile template: every job's h must fall in
// the same bucket as max_rows (1, 2, 4, 8, 16 chunks of 64 rows).
hipError_t launch_panel_batch(const PanelJob* d, int n, int ib, int max_rows, hipStream_t stream);
hipError_t launch_panel_apply_batch(const PanelJob* d, int n, int ib, int max_nt, hipStream_t stream);
hipError_t launch_t_backsolve_batch(const PanelJob* d, int n, int max_n, hipStream_t stream);
hipError_t launch_tall_apply_batch(const PanelJob* d, int n, int ib, int max_nt, int max_slices,
                                   hipStream_t stream);
