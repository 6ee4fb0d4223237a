// Matrix-core GEMM for gfx950: 256 threads = 4 waves in a 2 x 2 grid, each
// wave owning a (BM/2) x (BN/2) block of 16 x 16 MFMA tiles.  K advances in
// steps of 16 through LDS (k-major, padded), with the next step prefetched
// into registers while the matrix cores work on the current one.
#include "device_common.h"
#include "gemm.h"

namespace {

template <typename CT>
struct AccT;
template <>
struct AccT<double> {
  typedef v4d T;
};
template <>
struct AccT<float> {
  typedef v4f T;
};

__device__ __forceinline__ v4d mfma_op(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma_op(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double unit_lower_mask(double x, int64_t row, int64_t col) {
  return row > col ? x : (row == col ? 1.0 : 0.0);
}

template <typename CT, int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm(const GemmDesc* __restrict__ descs, int ndesc,
                                              const GemmSeg* __restrict__ segs) {
  constexpr int BK = 16;
  constexpr int PAD = 4;
  constexpr int AE = BM * BK / 256;
  constexpr int BE = BN * BK / 256;
  constexpr int TM = BM / 32;
  constexpr int TN = BN / 32;
  typedef typename AccT<CT>::T acc_t;

  __shared__ CT As[BK][BM + PAD];
  __shared__ CT Bs[BK][BN + PAD];

  const int wg = blockIdx.x;
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_begin <= wg)
      lo = mid;
    else
      hi = mid - 1;
  }
  const GemmDesc d = descs[lo];
  const int t = wg - d.tile_begin;
  const int m0 = (t % d.tilesM) * BM;
  const int n0 = (t / d.tilesM) * BN;
  const int M = d.M, N = d.N;
  if (n0 >= N || m0 >= M) return;
  if ((d.flags & DESC_LOWER_ONLY) && m0 + BM <= n0) return;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;

  for (int s = 0; s < d.nseg; ++s) {
    const GemmSeg sg = segs[d.seg_begin + s];
    const bool ta = sg.flags & SEG_TRANS_A;
    const bool tb = sg.flags & SEG_TRANS_B;
    const bool aul = sg.flags & SEG_A_UNIT_LOWER;
    const bool bul = sg.flags & SEG_B_UNIT_LOWER;
    int kbeg = 0, kend = sg.K;
    if (aul) {
      if (ta) kbeg = max(kbeg, m0);
      else kend = min(kend, m0 + BM);
    }
    if (sg.flags & SEG_A_UPPER) {
      if (ta) kend = min(kend, m0 + BM);
      else kbeg = max(kbeg, m0);
    }
    if (bul) {
      if (tb) kend = min(kend, n0 + BN);
      else kbeg = max(kbeg, n0);
    }
    kbeg = (kbeg / BK) * BK;
    if (kbeg >= kend) continue;

    const double* __restrict__ Ap = sg.A;
    const double* __restrict__ Bp = sg.B;
    const int64_t lda = sg.lda, ldb = sg.ldb;

    CT ra[AE], rb[BE];
    auto load = [&](int k0) {
#pragma unroll
      for (int i = 0; i < AE; ++i) {
        const int e = tid + 256 * i;
        const int mm = ta ? e / BK : e % BM;
        const int kk = ta ? e % BK : e / BM;
        const int gm = m0 + mm, gk = k0 + kk;
        double x = 0.0;
        if (gm < M && gk < kend) {
          const int64_t row = ta ? gk : gm, col = ta ? gm : gk;
          x = Ap[row + col * lda];
          if (aul) x = unit_lower_mask(x, row, col);
        }
        ra[i] = (CT)x;
      }
#pragma unroll
      for (int i = 0; i < BE; ++i) {
        const int e = tid + 256 * i;
        const int nn = tb ? e % BN : e / BK;
        const int kk = tb ? e / BN : e % BK;
        const int gn = n0 + nn, gk = k0 + kk;
        double x = 0.0;
        if (gn < N && gk < kend) {
          const int64_t row = tb ? gn : gk, col = tb ? gk : gn;
          x = Bp[row + col * ldb];
          if (bul) x = unit_lower_mask(x, row, col);
        }
        rb[i] = (CT)x;
      }
    };

    load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < AE; ++i) {
        const int e = tid + 256 * i;
        const int mm = ta ? e / BK : e % BM;
        const int kk = ta ? e % BK : e / BM;
        As[kk][mm] = ra[i];
      }
#pragma unroll
      for (int i = 0; i < BE; ++i) {
        const int e = tid + 256 * i;
        const int nn = tb ? e % BN : e / BK;
        const int kk = tb ? e / BN : e % BK;
        Bs[kk][nn] = rb[i];
      }
      __syncthreads();
      if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        CT af[TM], bf[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = As[kk + (lane >> 4)][wm * (BM / 2) + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < TN; ++j) bf[j] = Bs[kk + (lane >> 4)][wn * (BN / 2) + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = mfma_op(af[i], bf[j], acc[i][j]);
      }
    }
  }

  // epilogue: lane holds column lane%16 of each 16x16 tile; accumulator v is
  // row 4*(lane/16)+v for the FP32 instruction and row 4*v+lane/16 for the
  // FP64 instruction (measured layouts of v_mfma_f32/f64_16x16x4 on gfx950)
  constexpr bool f64out = sizeof(CT) == 8;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = n0 + wn * (BN / 2) + j * 16 + (lane & 15);
      if (col >= N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * (BM / 2) + i * 16 + (f64out ? v * 4 + (lane >> 4) : (lane >> 4) * 4 + v);
        if (row >= M) continue;
        const double raw = (double)acc[i][j][v];
        if (d.C) {
          double c = d.alpha * raw;
          if (d.Cin) c += d.beta * d.Cin[row + (int64_t)col * d.ldcin];
          d.C[row + (int64_t)col * d.ldc] = c;
        }
        if (d.D2) d.D2[row + (int64_t)col * d.ldd2] = raw;
      }
    }
  }
}

typedef double d2v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const d2v gd2v;
typedef __attribute__((address_space(1))) const double gdbl;

// Skinny products (N <= 16, FP64): the applications of Q^T / Q and the
// back-substitution sums with a few right-hand sides.  These read each tile of
// A once and do 2 * N flops per element, so they are bound by HBM; the
// 64 x 64 MFMA tile would compute four times the useful work.  A workgroup
// owns 64 rows of C and all (<= 16) columns; its four waves take interleaved
// 16-deep K blocks and sum their 64 x 16 partials through LDS in a fixed
// order.  Operands go straight from global memory into the MFMA registers:
// for A transposed a lane reads four consecutive k of one column (lane group
// g takes k = 4g .. 4g + 3 of each block and steps through them), otherwise
// sixteen lanes read sixteen consecutive rows of one k column.  On full
// 64-row tiles of segments whose K is a multiple of 16 (no unit-lower mask,
// 16-byte aligned operands, even leading dimensions) each wave keeps the
// next K block's loads in flight while it multiplies the current one, and
// the four consecutive k of a lane are read as two 16-byte vectors.
template <bool TA>
__global__ __launch_bounds__(256) void k_gemm_skinny(const GemmDesc* __restrict__ descs, int ndesc,
                                                     const GemmSeg* __restrict__ segs) {
  constexpr int BM = 64, BKS = 16;
  __shared__ double red[3][BM / 16][4][64];
  const int wg = blockIdx.x;
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_begin <= wg) lo = mid;
    else hi = mid - 1;
  }
  const GemmDesc d = descs[lo];
  const int m0 = (wg - d.tile_begin) * BM;
  const int M = d.M, N = d.N;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: K-block loops run on scalars
  const int lm = lane & 15, lg = lane >> 4;
  v4d acc[BM / 16];
#pragma unroll
  for (int i = 0; i < BM / 16; ++i) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < d.nseg; ++s) {
    const GemmSeg sg = segs[d.seg_begin + s];
    const bool aul = sg.flags & SEG_A_UNIT_LOWER;
    int kbeg = 0, kend = sg.K;
    if (aul) {
      if (TA) kbeg = max(kbeg, m0);
      else kend = min(kend, m0 + BM);
    }
    kbeg = (kbeg / BKS) * BKS;
    const double* __restrict__ Ap = sg.A;
    const double* __restrict__ Bp = sg.B;
    const int64_t lda = sg.lda, ldb = sg.ldb;
    const bool fast = !aul && m0 + BM <= M && kend % BKS == 0 && ((lda | ldb) & 1) == 0 &&
                      (((uintptr_t)Ap | (uintptr_t)Bp) & 15) == 0;
    if (fast) {
      // every load has a valid address (column min(lm, N - 1), the last block
      // again past the end), so each K block issues the same loads and the
      // wait before its products covers exactly the block before it
      // per-lane base addresses; a K block adds one uniform offset
      const double* bl = Bp + (int64_t)min(lm, N - 1) * ldb + 4 * lg;
      const double* al = TA ? Ap + (int64_t)(m0 + lm) * lda + 4 * lg : Ap + m0 + lm + (int64_t)(4 * lg) * lda;
      const int64_t ai = TA ? 16 * lda : 16;      // next 16 rows of C
      const int64_t ak = TA ? 1 : lda;            // next k
      auto ld = [&](int k0, double (&av)[BM / 16][4], double (&bv)[4]) {
        const double* bk = bl + k0;
        const d2v b0 = *(const gd2v*)bk;
        const d2v b1 = *(const gd2v*)(bk + 2);
        bv[0] = b0[0]; bv[1] = b0[1]; bv[2] = b1[0]; bv[3] = b1[1];
        const double* ak0 = al + (int64_t)k0 * ak;
#pragma unroll
        for (int i = 0; i < BM / 16; ++i) {
          if (TA) {
            const d2v a0 = *(const gd2v*)(ak0 + i * ai);
            const d2v a1 = *(const gd2v*)(ak0 + i * ai + 2);
            av[i][0] = a0[0]; av[i][1] = a0[1]; av[i][2] = a1[0]; av[i][3] = a1[1];
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) av[i][u] = *(const gdbl*)(ak0 + i * ai + u * ak);
          }
        }
      };
      auto mm = [&](const double (&av)[BM / 16][4], const double (&bv)[4]) {
        const bool live = lm < N;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double bu = live ? bv[u] : 0.0;
#pragma unroll
          for (int i = 0; i < BM / 16; ++i) acc[i] = mfma_op(av[i][u], bu, acc[i]);
        }
      };
      int k0 = kbeg + wave * BKS;
      if (k0 < kend) {
        double a0[BM / 16][4], b0[4], a1[BM / 16][4], b1[4];
        ld(k0, a0, b0);
        for (;;) {
          // the scheduling barriers keep each block's loads ahead of the
          // products of the block before it
          const int k1 = k0 + 4 * BKS;
          ld(k1 < kend ? k1 : k0, a1, b1);
          __builtin_amdgcn_sched_barrier(0);
          mm(a0, b0);
          if (k1 >= kend) break;
          const int k2 = k1 + 4 * BKS;
          ld(k2 < kend ? k2 : k1, a0, b0);
          __builtin_amdgcn_sched_barrier(0);
          mm(a1, b1);
          if (k2 >= kend) break;
          k0 = k2;
        }
      }
      continue;
    }
    for (int k0 = kbeg + wave * BKS; k0 < kend; k0 += 4 * BKS) {
      // B: lane (n = lm, group lg) holds k = k0 + 4 lg + u, u = 0..3
      double bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + 4 * lg + u;
        bv[u] = (lm < N && k < kend) ? Bp[k + (int64_t)lm * ldb] : 0.0;
      }
      double av[BM / 16][4];
#pragma unroll
      for (int i = 0; i < BM / 16; ++i) {
        const int m = m0 + 16 * i + lm;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + 4 * lg + u;
          double x = 0.0;
          if (m < M && k < kend) {
            const int64_t row = TA ? k : m, col = TA ? m : k;
            x = Ap[row + col * lda];
            if (aul) x = unit_lower_mask(x, row, col);
          }
          av[i][u] = x;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < BM / 16; ++i) acc[i] = mfma_op(av[i][u], bv[u], acc[i]);
    }
  }
  // waves 1..3 hand their partials to wave 0, which adds them in wave order
  if (wave > 0) {
#pragma unroll
    for (int i = 0; i < BM / 16; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[wave - 1][i][v][lane] = acc[i][v];
  }
  __syncthreads();
  if (wave != 0) return;
  const int col = lm;
  if (col >= N) return;
#pragma unroll
  for (int i = 0; i < BM / 16; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = m0 + 16 * i + 4 * v + lg;   // FP64 16x16x4 layout: row 4 v + lane / 16
      if (row >= M) continue;
      const double raw = ((acc[i][v] + red[0][i][v][lane]) + red[1][i][v][lane]) + red[2][i][v][lane];
      if (d.C) {
        double c = d.alpha * raw;
        if (d.Cin) c += d.beta * d.Cin[row + (int64_t)col * d.ldcin];
        d.C[row + (int64_t)col * d.ldc] = c;
      }
      if (d.D2) d.D2[row + (int64_t)col * d.ldd2] = raw;
    }
  }
}


// Order of the output tiles of a fast launch (128 x 128 tiles).  Workgroups
// are dispatched to the eight XCDs in turn (workgroup w on XCD w mod 8), and
// each XCD has its own L2.  Workgroup w takes position
//   L = (w mod 8) * T8 + w / 8   (w < 8 T8, T8 = floor(T / 8); the rest keep L = w)
// of the launch's T tiles, so every XCD works through one contiguous eighth of
// them: a product split into one descriptor per block column lands whole on
// one XCD, and no operand slab is fetched by all eight.  Inside a descriptor
// the tiles run in groups of 8 tile columns, row-major inside a group, so the
// workgroups resident on an XCD at one time cover about 8 x 8 tiles and share
// their A and B slabs in its L2.
__device__ __forceinline__ int xcd_tile_order(int w, int T) {
  constexpr int X = 8;
  const int T8 = T / X;
  return w < X * T8 ? (w % X) * T8 + w / X : w;
}
__device__ __forceinline__ void grouped_tile(int t, int tilesM, int tilesN, int* mt, int* nt) {
  constexpr int GN = 8;
  const int gsz = tilesM * GN;
  const int g = t / gsz, v = t - g * gsz;
  const int gw = min(GN, tilesN - g * GN);
  *mt = v / gw;
  *nt = g * GN + v % gw;
}

// Fast path for full 128 x 128 output tiles with one K segment (K a multiple
// of 16, 16-byte aligned operands, no masked triangles; an upper triangular A
// only prunes the K range).  Transposes are compile-time; global loads are
// 16-byte vectors from precomputed per-thread addresses; LDS is double
// buffered so each K step needs a single barrier.
template <typename CT, bool TA, bool TB, bool ACC64, int BK>
__device__ __forceinline__ void gemm_fast_body(const GemmDesc* __restrict__ descs, int ndesc,
                                               const GemmSeg* __restrict__ segs) {
  // row pad: a 144-element row stride puts the four K rows of one operand
  // fragment read on disjoint LDS banks (FP64: halves, FP32: quarters)
  constexpr int BM = 128, BN = 128, PAD = 16;
  constexpr int E = BK / 2;      // elements of each operand one thread moves per K step
  constexpr int NV = E / 2;      // ... as 16-byte vectors
  typedef typename AccT<CT>::T acc_t;
  __shared__ CT As[2][BK][BM + PAD];
  __shared__ CT Bs[2][BK][BN + PAD];

  const int wg = xcd_tile_order(blockIdx.x, gridDim.x);
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_begin <= wg) lo = mid;
    else hi = mid - 1;
  }
  const GemmDesc d = descs[lo];
  int mt, nt;
  grouped_tile(wg - d.tile_begin, d.tilesM, (d.N + BN - 1) / BN, &mt, &nt);
  const int m0 = mt * BM;
  const int n0 = nt * BN;
  if ((d.flags & DESC_LOWER_ONLY) && m0 + BM <= n0) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  // per-thread load coordinates: E consecutive elements per operand per K step
  // (along the operand's stored leading dimension)
  constexpr int TPL = 128 / E;   // threads along a 128-long contiguous run
  const int a_mk = TA ? (tid >> 1) : (tid / TPL);              // TA: m; else k
  const int a_8 = TA ? (tid & 1) * E : (tid % TPL) * E;        // TA: k offset; else m offset
  const int b_nk = TB ? (tid / TPL) : (tid >> 1);              // TB: k; else n
  const int b_8 = TB ? (tid % TPL) * E : (tid & 1) * E;        // TB: n offset; else k offset

  acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;
  // ACC64 (FP32 operands only): the matrix-core partial sums cover at most
  // 1024 of K (and at most one segment) before they are added into FP64
  // accumulators, so the FP32 rounding of long sums (K up to the stack
  // height) does not grow with K
  static_assert(!ACC64 || sizeof(CT) == 4, "FP64 accumulation is for FP32 operands");
  constexpr int kFlushSteps = 1024 / BK;
  double acc64[4][4][4];
  auto flush = [&]() {
    if constexpr (ACC64) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            acc64[i][j][v] += (double)acc[i][j][v];
            acc[i][j][v] = 0;
          }
    }
  };
  if constexpr (ACC64) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc64[i][j][v] = 0.0;
  }

  // PF2 (FP64 operands, A transposed): two register sets, the global loads
  // run two K steps ahead and the LDS writes of the next step are issued
  // after the first quarter of a step's matrix-core work, so both overlap the
  // rest of it.  The untransposed FP64 form (the trailing updates, which run
  // beside the panel kernels) keeps one set: at 216 registers two of its waves
  // leave room on each SIMD for one wave of the tall-panel column kernel.
  // FP32 operands keep one set (their occupancy depends on the registers).
  constexpr bool PF2 = sizeof(CT) == 8 && TA;
  d2v ra0[NV], rb0[NV];
  d2v ra1[PF2 ? NV : 1], rb1[PF2 ? NV : 1];
  for (int sgi = 0; sgi < d.nseg; ++sgi) {
    const GemmSeg sg = segs[d.seg_begin + sgi];
    int kbeg = 0, kend = sg.K;
    if (sg.flags & SEG_A_UPPER) {
      if (TA) kend = min(kend, m0 + BM);
      else kbeg = m0;
    }
    const double* ap = TA ? sg.A + (int64_t)(m0 + a_mk) * sg.lda + kbeg + a_8
                          : sg.A + (int64_t)(kbeg + a_mk) * sg.lda + m0 + a_8;
    const double* bp = TB ? sg.B + (int64_t)(kbeg + b_nk) * sg.ldb + n0 + b_8
                          : sg.B + (int64_t)(n0 + b_nk) * sg.ldb + kbeg + b_8;
    const int64_t astep = TA ? BK : (int64_t)BK * sg.lda;
    const int64_t bstep = TB ? (int64_t)BK * sg.ldb : BK;
    auto gload = [&](d2v (&ra)[NV], d2v (&rb)[NV], int step) {
      const gd2v* pa = (const gd2v*)(ap + step * astep);
      const gd2v* pb = (const gd2v*)(bp + step * bstep);
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        ra[q] = pa[q];
        rb[q] = pb[q];
      }
    };
    auto lstore = [&](const d2v (&ra)[NV], const d2v (&rb)[NV], int buf) {
#pragma unroll
      for (int q = 0; q < NV; ++q)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          if (TA) As[buf][a_8 + 2 * q + e][a_mk] = (CT)ra[q][e];
          else As[buf][a_mk][a_8 + 2 * q + e] = (CT)ra[q][e];
          if (TB) Bs[buf][b_nk][b_8 + 2 * q + e] = (CT)rb[q][e];
          else Bs[buf][b_8 + 2 * q + e][b_nk] = (CT)rb[q][e];
        }
    };
    auto kstep = [&](int buf, int kk) {
      CT af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[buf][kk + (lane >> 4)][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[buf][kk + (lane >> 4)][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma_op(af[i], bf[j], acc[i][j]);
    };
    // one K step from LDS buffer buf; the register set (na, nb) holds the
    // next step's tiles and goes to the other buffer
    auto step = [&](int st, int buf, const d2v (&na)[NV], const d2v (&nb)[NV], bool has_next) {
      kstep(buf, 0);
      if (has_next) lstore(na, nb, buf ^ 1);
#pragma unroll
      for (int kk = 4; kk < BK; kk += 4) kstep(buf, kk);
      __syncthreads();
      if (ACC64 && (st + 1) % kFlushSteps == 0) flush();
    };
    const int nsteps = (kend - kbeg) / BK;
    if (nsteps <= 0) continue;
    gload(ra0, rb0, 0);
    __syncthreads();  // previous segment's last reads of buffer 0 are done
    lstore(ra0, rb0, 0);
    if constexpr (PF2) {
      // pairs of steps with no branch inside: the loads past the end repeat
      // the last step and their LDS copies go to the buffer nobody reads, so
      // every pass has the same loads in flight and the wait before an LDS
      // write covers only the register set it writes
      const int last = nsteps - 1;
      gload(ra1, rb1, min(1, last));
      __syncthreads();
      for (int st = 0; st + 1 < nsteps; st += 2) {
        // even step: buffer 0; set 1 holds step st + 1, set 0 takes step st + 2
        gload(ra0, rb0, min(st + 2, last));
        step(st, 0, ra1, rb1, true);
        // odd step: buffer 1; set 0 holds step st + 2, set 1 takes step st + 3
        gload(ra1, rb1, min(st + 3, last));
        step(st + 1, 1, ra0, rb0, true);
      }
      if (nsteps & 1) {   // the last step, already in buffer 0
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) kstep(0, kk);
      }
    } else {
      // one register set: loads one step ahead, LDS writes after the step
      __syncthreads();
      for (int st = 0; st < nsteps; ++st) {
        const int buf = st & 1;
        const bool more = st + 1 < nsteps;
        if (more) gload(ra0, rb0, st + 1);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) kstep(buf, kk);
        if (more) lstore(ra0, rb0, buf ^ 1);
        __syncthreads();
        if (ACC64 && (st + 1) % kFlushSteps == 0) flush();
      }
    }
    if (ACC64 && nsteps % kFlushSteps != 0) flush();
  }

  // FP64 epilogue through LDS (the A tile buffers, free after the last K
  // step): in four passes of 16 rows of every wave's 64-row half, the
  // accumulators go to a column-major 128 x 32 staging tile, and each thread
  // then moves two consecutive rows of one column, so C, Cin and D2 are read
  // and written as 16-byte vectors, 256 contiguous bytes per 16 lanes,
  // instead of 8 bytes per lane spread over 16 columns.
  if constexpr (sizeof(CT) == 8 && !ACC64) {
    const bool al16 = ((((uintptr_t)d.C) | ((uintptr_t)d.Cin) | ((uintptr_t)d.D2)) & 15) == 0 &&
                      ((d.ldc | d.ldcin | d.ldd2) & 1) == 0;
    if (al16) {
      constexpr int LDW = 34;                   // staging column stride (doubles)
      static_assert(BN * LDW <= 2 * BK * (BM + PAD), "staging tile exceeds the A buffers");
      double* cs = &As[0][0][0];
      const int rr = (tid & 15) * 2;            // staging row pair: 0-15 from wm = 0, 16-31 from wm = 1
      const int grow = rr < 16 ? rr : 64 + rr - 16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        __syncthreads();   // the last K step's reads of As (or the previous pass's reads of cs) are done
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            cs[(wn * 64 + j * 16 + (lane & 15)) * LDW + wm * 16 + 4 * v + (lane >> 4)] = acc[i][j][v];
        __syncthreads();
#pragma unroll
        for (int it = 0; it < BN / 16; ++it) {
          const int c = it * 16 + (tid >> 4);
          const d2v raw = *(const d2v*)(cs + c * LDW + rr);
          const int row = m0 + grow + i * 16;
          const int col = n0 + c;
          if (d.C) {
            d2v cv = raw * d.alpha;
            if (d.Cin) cv += *(const gd2v*)(d.Cin + row + (int64_t)col * d.ldcin) * d.beta;
            *(d2v*)(d.C + row + (int64_t)col * d.ldc) = cv;
          }
          if (d.D2) *(d2v*)(d.D2 + row + (int64_t)col * d.ldd2) = raw;
        }
      }
      return;
    }
  }
  // FP32 operands, FP64 output: the same staging in the (FP32) A buffers,
  // which hold a 128 x 16 FP64 tile: eight passes of 8 rows of every wave's
  // half; the FP32 accumulator layout puts rows 4 g + v (g = lane / 16) in
  // lane group g, so a pass takes two of the four lane groups.
  if constexpr (sizeof(CT) == 4 && !ACC64) {
    const bool al16 = ((((uintptr_t)d.C) | ((uintptr_t)d.Cin) | ((uintptr_t)d.D2)) & 15) == 0 &&
                      ((d.ldc | d.ldcin | d.ldd2) & 1) == 0;
    if (al16) {
      constexpr int LDW = 18;
      static_assert(BN * LDW * 8 <= 2 * BK * (BM + PAD) * (int)sizeof(CT), "staging tile exceeds the A buffers");
      double* cs = (double*)&As[0][0][0];
      const int rr = (tid & 7) * 2;             // staging row pair: 0-7 from wm = 0, 8-15 from wm = 1
      const int grow = (rr < 8 ? rr : 64 + rr - 8);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          __syncthreads();
          if ((lane >> 5) == hh) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                cs[(wn * 64 + j * 16 + (lane & 15)) * LDW + wm * 8 + ((lane >> 4) & 1) * 4 + v] = (double)acc[i][j][v];
          }
          __syncthreads();
#pragma unroll
          for (int it = 0; it < BN / 32; ++it) {
            const int c = it * 32 + (tid >> 3);
            const d2v raw = *(const d2v*)(cs + c * LDW + rr);
            const int row = m0 + grow + i * 16 + hh * 8;
            const int col = n0 + c;
            if (d.C) {
              d2v cv = raw * d.alpha;
              if (d.Cin) cv += *(const gd2v*)(d.Cin + row + (int64_t)col * d.ldcin) * d.beta;
              *(d2v*)(d.C + row + (int64_t)col * d.ldc) = cv;
            }
            if (d.D2) *(d2v*)(d.D2 + row + (int64_t)col * d.ldd2) = raw;
          }
        }
      }
      return;
    }
  }
  constexpr bool f64out = sizeof(CT) == 8;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 64 + i * 16 + (f64out ? v * 4 + (lane >> 4) : (lane >> 4) * 4 + v);
        const double raw = ACC64 ? acc64[i][j][v] : (double)acc[i][j][v];
        if (d.C) {
          double c = d.alpha * raw;
          if (d.Cin) c += d.beta * d.Cin[row + (int64_t)col * d.ldcin];
          d.C[row + (int64_t)col * d.ldc] = c;
        }
        if (d.D2) d.D2[row + (int64_t)col * d.ldd2] = raw;
      }
    }
  }
}

#ifndef BLR_F64_WAVES
#define BLR_F64_WAVES 2
#endif
template <typename CT, bool TA, bool TB>
__global__ __launch_bounds__(256, sizeof(CT) == 8 ? BLR_F64_WAVES : 3) void k_gemm_fast(
    const GemmDesc* __restrict__ descs, int ndesc, const GemmSeg* __restrict__ segs) {
  gemm_fast_body<CT, TA, TB, false, sizeof(CT) == 8 ? kFastKStep64 : kFastKStep32>(descs, ndesc, segs);
}

// FP32 operands, FP64 accumulation across K (long sums); two waves per SIMD
// keep the extra accumulators resident without losing all latency hiding.
template <bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void k_gemm_fast_acc64(const GemmDesc* __restrict__ descs, int ndesc,
                                                            const GemmSeg* __restrict__ segs) {
  gemm_fast_body<float, TA, TB, true, kFastKStep32>(descs, ndesc, segs);
}

}  // namespace

hipError_t launch_gemm(const GemmDesc* d_descs, int ndesc, const GemmSeg* d_segs, int ntiles,
                       int mode, int fp32, hipStream_t stream) {
  if (ndesc <= 0 || ntiles <= 0) return hipSuccess;
  dim3 grid(ntiles), block(256);
#define BLR_FAST(CT, TA, TB)                                                                      \
  do {                                                                                            \
    if (sizeof(CT) == 4 && fp32 == 2)                                                             \
      hipLaunchKernelGGL((k_gemm_fast_acc64<TA, TB>), grid, block, 0, stream, d_descs, ndesc, d_segs); \
    else                                                                                          \
      hipLaunchKernelGGL((k_gemm_fast<CT, TA, TB>), grid, block, 0, stream, d_descs, ndesc, d_segs);   \
  } while (0)
  switch (mode) {
    case GEMM_SMALL:
      if (fp32) hipLaunchKernelGGL((k_gemm<float, 64, 64>), grid, block, 0, stream, d_descs, ndesc, d_segs);
      else hipLaunchKernelGGL((k_gemm<double, 64, 64>), grid, block, 0, stream, d_descs, ndesc, d_segs);
      break;
    case GEMM_BIG:
      if (fp32) hipLaunchKernelGGL((k_gemm<float, 128, 128>), grid, block, 0, stream, d_descs, ndesc, d_segs);
      else hipLaunchKernelGGL((k_gemm<double, 128, 128>), grid, block, 0, stream, d_descs, ndesc, d_segs);
      break;
    case GEMM_FAST_NN:
      if (fp32) BLR_FAST(float, false, false); else BLR_FAST(double, false, false);
      break;
    case GEMM_FAST_TN:
      if (fp32) BLR_FAST(float, true, false); else BLR_FAST(double, true, false);
      break;
    case GEMM_FAST_NT:
      if (fp32) BLR_FAST(float, false, true); else BLR_FAST(double, false, true);
      break;
    case GEMM_FAST_TT:
      if (fp32) BLR_FAST(float, true, true); else BLR_FAST(double, true, true);
      break;
    case GEMM_SKINNY_N:
      if (fp32) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_gemm_skinny<false>), grid, block, 0, stream, d_descs, ndesc, d_segs);
      break;
    case GEMM_SKINNY_T:
      if (fp32) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_gemm_skinny<true>), grid, block, 0, stream, d_descs, ndesc, d_segs);
      break;
    default:
      return hipErrorInvalidValue;
  }
#undef BLR_FAST
  return hipGetLastError();
}
