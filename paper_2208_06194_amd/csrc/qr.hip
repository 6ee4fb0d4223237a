// Householder reflector generation on tiles (Sections 3.4.1 and 3.4.3 of
// arXiv 2208.06194) and the compact-WY factor T (eq. compact_wy).
//
// k_panel factors IB consecutive columns of a tile held in registers (one
// workgroup, 256 threads; thread t owns rows t, t+256, ...).  Each column:
// one block reduction for the tail norm (wavefront shuffles + LDS), the
// larfg scalars, and one block reduction of IB dot products that serves
// both the update of the later panel columns and the Gram column needed by
// the forward T recurrence of this panel.
//
// Two modes:
//  * GEQRT: a (h x IB) panel of a dense tile; the pivot of column jj is local
//    row jj and the reflector is unit lower trapezoidal.
//  * TPQRT: the stack [R; B] with R upper triangular (only its IB x IB
//    diagonal block is touched here) and B an (hb x IB) panel; the reflector
//    of column jj is [e_jj; v] with v spanning all hb rows of B.
//
// k_t_backsolve fills the off-diagonal IB-blocks of the full upper
// triangular T from the Gram matrix G = V^T V: column c of T solves
// (diag(1/tau) + striu(G)) x = e_c, i.e. T[r][c] = -tau_r sum_{t=r+1..c} G[r][t] T[t][c].
#include "device_common.h"
#include "qr.h"

#include <algorithm>

namespace {

// Owner-wave panel factorization: 1024 threads, wave w owns panel columns
// w*CPW .. w*CPW+CPW-1 (IB = 16*CPW), lane l holds rows l + 64*s, s < RS.
// Column jj: the owner wave reduces the tail norm and writes the scaled
// reflector to LDS; every wave then forms the dot products of the reflector
// with its own columns by one wavefront reduction per column and applies the
// rank-one update in registers.
template <int RS, int CPW>
__device__ __forceinline__ void panel_body(const PanelArgs& a) {
  constexpr int IB = 16 * CPW;
  __shared__ double vbuf[64 * RS];
  __shared__ double top[IB][IB + 1];
  __shared__ double Tl[IB][IB + 1];
  __shared__ double gcol[IB];
  __shared__ double sc[2];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const bool tp = a.mode == PANEL_TPQRT;
  const int h = a.h;
  double* X = a.X;
  const int64_t ldx = a.ldx;

  double x[CPW][RS];
#pragma unroll
  for (int cc = 0; cc < CPW; ++cc)
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int r = lane + 64 * s;
      x[cc][s] = (r < h) ? X[r + (int64_t)(w * CPW + cc) * ldx] : 0.0;
    }
  for (int e = tid; e < IB * IB; e += 1024) {
    const int r = e % IB, c = e / IB;
    top[r][c] = (tp && r <= c) ? a.R[r + (int64_t)c * a.ldr] : 0.0;
    Tl[r][c] = 0.0;
  }
  __syncthreads();

  for (int jj = 0; jj < IB; ++jj) {
    const int ow = jj / CPW, oc = jj % CPW;
    const int ps = jj >> 6, pl = jj & 63;   // GEQRT pivot: slot and lane of row jj
    if (w == ow) {
      double val[RS];
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        double t = 0.0;
#pragma unroll
        for (int cc = 0; cc < CPW; ++cc) t = (cc == oc) ? x[cc][s] : t;
        val[s] = t;
      }
      double ss = 0.0, piv = 0.0;
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const int r = lane + 64 * s;
        const bool tail = tp ? (r < h) : (r > jj && r < h);
        ss += tail ? val[s] * val[s] : 0.0;
        piv = (s == ps) ? val[s] : piv;
      }
      ss = wave_sum(ss);
      const double alpha = tp ? top[jj][jj] : __shfl(piv, pl, 64);
      double beta, tau, scal;
      larfg_scalars(alpha, ss, &beta, &tau, &scal);
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const int r = lane + 64 * s;
        const bool tail = tp ? (r < h) : (r > jj && r < h);
        const double v = tail ? val[s] * scal : 0.0;
        vbuf[r] = v;
        const double nv = tail ? v : ((!tp && r == jj) ? beta : val[s]);
#pragma unroll
        for (int cc = 0; cc < CPW; ++cc)
          if (cc == oc) x[cc][s] = nv;
      }
      if (lane == 0) {
        sc[0] = tau;
        sc[1] = beta;
        Tl[jj][jj] = tau;
        a.tau[jj] = tau;
        if (tp) top[jj][jj] = beta;
      }
    }
    __syncthreads();
    const double tau = sc[0];
    double v[RS];
#pragma unroll
    for (int s = 0; s < RS; ++s) v[s] = vbuf[lane + 64 * s];
#pragma unroll
    for (int cc = 0; cc < CPW; ++cc) {
      const int c = w * CPW + cc;
      if (c == jj) continue;
      double d = 0.0, prow = 0.0;
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        d += v[s] * x[cc][s];
        prow = (s == ps) ? x[cc][s] : prow;
      }
      d = wave_sum(d);
      // pivot-row term: GEQRT row jj of column c; TPQRT R(jj, c) for c > jj
      const double pr = tp ? (c > jj ? top[jj][c] : 0.0) : __shfl(prow, pl, 64);
      const double wc = d + pr;
      if (c > jj && tau != 0.0) {
#pragma unroll
        for (int s = 0; s < RS; ++s) x[cc][s] -= tau * wc * v[s];
        if (!tp) {
#pragma unroll
          for (int s = 0; s < RS; ++s)
            if (s == ps && lane == pl) x[cc][s] -= tau * wc;
        } else if (lane == 0) {
          top[jj][c] -= tau * wc;
        }
      }
      if (c < jj && lane == 0) gcol[c] = wc;
    }
    __syncthreads();
    // T column jj of this panel: T[c][jj] = -tau * sum_{t=c}^{jj-1} T[c][t] g_t
    if (tid < jj) {
      double s = 0.0;
      for (int tt = tid; tt < jj; ++tt) s += Tl[tid][tt] * gcol[tt];
      Tl[tid][jj] = -tau * s;
    }
    __syncthreads();
  }

#pragma unroll
  for (int cc = 0; cc < CPW; ++cc)
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int r = lane + 64 * s;
      if (r < h) X[r + (int64_t)(w * CPW + cc) * ldx] = x[cc][s];
    }
  for (int e = tid; e < IB * IB; e += 1024) {
    const int r = e % IB, c = e / IB;
    if (r <= c) {
      if (tp) a.R[r + (int64_t)c * a.ldr] = top[r][c];
      a.T[r + (int64_t)c * a.ldt] = Tl[r][c];
    }
  }
}

// Trailing update of one panel, fused, on the matrix cores: for a block of
// NC = 32 trailing columns,
//   TPQRT: W = R_rows + V^T B;  W2 = T^T W;  R_rows -= W2;  B -= V W2
//   GEQRT: W = V^T C;           W2 = T^T W;  C -= V W2   (V unit lower)
// One workgroup (4 waves) per column block.  V and B are staged through LDS
// in chunks of 64 rows (column-contiguous global reads); V^T B splits each
// chunk's rows over the 4 waves (partial sums reduced in LDS), V W2 gives
// each wave 16 rows of the chunk.
template <int IB>
__device__ __forceinline__ void panel_apply_body(const PanelArgs& a, int nt, int cb) {
  constexpr int NC = 32, CH = 64, MT = IB / 16;
  __shared__ double Vs[CH][IB + 1];
  __shared__ double Bs[CH][NC + 1];
  __shared__ double Wp[4][IB][NC + 1];
  __shared__ double Tt[IB][IB + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const bool tp = a.mode == PANEL_TPQRT;
  const int c0 = cb * NC;
  const int nc = min(NC, nt - c0);
  const int h = a.h;
  const double* V = a.X;
  double* B = a.X + (int64_t)(IB + c0) * a.ldx;
  const int64_t ld = a.ldx;
  for (int e = tid; e < IB * IB; e += 256) Tt[e % IB][e / IB] = a.T[(e % IB) + (int64_t)(e / IB) * a.ldt];

  auto load_v = [&](int r0) {
    for (int e = tid; e < CH * IB; e += 256) {
      const int r = e % CH, l = e / CH, gr = r0 + r;
      double v = 0.0;
      if (gr < h) {
        v = V[gr + (int64_t)l * ld];
        if (!tp) v = gr > l ? v : (gr == l ? 1.0 : 0.0);
      }
      Vs[r][l] = v;
    }
  };

  // phase 1: W = V^T B
  v4d acc[MT][2];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[mt][j][v] = 0.0;
  for (int r0 = 0; r0 < h; r0 += CH) {
    __syncthreads();
    load_v(r0);
    for (int e = tid; e < CH * NC; e += 256) {
      const int r = e % CH, c = e / CH, gr = r0 + r;
      Bs[r][c] = (gr < h && c < nc) ? B[gr + (int64_t)c * ld] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kr = 16 * w + 4 * ks + (lane >> 4);
      double af[MT], bf[2];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) af[mt] = Vs[kr][mt * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = Bs[kr][j * 16 + (lane & 15)];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[mt][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mt], bf[j], acc[mt][j], 0, 0, 0);
    }
  }
  // f64 MFMA output layout: accumulator v of lane l is row 4v + l/16, column l%16
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) Wp[w][mt * 16 + 4 * v + (lane >> 4)][j * 16 + (lane & 15)] = acc[mt][j][v];
  __syncthreads();
  for (int e = tid; e < IB * NC; e += 256) {
    const int l = e % IB, c = e / IB;
    double s = Wp[0][l][c] + Wp[1][l][c] + Wp[2][l][c] + Wp[3][l][c];
    if (tp && c < nc) s += a.R[l + (int64_t)(IB + c0 + c) * a.ldr];
    Wp[0][l][c] = s;
  }
  __syncthreads();
  // W2 = T^T W (T upper triangular), kept in Wp[1]; R_rows -= W2
  for (int e = tid; e < IB * NC; e += 256) {
    const int l = e % IB, c = e / IB;
    double s = 0.0;
    for (int m = 0; m <= l; ++m) s += Tt[m][l] * Wp[0][m][c];
    Wp[1][l][c] = s;
    if (tp && c < nc) a.R[l + (int64_t)(IB + c0 + c) * a.ldr] -= s;
  }
  // phase 3: B -= V W2, 64 rows per chunk, wave w computes rows 16w..16w+15
  for (int r0 = 0; r0 < h; r0 += CH) {
    __syncthreads();
    load_v(r0);
    __syncthreads();
    v4d p[2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) p[j][v] = 0.0;
#pragma unroll
    for (int ks = 0; ks < IB / 4; ++ks) {
      const double af = Vs[16 * w + (lane & 15)][4 * ks + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const double bf = Wp[1][4 * ks + (lane >> 4)][j * 16 + (lane & 15)];
        p[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf, p[j], 0, 0, 0);
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) Bs[16 * w + 4 * v + (lane >> 4)][j * 16 + (lane & 15)] = p[j][v];
    __syncthreads();
    for (int e = tid; e < CH * NC; e += 256) {
      const int r = e % CH, c = e / CH, gr = r0 + r;
      if (gr < h && c < nc) B[gr + (int64_t)c * ld] -= Bs[r][c];
    }
  }
}

// One wave per column c of T (n x n); rows above the IB-block of c are
// filled by back-substitution in blocks of 8 rows: the 8 dot products with
// the already known part of the column are formed together (their loads and
// reductions overlap), then the 8 x 8 triangle is solved redundantly by every
// lane.  Lane l owns x[t] for t = l (mod 64) in LDS.
__device__ __forceinline__ void t_backsolve_body(const TBackArgs& a, int cb) {
  extern __shared__ double xs[];  // 4 waves x n
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = cb * 4 + wave;
  if (c >= a.n) return;
  double* x = xs + (size_t)wave * a.n;
  const int bs = (c / a.ib) * a.ib;
  const double* G = a.G;
  const int64_t ldg = a.ldg;
  for (int t = bs + ((lane - bs) & 63); t <= c; t += 64) x[t] = a.T[t + (int64_t)c * a.ldt];
  for (int r1 = bs - 1; r1 >= 0; r1 -= 8) {
    const int r0 = r1 - 7;   // block rows r0..r1 (bs is a multiple of 8)
    double d[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) d[q] = 0.0;
    for (int t = r1 + 1 + ((lane - (r1 + 1)) & 63); t <= c; t += 64) {
      const double xt = x[t];
#pragma unroll
      for (int q = 0; q < 8; ++q) d[q] += G[t + (int64_t)(r0 + q) * ldg] * xt;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) d[q] = wave_sum(d[q]);
    // within-block triangle: rows r1 down to r0
    double xb[8];
#pragma unroll
    for (int q = 7; q >= 0; --q) {
      double s = d[q];
#pragma unroll
      for (int u = q + 1; u < 8; ++u) s += G[(r0 + u) + (int64_t)(r0 + q) * ldg] * xb[u];
      xb[q] = -a.tau[r0 + q] * s;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = r0 + q;
      if ((r & 63) == lane) x[r] = xb[q];
      if (lane == q) a.T[r + (int64_t)c * a.ldt] = xb[q];
    }
  }
  for (int r = c + 1 + lane; r < a.n; r += 64) a.T[r + (int64_t)c * a.ldt] = 0.0;
}


// Split-K trailing update of a tall panel (V unit lower, h rows, IB columns)
// applied to the nt columns right of it: grid (nt/32 column blocks) x S row
// slices.  k_tall_apply_part writes each slice's V^T C into part;
// k_tall_apply_upd sums the slices, forms W2 = T^T W and updates its slice:
// C -= V W2.
template <int IB>
__device__ __forceinline__ void tall_apply_part_body(const PanelArgs& a, int nt, double* part, int cb, int sl,
                                                     int NB, int S) {
  constexpr int NC = 32, CH = 64, MT = IB / 16;
  __shared__ double Vs[CH][IB + 1];
  __shared__ double Bs[CH][NC + 1];
  __shared__ double Wp[4][IB][NC + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c0 = cb * NC, nc = min(NC, nt - c0);
  const int h = a.h;
  const int slice = ((h + S - 1) / S + CH - 1) / CH * CH;
  const int rb = sl * slice, rend = min(h, rb + slice);
  const double* V = a.X;
  const double* B = a.X + (int64_t)(IB + c0) * a.ldx;
  const int64_t ld = a.ldx;
  v4d acc[MT][2];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[mt][j][v] = 0.0;
  for (int r0 = rb; r0 < rend; r0 += CH) {
    __syncthreads();
    for (int e = tid; e < CH * IB; e += 256) {
      const int r = e % CH, l = e / CH, gr = r0 + r;
      double v = 0.0;
      if (gr < rend) {
        v = V[gr + (int64_t)l * ld];
        v = gr > l ? v : (gr == l ? 1.0 : 0.0);
      }
      Vs[r][l] = v;
    }
    for (int e = tid; e < CH * NC; e += 256) {
      const int r = e % CH, c = e / CH, gr = r0 + r;
      Bs[r][c] = (gr < rend && c < nc) ? B[gr + (int64_t)c * ld] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kr = 16 * w + 4 * ks + (lane >> 4);
      double af[MT], bf[2];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) af[mt] = Vs[kr][mt * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = Bs[kr][j * 16 + (lane & 15)];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[mt][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mt], bf[j], acc[mt][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) Wp[w][mt * 16 + 4 * v + (lane >> 4)][j * 16 + (lane & 15)] = acc[mt][j][v];
  __syncthreads();
  double* out = part + ((int64_t)sl * NB + cb) * IB * NC;
  for (int e = tid; e < IB * NC; e += 256) {
    const int l = e % IB, c = e / IB;
    out[e] = Wp[0][l][c] + Wp[1][l][c] + Wp[2][l][c] + Wp[3][l][c];
  }
}

template <int IB>
__device__ __forceinline__ void tall_apply_upd_body(const PanelArgs& a, int nt, const double* part, int cb, int sl,
                                                    int NB, int S) {
  constexpr int NC = 32, CH = 64;
  __shared__ double Vs[CH][IB + 1];
  __shared__ double Ps[CH][NC + 1];
  __shared__ double W[IB][NC + 1];
  __shared__ double W2[IB][NC + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c0 = cb * NC, nc = min(NC, nt - c0);
  const int h = a.h;
  const int slice = ((h + S - 1) / S + CH - 1) / CH * CH;
  const int rb = sl * slice, rend = min(h, rb + slice);
  const double* V = a.X;
  double* B = a.X + (int64_t)(IB + c0) * a.ldx;
  const int64_t ld = a.ldx;
  for (int e = tid; e < IB * NC; e += 256) {
    // eight independent partial sums keep eight loads in flight
    double s8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) s8[u] = 0.0;
    int q = 0;
    for (; q + 8 <= S; q += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) s8[u] += part[((int64_t)(q + u) * NB + cb) * IB * NC + e];
    }
    for (; q < S; ++q) s8[0] += part[((int64_t)q * NB + cb) * IB * NC + e];
    W[e % IB][e / IB] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
  }
  __syncthreads();
  for (int e = tid; e < IB * NC; e += 256) {
    const int l = e % IB, c = e / IB;
    double s = 0.0;
    for (int m = 0; m <= l; ++m) s += a.T[m + (int64_t)l * a.ldt] * W[m][c];
    W2[l][c] = s;
  }
  for (int r0 = rb; r0 < rend; r0 += CH) {
    __syncthreads();
    for (int e = tid; e < CH * IB; e += 256) {
      const int r = e % CH, l = e / CH, gr = r0 + r;
      double v = 0.0;
      if (gr < rend) {
        v = V[gr + (int64_t)l * ld];
        v = gr > l ? v : (gr == l ? 1.0 : 0.0);
      }
      Vs[r][l] = v;
    }
    __syncthreads();
    v4d pr[2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) pr[j][v] = 0.0;
#pragma unroll
    for (int ks = 0; ks < IB / 4; ++ks) {
      const double af = Vs[16 * w + (lane & 15)][4 * ks + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const double bf = W2[4 * ks + (lane >> 4)][j * 16 + (lane & 15)];
        pr[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf, pr[j], 0, 0, 0);
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) Ps[16 * w + 4 * v + (lane >> 4)][j * 16 + (lane & 15)] = pr[j][v];
    __syncthreads();
    for (int e = tid; e < CH * NC; e += 256) {
      const int r = e % CH, c = e / CH, gr = r0 + r;
      if (gr < rend && c < nc) B[gr + (int64_t)c * ld] -= Ps[r][c];
    }
  }
}

// ---------------------------------------------------------------------------
// Tall panels as a tree (TSQR) with Householder reconstruction (the tree and
// its buffers are described with TsqrTree in qr.h).  Row split of n items
// into parts balanced groups: group g covers [g base + min(g, rem), ...).
__device__ __forceinline__ int tsqr_first(int n, int parts, int g) {
  const int base = n / parts, rem = n % parts;
  return g * base + min(g, rem);
}
__device__ __forceinline__ int tsqr_parent(int i, int n, int parts) {
  const int base = n / parts, rem = n % parts, edge = rem * (base + 1);
  return i < edge ? i / (base + 1) : rem + (i - edge) / base;
}

// Householder QR (larfg convention) of one block of at most kTsqrRows rows
// and 16 columns: thread r holds row r.  Column j: one block reduction of
// the 16 dot products of the column's tail (rows below j) with every column
// gives the tail norm, the update coefficients w_t = x_jt + s d_t of the
// later columns and the Gram entries g_v = Y_v^T v_j of the T recurrence.
// The wave part of the reduction is a butterfly that halves the values at
// each exchange (8 + 4 + 2 + 1 + 2 shuffles instead of 16 x 6); the four
// wave partials and the pivot row go through double-buffered LDS, and every
// thread forms the larfg scalars itself, so a column costs one barrier.  T is
// formed after the last column from the saved Gram entries and taus.
__device__ __forceinline__ void tsqr_qr_body(const TsqrTree& tr, int level, int node) {
  constexpr int IB = kTsqrIB, NT = kTsqrRows, NW = NT / 64;
  __shared__ double red[2][NW][IB];
  __shared__ double piv[2][IB];
  __shared__ double Gs[IB][IB + 1];   // Gs[v][j]: Gram entry of reflector v with reflector j
  __shared__ double taus[IB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int L = tr.levels;
  double* X;
  int64_t ld;
  int rows;
  if (level == 0) {
    const int s0 = tsqr_first(tr.h, tr.count[0], node), s1 = tsqr_first(tr.h, tr.count[0], node + 1);
    X = tr.X + s0;
    ld = tr.ldx;
    rows = s1 - s0;
  } else {
    const int np = tr.count[level - 1], nc = tr.count[level];
    const int c0 = tsqr_first(np, nc, node), c1 = tsqr_first(np, nc, node + 1);
    ld = (int64_t)np * IB;
    X = tr.S[level] + (int64_t)c0 * IB;
    rows = (c1 - c0) * IB;
  }
  const bool own = tid < rows;
  double x[IB];
#pragma unroll
  for (int t = 0; t < IB; ++t) x[t] = own ? X[tid + (int64_t)t * ld] : 0.0;
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
#pragma unroll
  for (int j = 0; j < IB; ++j) {
    const int bf = j & 1;
    if (tid == j) {
#pragma unroll
      for (int t = 0; t < IB; ++t) piv[bf][t] = x[t];
    }
    // d_t = sum over rows r > j of x_rj x_rt, reduced over the wave
    const double xj = (own && tid > j) ? x[j] : 0.0;
    double a8[8], a4[4], a2[2], a1;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double lo = xj * x[u], hi = xj * x[u + 8];
      a8[u] = (b5 ? hi : lo) + __shfl_xor(b5 ? lo : hi, 32, 64);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) a4[u] = (b4 ? a8[u + 4] : a8[u]) + __shfl_xor(b4 ? a8[u] : a8[u + 4], 16, 64);
#pragma unroll
    for (int u = 0; u < 2; ++u) a2[u] = (b3 ? a4[u + 2] : a4[u]) + __shfl_xor(b3 ? a4[u] : a4[u + 2], 8, 64);
    a1 = (b2 ? a2[1] : a2[0]) + __shfl_xor(b2 ? a2[0] : a2[1], 4, 64);
    a1 += __shfl_xor(a1, 2, 64);
    a1 += __shfl_xor(a1, 1, 64);
    if ((lane & 3) == 0) red[bf][wave][lane >> 2] = a1;
    __syncthreads();
    // every thread: the larfg scalars of column j (the same sums in the same
    // order in every thread)
    double dj = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) dj += red[bf][q][j];
    double beta, tau, scal;
    larfg_scalars(piv[bf][j], dj, &beta, &tau, &scal);
    if (tid < j) {
      double d = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) d += red[bf][q][tid];
      Gs[tid][j] = piv[bf][tid] + scal * d;
    } else if (tid == j) {
      taus[j] = tau;
    }
    if (own && tid >= j) {
      const double v = tid > j ? x[j] * scal : 1.0;
#pragma unroll
      for (int t = j + 1; t < IB; ++t) {
        double d = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) d += red[bf][q][t];
        x[t] -= tau * (piv[bf][t] + scal * d) * v;
      }
      x[j] = tid > j ? v : beta;
    }
  }
  if (own) {
#pragma unroll
    for (int t = 0; t < IB; ++t) X[tid + (int64_t)t * ld] = x[t];
  }
  __syncthreads();
  if (tid < IB) {
    const int r = tid;
    if (level < L) {
      // R of this block into the next level's stack (zeros below the diagonal)
      double* Rn = tr.S[level + 1] + (int64_t)node * IB;
      const int64_t ldn = (int64_t)tr.count[level] * IB;
#pragma unroll
      for (int c = 0; c < IB; ++c) Rn[r + (int64_t)c * ldn] = c >= r ? x[c] : 0.0;
    }
    if (level == 0 && L > 0) {
      double* Y1 = tr.Y1 + (int64_t)node * IB * IB;
#pragma unroll
      for (int c = 0; c < IB; ++c) Y1[r + c * IB] = c < r ? x[c] : (c == r ? 1.0 : 0.0);
    }
    // row r of T: T[r][r] = tau_r, T[r][j] = -tau_j sum_{v=r}^{j-1} T[r][v] g_v^(j)
    double* Tout;
    int64_t ldt;
    if (L == 0) {
      Tout = tr.T;
      ldt = tr.ldt;
      tr.tau[r] = taus[r];
    } else {
      Tout = tr.Tn[level] + (int64_t)node * IB * IB;
      ldt = IB;
    }
    double trow[IB];
#pragma unroll
    for (int jj = 0; jj < IB; ++jj) {
      double sum = 0.0;
#pragma unroll
      for (int v = 0; v < jj; ++v)
        if (v >= r) sum += trow[v] * Gs[v][jj];
      trow[jj] = jj < r ? 0.0 : (jj == r ? taus[r] : -taus[jj] * sum);
      if (jj >= r) Tout[r + (int64_t)jj * ldt] = trow[jj];
    }
  }
}

// C of the leaf gg: the 16 rows of the explicit Q of each tree node above
// it, from the root (C = I) down, C_child = E_j C - Y_j T Y_1^T C with Y_j
// the node's reflector rows of child j and Y_1 its top (unit lower) block.
// Thread (i, k) = (tid / 16, tid % 16) holds one element.
__device__ __forceinline__ void tsqr_walk(const TsqrTree& tr, int gg, double (*C)[kTsqrIB + 1],
                                          double (*P)[kTsqrIB + 1], double (*M)[kTsqrIB + 1]) {
  constexpr int IB = kTsqrIB;
  const int tid = threadIdx.x, i = tid >> 4, k = tid & 15;
  C[i][k] = i == k ? 1.0 : 0.0;
  __syncthreads();
#pragma unroll 1
  for (int l = tr.levels; l >= 1; --l) {
    int child = gg;   // ancestor of gg at level l - 1
#pragma unroll 1
    for (int m = 1; m < l; ++m) child = tsqr_parent(child, tr.count[m - 1], tr.count[m]);
    const int np = tr.count[l - 1], nc = tr.count[l];
    const int node = tsqr_parent(child, np, nc);
    const int fc = tsqr_first(np, nc, node);
    const int j = child - fc;
    const int64_t ld = (int64_t)np * IB;
    const double* Y = tr.S[l] + (int64_t)fc * IB;
    const double* T = tr.Tn[l] + (int64_t)node * IB * IB;
    // fixed trip counts with masks: the loops unroll without versions
    double s = C[i][k];
#pragma unroll
    for (int m = 0; m < IB; ++m)
      if (m > i) s += Y[m + (int64_t)i * ld] * C[m][k];
    P[i][k] = s;
    __syncthreads();
    s = 0.0;
#pragma unroll
    for (int m = 0; m < IB; ++m)
      if (m >= i) s += T[i + m * IB] * P[m][k];
    M[i][k] = s;
    __syncthreads();
    double cn;
    if (j == 0) {
      cn = C[i][k] - M[i][k];
#pragma unroll
      for (int m = 0; m < IB; ++m)
        if (m < i) cn -= Y[i + (int64_t)m * ld] * M[m][k];
    } else {
      cn = 0.0;
      const double* Yr = Y + (int64_t)j * IB + i;
#pragma unroll
      for (int m = 0; m < IB; ++m) cn -= Yr[(int64_t)m * ld] * M[m][k];
    }
    __syncthreads();
    C[i][k] = cn;
    __syncthreads();
  }
}

// Leaf level of the same step: M = T_g Y1_g^T C (Y1_g explicit unit lower).
__device__ __forceinline__ void tsqr_leaf_m(const TsqrTree& tr, int g, double (*C)[kTsqrIB + 1],
                                            double (*P)[kTsqrIB + 1], double (*M)[kTsqrIB + 1]) {
  constexpr int IB = kTsqrIB;
  const int tid = threadIdx.x, i = tid >> 4, k = tid & 15;
  const double* Y1 = tr.Y1 + (int64_t)g * IB * IB;
  const double* T = tr.Tn[0] + (int64_t)g * IB * IB;
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < IB; ++m)
    if (m >= i) s += Y1[m + i * IB] * C[m][k];
  P[i][k] = s;
  __syncthreads();
  s = 0.0;
#pragma unroll
  for (int m = 0; m < IB; ++m)
    if (m >= i) s += T[i + m * IB] * P[m][k];
  M[i][k] = s;
  __syncthreads();
}

// Final step for leaf g (levels >= 1): its rows of Q = H_g [C_g; 0], then
// the reconstruction.  Q's top block A = Q(0:16, :) (leaf 0's first rows)
// is factored A - D = L U with d_i = -sign of the current pivot, so that
// the pivot U_ii = a_ii - d_i has magnitude at least 1; then the panel's
// Householder vectors are [L; Q(16:, :) U^-1], T = -U D L^-T, tau = diag(T)
// and R = D R_root.  Every leaf factors A itself (16 x 16, from leaf 0's
// side copies), so the step is one launch; leaf 0 writes the top rows, T
// and tau.
__device__ __forceinline__ void tsqr_final_body(const TsqrTree& tr, int g) {
  constexpr int IB = kTsqrIB;
  __shared__ double Cb[IB][IB + 1];
  __shared__ double Pb[IB][IB + 1];
  __shared__ double Mb[IB][IB + 1];
  __shared__ double A[IB][IB + 1];
  __shared__ double Lb[IB][IB + 1];
  __shared__ double dsg[IB], ipd[IB];
  const int tid = threadIdx.x, i = tid >> 4, k = tid & 15;
  const int s0 = tsqr_first(tr.h, tr.count[0], g), s1 = tsqr_first(tr.h, tr.count[0], g + 1);
  const int rows = s1 - s0;
  const bool own = tid < rows;
  double* X = tr.X + s0;
  const int64_t ld = tr.ldx;
  // 1. Q's top block from leaf 0, and its signed LU
  tsqr_walk(tr, 0, Cb, Pb, Mb);
  tsqr_leaf_m(tr, 0, Cb, Pb, Mb);
  {
    const double* Y10 = tr.Y1;
    double a = Cb[i][k];
#pragma unroll
    for (int m = 0; m < IB; ++m)
      if (m <= i) a -= Y10[i + m * IB] * Mb[m][k];
    A[i][k] = a;
    Lb[i][k] = i == k ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < IB; ++c) {
    const double acc = A[c][c];
    const double d = acc >= 0.0 ? -1.0 : 1.0;
    const double p = acc - d;
    const double aic = A[i][c], aci = A[c][k];
    __syncthreads();
    if (i > c) {
      const double l = aic / p;
      if (k == c) Lb[i][c] = l;
      else if (k > c) A[i][k] -= l * aci;
    }
    if (tid == 0) {
      dsg[c] = d;
      ipd[c] = 1.0 / p;
      A[c][c] = p;
    }
    __syncthreads();
  }
  // 2. this leaf's C and M
  tsqr_walk(tr, g, Cb, Pb, Mb);
  tsqr_leaf_m(tr, g, Cb, Pb, Mb);
  // 3. rows of the reconstructed reflectors: (E - y M) U^-1 with E this
  // row of [C_g; 0] and y its row of the leaf's reflectors (unit lower).
  // W = M U^-1 and E U^-1 (= C_g U^-1 on the leaf's first rows) are formed
  // once, by forward substitution, so that every row is one product with W.
  if (tid < 2 * IB) {
    double (*src)[IB + 1] = tid < IB ? Mb : Cb;
    const int r = tid & 15;
    for (int t = 0; t < IB; ++t) {
      double s = src[r][t];
      for (int m = 0; m < t; ++m) s -= src[r][m] * A[m][t];
      src[r][t] = s * ipd[t];
    }
  }
  __syncthreads();
  if (own) {
    if (s0 + tid >= IB) {
      double y[IB];
#pragma unroll
      for (int t = 0; t < IB; ++t) {
        const double v = X[tid + (int64_t)t * ld];
        y[t] = tid > t ? v : (tid == t ? 1.0 : 0.0);
      }
#pragma unroll
      for (int t = 0; t < IB; ++t) {
        double z = (tid < IB) ? Cb[tid][t] : 0.0;
#pragma unroll
        for (int m = 0; m < IB; ++m) z -= y[m] * Mb[m][t];
        X[tid + (int64_t)t * ld] = z;
      }
    } else {
      // top rows (leaf 0): L below the diagonal, D R_root on and above it
      const int r = tid;
      const double* Rr = tr.S[tr.levels];
      const int64_t ldr = (int64_t)tr.count[tr.levels - 1] * IB;
#pragma unroll
      for (int t = 0; t < IB; ++t)
        X[r + (int64_t)t * ld] = t < r ? Lb[r][t] : dsg[r] * Rr[r + (int64_t)t * ldr];
    }
  }
  // 4. T = -U D L^-T and tau (leaf 0): row r solves t L^T = -(U D)_r (the
  // row is built in Pb, which only thread r touches)
  if (g == 0 && tid < IB) {
    const int r = tid;
    for (int c = 0; c < IB; ++c) {
      double s = c >= r ? -A[r][c] * dsg[c] : 0.0;
      for (int m = 0; m < c; ++m) s -= Pb[r][m] * Lb[c][m];
      Pb[r][c] = s;
    }
    for (int c = r; c < IB; ++c) tr.T[r + (int64_t)c * tr.ldt] = Pb[r][c];
    tr.tau[r] = Pb[r][r];
  }
}

__device__ __forceinline__ int tsqr_item(const TsqrItem* items, int n, int wg) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].wg_begin <= wg) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kTsqrRows, 6) void k_tsqr_qr(const TsqrTree* __restrict__ trees,
                                                       const TsqrItem* __restrict__ items, int n) {
  const int it = tsqr_item(items, n, blockIdx.x);
  const TsqrItem I = items[it];
  tsqr_qr_body(trees[I.tree], I.level, blockIdx.x - I.wg_begin);
}
__global__ __launch_bounds__(kTsqrRows, 6) void k_tsqr_final(const TsqrTree* __restrict__ trees,
                                                          const TsqrItem* __restrict__ items, int n) {
  const int it = tsqr_item(items, n, blockIdx.x);
  const TsqrItem I = items[it];
  tsqr_final_body(trees[I.tree], blockIdx.x - I.wg_begin);
}

// Batched copy of column-major blocks (gather / scatter of the stacked
// block column), and the explicit unit-lower form of a packed reflector block.
__global__ void k_copy_blocks(const CopyDesc* __restrict__ d) {
  const CopyDesc D = d[blockIdx.y];
  if (D.unit_lower == 3) {   // one int32
    if (blockIdx.x == 0 && threadIdx.x == 0) *(int*)D.dst = *(const int*)D.src;
    return;
  }
  const int64_t n = (int64_t)D.rows * D.cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % D.rows, c = e / D.rows;
    double v = D.src[r + c * D.lds];
    for (int q = 1; q < D.nsum; ++q) v += D.src[r + c * D.lds + q * D.sstride];
    if (D.unit_lower == 1) v = r > c ? v : (r == c ? 1.0 : 0.0);
    else if (D.unit_lower == 2) v = r <= c ? v : 0.0;
    D.dst[r + c * D.ldd] = v;
  }
}

// Modified Gram-Schmidt QR of the stacked right factors of a block column
// (the comparison method, Section 2.1 Alg. 1 with Section 3.2), in one
// workgroup of 16 waves.  Column c: r_cc = ||x_c|| (block reduction),
// q_c = x_c / r_cc; then every later column d, one wave each, takes
// r_cd = q_c^T x_d (wave reduction over its rows, lanes striding) and
// x_d -= r_cd q_c.  The summation order is fixed.
__global__ __launch_bounds__(1024) void k_mgs_stack(double* X, int64_t ldx, int h, int w, double* R, int64_t ldr) {
  __shared__ double red[16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int c = 0; c < w; ++c) {
    double* xc = X + (int64_t)c * ldx;
    double s = 0.0;
    for (int r = tid; r < h; r += 1024) s += xc[r] * xc[r];
    const double rcc = sqrt(block_sum(s, red));
    for (int r = tid; r < h; r += 1024) xc[r] = xc[r] / rcc;
    if (tid == 0) R[c + (int64_t)c * ldr] = rcc;
    for (int r = c + 1 + tid; r < w; r += 1024) R[r + (int64_t)c * ldr] = 0.0;
    __syncthreads();   // q_c is written before the waves read it
    for (int d = c + 1 + wv; d < w; d += 16) {
      double* xd = X + (int64_t)d * ldx;
      double t = 0.0;
      for (int r = lane; r < h; r += 64) t += xc[r] * xd[r];
      t = wave_sum(t);
      for (int r = lane; r < h; r += 64) xd[r] -= t * xc[r];
      if (lane == 0) R[c + (int64_t)d * ldr] = t;
    }
    __syncthreads();   // the updates are done before the next column's norm
  }
}

// Single-problem kernels: the grid covers one problem.
template <int RS, int CPW>
__global__ __launch_bounds__(1024) void k_panel(PanelArgs a) { panel_body<RS, CPW>(a); }
template <int IB>
__global__ __launch_bounds__(256) void k_panel_apply(PanelArgs a, int nt) { panel_apply_body<IB>(a, nt, blockIdx.x); }
__global__ __launch_bounds__(256) void k_t_backsolve(TBackArgs a) { t_backsolve_body(a, blockIdx.x); }
template <int IB>
__global__ __launch_bounds__(256) void k_tall_apply_part(PanelArgs a, int nt, double* part) {
  tall_apply_part_body<IB>(a, nt, part, blockIdx.x, blockIdx.y, gridDim.x, gridDim.y);
}
template <int IB>
__global__ __launch_bounds__(256) void k_tall_apply_upd(PanelArgs a, int nt, const double* part) {
  tall_apply_upd_body<IB>(a, nt, part, blockIdx.x, blockIdx.y, gridDim.x, gridDim.y);
}

// Batched kernels: the last grid dimension indexes the job; the others span
// the largest job, and workgroups beyond a job's own extent exit at once
// (before any barrier).  Each job gets exactly the workgroups, and therefore
// the partitioning and summation order, of its single-problem launch.
template <int RS, int CPW>
__global__ __launch_bounds__(1024) void k_panel_batch(const PanelJob* __restrict__ jobs) {
  const PanelArgs a = jobs[blockIdx.x].a;
  panel_body<RS, CPW>(a);
}
template <int IB>
__global__ __launch_bounds__(256) void k_panel_apply_batch(const PanelJob* __restrict__ jobs) {
  const PanelArgs a = jobs[blockIdx.y].a;
  const int nt = jobs[blockIdx.y].nt;
  if ((int)blockIdx.x >= (nt + 31) / 32) return;
  panel_apply_body<IB>(a, nt, blockIdx.x);
}
__global__ __launch_bounds__(256) void k_t_backsolve_batch(const PanelJob* __restrict__ jobs) {
  const TBackArgs a = jobs[blockIdx.y].tb;
  if ((int)blockIdx.x >= (a.n + 3) / 4) return;
  t_backsolve_body(a, blockIdx.x);
}
template <int IB>
__global__ __launch_bounds__(256) void k_tall_apply_part_batch(const PanelJob* __restrict__ jobs) {
  const PanelJob& J = jobs[blockIdx.z];
  const PanelArgs a = J.a;
  const int nt = J.nt, S = J.groups, NB = (nt + 31) / 32;
  double* part = J.part;
  if ((int)blockIdx.x >= NB || (int)blockIdx.y >= S) return;
  tall_apply_part_body<IB>(a, nt, part, blockIdx.x, blockIdx.y, NB, S);
}
template <int IB>
__global__ __launch_bounds__(256) void k_tall_apply_upd_batch(const PanelJob* __restrict__ jobs) {
  const PanelJob& J = jobs[blockIdx.z];
  const PanelArgs a = J.a;
  const int nt = J.nt, S = J.groups, NB = (nt + 31) / 32;
  const double* part = J.part;
  if ((int)blockIdx.x >= NB || (int)blockIdx.y >= S) return;
  tall_apply_upd_body<IB>(a, nt, part, blockIdx.x, blockIdx.y, NB, S);
}

}  // namespace

hipError_t launch_tall_apply(const PanelArgs& a, int nt, int slices, double* part, hipStream_t stream) {
  if (nt <= 0) return hipSuccess;
  if (slices < 1 || slices > kTallApplySlices) return hipErrorInvalidValue;
  dim3 grid((nt + 31) / 32, slices), block(256);
  if (a.ib == 32) {
    hipLaunchKernelGGL((k_tall_apply_part<32>), grid, block, 0, stream, a, nt, part);
    hipLaunchKernelGGL((k_tall_apply_upd<32>), grid, block, 0, stream, a, nt, (const double*)part);
  } else if (a.ib == 16) {
    hipLaunchKernelGGL((k_tall_apply_part<16>), grid, block, 0, stream, a, nt, part);
    hipLaunchKernelGGL((k_tall_apply_upd<16>), grid, block, 0, stream, a, nt, (const double*)part);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tsqr_qr(const TsqrTree* trees, const TsqrItem* items, int n, int total_wg, hipStream_t stream) {
  if (n <= 0 || total_wg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tsqr_qr, dim3(total_wg), dim3(kTsqrRows), 0, stream, trees, items, n);
  return hipGetLastError();
}

hipError_t launch_tsqr_final(const TsqrTree* trees, const TsqrItem* items, int n, int total_wg,
                             hipStream_t stream) {
  if (n <= 0 || total_wg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tsqr_final, dim3(total_wg), dim3(kTsqrRows), 0, stream, trees, items, n);
  return hipGetLastError();
}

hipError_t launch_copy_blocks(const CopyDesc* d, int n, int64_t max_elems, hipStream_t stream) {
  if (n <= 0 || max_elems <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((max_elems + 255) / 256, 256);
  hipLaunchKernelGGL(k_copy_blocks, dim3(blocks, n), dim3(256), 0, stream, d);
  return hipGetLastError();
}

hipError_t launch_mgs_stack(double* X, int64_t ldx, int h, int w, double* R, int64_t ldr, hipStream_t stream) {
  if (h <= 0 || w <= 0) return hipSuccess;
  if (w > h || ldx < h || ldr < w) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mgs_stack, dim3(1), dim3(1024), 0, stream, X, ldx, h, w, R, ldr);
  return hipGetLastError();
}

hipError_t launch_panel(const PanelArgs& a, hipStream_t stream) {
  const int rs = (a.h + 63) / 64;
  dim3 grid(1), block(1024);
#define BLR_PANEL(RSV, CPWV) hipLaunchKernelGGL((k_panel<RSV, CPWV>), grid, block, 0, stream, a)
  if (a.ib == 32) {
    if (rs <= 1) BLR_PANEL(1, 2);
    else if (rs <= 2) BLR_PANEL(2, 2);
    else if (rs <= 4) BLR_PANEL(4, 2);
    else if (rs <= 8) BLR_PANEL(8, 2);
    else return hipErrorInvalidValue;  // tall panels use ib = 16 (register budget)
  } else if (a.ib == 16) {
    if (rs <= 1) BLR_PANEL(1, 1);
    else if (rs <= 2) BLR_PANEL(2, 1);
    else if (rs <= 4) BLR_PANEL(4, 1);
    else if (rs <= 8) BLR_PANEL(8, 1);
    else if (rs <= 16) BLR_PANEL(16, 1);
    else return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
#undef BLR_PANEL
  return hipGetLastError();
}

hipError_t launch_panel_apply(const PanelArgs& a, int nt, hipStream_t stream) {
  if (nt <= 0) return hipSuccess;
  dim3 grid((nt + 31) / 32), block(256);
  if (a.ib == 32) hipLaunchKernelGGL((k_panel_apply<32>), grid, block, 0, stream, a, nt);
  else if (a.ib == 16) hipLaunchKernelGGL((k_panel_apply<16>), grid, block, 0, stream, a, nt);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_t_backsolve(const TBackArgs& a, hipStream_t stream) {
  if (a.n <= a.ib) return hipSuccess;
  dim3 grid((a.n + 3) / 4), block(256);
  hipLaunchKernelGGL(k_t_backsolve, grid, block, (size_t)4 * a.n * sizeof(double), stream, a);
  return hipGetLastError();
}

hipError_t launch_panel_batch(const PanelJob* d, int n, int ib, int max_rows, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int rs = (max_rows + 63) / 64;
  dim3 grid(n), block(1024);
#define BLR_PANEL(RSV, CPWV) hipLaunchKernelGGL((k_panel_batch<RSV, CPWV>), grid, block, 0, stream, d)
  if (ib == 32) {
    if (rs <= 1) BLR_PANEL(1, 2);
    else if (rs <= 2) BLR_PANEL(2, 2);
    else if (rs <= 4) BLR_PANEL(4, 2);
    else if (rs <= 8) BLR_PANEL(8, 2);
    else return hipErrorInvalidValue;
  } else if (ib == 16) {
    if (rs <= 1) BLR_PANEL(1, 1);
    else if (rs <= 2) BLR_PANEL(2, 1);
    else if (rs <= 4) BLR_PANEL(4, 1);
    else if (rs <= 8) BLR_PANEL(8, 1);
    else if (rs <= 16) BLR_PANEL(16, 1);
    else return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
#undef BLR_PANEL
  return hipGetLastError();
}

hipError_t launch_panel_apply_batch(const PanelJob* d, int n, int ib, int max_nt, hipStream_t stream) {
  if (n <= 0 || max_nt <= 0) return hipSuccess;
  dim3 grid((max_nt + 31) / 32, n), block(256);
  if (ib == 32) hipLaunchKernelGGL((k_panel_apply_batch<32>), grid, block, 0, stream, d);
  else if (ib == 16) hipLaunchKernelGGL((k_panel_apply_batch<16>), grid, block, 0, stream, d);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_t_backsolve_batch(const PanelJob* d, int n, int max_n, hipStream_t stream) {
  if (n <= 0 || max_n <= 0) return hipSuccess;
  dim3 grid((max_n + 3) / 4, n), block(256);
  hipLaunchKernelGGL(k_t_backsolve_batch, grid, block, (size_t)4 * max_n * sizeof(double), stream, d);
  return hipGetLastError();
}

hipError_t launch_tall_apply_batch(const PanelJob* d, int n, int ib, int max_nt, int max_slices,
                                   hipStream_t stream) {
  if (n <= 0 || max_nt <= 0) return hipSuccess;
  if (max_slices < 1 || max_slices > kTallApplySlices) return hipErrorInvalidValue;
  dim3 grid((max_nt + 31) / 32, max_slices, n), block(256);
  if (ib == 32) {
    hipLaunchKernelGGL((k_tall_apply_part_batch<32>), grid, block, 0, stream, d);
    hipLaunchKernelGGL((k_tall_apply_upd_batch<32>), grid, block, 0, stream, d);
  } else if (ib == 16) {
    hipLaunchKernelGGL((k_tall_apply_part_batch<16>), grid, block, 0, stream, d);
    hipLaunchKernelGGL((k_tall_apply_upd_batch<16>), grid, block, 0, stream, d);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
