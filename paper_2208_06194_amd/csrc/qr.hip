// Householder reflector generation on tiles (Sections 3.3.1 and 3.3.3 of
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

namespace {

template <int ROWS, int IB>
__global__ __launch_bounds__(256) void k_panel(PanelArgs a) {
  __shared__ double red[4][IB];      // per-wave partial dot products
  __shared__ double prow[IB];        // pivot row (GEQRT) / R row (TPQRT)
  __shared__ double top[IB][IB + 1]; // TPQRT: R diagonal block
  __shared__ double Tl[IB][IB + 1];  // T of this panel
  __shared__ double gcol[IB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool tp = a.mode == PANEL_TPQRT;
  const int h = a.h;
  double* X = a.X;
  const int64_t ldx = a.ldx;

  double x[ROWS][IB];
#pragma unroll
  for (int rr = 0; rr < ROWS; ++rr) {
    const int r = tid + 256 * rr;
#pragma unroll
    for (int c = 0; c < IB; ++c) x[rr][c] = (r < h) ? X[r + c * ldx] : 0.0;
  }
  if (tp) {
    for (int e = tid; e < IB * IB; e += 256) {
      const int r = e % IB, c = e / IB;
      top[r][c] = (r <= c) ? a.R[r + c * a.ldr] : 0.0;
    }
  }
  for (int e = tid; e < IB * IB; e += 256) Tl[e % IB][e / IB] = 0.0;
  __syncthreads();

  for (int jj = 0; jj < IB; ++jj) {
    // extract column jj, pivot row values
    double v[ROWS];
    bool tail[ROWS];
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr) {
      const int r = tid + 256 * rr;
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < IB; ++c) s = (c == jj) ? x[rr][c] : s;
      v[rr] = s;
      tail[rr] = tp ? (r < h) : (r > jj && r < h);
      if (!tp && r == jj) {
#pragma unroll
        for (int c = 0; c < IB; ++c) prow[c] = x[rr][c];
      }
    }
    if (tp && tid < IB) prow[tid] = (tid > jj) ? top[jj][tid] : 0.0;
    double ss = 0.0;
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr) ss += tail[rr] ? v[rr] * v[rr] : 0.0;
    const double xnorm2 = block_sum(ss, &red[0][0]);   // has barriers: prow visible after
    const double alpha = tp ? top[jj][jj] : prow[jj];
    double beta, tau, scal;
    larfg_scalars(alpha, xnorm2, &beta, &tau, &scal);
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr) v[rr] = tail[rr] ? v[rr] * scal : 0.0;
    // dot products of the new reflector with every other panel column
    double part[IB];
#pragma unroll
    for (int c = 0; c < IB; ++c) {
      double s = 0.0;
#pragma unroll
      for (int rr = 0; rr < ROWS; ++rr) s += v[rr] * x[rr][c];
      part[c] = wave_sum(s);
    }
    __syncthreads();  // all reads of red / prow done
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < IB; ++c) red[wave][c] = part[c];
    }
    __syncthreads();
    double w[IB];
#pragma unroll
    for (int c = 0; c < IB; ++c) {
      const double pr = (!tp || c > jj) ? prow[c] : 0.0;
      w[c] = pr + red[0][c] + red[1][c] + red[2][c] + red[3][c];
    }
    // store the reflector into column jj and update the later columns
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr) {
      const int r = tid + 256 * rr;
#pragma unroll
      for (int c = 0; c < IB; ++c) {
        if (c == jj) {
          if (tail[rr]) x[rr][c] = v[rr];
          else if (!tp && r == jj) x[rr][c] = beta;
        } else if (c > jj) {
          if (tail[rr]) x[rr][c] -= tau * w[c] * v[rr];
          else if (!tp && r == jj) x[rr][c] -= tau * w[c];
        }
      }
    }
    if (tid < IB) {
      const double pr = (!tp || tid > jj) ? prow[tid] : 0.0;
      const double wt = pr + red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
      gcol[tid] = wt;
      if (tp && tid > jj) top[jj][tid] -= tau * wt;
    }
    if (tp && tid == 0) top[jj][jj] = beta;
    if (tid == 0) Tl[jj][jj] = tau;
    __syncthreads();
    // T column jj of this panel: T[c][jj] = -tau * sum_{t=c}^{jj-1} T[c][t] g_t
    if (tid < jj) {
      double s = 0.0;
      for (int tt = tid; tt < jj; ++tt) s += Tl[tid][tt] * gcol[tt];
      Tl[tid][jj] = -tau * s;
    }
    if (tid == 0) a.tau[jj] = tau;
    __syncthreads();
  }

#pragma unroll
  for (int rr = 0; rr < ROWS; ++rr) {
    const int r = tid + 256 * rr;
    if (r < h) {
#pragma unroll
      for (int c = 0; c < IB; ++c) X[r + c * ldx] = x[rr][c];
    }
  }
  if (tp) {
    for (int e = tid; e < IB * IB; e += 256) {
      const int r = e % IB, c = e / IB;
      if (r <= c) a.R[r + c * a.ldr] = top[r][c];
    }
  }
  for (int e = tid; e < IB * IB; e += 256) {
    const int r = e % IB, c = e / IB;
    if (r <= c) a.T[r + c * a.ldt] = Tl[r][c];
  }
}

// One wave per column c of T (n x n); rows above the IB-block of c.
__global__ __launch_bounds__(256) void k_t_backsolve(TBackArgs a) {
  extern __shared__ double xs[];  // 4 waves x n
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 4 + wave;
  if (c >= a.n) return;
  double* x = xs + (size_t)wave * a.n;
  const int bs = (c / a.ib) * a.ib;
  const double* G = a.G;
  const int64_t ldg = a.ldg;
  // lane l owns entries t = l (mod 64) of x: it is the only lane that writes
  // or reads them, so no cross-lane synchronisation is needed
  for (int t = bs + ((lane - bs) & 63); t <= c; t += 64) x[t] = a.T[t + (int64_t)c * a.ldt];
  for (int r = bs - 1; r >= 0; --r) {
    double s = 0.0;
    for (int t = r + 1 + ((lane - (r + 1)) & 63); t <= c; t += 64) s += G[t + (int64_t)r * ldg] * x[t];
    s = wave_sum(s);
    const double xr = -a.tau[r] * s;
    if ((r & 63) == lane) x[r] = xr;
    if (lane == 0) a.T[r + (int64_t)c * a.ldt] = xr;
  }
  // zero the strictly lower part of column c
  for (int r = c + 1 + lane; r < a.n; r += 64) a.T[r + (int64_t)c * a.ldt] = 0.0;
}

}  // namespace

hipError_t launch_panel(const PanelArgs& a, hipStream_t stream) {
  const int rows = (a.h + 255) / 256;
  dim3 grid(1), block(256);
  if (a.ib == 32) {
    if (rows <= 1) hipLaunchKernelGGL((k_panel<1, 32>), grid, block, 0, stream, a);
    else if (rows <= 2) hipLaunchKernelGGL((k_panel<2, 32>), grid, block, 0, stream, a);
    else return hipErrorInvalidValue;  // tall panels use ib = 16 (register budget)
  } else if (a.ib == 16) {
    if (rows <= 1) hipLaunchKernelGGL((k_panel<1, 16>), grid, block, 0, stream, a);
    else if (rows <= 2) hipLaunchKernelGGL((k_panel<2, 16>), grid, block, 0, stream, a);
    else if (rows <= 4) hipLaunchKernelGGL((k_panel<4, 16>), grid, block, 0, stream, a);
    else return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_t_backsolve(const TBackArgs& a, hipStream_t stream) {
  if (a.n <= a.ib) return hipSuccess;
  dim3 grid((a.n + 3) / 4), block(256);
  hipLaunchKernelGGL(k_t_backsolve, grid, block, (size_t)4 * a.n * sizeof(double), stream, a);
  return hipGetLastError();
}
