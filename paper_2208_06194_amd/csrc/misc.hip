// Element-wise and reduction kernels: kernel-matrix tiles, cluster boxes,
// the Gaussian test matrix of the range finder, finiteness checks,
// Frobenius norms and the triangular solve of the back-substitution.
#include "device_common.h"
#include "misc.h"

namespace {

__global__ void k_fill_tiles(const TileFillDesc* __restrict__ d, TileFillParams P) {
  const TileFillDesc D = d[blockIdx.y];
  const int b = P.b;
  const int64_t nel = (int64_t)b * b;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nel;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % b), c = (int)(e / b);
    const int64_t gi = (int64_t)D.ti * b + r, gj = (int64_t)D.tj * b + c;
    double v;
    if (gi >= P.mu || gj >= P.nu) {
      v = (gi >= P.mu && gj >= P.nu && gi - P.mu == gj - P.nu) ? 1.0 : 0.0;
    } else if (P.src_dense) {
      v = P.A[gi + gj * P.lda];
    } else {
      double d2 = 0.0;
      for (int k = 0; k < P.dim; ++k) {
        const double df = P.x[gi * P.dim + k] - P.y[gj * P.dim + k];
        d2 += df * df;
      }
      const double dist = sqrt(d2) + P.reg;
      v = (P.kernel == 0) ? -log(dist) : 1.0 / dist;
    }
    D.dst[e] = v;
  }
}

__global__ void k_boxes(const double* __restrict__ pts, int npts, int dim, int b, double* lo,
                        double* hi) {
  __shared__ double smn[256], smx[256];
  const int cl = blockIdx.x;
  const int cnt = min(b, npts - cl * b);   // the last cluster may hold fewer points
  for (int k = 0; k < dim; ++k) {
    double mn = 1e300, mx = -1e300;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
      const double v = pts[((int64_t)cl * b + i) * dim + k];
      mn = fmin(mn, v);
      mx = fmax(mx, v);
    }
    smn[threadIdx.x] = mn;
    smx[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + s]);
        smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + s]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      lo[cl * dim + k] = smn[0];
      hi[cl * dim + k] = smx[0];
    }
    __syncthreads();
  }
}

__device__ __forceinline__ unsigned long long sm_mix(unsigned long long z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

// Standard normals from the counter-based splitmix64 stream (seed, stream):
// key = mix(seed*G + stream*G2 + 1), word i = mix(key + (i+1)*G),
// g_i = sqrt(-2 ln(1 - U(w_2i))) cos(2 pi U(w_2i+1)), U(w) = (w >> 11) 2^-53.
__global__ void k_gaussian(double* out, int64_t n, unsigned long long seed, unsigned long long stream) {
  const unsigned long long G = 0x9E3779B97F4A7C15ull, G2 = 0xD1B54A32D192ED03ull;
  const unsigned long long key = sm_mix(seed * G + stream * G2 + 1ull);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long w0 = sm_mix(key + (unsigned long long)(2 * i + 1) * G);
    const unsigned long long w1 = sm_mix(key + (unsigned long long)(2 * i + 2) * G);
    const double u1 = 1.0 - (double)(w0 >> 11) * 0x1.0p-53;
    const double u2 = (double)(w1 >> 11) * 0x1.0p-53;
    out[i] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
  }
}

__global__ void k_nonfinite(const double* __restrict__ a, int64_t rows, int64_t cols, int64_t ld,
                            int* flag) {
  const int64_t n = rows * cols;
  int bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double v = a[(e % rows) + (e / rows) * ld];
    bad |= !isfinite(v);
  }
  if (bad) atomicOr(flag, 1);
}

// sum of squares of each matrix in a batch: out[i] = ||M_i||_F^2
__global__ void k_frob2(const Frob2Desc* __restrict__ d) {
  __shared__ double red[16];
  const Frob2Desc D = d[blockIdx.x];
  double s = 0.0;
  const int64_t n = (int64_t)D.rows * D.cols;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const double v = D.M[(e % D.rows) + (e / D.rows) * D.ld];
    s += v * v;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) *D.out = s;
}

// Blocked triangular solves with the upper triangular R (n x n, ld ldr):
// TRANS = false solves R X = C (back substitution, 64-row blocks from the
// bottom), TRANS = true solves R^T X = C (forward substitution, blocks from
// the top).  One workgroup of 8 waves per group of up to 16 right-hand
// sides, X overwritten in place.  Each diagonal block is staged in LDS with
// the reciprocals of its diagonal and solved by four waves, four right-hand
// sides each (lanes on rows; the solved value of each step read from its
// lane with readlane).  Then all waves subtract the block's contribution from
// the rows still to be solved (right-looking) as a matrix-core product:
// op(R)(rows, block), 16-row tiles loaded from global memory eight K steps at
// a time, times the block's solution from LDS.
constexpr int kTrsmB = 64, kTrsmR = 16, kTrsmThreads = 512;
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <bool TRANS>
__device__ __forceinline__ void trsm_body(const double* __restrict__ R, int64_t ldr, int n, double* X, int64_t ldx,
                                          int nrhs, int cb) {
  constexpr int NW = kTrsmThreads / 64;
  __shared__ double Rs[kTrsmB][kTrsmB + 1];   // op(R) of the diagonal block: Rs[row][col]
  __shared__ double dinv[kTrsmB];
  __shared__ double xs[kTrsmB][kTrsmR];       // the block's solution (zero past the block and nrhs)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lm = lane & 15, lg = lane >> 4;
  const int c0 = cb * kTrsmR;
  const int nr = min(kTrsmR, nrhs - c0);
  double* Xc = X + (int64_t)c0 * ldx;
  const int nb = (n + kTrsmB - 1) / kTrsmB;
  for (int bi = 0; bi < nb; ++bi) {
    const int blk = TRANS ? bi : nb - 1 - bi;
    const int r0 = blk * kTrsmB, r1 = min(n, r0 + kTrsmB), bs = r1 - r0;
    for (int e = tid; e < kTrsmB * kTrsmB; e += kTrsmThreads) {
      const int i = e % kTrsmB, j = e / kTrsmB;
      double v = 0.0;
      if (i < bs && j < bs)
        v = TRANS ? R[(r0 + j) + (int64_t)(r0 + i) * ldr] : R[(r0 + i) + (int64_t)(r0 + j) * ldr];
      Rs[i][j] = v;
    }
    if (tid < kTrsmB) {
      const double d = tid < bs ? (TRANS ? R[(r0 + tid) + (int64_t)(r0 + tid) * ldr]
                                         : R[(r0 + tid) + (int64_t)(r0 + tid) * ldr])
                                : 1.0;
      dinv[tid] = 1.0 / d;
    }
    __syncthreads();
    if (wave < kTrsmR / 4) {
      // wave w solves right-hand sides 4w .. 4w + 3 of the group
      const int r = r0 + lane;
      double c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int cu = 4 * wave + u;
        c[u] = (lane < bs && cu < nr) ? Xc[r + (int64_t)cu * ldx] : 0.0;
      }
      for (int st = 0; st < bs; ++st) {
        const int i = TRANS ? st : bs - 1 - st;
        const double rinv = dinv[i];
        const double a = Rs[lane][i];
        const bool upd = TRANS ? (lane > i) : (lane < i);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double xi = readlane_f64(c[u], i) * rinv;
          if (upd) c[u] -= a * xi;
          if (lane == i) c[u] = xi;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int cu = 4 * wave + u;
        xs[lane][cu] = c[u];
        if (lane < bs && cu < nr) Xc[r + (int64_t)cu * ldx] = c[u];
      }
    }
    __syncthreads();
    // rows [ua, ub) still to solve: C(rows) -= op(R)(rows, r0:r1) x_block
    const int ua = TRANS ? r1 : 0, ub = TRANS ? n : r0;
    const int ntile = (ub - ua + 15) / 16;
    for (int t0 = wave * 4; t0 < ntile; t0 += 4 * NW) {
      v4d acc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
      for (int half = 0; half < 2; ++half) {
        double av[4][8];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) {
            const int k = 4 * (8 * half + kk) + lg;
            const int row = ua + 16 * (t0 + q) + lm;
            double v = 0.0;
            if (t0 + q < ntile && row < ub && k < bs)
              v = TRANS ? R[(r0 + k) + (int64_t)row * ldr] : R[row + (int64_t)(r0 + k) * ldr];
            av[q][kk] = v;
          }
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          const double bv = xs[4 * (8 * half + kk) + lg][lm];
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q][kk], bv, acc[q], 0, 0, 0);
        }
      }
      // FP64 16x16x4 layout: lane holds column lane % 16, accumulator v row 4 v + lane / 16
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = ua + 16 * (t0 + q) + 4 * v + lg;
          if (t0 + q < ntile && row < ub && lm < nr) Xc[row + (int64_t)lm * ldx] -= acc[q][v];
        }
    }
    __syncthreads();
  }
}

template <bool TRANS>
__global__ __launch_bounds__(kTrsmThreads) void k_trsm_blk(const double* __restrict__ R, int64_t ldr, int n,
                                                           double* X, int64_t ldx, int nrhs) {
  trsm_body<TRANS>(R, ldr, n, X, ldx, nrhs, blockIdx.x);
}

// Batched form: job blockIdx.y; workgroups past the job's right-hand sides exit.
template <bool TRANS>
__global__ __launch_bounds__(kTrsmThreads) void k_trsm_blk_batch(const TrsmJob* __restrict__ jobs) {
  const TrsmJob J = jobs[blockIdx.y];
  if ((int)blockIdx.x * kTrsmR >= J.nrhs) return;
  trsm_body<TRANS>(J.R, J.ldr, J.n, J.X, J.ldx, J.nrhs, blockIdx.x);
}

// out = a x + b y + c z over a rows x cols column-major block (y, z may be null).
__device__ __forceinline__ void lincomb_one(const LincombDesc& D, int64_t e0, int64_t stride) {
  const int64_t n = (int64_t)D.rows * D.cols;
  for (int64_t e = e0; e < n; e += stride) {
    const int64_t r = e % D.rows, col = e / D.rows;
    double v = D.a * D.x[r + col * D.ldx];
    if (D.y) v += D.b * D.y[r + col * D.ldy];
    if (D.z) v += D.c * D.z[r + col * D.ldz];
    D.out[r + col * D.ldo] = v;
  }
}

__global__ void k_lincomb_batch(const LincombDesc* __restrict__ d) {
  const LincombDesc D = d[blockIdx.y];
  lincomb_one(D, blockIdx.x * (int64_t)blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

__global__ void k_lincomb(double* out, int64_t ldo, const double* x, int64_t ldx, const double* y, int64_t ldy,
                          const double* z, int64_t ldz, double a, double b, double c, int rows, int cols) {
  const LincombDesc D{out, ldo, x, ldx, y, ldy, z, ldz, a, b, c, rows, cols};
  lincomb_one(D, blockIdx.x * (int64_t)blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

__global__ void k_diag_absmin(const DiagDesc* __restrict__ d, int b, double* out) {
  // out[2*i] = min |diag|, out[2*i+1] = ||upper triangle||_F^2 of tile i
  __shared__ double red[16];
  __shared__ double smn[256];
  const DiagDesc D = d[blockIdx.x];
  double mn = 1e300, s = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)b * b; e += blockDim.x) {
    const int r = (int)(e % b), c = (int)(e / b);
    if (r <= c && c < D.ncols) {
      const double v = D.R[r + (int64_t)c * b];
      s += v * v;
      if (r == c) mn = fmin(mn, fabs(v));
    }
  }
  s = block_sum(s, red);
  smn[threadIdx.x] = mn;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = smn[0];
    out[2 * blockIdx.x + 1] = s;
  }
}

}  // namespace

hipError_t launch_fill_tiles(const TileFillDesc* d, int n, const TileFillParams& p, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(((int64_t)p.b * p.b + 255) / 256, 64);
  hipLaunchKernelGGL(k_fill_tiles, dim3(blocks, n), dim3(256), 0, s, d, p);
  return hipGetLastError();
}

hipError_t launch_boxes(const double* pts, int npts, int dim, int b, double* lo, double* hi,
                        hipStream_t s) {
  const int ncl = (npts + b - 1) / b;
  if (ncl <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_boxes, dim3(ncl), dim3(256), 0, s, pts, npts, dim, b, lo, hi);
  return hipGetLastError();
}

hipError_t launch_gaussian(double* out, int64_t n, unsigned long long seed, unsigned long long stream,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_gaussian, dim3(blocks), dim3(256), 0, s, out, n, seed, stream);
  return hipGetLastError();
}

hipError_t launch_nonfinite(const double* a, int64_t rows, int64_t cols, int64_t ld, int* flag,
                            hipStream_t s) {
  if (rows * cols <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((rows * cols + 255) / 256, 2048);
  hipLaunchKernelGGL(k_nonfinite, dim3(blocks), dim3(256), 0, s, a, rows, cols, ld, flag);
  return hipGetLastError();
}

hipError_t launch_frob2(const Frob2Desc* d, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_frob2, dim3(n), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_trsm_upper(const double* R, int64_t ldr, int n, double* X, int64_t ldx, int nrhs,
                             hipStream_t s) {
  if (nrhs <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trsm_blk<false>, dim3((nrhs + kTrsmR - 1) / kTrsmR), dim3(kTrsmThreads), 0, s, R, ldr, n,
                     X, ldx, nrhs);
  return hipGetLastError();
}

hipError_t launch_trsm_upper_t(const double* R, int64_t ldr, int n, double* X, int64_t ldx, int nrhs,
                               hipStream_t s) {
  if (nrhs <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trsm_blk<true>, dim3((nrhs + kTrsmR - 1) / kTrsmR), dim3(kTrsmThreads), 0, s, R, ldr, n,
                     X, ldx, nrhs);
  return hipGetLastError();
}

hipError_t launch_lincomb(double* out, int64_t ldo, const double* x, int64_t ldx, const double* y, int64_t ldy,
                          const double* z, int64_t ldz, double a, double b, double c, int rows, int cols,
                          hipStream_t s) {
  const int64_t n = (int64_t)rows * cols;
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_lincomb, dim3(blocks), dim3(256), 0, s, out, ldo, x, ldx, y, ldy, z, ldz, a, b, c, rows,
                     cols);
  return hipGetLastError();
}

hipError_t launch_trsm_batch(const TrsmJob* d, int count, int trans, int max_nrhs, hipStream_t s) {
  if (count <= 0 || max_nrhs <= 0) return hipSuccess;
  dim3 grid((max_nrhs + kTrsmR - 1) / kTrsmR, count), block(kTrsmThreads);
  if (trans) hipLaunchKernelGGL(k_trsm_blk_batch<true>, grid, block, 0, s, d);
  else hipLaunchKernelGGL(k_trsm_blk_batch<false>, grid, block, 0, s, d);
  return hipGetLastError();
}

hipError_t launch_lincomb_batch(const LincombDesc* d, int count, int64_t max_elems, hipStream_t s) {
  if (count <= 0 || max_elems <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((max_elems + 255) / 256, 4096);
  hipLaunchKernelGGL(k_lincomb_batch, dim3(blocks, count), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_diag_absmin(const DiagDesc* d, int n, int b, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_absmin, dim3(n), dim3(256), 0, s, d, b, out);
  return hipGetLastError();
}
