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
    if (P.src_dense) {
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
  for (int k = 0; k < dim; ++k) {
    double mn = 1e300, mx = -1e300;
    for (int i = threadIdx.x; i < b; i += blockDim.x) {
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
  (void)npts;
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

// X <- R^{-1} X for upper-triangular R (n x n, ld ldr), X n x nrhs.  One
// wave per right-hand side; lane l keeps the solution entries t = l mod 64
// in LDS, so every lane only ever reads what it wrote itself.
__global__ __launch_bounds__(256) void k_trsm_upper(const double* __restrict__ R, int64_t ldr, int n,
                                                    double* X, int64_t ldx, int nrhs) {
  extern __shared__ double xs[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 4 + wave;
  if (c >= nrhs) return;
  double* xl = xs + (size_t)wave * n;
  double* x = X + (int64_t)c * ldx;
  for (int r = n - 1; r >= 0; --r) {
    double s = 0.0;
    for (int t = r + 1 + ((lane - (r + 1)) & 63); t < n; t += 64) s += R[r + (int64_t)t * ldr] * xl[t];
    s = wave_sum(s);
    const double xr = (x[r] - s) / R[r + (int64_t)r * ldr];
    if ((r & 63) == lane) xl[r] = xr;
  }
  for (int t = lane; t < n; t += 64) x[t] = xl[t];
}

// R^T x = c for upper triangular R (forward substitution), one wave per
// right-hand side; column r of R is contiguous, so the dot product of step r
// reads it coalesced.
__global__ __launch_bounds__(256) void k_trsm_upper_t(const double* __restrict__ R, int64_t ldr, int n,
                                                      double* X, int64_t ldx, int nrhs) {
  extern __shared__ double xs[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 4 + wave;
  if (c >= nrhs) return;
  double* xl = xs + (size_t)wave * n;
  double* x = X + (int64_t)c * ldx;
  for (int r = 0; r < n; ++r) {
    double s = 0.0;
    for (int t = lane; t < r; t += 64) s += R[t + (int64_t)r * ldr] * xl[t];
    s = wave_sum(s);
    const double xr = (x[r] - s) / R[r + (int64_t)r * ldr];
    if ((r & 63) == lane) xl[r] = xr;
    __builtin_amdgcn_wave_barrier();
  }
  for (int t = lane; t < n; t += 64) x[t] = xl[t];
}

// out = a x + b y + c z over a rows x cols column-major block (y, z may be null).
__global__ void k_lincomb(double* out, int64_t ldo, const double* x, int64_t ldx, const double* y, int64_t ldy,
                          const double* z, int64_t ldz, double a, double b, double c, int rows, int cols) {
  const int64_t n = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % rows, col = e / rows;
    double v = a * x[r + col * ldx];
    if (y) v += b * y[r + col * ldy];
    if (z) v += c * z[r + col * ldz];
    out[r + col * ldo] = v;
  }
}

__global__ void k_diag_absmin(const DiagDesc* __restrict__ d, int b, double* out) {
  // out[2*i] = min |diag|, out[2*i+1] = ||upper triangle||_F^2 of tile i
  __shared__ double red[16];
  __shared__ double smn[256];
  const DiagDesc D = d[blockIdx.x];
  double mn = 1e300, s = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)b * b; e += blockDim.x) {
    const int r = (int)(e % b), c = (int)(e / b);
    if (r <= c) {
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
  const int ncl = npts / b;
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
  if (nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trsm_upper, dim3((nrhs + 3) / 4), dim3(256), (size_t)4 * n * sizeof(double), s, R,
                     ldr, n, X, ldx, nrhs);
  return hipGetLastError();
}

hipError_t launch_trsm_upper_t(const double* R, int64_t ldr, int n, double* X, int64_t ldx, int nrhs,
                               hipStream_t s) {
  if (nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trsm_upper_t, dim3((nrhs + 3) / 4), dim3(256), (size_t)4 * n * sizeof(double), s, R,
                     ldr, n, X, ldx, nrhs);
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

hipError_t launch_diag_absmin(const DiagDesc* d, int n, int b, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_absmin, dim3(n), dim3(256), 0, s, d, b, out);
  return hipGetLastError();
}
