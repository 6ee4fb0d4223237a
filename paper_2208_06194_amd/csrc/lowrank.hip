// Low-rank kernels for gfx950, one workgroup (256 threads) per problem.
//
// k_recompress: rounded addition of up to three low-rank terms (Alg. 6):
//   stack U = [U_1 U_2 ...] and V = [V_1 V_2 ...] (actual ranks, compacted),
//   Householder QR of each stack (reflectors kept), core Z = R_V R_U^T,
//   one-sided Jacobi (Hestenes) on the columns of Z:  Z J = W with W = v sigma
//   and J = u (left singular vectors of R_U R_V^T), eps-truncation relative
//   to the Frobenius norm of the sum, U_C = Q_U u_r, V_C = Q_V v_r sigma_r.
//
// k_rangefinder / k_comp_svd: truncated SVD of a dense tile for compression:
//   Q = orth(A Omega) by Householder QR, B = Q^T A, one-sided Jacobi on B^T,
//   and the rank is the smallest r with
//   ||A - Q B||_F^2 + sum_{l >= r} sigma_l^2 <= eps^2 ||A||_F^2,
//   so the truncation error of the stored U V^T is bounded exactly.
#include "device_common.h"
#include "lowrank.h"

namespace {

constexpr double JACOBI_TOL = 1e-15;
constexpr int JACOBI_MAX_SWEEPS = 40;
constexpr int LDS_DIM = 64;      // Jacobi matrices of the compression SVD held in LDS up to this order
constexpr int RC_LDS_DIM = 96;   // the rounded addition's core and rotations in LDS up to this order

// Householder QR of rows x cols column-major X (global memory), in place:
// R in the upper triangle, reflector tails below, tau[0 .. min(rows,cols)).
// Each wave updates four trailing columns at a time (independent loads and
// reductions in flight).
__device__ void wg_hqr(double* X, int64_t ld, int rows, int cols, double* tau, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kmax = min(rows, cols);
  for (int c = 0; c < kmax; ++c) {
    double ss = 0.0;
    for (int i = c + 1 + tid; i < rows; i += 256) {
      const double x = X[i + c * ld];
      ss += x * x;
    }
    const double xn2 = block_sum(ss, red);
    const double alpha = X[c + c * ld];
    double beta, t, scal;
    larfg_scalars(alpha, xn2, &beta, &t, &scal);
    __syncthreads();
    for (int i = c + 1 + tid; i < rows; i += 256) X[i + c * ld] *= scal;
    if (tid == 0) {
      X[c + c * ld] = beta;
      tau[c] = t;
    }
    __syncthreads();
    if (t != 0.0) {
      for (int c0 = c + 1 + 4 * wave; c0 < cols; c0 += 16) {
        double sv[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i = c + 1 + lane; i < rows; i += 64) {
          const double v = X[i + c * ld];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (c0 + u < cols) sv[u] += v * X[i + (c0 + u) * ld];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) sv[u] = wave_sum(sv[u]) + ((c0 + u < cols) ? X[c + (c0 + u) * ld] : 0.0);
        for (int i = c + 1 + lane; i < rows; i += 64) {
          const double v = X[i + c * ld];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (c0 + u < cols) X[i + (c0 + u) * ld] -= t * sv[u] * v;
        }
        if (lane == 0) {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (c0 + u < cols) X[c + (c0 + u) * ld] -= t * sv[u];
        }
      }
    }
    __syncthreads();
  }
}

// C <- Q C with Q = H_0 ... H_{k-1} stored as reflectors in X (rows x k);
// four columns of C per wave at a time.
__device__ void wg_apply_q(const double* X, int64_t ld, int rows, int k, const double* tau,
                           double* C, int64_t ldc, int nc) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c = k - 1; c >= 0; --c) {
    const double t = tau[c];
    if (t != 0.0) {
      for (int j0 = 4 * wave; j0 < nc; j0 += 16) {
        double sv[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i = c + 1 + lane; i < rows; i += 64) {
          const double v = X[i + c * ld];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (j0 + u < nc) sv[u] += v * C[i + (j0 + u) * ldc];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) sv[u] = wave_sum(sv[u]) + ((j0 + u < nc) ? C[c + (j0 + u) * ldc] : 0.0);
        for (int i = c + 1 + lane; i < rows; i += 64) {
          const double v = X[i + c * ld];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (j0 + u < nc) C[i + (j0 + u) * ldc] -= t * sv[u] * v;
        }
        if (lane == 0) {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (j0 + u < nc) C[c + (j0 + u) * ldc] -= t * sv[u];
        }
      }
    }
    __syncthreads();
  }
}

// Round-robin (circle method) pairing of n2 (even) columns, round r in [0, n2-1).
__device__ __forceinline__ void rr_pair(int pi, int r, int n2, int* a, int* b) {
  *a = (pi == 0) ? 0 : ((pi + r - 1) % (n2 - 1)) + 1;
  *b = ((n2 - 2 - pi + r) % (n2 - 1)) + 1;
}

// One-sided Jacobi: orthogonalise the nc columns (length nr) of Z by plane
// rotations, accumulating them in J (nc x nc, starts at I).  Groups of 16
// lanes process disjoint column pairs of one round concurrently.
__device__ void wg_jacobi(double* Z, int64_t ldz, int nr, int nc, double* J, int64_t ldj,
                          int* flag) {
  const int tid = threadIdx.x;
  for (int e = tid; e < nc * nc; e += 256) {
    const int i = e % nc, j = e / nc;
    J[i + j * ldj] = (i == j) ? 1.0 : 0.0;
  }
  if (nc < 2) {
    __syncthreads();
    return;
  }
  const int n2 = nc + (nc & 1);
  // lanes per column pair: every pair of a round in one batch once there
  // are at least 16 pairs (64 groups of 4 lanes), else groups of 16 lanes
  const int GW = (n2 / 2 >= 16) ? 4 : 16;
  const int NG = 256 / GW;
  const int g = tid / GW, gl = tid % GW;
  for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int round = 0; round < n2 - 1; ++round) {
      for (int pi = g; pi < n2 / 2; pi += NG) {
        int a, bq;
        rr_pair(pi, round, n2, &a, &bq);
        if (a >= nc || bq >= nc) continue;
        const int p = min(a, bq), q = max(a, bq);
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = gl; i < nr; i += GW) {
          const double zp = Z[i + p * ldz], zq = Z[i + q * ldz];
          al += zp * zp;
          be += zq * zq;
          ga += zp * zq;
        }
        al = group_sum(al, GW);
        be = group_sum(be, GW);
        ga = group_sum(ga, GW);
        if (ga != 0.0 && fabs(ga) > JACOBI_TOL * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
          for (int i = gl; i < nr; i += GW) {
            const double zp = Z[i + p * ldz], zq = Z[i + q * ldz];
            Z[i + p * ldz] = cs * zp - sn * zq;
            Z[i + q * ldz] = sn * zp + cs * zq;
          }
          for (int i = gl; i < nc; i += GW) {
            const double jp = J[i + p * ldj], jq = J[i + q * ldj];
            J[i + p * ldj] = cs * jp - sn * jq;
            J[i + q * ldj] = sn * jp + cs * jq;
          }
          if (gl == 0) *flag = 1;
        }
      }
      __syncthreads();
    }
    const int rotated = *flag;
    __syncthreads();
    if (!rotated) break;
  }
}

// Column norms of Z (nr x nc) into sig, and perm sorting them descending
// (ties by index).
__device__ void wg_sort_sigma(const double* Z, int64_t ldz, int nr, int nc, double* sig, int* perm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = wave; j < nc; j += 4) {
    double s = 0.0;
    for (int i = lane; i < nr; i += 64) {
      const double z = Z[i + j * ldz];
      s += z * z;
    }
    s = wave_sum(s);
    if (lane == 0) sig[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < nc; j += 256) {
    int rk = 0;
    const double sj = sig[j];
    for (int l = 0; l < nc; ++l) rk += (sig[l] > sj) || (sig[l] == sj && l < j);
    perm[rk] = j;
  }
  __syncthreads();
}

__device__ void record_overflow(const RcParams& P, unsigned long long* own, double dropped_rel) {
  unsigned long long* c = own ? own : P.overflow_count;
  unsigned long long* m = own ? own + 1 : P.max_dropped_bits;
  atomicAdd(c, 1ull);
  atomicMax(m, (unsigned long long)__double_as_longlong(dropped_rel));
}

__global__ __launch_bounds__(256) void k_recompress(const RcDesc* __restrict__ descs, RcParams P) {
  __shared__ double red[16];
  // the core Z and the rotations J in LDS up to order RC_LDS_DIM; beyond
  // that (up to order 135) Z alone, J in global memory
  __shared__ double zjl[2 * RC_LDS_DIM * RC_LDS_DIM];
  double* zl = zjl;
  double* jl = zjl + RC_LDS_DIM * RC_LDS_DIM;
  __shared__ double sig[384];
  __shared__ int perm[384];
  __shared__ int ranks[3];
  __shared__ int flag, rsel;

  const RcDesc& D = descs[blockIdx.x];
  const int tid = threadIdx.x;
  const int b = P.b, rc = P.rc, smax = 3 * rc;
  double* WU = D.work;
  double* WV = WU + (size_t)b * smax;
  double* Zg = WV + (size_t)b * smax;
  double* Jg = Zg + (size_t)smax * smax;
  double* tauU = Jg + (size_t)smax * smax;
  double* tauV = tauU + smax;

  if (tid < 3) {
    int r = 0;
    if (tid < D.nterm) {
      const RcTerm& T = D.t[tid];
      r = T.rank_ptr ? *T.rank_ptr : T.rank;
      r = max(0, min(r, rc));
    }
    ranks[tid] = r;
  }
  __syncthreads();
  const int s = ranks[0] + ranks[1] + ranks[2];
  if (s == 0) {
    for (int e = tid; e < b * rc; e += 256) {
      D.Uout[e] = 0.0;
      D.Vtout[e] = 0.0;
    }
    if (tid == 0) *D.rank_out = 0;
    return;
  }
  int off = 0;
  for (int tt = 0; tt < D.nterm; ++tt) {
    const RcTerm& T = D.t[tt];
    const int r = ranks[tt];
    for (int e = tid; e < b * r; e += 256) {
      const int i = e % b, l = e / b;
      const double u = T.transU ? T.U[l + (int64_t)i * T.ldu] : T.U[i + (int64_t)l * T.ldu];
      WU[i + (size_t)(off + l) * b] = T.sign * u;
      WV[i + (size_t)(off + l) * b] = T.Vt[l + (int64_t)i * T.ldvt];
    }
    off += r;
  }
  __syncthreads();
  wg_hqr(WU, b, b, s, tauU, red);
  wg_hqr(WV, b, b, s, tauV, red);
  const int k = min(b, s);
  const bool lds = k <= RC_LDS_DIM && s <= RC_LDS_DIM;
  double* Z = lds ? zl : Zg;
  double* J = lds ? jl : Jg;
  const int64_t ldz = k, ldj = k;
  // Z = R_V R_U^T  (k x k)
  if (lds) {
    // R_V and R_U (k x s upper triangles) staged in LDS; the products are
    // held in registers until both stagings are no longer read
    for (int e = tid; e < k * s; e += 256) {
      const int i = e % k, l = e / k;
      zl[e] = (l >= i) ? WV[i + (size_t)l * b] : 0.0;
      jl[e] = (l >= i) ? WU[i + (size_t)l * b] : 0.0;
    }
    __syncthreads();
    constexpr int ZPT = (RC_LDS_DIM * RC_LDS_DIM + 255) / 256;
    double zr[ZPT];
#pragma unroll
    for (int u = 0; u < ZPT; ++u) {
      const int e = tid + 256 * u;
      double acc = 0.0;
      if (e < k * k) {
        const int i = e % k, j = e / k;
        for (int l = max(i, j); l < s; ++l) acc += zl[i + l * k] * jl[j + l * k];
      }
      zr[u] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < ZPT; ++u) {
      const int e = tid + 256 * u;
      if (e < k * k) zl[e] = zr[u];
    }
  } else {
    for (int e = tid; e < k * k; e += 256) {
      const int i = e % k, j = e / k;
      double acc = 0.0;
      for (int l = max(i, j); l < s; ++l) acc += WV[i + (size_t)l * b] * WU[j + (size_t)l * b];
      Z[i + j * ldz] = acc;
    }
  }
  __syncthreads();
  if (!lds && (int64_t)k * k <= 2 * RC_LDS_DIM * RC_LDS_DIM) {
    // the rotations touch Z's columns four times for each of J's: Z into LDS
    for (int e = tid; e < k * k; e += 256) zjl[e] = Zg[e];
    __syncthreads();
    Z = zjl;
  }
  wg_jacobi(Z, ldz, k, k, J, ldj, &flag);
  wg_sort_sigma(Z, ldz, k, k, sig, perm);
  if (tid == 0) {
    double total2 = 0.0;
    for (int l = 0; l < k; ++l) total2 += sig[l] * sig[l];
    int r = k;
    if (total2 == 0.0) {
      r = 0;
    } else {
      const double thr2 = P.eps * P.eps * total2;
      double tail2 = 0.0;
      while (r > 0) {
        const double sv = sig[perm[r - 1]];
        if (tail2 + sv * sv > thr2) break;
        tail2 += sv * sv;
        --r;
      }
      if (r > P.cap) {
        double drop2 = 0.0;
        for (int l = P.cap; l < k; ++l) drop2 += sig[perm[l]] * sig[perm[l]];
        record_overflow(P, D.counters, sqrt(drop2 / total2));
        r = P.cap;
      }
    }
    rsel = r;
  }
  __syncthreads();
  const int r = rsel;
  // U_C = Q_U [u_r; 0]
  for (int e = tid; e < b * rc; e += 256) {
    const int i = e % b, l = e / b;
    D.Uout[e] = (l < r && i < k) ? J[i + perm[l] * ldj] : 0.0;
  }
  __syncthreads();
  wg_apply_q(WU, b, b, k, tauU, D.Uout, b, r);
  // V_C = Q_V [v_r sigma_r; 0], staged in WU, then transposed into Vt
  for (int e = tid; e < b * r; e += 256) {
    const int i = e % b, l = e / b;
    WU[i + (size_t)l * b] = (i < k) ? Z[i + perm[l] * ldz] : 0.0;
  }
  __syncthreads();
  wg_apply_q(WV, b, b, k, tauV, WU, b, r);
  for (int e = tid; e < rc * b; e += 256) {
    const int l = e % rc, i = e / rc;
    D.Vtout[e] = (l < r) ? WU[i + (size_t)l * b] : 0.0;
  }
  if (tid == 0) *D.rank_out = r;
}

__global__ __launch_bounds__(256) void k_rangefinder(const CompDesc* __restrict__ descs, int b, int l) {
  __shared__ double red[16];
  const CompDesc& D = descs[blockIdx.x];
  double* tau = D.work;
  wg_hqr(D.Y, b, b, l, tau, red);
  for (int e = threadIdx.x; e < b * l; e += 256) {
    const int i = e % b, j = e / b;
    D.Q[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  wg_apply_q(D.Y, b, b, min(b, l), tau, D.Q, b, l);
}

__global__ __launch_bounds__(256) void k_comp_svd(const CompDesc* __restrict__ descs, CompParams P) {
  __shared__ double jl[LDS_DIM * LDS_DIM];
  __shared__ double sig[192];
  __shared__ int perm[192];
  __shared__ int flag, rsel, stat;
  const CompDesc& D = descs[blockIdx.x];
  const int tid = threadIdx.x;
  const int b = P.b, l = P.l, rc = P.rc;
  double* Z = D.work;                    // b x l = B^T
  double* Jg = Z + (size_t)b * l;        // l x l
  for (int e = tid; e < b * l; e += 256) {
    const int i = e % b, j = e / b;
    Z[e] = D.B[j + (int64_t)i * l];
  }
  __syncthreads();
  double* J = (l <= LDS_DIM) ? jl : Jg;
  wg_jacobi(Z, b, b, l, J, l, &flag);
  wg_sort_sigma(Z, b, b, l, sig, perm);
  if (tid == 0) {
    const double a2 = *D.anorm2, e2 = *D.enorm2;
    const double thr2 = P.eps * P.eps * a2;
    int r = l, st = 0;
    if (a2 == 0.0) {
      r = 0;
    } else if (e2 > thr2) {
      st = 1;  // the sampled range misses more than the tolerance
      r = l;
    } else {
      double tail2 = e2;
      while (r > 0) {
        const double sv = sig[perm[r - 1]];
        if (tail2 + sv * sv > thr2) break;
        tail2 += sv * sv;
        --r;
      }
    }
    if (r > P.cap) {
      st = 1;
      r = P.cap;
    }
    if (st && P.truncate) st = 2;  // kept at the cap: counted, stays low-rank
    rsel = r;
    stat = st;
  }
  __syncthreads();
  const int r = rsel;
  // U = Q J[:, perm[:r]]
  for (int e = tid; e < b * rc; e += 256) {
    const int i = e % b, c = e / b;
    double acc = 0.0;
    if (c < r) {
      const int pc = perm[c];
      for (int m = 0; m < l; ++m) acc += D.Q[i + (int64_t)m * b] * J[m + pc * l];
    }
    D.Uout[e] = acc;
  }
  for (int e = tid; e < rc * b; e += 256) {
    const int c = e % rc, i = e / rc;
    D.Vtout[e] = (c < r) ? Z[i + (int64_t)perm[c] * b] : 0.0;
  }
  if (tid == 0) {
    *D.rank_out = r;
    *D.status_out = stat;
  }
}

}  // namespace

size_t rc_work_doubles(int b, int rc) {
  const size_t smax = 3 * (size_t)rc;
  return 2 * (size_t)b * smax + 2 * smax * smax + 2 * smax;
}

size_t comp_work_doubles(int b, int l) { return (size_t)b * l + (size_t)l * l + (size_t)l; }

hipError_t launch_recompress(const RcDesc* d, int n, const RcParams& p, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_recompress, dim3(n), dim3(256), 0, stream, d, p);
  return hipGetLastError();
}

hipError_t launch_rangefinder(const CompDesc* d, int n, int b, int l, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rangefinder, dim3(n), dim3(256), 0, stream, d, b, l);
  return hipGetLastError();
}

hipError_t launch_comp_svd(const CompDesc* d, int n, const CompParams& p, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_comp_svd, dim3(n), dim3(256), 0, stream, d, p);
  return hipGetLastError();
}
