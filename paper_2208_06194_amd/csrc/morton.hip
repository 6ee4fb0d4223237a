// Morton (Z-order) keys of a point set and a stable sort by key on the
// device (rocPRIM radix sort), for blr_morton_sort.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include <stdint.h>

#include "morton.h"

namespace {

__global__ void k_morton_keys(const double* __restrict__ pts, int64_t n, int dim, uint64_t* __restrict__ keys,
                              int64_t* __restrict__ idx) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t q[3] = {0, 0, 0};
    for (int c = 0; c < dim; ++c) {
      double v = floor(pts[i * dim + c] * 2097152.0);   // 2^21 levels
      v = fmin(fmax(v, 0.0), 2097151.0);
      q[c] = (uint64_t)v;
    }
    uint64_t key = 0;
    for (int level = 20; level >= 0; --level)
      for (int c = 0; c < dim; ++c) key = (key << 1) | ((q[c] >> level) & 1ull);
    keys[i] = key;
    idx[i] = i;
  }
}

__global__ void k_gather_points(const double* __restrict__ pts, int64_t n, int dim, const int64_t* __restrict__ perm,
                                double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * dim; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / dim, c = e % dim;
    out[e] = pts[perm[r] * dim + c];
  }
}

}  // namespace

hipError_t morton_sort(const double* pts, int64_t n, int dim, int64_t* perm, double* sorted, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  uint64_t *k0 = nullptr, *k1 = nullptr;
  int64_t* i0 = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  // scratch is stream-ordered memory on s: nothing here waits for other work
  hipError_t e = hipMallocAsync((void**)&k0, n * sizeof(uint64_t), s);
  if (e == hipSuccess) e = hipMallocAsync((void**)&k1, n * sizeof(uint64_t), s);
  if (e == hipSuccess) e = hipMallocAsync((void**)&i0, n * sizeof(int64_t), s);
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_morton_keys, dim3(blocks), dim3(256), 0, s, pts, n, dim, k0, i0);
    e = hipGetLastError();
  }
  // radix sort is stable: equal keys keep the original index order
  if (e == hipSuccess)
    e = rocprim::radix_sort_pairs(nullptr, tmp_bytes, k0, k1, i0, perm, (size_t)n, 0, 21 * dim, s);
  if (e == hipSuccess) e = hipMallocAsync(&tmp, std::max<size_t>(tmp_bytes, 1), s);
  if (e == hipSuccess)
    e = rocprim::radix_sort_pairs(tmp, tmp_bytes, k0, k1, i0, perm, (size_t)n, 0, 21 * dim, s);
  if (e == hipSuccess && sorted) {
    const int gb = (int)std::min<int64_t>((n * dim + 255) / 256, 8192);
    hipLaunchKernelGGL(k_gather_points, dim3(gb), dim3(256), 0, s, pts, n, dim, perm, sorted);
    e = hipGetLastError();
  }
  if (tmp) (void)hipFreeAsync(tmp, s);
  if (i0) (void)hipFreeAsync(i0, s);
  if (k1) (void)hipFreeAsync(k1, s);
  if (k0) (void)hipFreeAsync(k0, s);
  return e;
}
