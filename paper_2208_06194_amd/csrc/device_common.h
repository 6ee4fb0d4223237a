// Device helpers shared by the HIP kernels of libblrqr (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

#define BLR_WAVE 64

// Sum over the 64 lanes of a wave (every lane receives the result).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over groups of `width` consecutive lanes (width a power of two <= 64).
__device__ __forceinline__ double group_sum(double v, int width) {
  for (int off = width >> 1; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum of one value (blockDim.x a multiple of 64, <= 1024).
// `red` is LDS scratch of at least 16 doubles.  All threads get the result.
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// LAPACK larfg convention: given pivot alpha and ||x||^2, produce beta,
// tau and the scale 1/(alpha - beta) of the reflector tail.
__device__ __forceinline__ void larfg_scalars(double alpha, double xnorm2, double* beta,
                                              double* tau, double* scal) {
  if (xnorm2 == 0.0) {
    *beta = alpha;
    *tau = 0.0;
    *scal = 0.0;
    return;
  }
  const double norm = sqrt(alpha * alpha + xnorm2);
  const double b = (alpha >= 0.0) ? -norm : norm;
  *beta = b;
  *tau = (b - alpha) / b;
  *scal = 1.0 / (alpha - b);
}
