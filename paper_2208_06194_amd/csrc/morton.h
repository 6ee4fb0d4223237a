// Morton ordering of a point set on the device (blr_morton_sort).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// perm[r] = original index of the r-th point in Morton order; sorted (may be
// null) = the points in that order.  Synchronises s; frees its temporaries.
hipError_t morton_sort(const double* pts, int64_t n, int dim, int64_t* perm, double* sorted, hipStream_t s);
