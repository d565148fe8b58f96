// Fixed-order block reduction shared by the sampling kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace mrf {

// Sum of x over a 256-thread block (tree order fixed, so the result does not
// depend on scheduling); every thread returns the total.
__device__ __forceinline__ double block_sum_f64(double x, double *red) {
  const int tid = threadIdx.x;
  red[tid] = x;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  return red[0];
}

}  // namespace mrf
