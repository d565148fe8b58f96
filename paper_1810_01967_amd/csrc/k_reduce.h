// Helpers shared by the sampling kernels: a fixed-order block reduction and
// the map from a virtual (slice, coil, frame) pair to its sampling pattern.
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

// Virtual pair pv = (slice * ncoil + coil) * L + frame: the CSR pair
// slice * L + frame whose pattern every coil shares, and the offset of the
// coil's samples in coil-major sample arrays ([ncoil][M]).
struct VPair {
  int p;
  int64_t qoff;
};
__device__ __forceinline__ VPair vpair(int pv, int L, int ncoil, int64_t M) {
  const int vs = pv / L, t = pv - vs * L;
  const int sl = vs / ncoil, q = vs - sl * ncoil;
  return {sl * L + t, (int64_t)q * M};
}

}  // namespace mrf
