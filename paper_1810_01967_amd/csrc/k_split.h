// Split BF16 encoding shared by the kernels that produce split rows: x is
// carried as hi + lo with hi = RNE_bf16(x) and lo = RNE_bf16(x - hi), so
// |x - hi - lo| <= 2^-16 |x|.  Rows are stored as Kx/32 chunks
// [hi 32 | lo 32] (one 128-byte line per 32-element chunk).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrf {

__device__ __forceinline__ uint16_t bf16_rne_split(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ void split_bf16(float x, uint16_t &hi, uint16_t &lo) {
  hi = bf16_rne_split(x);
  lo = bf16_rne_split(x - __uint_as_float((uint32_t)hi << 16));
}

// element offset of column k of a split row (hi; the lo value is 32 further)
__device__ __forceinline__ int64_t split_off(int k) { return (int64_t)(k >> 5) * 64 + (k & 31); }

// Atom splits of the split-BF16 exhaustive filter when its voxel count is only
// known on the device (nvt voxel tiles, ntiles tiles of 256 atoms): about
// 1,024 work items, at most 64 splits and one split per atom tile.
__device__ __forceinline__ int x3_device_splits(int nvt, int ntiles) {
  const int nvt8 = (nvt + 7) / 8 * 8;
  const int s = nvt8 > 0 ? (1024 + nvt8 - 1) / nvt8 : 1;
  return max(1, min(s, min(ntiles, 64)));
}

}  // namespace mrf
