// Register-resident sorted candidate lists for the scoring kernels' epilogues
// (the input of the exactness certificate of eq. exactP): a list holds the
// kCertK best (score, atom) pairs seen so far, best first, equal scores in
// increasing atom order, empty slots (-inf, -1) at the end.  All indexing is
// static, so the lists stay in registers.
#pragma once

#include <hip/hip_runtime.h>

namespace mrf {

constexpr int kCertK = 8;

// epilogues of the exhaustive scoring kernels
enum { SC_TOP1 = 0, SC_TOPK = 1, SC_COLLECT = 2 };

// (s1, j1) ranks before (s0, j0): higher score, or the same score and a lower
// valid index.  NaN never ranks before anything.
__device__ __forceinline__ bool rank_before(float s1, int j1, float s0, int j0) {
  return (s1 > s0) || (s1 == s0 && j1 >= 0 && (j0 < 0 || j1 < j0));
}

__device__ __forceinline__ void topk_clear(float (&ls)[kCertK], int (&lj)[kCertK]) {
#pragma unroll
  for (int i = 0; i < kCertK; ++i) {
    ls[i] = -INFINITY;
    lj[i] = -1;
  }
}

// Insert an atom that arrives after every atom already in the list (atoms
// scanned in increasing index order): a strict '>' keeps it behind equal
// scores.  The caller has checked s > ls[kCertK - 1].
__device__ __forceinline__ void topk_push_ordered(float (&ls)[kCertK], int (&lj)[kCertK], float s, int j) {
#pragma unroll
  for (int i = 0; i < kCertK; ++i) {
    if (s > ls[i]) {
      const float ts = ls[i];
      const int tj = lj[i];
      ls[i] = s;
      lj[i] = j;
      s = ts;
      j = tj;
    }
  }
}

// Insert any pair (full ordering with the index tie-break).
__device__ __forceinline__ void topk_push(float (&ls)[kCertK], int (&lj)[kCertK], float s, int j) {
  if (j < 0 || !rank_before(s, j, ls[kCertK - 1], lj[kCertK - 1])) return;
#pragma unroll
  for (int i = 0; i < kCertK; ++i) {
    if (rank_before(s, j, ls[i], lj[i])) {
      const float ts = ls[i];
      const int tj = lj[i];
      ls[i] = s;
      lj[i] = j;
      s = ts;
      j = tj;
    }
  }
}

// Merge the list of the lane `mask` lanes away (a disjoint set of atoms).
__device__ __forceinline__ void topk_merge_xor(float (&ls)[kCertK], int (&lj)[kCertK], int mask) {
  float ps[kCertK];
  int pj[kCertK];
#pragma unroll
  for (int i = 0; i < kCertK; ++i) {
    ps[i] = __shfl_xor(ls[i], mask, 64);
    pj[i] = __shfl_xor(lj[i], mask, 64);
  }
#pragma unroll
  for (int i = 0; i < kCertK; ++i) topk_push(ls, lj, ps[i], pj[i]);
}

}  // namespace mrf
