// The per-voxel end of a matched filter: best (score, atom) -> index, PD
// (eq. exactPs), normalised correlation and parameter look-up.  Shared by
// the exhaustive merge and the learned path's last passes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrf {

__device__ __forceinline__ void finish_voxel(int64_t v, float sc, int j, int d, const float *znorm,
                                             const int32_t *warm, const float *inv_norm,
                                             const float *params, int nparam, int32_t *idx,
                                             float *pd, float *corr, float *params_out,
                                             float *gamma_hat) {
  const float zn = znorm[v];
  float g = 0.f, c = 0.f;
  if (zn < 0.f || j < 0) {
    j = -1;  // non-finite voxel
  } else if (zn == 0.f) {
    j = warm ? warm[v] : 0;
    if (j < 0 || j >= d) j = 0;  // an out-of-range warm index is not trusted
  } else {
    g = fmaxf(sc, 0.f);
    c = sc / zn;
  }
  idx[v] = j;
  if (pd) pd[v] = j >= 0 ? g * inv_norm[j] : 0.f;
  if (corr) corr[v] = c;
  gamma_hat[v] = g;
  if (params_out)
    for (int p = 0; p < nparam; ++p)
      params_out[v * nparam + p] = j >= 0 ? params[(int64_t)j * nparam + p] : 0.f;
}

// The outputs finish_voxel writes, and what it reads besides the best pair.
struct FinishArgs {
  int d;
  const float *znorm;
  const int32_t *warm;
  const float *inv_norm;
  const float *params;
  int nparam;
  int32_t *idx;  // null: nothing to finish
  float *pd;
  float *corr;
  float *params_out;
  float *gamma_hat;
};

// finish_voxel of a single (score, atom) candidate taken as a one-split merge
// (a candidate with no atom or a NaN score counts as none).
__device__ __forceinline__ void finish_single(int64_t v, float sc, int j, const FinishArgs &f) {
  const bool has = j >= 0 && !(sc != sc);
  finish_voxel(v, has ? sc : -INFINITY, has ? j : -1, f.d, f.znorm, f.warm, f.inv_norm, f.params, f.nparam,
               f.idx, f.pd, f.corr, f.params_out, f.gamma_hat);
}

}  // namespace mrf
