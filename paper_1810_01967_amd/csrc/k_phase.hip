// Phase alignment for a complex proton density (Section "CoverBLIP
// algorithm", the phase-alignment paragraph): per voxel the phase of its
// coefficient on the dictionary's first principal direction u,
// theta_v = angle(u^H Z_v), as the unit factor e^{i theta_v}; and the phase
// of the complex PD from it and the chosen atom's alignment factor.
#include "mrf_internal.h"

namespace mrf {

__device__ __forceinline__ float2 unit_of(double cx, double cy) {
  const double m = sqrt(cx * cx + cy * cy);
  if (!(m > 0.0) || !isfinite(m)) return make_float2(1.f, 0.f);
  return make_float2((float)(cx / m), (float)(cy / m));
}

// voxel-major Z [n][L]: one thread per voxel, FP64 accumulation over frames
__global__ __launch_bounds__(256) void k_voxel_phase(const float2 *__restrict__ Z, int64_t n, int L,
                                                     const float2 *__restrict__ u, float2 *__restrict__ vphase) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= n) return;
  const float2 *z = Z + v * L;
  double cx = 0.0, cy = 0.0;
  for (int t = 0; t < L; ++t) {
    const float2 a = u[t], b = z[t];  // conj(a) * b
    cx += (double)a.x * b.x + (double)a.y * b.y;
    cy += (double)a.x * b.y - (double)a.y * b.x;
  }
  vphase[v] = unit_of(cx, cy);
}

// frame-major X - mu G: coalesced across the voxels of a slice
__global__ __launch_bounds__(256) void k_voxel_phase_frames(const float2 *__restrict__ X, const float2 *__restrict__ G,
                                                            float mu, int64_t n, int64_t npix, int L,
                                                            const float2 *__restrict__ u,
                                                            float2 *__restrict__ vphase) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= n) return;
  const int64_t sl = v / npix, p = v - sl * npix;
  double cx = 0.0, cy = 0.0;
  for (int t = 0; t < L; ++t) {
    const int64_t e = (sl * L + t) * npix + p;
    float2 b = X[e];
    if (G) {
      const float2 g = G[e];
      b.x = b.x - mu * g.x;
      b.y = b.y - mu * g.y;
    }
    const float2 a = u[t];
    cx += (double)a.x * b.x + (double)a.y * b.y;
    cy += (double)a.x * b.y - (double)a.y * b.x;
  }
  vphase[v] = unit_of(cx, cy);
}

__global__ void k_pd_phase(const int32_t *__restrict__ idx, const float2 *__restrict__ vphase,
                           const float2 *__restrict__ afac, int64_t n, float *__restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= n) return;
  const int j = idx[v];
  float r = 0.f;
  if (j >= 0) {
    const float2 e = vphase[v], f = afac[j];
    r = atan2f(e.x * f.y + e.y * f.x, e.x * f.x - e.y * f.y);
  }
  out[v] = r;
}

void launch_voxel_phase(const float2 *Z, int64_t n, int L, const float2 *u, float2 *vphase, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_voxel_phase, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Z, n, L, u, vphase);
}

void launch_voxel_phase_frames(const float2 *X, const float2 *G, float mu, int64_t n, int64_t npix, int L,
                               const float2 *u, float2 *vphase, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_voxel_phase_frames, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, G, mu, n, npix,
                     L, u, vphase);
}

void launch_pd_phase(const int32_t *idx, const float2 *vphase, const float2 *afac, int64_t n, float *out,
                     hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pd_phase, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, idx, vphase, afac, n, out);
}

}  // namespace mrf
