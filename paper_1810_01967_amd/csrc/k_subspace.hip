// Temporal subspace compression on gfx950 (eq. CS1, eq. gradupdate, eq.
// gradcompression): X_t = sum_k V[t, k] Xc_k and Xc_k = sum_t conj(V[t, k]) X_t
// per pixel; the 2-D Fourier transform acts per frame and commutes with both.
//   * k_widen: FP32 normalised dictionary rows -> FP64 complex rows (the
//     Gram matrix and the compressed atoms are formed in FP64);
//   * k_sample_sub: the compressed forward operator at the samples, y_i =
//     sum_k V[t_i, k] Kc_k(kappa_i) over the s compressed k-space images of
//     the sample's (slice, coil) (fixed order), minus Y, with per-(slice,
//     coil, frame) weighted squared norms as in the uncompressed sampler;
//   * k_compress_frames: per pixel, Kc_k = sum_t conj(V[t, k]) K_t over the L
//     full frames (fixed order), 32 compressed frames per thread.
#include "k_reduce.h"
#include "mrf_internal.h"

namespace mrf {

__global__ void k_widen(const float *__restrict__ dhat, int Kp, int is_complex, int64_t rows, int L,
                        double2 *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= rows * L) return;
  const int64_t r = q / L;
  const int t = (int)(q - r * L);
  const float *a = dhat + r * Kp;
  out[q] = is_complex ? make_double2(a[2 * t], a[2 * t + 1]) : make_double2(a[t], 0.0);
}

void launch_widen(const float *dhat, int Kp, int is_complex, int64_t rows, int L, double2 *out, hipStream_t s) {
  const int64_t n = rows * L;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_widen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dhat, Kp, is_complex, rows, L,
                     out);
}

__global__ __launch_bounds__(256) void k_sample_sub(const float2 *__restrict__ Kc, int64_t npix, int L, int sdim,
                                                    const float2 *__restrict__ V, const int64_t *__restrict__ off,
                                                    const int32_t *__restrict__ sidx, const float2 *__restrict__ Y,
                                                    const float *__restrict__ w, float2 *__restrict__ R,
                                                    double *part, int64_t M, int ncoil) {
  __shared__ double red[256];
  __shared__ float2 vrow[kMaxSubspace];
  const int pv = blockIdx.x;  // virtual (slice, coil, frame) pair
  const VPair vp = vpair(pv, L, ncoil, M);
  const int vs = pv / L, t = pv - vs * L;
  for (int k = threadIdx.x; k < sdim; k += 256) vrow[k] = V[(int64_t)t * sdim + k];
  __syncthreads();
  const int64_t b = min(max(off[vp.p], (int64_t)0), M), e = min(max(off[vp.p + 1], b), M);
  const float2 *img = Kc + (int64_t)vs * sdim * npix;
  double acc = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) {
    const uint32_t kap = (uint32_t)sidx[i];
    float2 r = make_float2(0.f, 0.f);
    if (kap < (uint32_t)npix) {
      for (int k = 0; k < sdim; ++k) {
        const float2 v = vrow[k], x = img[(int64_t)k * npix + kap];
        r.x = fmaf(v.x, x.x, fmaf(-v.y, x.y, r.x));
        r.y = fmaf(v.x, x.y, fmaf(v.y, x.x, r.y));
      }
    }
    if (Y) {
      const float2 y = Y[vp.qoff + i];
      r.x -= y.x;
      r.y -= y.y;
    }
    R[vp.qoff + i] = r;
    const double m2 = (double)r.x * r.x + (double)r.y * r.y;
    acc += w ? (double)w[i] * m2 : m2;
  }
  const double sum = block_sum_f64(acc, red);
  if (threadIdx.x == 0 && part) part[pv] = sum;
}

void launch_sample_sub(const float2 *Kc, int64_t npix, int L, int sdim, const float2 *V, const int64_t *off,
                       const int32_t *sidx, const float2 *Y, const float *w, float2 *R, double *part, int nvpairs,
                       int64_t M, int ncoil, hipStream_t s) {
  hipLaunchKernelGGL(k_sample_sub, dim3(nvpairs), dim3(256), 0, s, Kc, npix, L, sdim, V, off, sidx, Y, w, R, part,
                     M, ncoil);
}

constexpr int SUB_KC = 32;  // compressed frames per block of k_compress_frames

// Kfull [S][L][npix] -> Kc [S][sdim][npix]; block = (slice, 256 pixels, chunk
// of SUB_KC compressed frames).  V entries are read at wave-uniform addresses
// (one V row segment per frame), so no frame-count limit applies.
__global__ __launch_bounds__(256) void k_compress_frames(const float2 *__restrict__ Kfull, int64_t npix, int L,
                                                         int sdim, const float2 *__restrict__ V,
                                                         float2 *__restrict__ Kc) {
  const int nchunk = (sdim + SUB_KC - 1) / SUB_KC;
  const int64_t tiles = (npix + 255) / 256;
  const int64_t bid = blockIdx.x;
  const int chunk = (int)(bid % nchunk);
  const int64_t rest = bid / nchunk;
  const int64_t tile = rest % tiles;
  const int sl = (int)(rest / tiles);
  const int k0 = chunk * SUB_KC;
  const int kn = min(SUB_KC, sdim - k0);
  const int64_t pix = tile * 256 + threadIdx.x;
  if (pix >= npix) return;
  float ar[SUB_KC], ai[SUB_KC];
#pragma unroll
  for (int kk = 0; kk < SUB_KC; ++kk) {
    ar[kk] = 0.f;
    ai[kk] = 0.f;
  }
  const float2 *src = Kfull + (int64_t)sl * L * npix + pix;
  for (int t = 0; t < L; ++t) {
    const float2 x = src[(int64_t)t * npix];
    if (x.x == 0.f && x.y == 0.f) continue;  // unsampled (exact zero): contributes nothing
    const float2 *vt = V + (int64_t)t * sdim + k0;
#pragma unroll
    for (int kk = 0; kk < SUB_KC; ++kk) {
      if (kk < kn) {
        const float2 v = vt[kk];  // conj(v) * x
        ar[kk] = fmaf(v.x, x.x, fmaf(v.y, x.y, ar[kk]));
        ai[kk] = fmaf(v.x, x.y, fmaf(-v.y, x.x, ai[kk]));
      }
    }
  }
  float2 *dst = Kc + (int64_t)sl * sdim * npix + pix;
#pragma unroll
  for (int kk = 0; kk < SUB_KC; ++kk)
    if (kk < kn) dst[(int64_t)(k0 + kk) * npix] = make_float2(ar[kk], ai[kk]);
}

// X [S][L][npix] = per pixel sum_k V[t, k] Xc [S][sdim][npix]: 32 frames per
// thread, V read at wave-uniform addresses, compressed frames in order.
__global__ __launch_bounds__(256) void k_expand_frames(const float2 *__restrict__ Xc, int64_t npix, int L, int sdim,
                                                       const float2 *__restrict__ V, float2 *__restrict__ X) {
  const int nchunk = (L + SUB_KC - 1) / SUB_KC;
  const int64_t tiles = (npix + 255) / 256;
  const int64_t bid = blockIdx.x;
  const int chunk = (int)(bid % nchunk);
  const int64_t rest = bid / nchunk;
  const int64_t tile = rest % tiles;
  const int sl = (int)(rest / tiles);
  const int t0 = chunk * SUB_KC;
  const int tn = min(SUB_KC, L - t0);
  const int64_t pix = tile * 256 + threadIdx.x;
  if (pix >= npix) return;
  float ar[SUB_KC], ai[SUB_KC];
#pragma unroll
  for (int tt = 0; tt < SUB_KC; ++tt) {
    ar[tt] = 0.f;
    ai[tt] = 0.f;
  }
  const float2 *src = Xc + (int64_t)sl * sdim * npix + pix;
  for (int k = 0; k < sdim; ++k) {
    const float2 x = src[(int64_t)k * npix];
#pragma unroll
    for (int tt = 0; tt < SUB_KC; ++tt) {
      if (tt < tn) {
        const float2 v = V[(int64_t)(t0 + tt) * sdim + k];  // v * x
        ar[tt] = fmaf(v.x, x.x, fmaf(-v.y, x.y, ar[tt]));
        ai[tt] = fmaf(v.x, x.y, fmaf(v.y, x.x, ai[tt]));
      }
    }
  }
  float2 *dst = X + (int64_t)sl * L * npix + pix;
#pragma unroll
  for (int tt = 0; tt < SUB_KC; ++tt)
    if (tt < tn) dst[(int64_t)(t0 + tt) * npix] = make_float2(ar[tt], ai[tt]);
}

void launch_expand_frames(const float2 *Xc, int64_t npix, int S, int L, int sdim, const float2 *V, float2 *X,
                          hipStream_t s) {
  const int nchunk = (L + SUB_KC - 1) / SUB_KC;
  const int64_t tiles = (npix + 255) / 256;
  const int64_t blocks = (int64_t)S * tiles * nchunk;
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_expand_frames, dim3((unsigned)blocks), dim3(256), 0, s, Xc, npix, L, sdim, V, X);
}

void launch_compress_frames(const float2 *Kfull, int64_t npix, int S, int L, int sdim, const float2 *V, float2 *Kc,
                            hipStream_t s) {
  const int nchunk = (sdim + SUB_KC - 1) / SUB_KC;
  const int64_t tiles = (npix + 255) / 256;
  const int64_t blocks = (int64_t)S * tiles * nchunk;
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_compress_frames, dim3((unsigned)blocks), dim3(256), 0, s, Kfull, npix, L, sdim, V, Kc);
}

}  // namespace mrf
