// Non-uniform Fourier transform for non-Cartesian (spiral) sampling on
// gfx950: the forward model's F at arbitrary k-space coordinates (Section
// "In-vivo data with variable-density spiral acquisition"), by gridding on a
// 2x oversampled grid with the "exponential of semicircle" kernel
// phi(z) = exp(beta (sqrt(1 - z^2) - 1)), |z| <= 1, of width W fine cells
// (Barnett, Magland, af Klinteberg, SIAM J. Sci. Comput. 2019), beta = 2.30 W:
//   forward  y(k) = e^{-2 pi i k.c} sum_{taps g} phi_y phi_x FFT_N(pad(x / phihat))[g]
//   adjoint  x = crop(IFFT_N(spread(w y e^{+2 pi i k.c}))) / phihat
// with the image centred (c = (ny/2, nx/2)) so that the deapodisation
// 1/phihat stays bounded, and the scale making y the unitary transform of the
// ny x nx image.  The tap set of a sample at fine position u is the W
// integers from ceil(u - W/2); interpolation and spreading use the same
// taps and weights, so they are adjoint to each other exactly (up to
// rounding).  Spreading gathers per fine-grid point over the samples of the
// neighbouring bins (8 x 8 fine cells, samples sorted by bin at plan
// creation), in a fixed order: deterministic, no atomics.
#include "k_reduce.h"
#include "mrf_internal.h"

namespace mrf {

constexpr int NUFFT_BIN = kNufftBin;

__device__ __forceinline__ float es_kernel(float z, float beta) {
  const float q = 1.f - z * z;
  return q > 0.f ? expf(beta * (sqrtf(q) - 1.f)) : 0.f;
}

// e^{-2 pi i (ky cy + kx cx)}, each product exact (c a power of two), the two
// phases multiplied
__device__ __forceinline__ float2 centre_phase(float2 k, float cy, float cx) {
  float sy, cyv, sx, cxv;
  sincospif(-2.f * (k.x * cy), &sy, &cyv);
  sincospif(-2.f * (k.y * cx), &sx, &cxv);
  return make_float2(cyv * cxv - sy * sx, cyv * sx + sy * cxv);
}

// out [nimg][Ny][Nx] (Ny = 2 ny): x at ((ry - ny/2) mod Ny, (rx - nx/2) mod Nx)
// times dy[ry] dx[rx], zero elsewhere
__global__ __launch_bounds__(256) void k_nufft_pad(const float2 *__restrict__ X, int64_t nimg, int ny, int nx,
                                                   const float *__restrict__ dy, const float *__restrict__ dx,
                                                   float2 *__restrict__ out) {
  const int Ny = 2 * ny, Nx = 2 * nx;
  const int64_t total = nimg * Ny * Nx;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int64_t img = e / ((int64_t)Ny * Nx);
  const int r = (int)(e - img * Ny * Nx);
  const int gy = r / Nx, gx = r - gy * Nx;
  const int sy = gy < Ny / 2 ? gy : gy - Ny, sx = gx < Nx / 2 ? gx : gx - Nx;  // signed fine index
  const int ry = sy + ny / 2, rx = sx + nx / 2;
  float2 v = make_float2(0.f, 0.f);
  if (ry >= 0 && ry < ny && rx >= 0 && rx < nx) {
    const float2 x = X[(img * ny + ry) * nx + rx];
    const float f = dy[ry] * dx[rx];
    v = make_float2(x.x * f, x.y * f);
  }
  out[e] = v;
}

// X [nimg][ny][nx] = K [nimg][Ny][Nx] at ((ry - ny/2) mod Ny, (rx - nx/2) mod Nx) times dy dx
__global__ __launch_bounds__(256) void k_nufft_crop(const float2 *__restrict__ K, int64_t nimg, int ny, int nx,
                                                    const float *__restrict__ dy, const float *__restrict__ dx,
                                                    float2 *__restrict__ X) {
  const int Ny = 2 * ny, Nx = 2 * nx;
  const int64_t total = nimg * ny * nx;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int64_t img = e / ((int64_t)ny * nx);
  const int r = (int)(e - img * ny * nx);
  const int ry = r / nx, rx = r - ry * nx;
  const int gy = (ry - ny / 2 + Ny) % Ny, gx = (rx - nx / 2 + Nx) % Nx;
  const float2 k = K[(img * Ny + gy) * Nx + gx];
  const float f = dy[ry] * dx[rx];
  X[e] = make_float2(k.x * f, k.y * f);
}

// One block per virtual (slice, coil, frame) pair, one thread per sample:
// y = centre phase x sum of the W x W taps of the pair's fine grid (SUB:
// of the sdim compressed fine grids of its (slice, coil), combined with the
// frame's row of V), R = y - Y, per-pair weighted squared norms.
template <bool SUB>
__global__ __launch_bounds__(256) void k_nufft_interp(const float2 *__restrict__ K, int Ny, int Nx, int W,
                                                      float beta, float cy, float cx,
                                                      const int64_t *__restrict__ off,
                                                      const float2 *__restrict__ coords,
                                                      const float2 *__restrict__ Y, const float *__restrict__ w,
                                                      float2 *__restrict__ R, double *part, int64_t M, int L,
                                                      int ncoil, const float2 *__restrict__ V, int sdim) {
  __shared__ double red[256];
  __shared__ float2 vrow[SUB ? kMaxSubspace : 1];
  const int pv = blockIdx.x;
  const VPair vp = vpair(pv, L, ncoil, M);
  const int vs = pv / L, t = pv - vs * L;
  if (SUB) {
    for (int k = threadIdx.x; k < sdim; k += 256) vrow[k] = V[(int64_t)t * sdim + k];
    __syncthreads();
  }
  const int64_t b = min(max(off[vp.p], (int64_t)0), M), e = min(max(off[vp.p + 1], b), M);
  const int64_t plane = (int64_t)Ny * Nx;
  const float2 *img = SUB ? K + (int64_t)vs * sdim * plane : K + (int64_t)pv * plane;
  const float half = 0.5f * W, zs = 2.f / W;
  double acc = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) {
    const float2 k = coords[i];
    const float uy = k.x * Ny, ux = k.y * Nx;
    const int jy0 = (int)ceilf(uy - half), jx0 = (int)ceilf(ux - half);
    float wy[8], wx[8];
    int iy[8], ix[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      if (m < W) {
        wy[m] = es_kernel(((float)(jy0 + m) - uy) * zs, beta);
        wx[m] = es_kernel(((float)(jx0 + m) - ux) * zs, beta);
        iy[m] = ((jy0 + m) % Ny + Ny) % Ny;
        ix[m] = ((jx0 + m) % Nx + Nx) % Nx;
      }
    }
    float2 y = make_float2(0.f, 0.f);
    const int nk = SUB ? sdim : 1;
    for (int kk = 0; kk < nk; ++kk) {
      const float2 *g = img + (int64_t)kk * plane;
      float2 a = make_float2(0.f, 0.f);
      for (int my = 0; my < W; ++my) {
        const float2 *row = g + (int64_t)iy[my] * Nx;
        float2 ra = make_float2(0.f, 0.f);
#pragma unroll
        for (int mx = 0; mx < 8; ++mx) {
          if (mx < W) {
            const float2 v = row[ix[mx]];
            ra.x = fmaf(wx[mx], v.x, ra.x);
            ra.y = fmaf(wx[mx], v.y, ra.y);
          }
        }
        a.x = fmaf(wy[my], ra.x, a.x);
        a.y = fmaf(wy[my], ra.y, a.y);
      }
      if (SUB) {
        const float2 v = vrow[kk];
        y.x = fmaf(v.x, a.x, fmaf(-v.y, a.y, y.x));
        y.y = fmaf(v.x, a.y, fmaf(v.y, a.x, y.y));
      } else {
        y = a;
      }
    }
    const float2 ph = centre_phase(k, cy, cx);
    float2 r = make_float2(ph.x * y.x - ph.y * y.y, ph.x * y.y + ph.y * y.x);
    if (Y) {
      const float2 yy = Y[vp.qoff + i];
      r.x -= yy.x;
      r.y -= yy.y;
    }
    R[vp.qoff + i] = r;
    const double m2 = (double)r.x * r.x + (double)r.y * r.y;
    acc += w ? (double)w[i] * m2 : m2;
  }
  const double sum = block_sum_f64(acc, red);
  if (threadIdx.x == 0 && part) part[pv] = sum;
}

// out [S' L][Ny][Nx]: per fine-grid point of virtual pair pv, the sum over
// the pair's samples whose taps include it of phi_y phi_x conj(centre phase)
// w_i R_i; samples visited bin by bin (at most 3 x 3 bins around the point,
// rows then columns), each bin in increasing sample order.
__global__ __launch_bounds__(256) void k_nufft_spread(const float2 *__restrict__ R, const float *__restrict__ w,
                                                      const int64_t *__restrict__ off,
                                                      const float2 *__restrict__ coords,
                                                      const int32_t *__restrict__ bperm,
                                                      const int32_t *__restrict__ boff, int Ny, int Nx, int W,
                                                      float beta, float cy, float cx, int64_t M, int L, int ncoil,
                                                      int64_t nvpairs, float2 *__restrict__ out) {
  const int64_t plane = (int64_t)Ny * Nx;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nvpairs * plane) return;
  const int pv = (int)(e / plane);
  const int r = (int)(e - (int64_t)pv * plane);
  const int gy = r / Nx, gx = r - gy * Nx;
  const VPair vp = vpair(pv, L, ncoil, M);
  const int nby = Ny / NUFFT_BIN, nbx = Nx / NUFFT_BIN, nb = nby * nbx;
  const int64_t b0 = min(max(off[vp.p], (int64_t)0), M);
  const int32_t *bo = boff + (int64_t)vp.p * (nb + 1);
  const float half = 0.5f * W, zs = 2.f / W;
  const int hw = (W + 1) / 2 + 1;  // bin search margin in fine cells
  const int by_lo = (gy - hw + 8 * Ny) / NUFFT_BIN, by_hi = (gy + hw + 8 * Ny) / NUFFT_BIN;
  const int bx_lo = (gx - hw + 8 * Nx) / NUFFT_BIN, bx_hi = (gx + hw + 8 * Nx) / NUFFT_BIN;
  float ax = 0.f, ay = 0.f;
  for (int byr = by_lo; byr <= by_hi; ++byr) {
    const int by = byr % nby;
    for (int bxr = bx_lo; bxr <= bx_hi; ++bxr) {
      const int bx = bxr % nbx;
      const int bin = by * nbx + bx;
      const int64_t s0 = b0 + bo[bin], s1 = b0 + bo[bin + 1];
      for (int64_t q = s0; q < s1; ++q) {
        const int64_t i = bperm[q];
        if (i < 0 || i >= M) continue;
        const float2 k = coords[i];
        const float uy = k.x * Ny, ux = k.y * Nx;
        const int jy0 = (int)ceilf(uy - half), jx0 = (int)ceilf(ux - half);
        const int dy = ((gy - jy0) % Ny + Ny) % Ny, dx = ((gx - jx0) % Nx + Nx) % Nx;
        if (dy >= W || dx >= W) continue;
        const float f = es_kernel(((float)(jy0 + dy) - uy) * zs, beta) *
                        es_kernel(((float)(jx0 + dx) - ux) * zs, beta);
        float2 v = R[vp.qoff + i];
        if (w) {
          const float a = w[i];
          v.x *= a;
          v.y *= a;
        }
        const float2 ph = centre_phase(k, cy, cx);  // conj(ph) * v
        ax = fmaf(f, ph.x * v.x + ph.y * v.y, ax);
        ay = fmaf(f, ph.x * v.y - ph.y * v.x, ay);
      }
    }
  }
  out[e] = make_float2(ax, ay);
}

void launch_nufft_pad(const float2 *X, int64_t nimg, int ny, int nx, const float *dy, const float *dx, float2 *out,
                      hipStream_t s) {
  const int64_t total = nimg * 4 * (int64_t)ny * nx;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_nufft_pad, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, X, nimg, ny, nx, dy, dx,
                     out);
}

void launch_nufft_crop(const float2 *K, int64_t nimg, int ny, int nx, const float *dy, const float *dx, float2 *X,
                       hipStream_t s) {
  const int64_t total = nimg * (int64_t)ny * nx;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_nufft_crop, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, K, nimg, ny, nx, dy, dx,
                     X);
}

void launch_nufft_interp(const float2 *K, int ny, int nx, int W, float beta, const int64_t *off,
                         const float2 *coords, const float2 *Y, const float *w, float2 *R, double *part,
                         int nvpairs, int64_t M, int L, int ncoil, const float2 *V, int sdim, hipStream_t s) {
  if (nvpairs <= 0) return;
  const float cy = 0.5f * ny, cx = 0.5f * nx;
  if (V)
    hipLaunchKernelGGL(k_nufft_interp<true>, dim3(nvpairs), dim3(256), 0, s, K, 2 * ny, 2 * nx, W, beta, cy, cx,
                       off, coords, Y, w, R, part, M, L, ncoil, V, sdim);
  else
    hipLaunchKernelGGL(k_nufft_interp<false>, dim3(nvpairs), dim3(256), 0, s, K, 2 * ny, 2 * nx, W, beta, cy, cx,
                       off, coords, Y, w, R, part, M, L, ncoil, nullptr, 1);
}

void launch_nufft_spread(const float2 *R, const float *w, const int64_t *off, const float2 *coords,
                         const int32_t *bperm, const int32_t *boff, int ny, int nx, int W, float beta, int64_t M,
                         int L, int ncoil, int64_t nvpairs, float2 *out, hipStream_t s) {
  const int64_t total = nvpairs * 4 * (int64_t)ny * nx;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_nufft_spread, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, R, w, off, coords,
                     bperm, boff, 2 * ny, 2 * nx, W, beta, 0.5f * ny, 0.5f * nx, M, L, ncoil, nvpairs, out);
}

}  // namespace mrf
