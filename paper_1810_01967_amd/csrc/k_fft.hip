// Forward model kernels for gfx950: batched unitary 2-D DFT of frames (two
// passes of 1-D radix-2 transforms staged in LDS), sample gather / residual,
// zero-filled scatter (the adjoint of the sampling), and fixed-order FP64
// reductions for the step-size rule.
#include "k_reduce.h"
#include "mrf_internal.h"

namespace mrf {

// ---------------------------------------------------------------------------
// 1-D FFT of many lines held in LDS
// ---------------------------------------------------------------------------
// A block transforms C = 4096/N lines of length N.  Lines are either rows of
// a frame (consecutive elements) or columns (elements nx apart); the load and
// store loops put the unit-stride index on consecutive threads so both stay
// coalesced.  In LDS: bit-reversed placement, then log2(N) in-place
// decimation-in-time stages.  Twiddles exp(-2 pi i k/N) are computed once per
// block in FP64 and rounded to FP32.
template <int N>
struct FftCfg {
  static constexpr int C = 4096 / N;
  static constexpr int LOG = (N == 16) ? 4 : (N == 32) ? 5 : (N == 64) ? 6 : (N == 128) ? 7 : (N == 256) ? 8 : 9;
};

template <int N, bool COLS>
__global__ __launch_bounds__(256) void k_fft_lines(float2 *__restrict__ data, int64_t nimg,
                                                   int ny, int nx, int inverse) {
  constexpr int C = FftCfg<N>::C;
  constexpr int LOG = FftCfg<N>::LOG;
  __shared__ float2 buf[C][N + 1];
  __shared__ float2 tw[N / 2];
  const int tid = threadIdx.x;
  for (int k = tid; k < N / 2; k += 256) {
    double sn, cs;
    sincospi(-2.0 * k / N, &sn, &cs);
    tw[k] = make_float2((float)cs, inverse ? -(float)sn : (float)sn);
  }
  // lines of this block: line l -> (image l / lpi, index l % lpi)
  const int lpi = COLS ? nx : ny;
  const int64_t nlines = nimg * lpi;
  const int64_t line0 = (int64_t)blockIdx.x * C;
  const int64_t npix = (int64_t)nx * ny;
  const float scale = rsqrtf((float)N);
  auto addr = [&](int c, int e) -> int64_t {
    const int64_t l = line0 + c;
    const int64_t img = l / lpi;
    const int j = (int)(l - img * lpi);
    return img * npix + (COLS ? ((int64_t)e * nx + j) : ((int64_t)j * nx + e));
  };
  for (int i = tid; i < C * N; i += 256) {
    int c, e;
    if (COLS) {
      e = i / C;
      c = i - e * C;
    } else {
      c = i / N;
      e = i - c * N;
    }
    if (line0 + c >= nlines) continue;
    const int r = (int)(__builtin_bitreverse32((unsigned)e) >> (32 - LOG));
    buf[c][r] = data[addr(c, e)];
  }
  __syncthreads();
#pragma unroll
  for (int st = 0; st < LOG; ++st) {
    const int m = 1 << st;
    for (int b = tid; b < C * (N / 2); b += 256) {
      const int c = b / (N / 2);
      const int k = b - c * (N / 2);
      const int g = k >> st, r = k & (m - 1);
      const int i0 = g * 2 * m + r, i1 = i0 + m;
      const float2 w = tw[r << (LOG - 1 - st)];
      const float2 a = buf[c][i0], x = buf[c][i1];
      const float2 bw = make_float2(x.x * w.x - x.y * w.y, x.x * w.y + x.y * w.x);
      buf[c][i0] = make_float2(a.x + bw.x, a.y + bw.y);
      buf[c][i1] = make_float2(a.x - bw.x, a.y - bw.y);
    }
    __syncthreads();
  }
  for (int i = tid; i < C * N; i += 256) {
    int c, e;
    if (COLS) {
      e = i / C;
      c = i - e * C;
    } else {
      c = i / N;
      e = i - c * N;
    }
    if (line0 + c >= nlines) continue;
    const float2 v = buf[c][e];
    data[addr(c, e)] = make_float2(v.x * scale, v.y * scale);
  }
}

// 256-point lines as 16 x 16 (four-step Cooley-Tukey): with n = 16 n1 + q
// and k = k1 + 16 k2, X[k] = sum_q W256^(q k1) W16^(q k2) sum_n1 x[n] W16^(n1 k1).
// Thread q of a line holds x[16 n1 + q] for all n1, takes the inner 16-point
// DFT in registers, applies W256^(q k1), and the line is transposed once
// through LDS so that thread k1 takes the outer 16-point DFT over q and holds
// X[k1 + 16 k2].  A 16-point DFT is itself 4 x 4 (n = 4 a + b, k = c + 4 d).
// One LDS round trip per element instead of log2(256) = 8 radix-2 stages.
__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
  return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// 4-point DFT in place, W4 = exp(-+ i pi / 2): u = +1 forward (multiply by
// -i), u = -1 inverse (by +i)
__device__ __forceinline__ void dft4(float2 &x0, float2 &x1, float2 &x2, float2 &x3, float u) {
  const float2 a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = csub(x1, x3);
  const float2 dm = make_float2(u * d.y, -u * d.x);  // d W4 (= -i d forward)
  x0 = cadd(a, c);
  x2 = csub(a, c);
  x1 = cadd(b, dm);
  x3 = csub(b, dm);
}
// 16-point DFT of v[0..15] (natural order in and out); w16[m] = W16^m
__device__ __forceinline__ void dft16(float2 *v, const float2 *w16, float u) {
  float2 t[4][4];  // t[b][c]
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    float2 x0 = v[b], x1 = v[4 + b], x2 = v[8 + b], x3 = v[12 + b];
    dft4(x0, x1, x2, x3, u);
    t[b][0] = x0;
    t[b][1] = cmul(x1, w16[b]);
    t[b][2] = cmul(x2, w16[2 * b]);
    t[b][3] = cmul(x3, w16[3 * b]);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float2 x0 = t[0][c], x1 = t[1][c], x2 = t[2][c], x3 = t[3][c];
    dft4(x0, x1, x2, x3, u);
    v[c] = x0;
    v[c + 4] = x1;
    v[c + 8] = x2;
    v[c + 12] = x3;
  }
}

template <bool COLS>
__global__ __launch_bounds__(256) void k_fft256(float2 *__restrict__ data, int64_t nimg, int ny, int nx,
                                                int inverse) {
  constexpr int N = 256;
  __shared__ float2 tw[N];               // W256^m
  __shared__ float2 buf[16][16][17];     // [line][k1][q], padded
  const int tid = threadIdx.x;
  {
    double sn, cs;
    sincospi(-2.0 * tid / N, &sn, &cs);
    tw[tid] = make_float2((float)cs, inverse ? -(float)sn : (float)sn);
  }
  const float u = inverse ? -1.f : 1.f;
  // thread (c, q): line c of the block, position q in it; consecutive
  // threads take consecutive elements (rows) or consecutive columns
  const int c = COLS ? (tid & 15) : (tid >> 4), q = COLS ? (tid >> 4) : (tid & 15);
  const int lpi = COLS ? nx : ny;
  const int64_t nlines = nimg * lpi;
  const int64_t l = (int64_t)blockIdx.x * 16 + c;
  const bool live = l < nlines;
  const int64_t img = live ? l / lpi : 0;
  const int j = live ? (int)(l - img * lpi) : 0;
  float2 *base = data + img * (int64_t)nx * ny + (COLS ? j : (int64_t)j * nx);
  const int64_t es = COLS ? nx : 1;  // element stride
  float2 v[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) v[n1] = live ? base[(16 * n1 + q) * es] : make_float2(0.f, 0.f);
  __syncthreads();  // the twiddle table
  float2 w16[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) w16[m] = tw[16 * m];
  dft16(v, w16, u);
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) buf[c][k1][q] = cmul(v[k1], tw[(q * k1) & (N - 1)]);
  __syncthreads();
  // now thread (c, q) takes k1 = q
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) v[n2] = buf[c][q][n2];
  dft16(v, w16, u);
  if (live) {
    const float sc = 1.f / 16.f;  // 1 / sqrt(256)
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) base[(q + 16 * k2) * es] = make_float2(v[k2].x * sc, v[k2].y * sc);
  }
}

template <int N, bool COLS>
static void fft_pass(float2 *data, int64_t nimg, int ny, int nx, int inverse, hipStream_t s) {
  constexpr int C = FftCfg<N>::C;
  const int64_t lines = nimg * (COLS ? nx : ny);
  const int64_t blocks = (lines + C - 1) / C;
  hipLaunchKernelGGL((k_fft_lines<N, COLS>), dim3((unsigned)blocks), dim3(256), 0, s, data, nimg,
                     ny, nx, inverse);
}

template <bool COLS>
static void fft_pass_n(int N, float2 *data, int64_t nimg, int ny, int nx, int inverse,
                       hipStream_t s) {
  if (N == 256) {
    const int64_t lines = nimg * (COLS ? nx : ny);
    hipLaunchKernelGGL(k_fft256<COLS>, dim3((unsigned)((lines + 15) / 16)), dim3(256), 0, s, data, nimg, ny, nx,
                       inverse);
    return;
  }
  switch (N) {
    case 16: fft_pass<16, COLS>(data, nimg, ny, nx, inverse, s); break;
    case 32: fft_pass<32, COLS>(data, nimg, ny, nx, inverse, s); break;
    case 64: fft_pass<64, COLS>(data, nimg, ny, nx, inverse, s); break;
    case 128: fft_pass<128, COLS>(data, nimg, ny, nx, inverse, s); break;
    case 256: fft_pass<256, COLS>(data, nimg, ny, nx, inverse, s); break;
    case 512: fft_pass<512, COLS>(data, nimg, ny, nx, inverse, s); break;
    default: break;
  }
}

void launch_fft2(float2 *data, int64_t nimg, int ny, int nx, int inverse, hipStream_t s) {
  fft_pass_n<false>(nx, data, nimg, ny, nx, inverse, s);
  fft_pass_n<true>(ny, data, nimg, ny, nx, inverse, s);
}

// ---------------------------------------------------------------------------
// sampling
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_sample(const float2 *__restrict__ K, int64_t npix,
                                                const int64_t *__restrict__ off,
                                                const int32_t *__restrict__ sidx,
                                                const float2 *__restrict__ Y,
                                                const float *__restrict__ w,
                                                float2 *__restrict__ R, double *part, int64_t M, int L,
                                                int ncoil) {
  __shared__ double red[256];
  const int pv = blockIdx.x;
  const VPair vp = vpair(pv, L, ncoil, M);
  const int64_t b = min(max(off[vp.p], (int64_t)0), M), e = min(max(off[vp.p + 1], b), M);
  const float2 *img = K + (int64_t)pv * npix;
  double acc = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) {
    const uint32_t k = (uint32_t)sidx[i];
    float2 r = k < (uint32_t)npix ? img[k] : make_float2(0.f, 0.f);
    if (Y) {
      const float2 y = Y[vp.qoff + i];
      r.x -= y.x;
      r.y -= y.y;
    }
    R[vp.qoff + i] = r;
    const double m = (double)r.x * r.x + (double)r.y * r.y;
    acc += w ? (double)w[i] * m : m;
  }
  const double s = block_sum_f64(acc, red);
  if (threadIdx.x == 0 && part) part[pv] = s;
}

void launch_sample(const float2 *K, int64_t npix, const int64_t *off, const int32_t *sidx,
                   const float2 *Y, const float *w, float2 *R, double *part, int nvpairs,
                   int64_t M, int L, int ncoil, hipStream_t s) {
  hipLaunchKernelGGL(k_sample, dim3(nvpairs), dim3(256), 0, s, K, npix, off, sidx, Y, w, R, part, M, L, ncoil);
}

__global__ __launch_bounds__(256) void k_zero(float4 *p, int64_t n4) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}
__global__ void k_zero_bytes(unsigned char *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0;
}

void launch_zero(void *p, int64_t bytes, hipStream_t s) {
  if (bytes <= 0) return;
  const int64_t n4 = bytes / 16;
  if (n4 > 0) {
    int64_t blocks = (n4 + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<float4 *>(p), n4);
  }
  const int64_t rem = bytes - n4 * 16;
  if (rem > 0)
    hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(256), 0, s,
                       reinterpret_cast<unsigned char *>(p) + n4 * 16, rem);
}

__global__ __launch_bounds__(256) void k_scatter(const float2 *__restrict__ R,
                                                 const float *__restrict__ w,
                                                 const int64_t *__restrict__ off,
                                                 const int32_t *__restrict__ sidx,
                                                 float2 *__restrict__ K, int64_t npix, int64_t M, int L,
                                                 int ncoil) {
  const int pv = blockIdx.x;
  const VPair vp = vpair(pv, L, ncoil, M);
  const int64_t b = min(max(off[vp.p], (int64_t)0), M), e = min(max(off[vp.p + 1], b), M);
  float2 *img = K + (int64_t)pv * npix;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) {
    const uint32_t k = (uint32_t)sidx[i];
    if (k >= (uint32_t)npix) continue;
    float2 r = R[vp.qoff + i];
    if (w) {
      const float a = w[i];
      r.x *= a;
      r.y *= a;
    }
    img[k] = r;
  }
}

void launch_scatter(const float2 *R, const float *w, const int64_t *off, const int32_t *sidx,
                    float2 *K, int64_t npix, int nvpairs, int64_t total, int64_t M, int L, int ncoil,
                    hipStream_t s) {
  launch_zero(K, total * (int64_t)sizeof(float2), s);
  hipLaunchKernelGGL(k_scatter, dim3(nvpairs), dim3(256), 0, s, R, w, off, sidx, K, npix, M, L, ncoil);
}

__global__ __launch_bounds__(256) void k_step_norms(const float2 *__restrict__ R,
                                                    const float2 *__restrict__ A,
                                                    const float *__restrict__ w,
                                                    const int64_t *__restrict__ off, int64_t M,
                                                    int L, int ncoil, double *part_a, double *part_ra,
                                                    float2 *R_update) {
  __shared__ double red[256];
  const int pv = blockIdx.x;
  const VPair vp = vpair(pv, L, ncoil, M);
  const int64_t b = min(max(off[vp.p], (int64_t)0), M), e = min(max(off[vp.p + 1], b), M);
  double sa = 0.0, sra = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) {
    const float2 a = A[vp.qoff + i];
    const float2 r = R[vp.qoff + i];
    const double wi = w ? (double)w[i] : 1.0;
    sa += wi * ((double)a.x * a.x + (double)a.y * a.y);
    const double qx = (double)r.x + a.x, qy = (double)r.y + a.y;
    sra += wi * (qx * qx + qy * qy);
    if (R_update) R_update[vp.qoff + i] = make_float2(r.x + a.x, r.y + a.y);
  }
  const double t1 = block_sum_f64(sa, red);
  if (threadIdx.x == 0) part_a[pv] = t1;
  __syncthreads();
  const double t2 = block_sum_f64(sra, red);
  if (threadIdx.x == 0) part_ra[pv] = t2;
}

void launch_step_norms(const float2 *R, const float2 *A, const float *w, const int64_t *off,
                       int nvpairs, int64_t M, int L, int ncoil, double *part_a, double *part_ra,
                       float2 *R_update, hipStream_t s) {
  hipLaunchKernelGGL(k_step_norms, dim3(nvpairs), dim3(256), 0, s, R, A, w, off, M, L, ncoil, part_a,
                     part_ra, R_update);
}

// ---------------------------------------------------------------------------
// coil sensitivities (eq. forward, c coils)
// ---------------------------------------------------------------------------
// out [S][c][F][npix] = S_q (pixel-wise) x X [S][F][npix]
__global__ __launch_bounds__(256) void k_coil_expand(const float2 *__restrict__ X,
                                                     const float2 *__restrict__ maps, int64_t npix, int F,
                                                     int ncoil, int64_t total, float2 *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int64_t pix = e % npix;
  const int64_t r = e / npix;  // (sl * c + q) * F + f
  const int f = (int)(r % F);
  const int64_t vs = r / F;
  const int64_t sl = vs / ncoil;
  const float2 m = maps[vs * npix + pix], x = X[(sl * F + f) * npix + pix];
  out[e] = make_float2(m.x * x.x - m.y * x.y, m.x * x.y + m.y * x.x);
}

void launch_coil_expand(const float2 *X, const float2 *maps, int S, int ncoil, int F, int64_t npix, float2 *out,
                        hipStream_t s) {
  const int64_t total = (int64_t)S * ncoil * F * npix;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_coil_expand, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, X, maps, npix, F,
                     ncoil, total, out);
}

// G [S][F][npix] = sum_q conj(S_q) x Gc [S][c][F][npix], coils in increasing order
__global__ __launch_bounds__(256) void k_coil_combine(const float2 *__restrict__ Gc,
                                                      const float2 *__restrict__ maps, int64_t npix, int F,
                                                      int ncoil, int64_t total, float2 *__restrict__ G) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int64_t pix = e % npix;
  const int64_t r = e / npix;  // sl * F + f
  const int f = (int)(r % F);
  const int64_t sl = r / F;
  float gx = 0.f, gy = 0.f;
  for (int q = 0; q < ncoil; ++q) {
    const int64_t vs = sl * ncoil + q;
    const float2 m = maps[vs * npix + pix], g = Gc[(vs * F + f) * npix + pix];
    gx = fmaf(m.x, g.x, fmaf(m.y, g.y, gx));
    gy = fmaf(m.x, g.y, fmaf(-m.y, g.x, gy));
  }
  G[e] = make_float2(gx, gy);
}

void launch_coil_combine(const float2 *Gc, const float2 *maps, int S, int ncoil, int F, int64_t npix, float2 *G,
                         hipStream_t s) {
  const int64_t total = (int64_t)S * F * npix;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_coil_combine, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, Gc, maps, npix, F,
                     ncoil, total, G);
}

__global__ __launch_bounds__(256) void k_reduce_sum(const double *__restrict__ part,
                                                    int64_t count, double *out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) acc += part[i];
  const double s = block_sum_f64(acc, red);
  if (threadIdx.x == 0) out[0] = s;
}

void launch_reduce_sum(const double *part, int64_t count, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, s, part, count, out);
}

__global__ __launch_bounds__(256) void k_scale(float2 *x, int64_t count, float a) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    float2 v = x[i];
    x[i] = make_float2(v.x * a, v.y * a);
  }
}

void launch_scale(float2 *x, int64_t count, float a, hipStream_t s) {
  int64_t blocks = (count + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks > 0) hipLaunchKernelGGL(k_scale, dim3((unsigned)blocks), dim3(256), 0, s, x, count, a);
}

}  // namespace mrf

namespace mrf {

__global__ __launch_bounds__(256) void k_norm2(const float2 *__restrict__ x, int64_t count,
                                               double *part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    const float2 v = x[i];
    acc += (double)v.x * v.x + (double)v.y * v.y;
  }
  const double sum = block_sum_f64(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

void launch_norm2(const float2 *x, int64_t count, double *part, int *nblocks_out, hipStream_t s) {
  int64_t blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  *nblocks_out = (int)blocks;
  hipLaunchKernelGGL(k_norm2, dim3((unsigned)blocks), dim3(256), 0, s, x, count, part);
}

}  // namespace mrf
