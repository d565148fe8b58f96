// Learned-proposal network kernels for gfx950: a general FP32 GEMM on MFMA
// (v_mfma_f32_32x32x2f32) with fused bias / row-scale / GELU / GELU-gradient
// epilogues, the loss and its gradient, bias-gradient column sums, the Adam
// update, the on-device generator of noisy training atoms, and the map from
// network outputs to grid cells.
#include <cmath>

#include "mrf_internal.h"

namespace mrf {

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float gelu_f(float a) { return 0.5f * a * (1.f + erff(a * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float a) {
  return 0.5f * (1.f + erff(a * 0.70710678118654752f)) + a * expf(-0.5f * a * a) * 0.3989422804014327f;
}

// ---------------------------------------------------------------------------
// GEMM: C[m][n] = epi( sum_k A(m,k) B(n,k) )
//   A(m,k) = AK ? A[m*lda + k] : A[k*lda + m];  B(n,k) = BK ? B[n*ldb + k] : B[k*ldb + n]
// Block tile 64 x 64, K chunks of 16 in LDS (zero-filled past M, N, K); four
// waves, each one 32x32 MFMA tile.
// ---------------------------------------------------------------------------
constexpr int G_T = 64, G_BK = 16, G_LD = 20;

// Split K: block z of grid.z sums k in [z kchunk, (z+1) kchunk) into
// C + z cstride (plain store; the partial sums are added by k_sum_parts).
template <bool AK, bool BK>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float *__restrict__ A,
                                              int64_t lda, const float *__restrict__ B, int64_t ldb,
                                              float *__restrict__ C, int64_t ldc, GemmEpi epi, int kchunk,
                                              int64_t cstride) {
  __shared__ float As[G_T][G_LD];
  __shared__ float Bs[G_T][G_LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int m0 = blockIdx.y * G_T, n0 = blockIdx.x * G_T;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  C += blockIdx.z * cstride;
  for (int k0 = kb; k0 < ke; k0 += G_BK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = tid + 256 * q;
      int r, c;  // r: row within tile (m or n), c: k within chunk
      if (AK) { r = i >> 4; c = i & 15; } else { c = i >> 6; r = i & 63; }
      const int gm = m0 + r, gk = k0 + c;
      float va = 0.f;
      if (gm < M && gk < ke) va = AK ? A[(int64_t)gm * lda + gk] : A[(int64_t)gk * lda + gm];
      As[r][c] = va;
      if (BK) { r = i >> 4; c = i & 15; } else { c = i >> 6; r = i & 63; }
      const int gn = n0 + r, gk2 = k0 + c;
      float vb = 0.f;
      if (gn < N && gk2 < ke) vb = BK ? B[(int64_t)gn * ldb + gk2] : B[(int64_t)gk2 * ldb + gn];
      Bs[r][c] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 8; ++s)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[wm + l32][h * 8 + s], Bs[wn + l32][h * 8 + s], acc, 0, 0, 0);
    __syncthreads();
  }
  const int n = n0 + wn + l32;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int m = m0 + wm + 8 * (i >> 2) + 4 * h + (i & 3);
    if (m >= M || n >= N) continue;
    float v = acc[i];
    if (epi.rowscale) v *= epi.rowscale[m];
    if (epi.bias) v += epi.bias[n];
    if (epi.kind == GEMM_GELU) {
      if (epi.pre) epi.pre[(int64_t)m * ldc + n] = v;
      v = gelu_f(v);
    } else if (epi.kind == GEMM_GELU_GRAD) {
      v *= gelu_grad_f(epi.gpre[(int64_t)m * ldc + n]);
    }
    C[(int64_t)m * ldc + n] = v;
  }
}

static void gemm_dispatch(dim3 grid, int M, int N, int K, const float *A, int64_t lda, bool a_kcontig,
                          const float *B, int64_t ldb, bool b_kcontig, float *C, int64_t ldc, const GemmEpi &epi,
                          int kchunk, int64_t cstride, hipStream_t s) {
  if (a_kcontig && b_kcontig)
    hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, epi, kchunk,
                       cstride);
  else if (a_kcontig)
    hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, epi, kchunk,
                       cstride);
  else if (b_kcontig)
    hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, epi, kchunk,
                       cstride);
  else
    hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, epi, kchunk,
                       cstride);
}

void launch_gemm(int M, int N, int K, const float *A, int64_t lda, bool a_kcontig, const float *B,
                 int64_t ldb, bool b_kcontig, float *C, int64_t ldc, const GemmEpi &epi,
                 hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  dim3 grid((unsigned)((N + G_T - 1) / G_T), (unsigned)((M + G_T - 1) / G_T));
  gemm_dispatch(grid, M, N, K, A, lda, a_kcontig, B, ldb, b_kcontig, C, ldc, epi, K, 0, s);
}

// out[i] = sum_z part[z][i] (z in order)
__global__ void k_sum_parts(const float *__restrict__ part, int splits, int64_t count, float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float acc = 0.f;
  for (int z = 0; z < splits; ++z) acc += part[z * count + i];
  out[i] = acc;
}

void launch_gemm_splitk(int M, int N, int K, const float *A, int64_t lda, bool a_kcontig, const float *B,
                        int64_t ldb, bool b_kcontig, float *C, int splits, float *part, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  const int kchunk = (int)round_up((K + splits - 1) / splits, G_BK);
  splits = (K + kchunk - 1) / kchunk;
  dim3 grid((unsigned)((N + G_T - 1) / G_T), (unsigned)((M + G_T - 1) / G_T), (unsigned)splits);
  const int64_t count = (int64_t)M * N;
  gemm_dispatch(grid, M, N, K, A, lda, a_kcontig, B, ldb, b_kcontig, part, N, GemmEpi(), kchunk, count, s);
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, part, splits, count, C);
}

// ---------------------------------------------------------------------------
// loss, bias gradients, Adam
// ---------------------------------------------------------------------------
// dy = 2 (y - t) / (B P); part[block] = sum (y - t)^2 (FP64)
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y, const float *__restrict__ t,
                                             int64_t count, float scale, float *__restrict__ dy,
                                             double *part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) {
    const float r = y[i] - t[i];
    dy[i] = scale * r;
    acc += (double)r * r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

void launch_mse(const float *y, const float *t, int64_t count, float scale, float *dy, double *part,
                int *nblocks, hipStream_t s) {
  int64_t b = (count + 255) / 256;
  if (b > 256) b = 256;
  *nblocks = (int)b;
  hipLaunchKernelGGL(k_mse, dim3((unsigned)b), dim3(256), 0, s, y, t, count, scale, dy, part);
}

// out[n] = sum_b x[b][n] in a fixed order: a block of 1024 threads takes 16
// columns; thread (g, c) sums rows g, g + 64, g + 128, ... of column c, then
// the 64 partial sums of a column are added in order of g.
__global__ __launch_bounds__(1024) void k_colsum(const float *__restrict__ x, int rows, int cols,
                                                 float *__restrict__ out) {
  __shared__ float part[64][17];
  const int cl = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int c = blockIdx.x * 16 + cl;
  float acc = 0.f;
  if (c < cols)
    for (int r = g; r < rows; r += 64) acc += x[(int64_t)r * cols + c];
  part[g][cl] = acc;
  __syncthreads();
  if (threadIdx.x < 16 && c < cols) {
    float t = 0.f;
    for (int i = 0; i < 64; ++i) t += part[i][cl];
    out[c] = t;
  }
}

void launch_colsum(const float *x, int rows, int cols, float *out, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)((cols + 15) / 16)), dim3(1024), 0, s, x, rows, cols, out);
}

__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t count, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

void launch_adam(float *w, const float *g, float *m, float *v, int64_t count, float lr, float b1,
                 float b2, float eps, int64_t t, hipStream_t s) {
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)t));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)t));
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, s, w, g, m, v, count, lr, b1, b2,
                     eps, c1, c2);
}

// inv[v] = 1/znorm[v] (0 for zero or non-finite rows)
__global__ void k_inv_norm(const float *__restrict__ zn, int64_t n, float *__restrict__ inv) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) inv[v] = zn[v] > 0.f ? 1.f / zn[v] : 0.f;
}

void launch_inv_norm(const float *znorm, int64_t n, float *inv, hipStream_t s) {
  hipLaunchKernelGGL(k_inv_norm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, znorm, n, inv);
}

// ---------------------------------------------------------------------------
// noisy training atoms
// ---------------------------------------------------------------------------
// Counter-based SplitMix64 (Steele, Lea, Flood 2014) as a stateless hash:
// draw i of stream `key` is mix(key + (i+1) * 0x9E3779B97F4A7C15).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double u01(uint64_t key, uint64_t i) {
  return (double)(mix64(key + (i + 1) * 0x9E3779B97F4A7C15ull) >> 11) * 0x1.0p-53;
}

// One block per sample s: atom j ~ U{0..d-1}, SNR ~ U(lo, hi) dB, x = Dhat_j +
// circular complex Gaussian noise of per-entry variance 10^(-SNR/10)/L;
// input row = x / ||x|| in the contraction layout (interleaved complex, or
// the real part for real atoms with the norm over the complex entries);
// target row = standardised parameters of atom j.
__global__ __launch_bounds__(256) void k_noisy_batch(
    const float *__restrict__ Dhat, int Kp, int L, int real_atoms, int d,
    const float *__restrict__ params, int nparam, const float *__restrict__ mean,
    const float *__restrict__ stdv, const int *__restrict__ logm, uint64_t key_atom,
    uint64_t key_snr, uint64_t key_noise, int64_t offset, float snr_lo, float snr_hi,
    float *__restrict__ X, int ldx, float *__restrict__ T, int32_t *__restrict__ atom_out) {
  __shared__ double red[256];
  const int64_t s = blockIdx.x;
  const int64_t gs = offset + s;
  int j = (int)(u01(key_atom, (uint64_t)gs) * (double)d);
  if (j >= d) j = d - 1;
  const double snr = (double)snr_lo + ((double)snr_hi - (double)snr_lo) * u01(key_snr, (uint64_t)gs);
  const double sig = sqrt(pow(10.0, -snr / 10.0) / (double)L * 0.5);
  const float *a = Dhat + (int64_t)j * Kp;
  const int K = real_atoms ? L : 2 * L;
  float *x = X + s * ldx;
  double acc = 0.0;
  for (int t = threadIdx.x; t < L; t += 256) {
    const uint64_t c = (uint64_t)gs * (uint64_t)L + (uint64_t)t;
    const double v1 = 1.0 - u01(key_noise, 2 * c);
    const double v2 = u01(key_noise, 2 * c + 1);
    const double rr = sqrt(-2.0 * log(v1));
    double sn, cs;
    sincospi(2.0 * v2, &sn, &cs);
    const double nre = sig * rr * cs, nim = sig * rr * sn;
    double xr, xi;
    if (real_atoms) {
      xr = (double)a[t] + nre;
      xi = nim;
      x[t] = (float)xr;
    } else {
      xr = (double)a[2 * t] + nre;
      xi = (double)a[2 * t + 1] + nim;
      x[2 * t] = (float)xr;
      x[2 * t + 1] = (float)xi;
    }
    acc += xr * xr + xi * xi;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const float inv = (float)(1.0 / sqrt(red[0]));
  for (int k = threadIdx.x; k < K; k += 256) x[k] *= inv;
  if (threadIdx.x < nparam && T) {
    const int p = threadIdx.x;
    float th = params[(int64_t)j * nparam + p];
    if (logm[p]) th = logf(th);
    T[s * nparam + p] = (th - mean[p]) / stdv[p];
  }
  if (threadIdx.x == 0 && atom_out) atom_out[s] = j;
}

void launch_noisy_batch(const float *Dhat, int Kp, int L, int real_atoms, int d, const float *params,
                        int nparam, const float *mean, const float *stdv, const int *logm,
                        uint64_t key_atom, uint64_t key_snr, uint64_t key_noise, int64_t offset,
                        int64_t B, float snr_lo, float snr_hi, float *X, int ldx, float *T,
                        int32_t *atom_out, hipStream_t s) {
  hipLaunchKernelGGL(k_noisy_batch, dim3((unsigned)B), dim3(256), 0, s, Dhat, Kp, L, real_atoms, d,
                     params, nparam, mean, stdv, logm, key_atom, key_snr, key_noise, offset, snr_lo,
                     snr_hi, X, ldx, T, atom_out);
}

// ---------------------------------------------------------------------------
// network output -> nearest grid cell per parameter
// ---------------------------------------------------------------------------
// axes: concatenated per-parameter grid values (ascending), axis p at
// axes[aoff[p] .. aoff[p] + dims[p]); comparisons in the transformed space
// (log where logm[p]), ties to the lower index.
// prep (optional): the start-of-call initialisation of k_learned_prep done by
// the same threads (the grid then covers its counter ranges too).
__global__ void k_cells(const float *__restrict__ Y, int64_t n, int P, const float *__restrict__ mean,
                        const float *__restrict__ stdv, const int *__restrict__ logm,
                        const float *__restrict__ axes, const int *__restrict__ aoff,
                        const int *__restrict__ dims, int32_t *__restrict__ cells, LearnedPrep prep) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (prep.list) learned_prep_at(v, prep, n);
  if (v >= n) return;
  for (int p = 0; p < P; ++p) {
    const float val = Y[v * P + p] * stdv[p] + mean[p];
    const float *ax = axes + aoff[p];
    const int N = dims[p];
    // first index with transformed axis value >= val
    int lo = 0, hi = N;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const float fa = logm[p] ? logf(ax[mid]) : ax[mid];
      if (fa < val) lo = mid + 1; else hi = mid;
    }
    int c;
    if (lo <= 0) c = 0;
    else if (lo >= N) c = N - 1;
    else {
      const float f0 = logm[p] ? logf(ax[lo - 1]) : ax[lo - 1];
      const float f1 = logm[p] ? logf(ax[lo]) : ax[lo];
      c = (val - f0 <= f1 - val) ? lo - 1 : lo;
    }
    if (!(val == val)) c = 0;
    cells[v * P + p] = c;
  }
}

void launch_cells(const float *Y, int64_t n, int P, const float *mean, const float *stdv,
                  const int *logm, const float *axes, const int *aoff, const int *dims, int32_t *cells,
                  hipStream_t s, const LearnedPrep *prep) {
  const LearnedPrep pp = prep ? *prep : LearnedPrep{};
  const int64_t m = prep ? std::max<int64_t>(n, std::max(pp.nz, pp.nz2)) : n;
  if (m <= 0) return;
  hipLaunchKernelGGL(k_cells, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, Y, n, P, mean,
                     stdv, logm, axes, aoff, dims, cells, pp);
}

}  // namespace mrf
