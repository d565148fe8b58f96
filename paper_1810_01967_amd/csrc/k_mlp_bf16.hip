// BF16 inference of the proposal network on gfx950 (v_mfma_f32_32x32x16_bf16,
// FP32 accumulation), for hidden width 256:
//   layer 1: h1 = GELU(x W1^T + b1), x = rowscale * X rounded to BF16, W1 in
//            BF16; h1 is written in BF16.  The split-row form reads the BF16
//            high parts of split voxel rows instead and scales the FP32
//            accumulator: h1 = GELU(rowscale * (RNE_bf16(X) W1^T) + b1), the
//            same network (linear in x before the bias) with the rounding
//            taken before the scale;
//   layer 2: h2 = GELU(h1 W2^T + b2) kept in FP32 and the output layer
//            y = h2 W3^T + b3 (FP32 W3) fused into the same block.
// A block computes all 256 hidden units of 256 rows (layer 1, sixteen waves)
// or 128 rows (layer 2, eight waves, its FP32 h2 tile in LDS); each wave owns
// 64 rows x 64 units (2 x 2 tiles of 32 x 32); K is staged through LDS in
// chunks of 32.  Larger row tiles read the weights fewer times.
#include <cmath>

#include "k_split.h"
#include "mrf_internal.h"

namespace mrf {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int MB_H = 256;   // hidden units (= block columns)
constexpr int MB_BK = kMlpBK;    // K per stage
constexpr int MB_LD = MB_BK + 8; // LDS row pitch in BF16 (8 of padding)
constexpr int MB_PC = MB_BK / 32;  // 8-element pieces per thread and row per stage
constexpr int MB_HLD = 260; // LDS row pitch of the FP32 h2 tile: 4 quarters of 64 units at stride 65
__device__ __forceinline__ int hq(int n) { return (n >> 6) * 65 + (n & 63); }  // unit n within a row
// rows per block of the two launches (tuning constants: 4 threads per row)
#ifndef MRF_MLP_M1
#define MRF_MLP_M1 256
#endif
#ifndef MRF_MLP_M2
#define MRF_MLP_M2 128
#endif
#ifndef MRF_MLP_WR1
#define MRF_MLP_WR1 64
#endif

__device__ __forceinline__ uint16_t to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float gelu_exact(float a) { return 0.5f * a * (1.f + erff(a * 0.70710678118654752f)); }

// FP32 [rows][cols] (leading dimension lds) -> BF16 [rows][ldd], zero beyond cols.
__global__ void k_to_bf16(const float *__restrict__ src, int rows, int cols, int64_t lds,
                          uint16_t *__restrict__ dst, int ldd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * ldd) return;
  const int64_t r = i / ldd;
  const int c = (int)(i - r * ldd);
  dst[i] = c < cols ? to_bf16(src[r * lds + c]) : (uint16_t)0;
}

void launch_to_bf16(const float *src, int rows, int cols, int64_t lds, uint16_t *dst, int ldd, hipStream_t s) {
  const int64_t n = (int64_t)rows * ldd;
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, rows, cols, lds, dst, ldd);
}

// LAYER1 = true: A = FP32 rows X (pitch ldx, K valid columns, K % 8 == 0,
// ldx % 4 == 0) times rowscale, W = W1 BF16 [256][Kx]; writes H1 BF16 [B][256].
// LAYER1 and SPLIT: A = the high parts of split rows H1in (2 Kx BF16 per row,
// pitch ldx elements; zero beyond the valid columns), rowscale applied to
// the accumulator.
// LAYER1 = false: A = H1 BF16 [B][256], W = W2 BF16 [256][256]; writes Y [B][P].
// WR: rows per wave (64, or 32 for twice the waves on the same row tile).
template <bool LAYER1, int MB_M, int WR, bool SPLIT = false>
__global__ __launch_bounds__(4 * MB_M * (64 / WR)) void k_mlp_bf16(int64_t B, const float *__restrict__ X, int64_t ldx, int K,
                                                     int Kx, const float *__restrict__ rowscale,
                                                     const uint16_t *__restrict__ H1in,
                                                     const uint16_t *__restrict__ W, const float *__restrict__ bias,
                                                     uint16_t *__restrict__ H1out, const float *__restrict__ W3,
                                                     const float *__restrict__ b3, int P, float *__restrict__ Y) {
  // MB_M rows per block, one wave per WR rows x 64 units
  constexpr int NT = 4 * MB_M * (64 / WR);      // threads per block
  constexpr int MI = WR / 32;                   // 32-row tiles per wave
  constexpr int NW = MB_H * 4 / NT;             // W chunks of 8 per thread per stage
  constexpr int STAGE = (MB_M + MB_H) * MB_LD;  // BF16 elements per stage
  // layer 2: the FP32 h2 tile and W3 (at most 8 rows) share the stage space
  constexpr int SMEM = LAYER1 ? 2 * STAGE * 2
                              : ((MB_M + 8) * MB_HLD * 4 > 2 * STAGE * 2 ? (MB_M + 8) * MB_HLD * 4 : 2 * STAGE * 2);
  __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int wr = (wave >> 2) * WR, wn = (wave & 3) * 64;  // the wave's rows and units
  const int64_t m0 = (int64_t)blockIdx.x * MB_M;
  const int nk = (LAYER1 ? Kx : MB_H) / MB_BK;
  const int ldw = LAYER1 ? Kx : MB_H;

  // loader: thread t covers row t/4 (A, the first 4 MB_M threads) and rows
  // t/4 + (NT/4) i (W), 8 MB_PC elements at (t & 3) * 8 MB_PC
  const int lr = tid >> 2, lc = (tid & 3) * 8 * MB_PC;
  const bool aload = lr < MB_M;
  const int64_t arow = m0 + lr;
  const bool avalid = aload && arow < B;
  const float sc = (LAYER1 && !SPLIT && avalid) ? (rowscale ? rowscale[arow] : 1.f) : 0.f;
  uint4 ra[MB_PC], rw[NW][MB_PC];
  auto gload = [&](int kc) {
#pragma unroll
    for (int c = 0; c < MB_PC; ++c) {
      const int k = kc * MB_BK + lc + 8 * c;
      if constexpr (LAYER1 && SPLIT) {  // 8 high parts of one 32-column chunk
        ra[c] = avalid ? *reinterpret_cast<const uint4 *>(H1in + arow * ldx + split_off(k))
                       : make_uint4(0u, 0u, 0u, 0u);
      } else if constexpr (LAYER1) {
        float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (avalid && k < K) {
          const float4 x0 = *reinterpret_cast<const float4 *>(X + arow * ldx + k);
          const float4 x1 = *reinterpret_cast<const float4 *>(X + arow * ldx + k + 4);
          v[0] = x0.x; v[1] = x0.y; v[2] = x0.z; v[3] = x0.w;
          v[4] = x1.x; v[5] = x1.y; v[6] = x1.z; v[7] = x1.w;
        }
        uint32_t p[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          p[i] = (uint32_t)to_bf16(v[2 * i] * sc) | ((uint32_t)to_bf16(v[2 * i + 1] * sc) << 16);
        ra[c] = make_uint4(p[0], p[1], p[2], p[3]);
      } else {
        ra[c] = avalid ? *reinterpret_cast<const uint4 *>(H1in + arow * MB_H + k) : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int i = 0; i < NW; ++i)
        rw[i][c] = *reinterpret_cast<const uint4 *>(W + (int64_t)(lr + (NT / 4) * i) * ldw + k);
    }
  };
  auto sstore = [&](int buf) {
    uint16_t *S = reinterpret_cast<uint16_t *>(smem) + buf * STAGE;
#pragma unroll
    for (int c = 0; c < MB_PC; ++c) {
      if (aload) *reinterpret_cast<uint4 *>(S + lr * MB_LD + lc + 8 * c) = ra[c];
#pragma unroll
      for (int i = 0; i < NW; ++i)
        *reinterpret_cast<uint4 *>(S + (MB_M + lr + (NT / 4) * i) * MB_LD + lc + 8 * c) = rw[i][c];
    }
  };

  f32x16 acc[MI][2];
#pragma unroll
  for (int a = 0; a < MI; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;

  gload(0);
  sstore(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) gload(kc + 1);
    const __bf16 *S = reinterpret_cast<const __bf16 *>(smem) + buf * STAGE;
#pragma unroll
    for (int ks = 0; ks < MB_BK / 16; ++ks) {
      bf16x8 a[MI], w[2];
#pragma unroll
      for (int mi = 0; mi < MI; ++mi)
        a[mi] = *reinterpret_cast<const bf16x8 *>(S + (wr + mi * 32 + l32) * MB_LD + ks * 16 + h * 8);
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
        w[ni] = *reinterpret_cast<const bf16x8 *>(S + (MB_M + wn + ni * 32 + l32) * MB_LD + ks * 16 + h * 8);
#pragma unroll
      for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mi], w[ni], acc[mi][ni], 0, 0, 0);
    }
    if (kc + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }
  // output element (row 8 (i / 4) + 4 h + (i % 4) of tile mi, unit l32 of tile ni)
  if constexpr (LAYER1) {
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
      const int n = wn + ni * 32 + l32;
      const float bn = bias[n];
#pragma unroll
      for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int64_t m = m0 + wr + mi * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
          if (m < B) {
            const float a = SPLIT ? acc[mi][ni][i] * (rowscale ? rowscale[m] : 1.f) : acc[mi][ni][i];
            H1out[m * MB_H + n] = to_bf16(gelu_exact(a + bn));
          }
        }
    }
  } else {
    float *Hs = reinterpret_cast<float *>(smem);
    float *W3s = Hs + MB_M * MB_HLD;  // [P][MB_HLD], the h2 row layout
    for (int e = tid; e < P * MB_H; e += NT) W3s[(e / MB_H) * MB_HLD + hq(e % MB_H)] = W3[e];
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
      const int n = wn + ni * 32 + l32;
      const float bn = bias[n];
#pragma unroll
      for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int i = 0; i < 16; ++i)
          Hs[(wr + mi * 32 + 8 * (i >> 2) + 4 * h + (i & 3)) * MB_HLD + hq(n)] = gelu_exact(acc[mi][ni][i] + bn);
    }
    __syncthreads();
    // y[m][p]: thread t < 4 MB_M sums units [64 (t & 3), +64) of row t / 4 in
    // a fixed order, then the four partial sums are added in a fixed order;
    // the 65-word quarter stride puts a wave's 16 rows x 4 quarters in 64
    // distinct banks, and W3 reads are broadcasts
    if (tid >= 4 * MB_M) return;  // whole waves
    const int row = tid >> 2, part = tid & 3;
    float yp[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) yp[p] = 0.f;
    for (int c = 0; c < 64; ++c) {
      const int q = part * 65 + c;
      const float hv = Hs[row * MB_HLD + q];
#pragma unroll
      for (int p = 0; p < 8; ++p)
        if (p < P) yp[p] = fmaf(hv, W3s[p * MB_HLD + q], yp[p]);
    }
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const float q1 = __shfl_down(yp[p], 1, 64);
      const float q2 = __shfl_down(yp[p], 2, 64);
      const float q3 = __shfl_down(yp[p], 3, 64);
      yp[p] = ((yp[p] + q1) + q2) + q3;
    }
    const int64_t m = m0 + row;
    if (part == 0 && m < B)
      for (int p = 0; p < P; ++p) Y[m * P + p] = yp[p] + b3[p];
  }
}

void launch_mlp_bf16(int64_t B, const float *X, int64_t ldx, int K, int Kx, const float *rowscale,
                     const uint16_t *W1b, const float *b1, uint16_t *H1, const uint16_t *W2b, const float *b2,
                     const float *W3, const float *b3, int P, float *Y, hipStream_t s) {
  if (B <= 0) return;
  constexpr int M1 = MRF_MLP_M1, M2 = MRF_MLP_M2;
#ifndef MRF_MLP_WR2
#define MRF_MLP_WR2 32
#endif
  constexpr int WR2 = MRF_MLP_WR2;  // rows per wave of the second layer (a tuning constant)
  constexpr int WR1 = MRF_MLP_WR1;  // rows per wave of the first layer (a tuning constant)
  hipLaunchKernelGGL((k_mlp_bf16<true, M1, WR1>), dim3((unsigned)((B + M1 - 1) / M1)), dim3(4 * M1 * (64 / WR1)), 0, s, B, X, ldx, K,
                     Kx, rowscale, nullptr, W1b, b1, H1, nullptr, nullptr, P, nullptr);
  hipLaunchKernelGGL((k_mlp_bf16<false, M2, WR2>), dim3((unsigned)((B + M2 - 1) / M2)), dim3(4 * M2 * (64 / WR2)), 0,
                     s, B, nullptr,
                     (int64_t)0, MB_H, MB_H, nullptr, H1, W2b, b2, nullptr, W3, b3, P, Y);
}

void launch_mlp_bf16_split(int64_t B, const uint16_t *Xs, int64_t ldxs, int Kx, const float *rowscale,
                           const uint16_t *W1b, const float *b1, uint16_t *H1, const uint16_t *W2b, const float *b2,
                           const float *W3, const float *b3, int P, float *Y, hipStream_t s) {
  if (B <= 0) return;
  constexpr int M1 = MRF_MLP_M1, M2 = MRF_MLP_M2, WR2 = MRF_MLP_WR2, WR1 = MRF_MLP_WR1;
  hipLaunchKernelGGL((k_mlp_bf16<true, M1, WR1, true>), dim3((unsigned)((B + M1 - 1) / M1)), dim3(4 * M1 * (64 / WR1)), 0, s, B,
                     nullptr, ldxs, Kx, Kx, rowscale, Xs, W1b, b1, H1, nullptr, nullptr, P, nullptr);
  hipLaunchKernelGGL((k_mlp_bf16<false, M2, WR2>), dim3((unsigned)((B + M2 - 1) / M2)), dim3(4 * M2 * (64 / WR2)), 0,
                     s, B, nullptr,
                     (int64_t)0, MB_H, MB_H, nullptr, H1, W2b, b2, nullptr, W3, b3, P, Y);
}

}  // namespace mrf
