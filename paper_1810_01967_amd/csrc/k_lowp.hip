// Reduced-precision row encoders for gfx950: BF16 (round to nearest even) and
// FP8-E4M3 with a per-row scale, plus the FP64 norms of each encoded row and
// of its rounding error (the terms of the exactness certificate's bound).
// The matrix-core scoring of the encoded rows is in k_score_mx.hip.
#include "mrf_internal.h"

namespace mrf {

// ---------------------------------------------------------------------------
// encoders
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// E4M3 (OCP, no infinities): round to nearest even, saturate to +-448, NaN -> 0x7F.
__device__ __forceinline__ uint8_t e4m3_rne(float q) {
  const uint32_t u = __float_as_uint(q);
  const uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
  const float a = fabsf(q);
  if (a != a) return 0x7F;
  if (a >= 448.f) return (uint8_t)(sign | 0x7E);
  if (a < 0.015625f) {  // below 2^-6: subnormal quantum 2^-9 (m = 8 is the smallest normal)
    const int m = (int)rintf(a * 512.f);
    return (uint8_t)(sign | m);
  }
  int e = (int)((u >> 23) & 0xFF) - 127;   // -6..8
  float r = rintf(ldexpf(a, 3 - e));       // 8..16, exact scaling then RNE
  if (r >= 16.f) {
    r = 8.f;
    ++e;
  }
  return (uint8_t)(sign | ((e + 7) << 3) | ((int)r - 8));
}

__device__ __forceinline__ double e4m3_to_double(uint8_t c) {
  const int e = (c >> 3) & 0xF, m = c & 7;
  const double mag = e == 0 ? ldexp((double)m, -9) : ldexp((double)(8 + m), e - 10);
  return (c & 0x80) ? -mag : mag;
}

// ||q||^2 and ||x - q||^2 of one row in FP64 (q the decoded value), reduced
// over the block in a fixed order; thread 0 writes their square roots.
__device__ __forceinline__ void row_norms(double q2, double e2, double *red, double2 *out) {
  red[threadIdx.x] = q2;
  red[256 + threadIdx.x] = e2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[threadIdx.x] += red[threadIdx.x + o];
      red[256 + threadIdx.x] += red[256 + threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = make_double2(sqrt(red[0]), sqrt(red[256]));
}

// One block per row; FP8 rows first reduce amax for the scale.  norms
// (optional): per row (||q||, ||x - q||) of the decoded row q (FP8: scale *
// E4M3 value), for the error bound of the reduced-precision scores.
__global__ __launch_bounds__(256) void k_quantize_rows(const float *__restrict__ in, int64_t rows,
                                                       int K, int64_t in_pitch, int fp8,
                                                       void *__restrict__ out, int64_t out_pitch,
                                                       float *__restrict__ scales, double2 *__restrict__ norms) {
  __shared__ float red[256];
  __shared__ double dred[512];
  const int64_t r = blockIdx.x;
  if (r >= rows) return;
  const float *x = in + r * in_pitch;
  if (!fp8) {
    uint16_t *o = static_cast<uint16_t *>(out) + r * out_pitch;
    double q2 = 0.0, e2 = 0.0;
    for (int64_t k = threadIdx.x; k < out_pitch; k += 256) {
      const uint16_t c = k < K ? bf16_rne(x[k]) : 0;
      o[k] = c;
      if (norms && k < K) {
        const double q = (double)__uint_as_float((uint32_t)c << 16), e = (double)x[k] - q;
        q2 += q * q;
        e2 += e * e;
      }
    }
    if (norms) row_norms(q2, e2, dred, norms + r);
    return;
  }
  float m = 0.f;
  for (int k = threadIdx.x; k < K; k += 256) m = fmaxf(m, fabsf(x[k]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  const float amax = red[0];
  const float sc = amax > 0.f ? __fdiv_rn(amax, 448.f) : 1.f;
  if (threadIdx.x == 0) scales[r] = sc;
  uint8_t *o = static_cast<uint8_t *>(out) + r * out_pitch;
  double q2 = 0.0, e2 = 0.0;
  for (int64_t k = threadIdx.x; k < out_pitch; k += 256) {
    const uint8_t c = k < K ? e4m3_rne(__fdiv_rn(x[k], sc)) : (uint8_t)0;
    o[k] = c;
    if (norms && k < K) {
      const double q = (double)sc * e4m3_to_double(c), e = (double)x[k] - q;
      q2 += q * q;
      e2 += e * e;
    }
  }
  if (norms) row_norms(q2, e2, dred, norms + r);
}

void launch_quantize_rows(const float *in, int64_t rows, int K, int64_t in_pitch, int precision,
                          void *out, int64_t out_pitch, float *scales, hipStream_t s, double2 *norms) {
  hipLaunchKernelGGL(k_quantize_rows, dim3((unsigned)rows), dim3(256), 0, s, in, rows, K, in_pitch,
                     precision == MRF_FP8 ? 1 : 0, out, out_pitch, scales, norms);
}

}  // namespace mrf
