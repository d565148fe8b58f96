// Reduced-precision matched filter for gfx950: BF16 / FP8-E4M3 row encoders
// and scoring on MFMA (v_mfma_f32_32x32x16_bf16,
// v_mfma_scale_f32_32x32x64_f8f6f4) with FP32 accumulation.  The scoring
// kernel's epilogues: the per-voxel maximum, or every atom at or above a
// per-voxel line (the candidates the exactness certificate rescores).
#include "k_topk.h"
#include "mrf_internal.h"

namespace mrf {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
// staging registers are native vectors: a struct type (uint4) is copied
// through private memory, which serialises every load on its own wait
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

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

// ---------------------------------------------------------------------------
// scoring
// ---------------------------------------------------------------------------
// Block tile 128 atoms x 128 voxels; K chunks of 128 bytes per row (64 BF16
// or 128 FP8 values) double-buffered in LDS; four waves 2 x 2, each with
// 2 x 2 MFMA 32x32 tiles (atoms = rows, voxels = columns, as in the FP32
// kernel), so a lane folds one voxel column per tile.  FP8 scores are the
// E4M3 products times the atom's scale (the voxel's scale, common to all its
// scores, is left out: lines are given in the same unit).
// MODE SC_TOP1: per split and voxel the best (score, atom), lowest atom on
// equal scores; SC_COLLECT: every atom with score >= thr[v] appended to
// cand[v][0..ccap) (count[v] counts them all).
constexpr int Q_BA = 128, Q_BV = 128, Q_CB = 128, Q_LDB = 144;  // bytes per LDS row

struct LowpCollect {
  const float *thr;
  unsigned int *count;
  int32_t *cand;
  int ccap;
};

template <bool FP8, int MODE>
__global__ __launch_bounds__(256, 2) void k_score_lowp(const uint8_t *__restrict__ Dq,
                                                       const float *__restrict__ dscale,
                                                       const uint8_t *__restrict__ Zq, int d,
                                                       int ntiles_total, int64_t n, int nvt,
                                                       int row_bytes, int splits,
                                                       int tiles_per_split,
                                                       float *__restrict__ part_s,
                                                       int *__restrict__ part_j, LowpCollect col) {
  const int bid = blockIdx.x;
  const int xcd = bid & 7, local = bid >> 3;
  const int split = local % splits;
  const int vt = (local / splits) * 8 + xcd;
  if (vt >= nvt) return;
  const int tb = split * tiles_per_split;
  const int te = min(tb + tiles_per_split, ntiles_total);

  __shared__ __attribute__((aligned(16))) uint8_t As[2][Q_BA * Q_LDB];
  __shared__ __attribute__((aligned(16))) uint8_t Zs[2][Q_BV * Q_LDB];
  __shared__ float tscale[2][Q_BA];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wa = wave >> 1, wv = wave & 1;
  const int h = lane >> 5, l32 = lane & 31;
  const int64_t v0 = (int64_t)vt * Q_BV;
  const int nkc = row_bytes / Q_CB;
  const int nq = te > tb ? (te - tb) * nkc : 0;

  // global -> LDS: 128 rows x 128 bytes per operand = 1024 x 16 B, 4 per thread
  const int lr = tid >> 3, lc = (tid & 7) * 16;
  u32x4 ra[4], rz[4];
  auto gload = [&](int q) {
    const int tile = tb + q / nkc, kc = q - (q / nkc) * nkc;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ra[i] = *reinterpret_cast<const u32x4 *>(Dq + (int64_t)(tile * Q_BA + lr + 32 * i) * row_bytes +
                                               kc * Q_CB + lc);
      rz[i] = *reinterpret_cast<const u32x4 *>(Zq + (v0 + lr + 32 * i) * row_bytes + kc * Q_CB + lc);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      *reinterpret_cast<u32x4 *>(&As[buf][(lr + 32 * i) * Q_LDB + lc]) = ra[i];
      *reinterpret_cast<u32x4 *>(&Zs[buf][(lr + 32 * i) * Q_LDB + lc]) = rz[i];
    }
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;
  float best[2] = {-INFINITY, -INFINITY};
  int bidx[2] = {-1, -1};
  float vthr[2] = {INFINITY, INFINITY};
  if (MODE == SC_COLLECT) {
#pragma unroll
    for (int nv = 0; nv < 2; ++nv) {
      const int64_t v = v0 + wv * 64 + nv * 32 + l32;
      if (v < n) vthr[nv] = col.thr[v];
    }
  }

  if (nq > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  for (int q = 0; q < nq; ++q) {
    const int buf = q & 1;
    const int kc = q % nkc;
    if (FP8 && kc == 0) {  // the tile's atom scales, double-buffered by tile parity
      const int tile = tb + q / nkc;
      if (tid < Q_BA) tscale[tile & 1][tid] = dscale[tile * Q_BA + tid];
    }
    if (q + 1 < nq) gload(q + 1);
    if (FP8) {
      // two k-steps of 64: lane supplies 32 bytes (k = h*32 .. h*32+31 of the step)
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        i32x8 af[2], zf[2];
#pragma unroll
        for (int ma = 0; ma < 2; ++ma) {
          const uint8_t *src = &As[buf][(wa * 64 + ma * 32 + l32) * Q_LDB + ks * 64 + h * 32];
          const u32x4 x0 = *reinterpret_cast<const u32x4 *>(src);
          const u32x4 x1 = *reinterpret_cast<const u32x4 *>(src + 16);
          af[ma] = i32x8{(int)x0.x, (int)x0.y, (int)x0.z, (int)x0.w,
                         (int)x1.x, (int)x1.y, (int)x1.z, (int)x1.w};
        }
#pragma unroll
        for (int nv = 0; nv < 2; ++nv) {
          const uint8_t *src = &Zs[buf][(wv * 64 + nv * 32 + l32) * Q_LDB + ks * 64 + h * 32];
          const u32x4 x0 = *reinterpret_cast<const u32x4 *>(src);
          const u32x4 x1 = *reinterpret_cast<const u32x4 *>(src + 16);
          zf[nv] = i32x8{(int)x0.x, (int)x0.y, (int)x0.z, (int)x0.w,
                         (int)x1.x, (int)x1.y, (int)x1.z, (int)x1.w};
        }
#pragma unroll
        for (int ma = 0; ma < 2; ++ma)
#pragma unroll
          for (int nv = 0; nv < 2; ++nv)
            acc[ma][nv] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                af[ma], zf[nv], acc[ma][nv], 0, 0, 0, 0x7F, 0, 0x7F);
      }
    } else {
      // four k-steps of 16: lane supplies 8 BF16 (k = h*8 .. h*8+7 of the step)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        bf16x8 af[2], zf[2];
#pragma unroll
        for (int ma = 0; ma < 2; ++ma)
          af[ma] = *reinterpret_cast<const bf16x8 *>(
              &As[buf][(wa * 64 + ma * 32 + l32) * Q_LDB + ks * 32 + h * 16]);
#pragma unroll
        for (int nv = 0; nv < 2; ++nv)
          zf[nv] = *reinterpret_cast<const bf16x8 *>(
              &Zs[buf][(wv * 64 + nv * 32 + l32) * Q_LDB + ks * 32 + h * 16]);
#pragma unroll
        for (int ma = 0; ma < 2; ++ma)
#pragma unroll
          for (int nv = 0; nv < 2; ++nv)
            acc[ma][nv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[ma], zf[nv], acc[ma][nv], 0, 0, 0);
      }
    }
    if (kc == nkc - 1) {
      if (FP8 && nkc == 1) __syncthreads();  // the scales written above, this same step
      const int tile = tb + q / nkc;
      const int abase = tile * Q_BA + wa * 64;
#pragma unroll
      for (int nv = 0; nv < 2; ++nv) {
        const int64_t v = v0 + wv * 64 + nv * 32 + l32;
#pragma unroll
        for (int ma = 0; ma < 2; ++ma) {
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int m = wa * 64 + ma * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
            const int j = abase + ma * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
            float sc = acc[ma][nv][i];
            if (FP8) sc *= tscale[tile & 1][m];
            if (MODE == SC_TOP1) {
              if (j < d && sc > best[nv]) {  // atoms in increasing order: '>' keeps the lowest index
                best[nv] = sc;
                bidx[nv] = j;
              }
            } else if (j < d && v < n && sc >= vthr[nv]) {
              const unsigned int pos = atomicAdd(&col.count[v], 1u);
              if ((int)pos < col.ccap) col.cand[v * col.ccap + pos] = j;
            }
          }
        }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;
    }
    if (q + 1 < nq) sstore(buf ^ 1);
    __syncthreads();
  }
  if (MODE == SC_COLLECT) return;

  // the half-waves, then the two atom halves of the block through LDS
#pragma unroll
  for (int nv = 0; nv < 2; ++nv) {
    const float ps = __shfl_xor(best[nv], 32, 64);
    const int pj = __shfl_xor(bidx[nv], 32, 64);
    if (rank_before(ps, pj, best[nv], bidx[nv])) {
      best[nv] = ps;
      bidx[nv] = pj;
    }
  }
  float *rs = reinterpret_cast<float *>(&As[0][0]);
  int *rj = reinterpret_cast<int *>(&Zs[0][0]);
  if (wa == 1 && h == 0) {
#pragma unroll
    for (int nv = 0; nv < 2; ++nv) {
      rs[wv * 64 + nv * 32 + l32] = best[nv];
      rj[wv * 64 + nv * 32 + l32] = bidx[nv];
    }
  }
  __syncthreads();
  if (wa == 0 && h == 0) {
#pragma unroll
    for (int nv = 0; nv < 2; ++nv) {
      const int c = wv * 64 + nv * 32 + l32;
      if (rank_before(rs[c], rj[c], best[nv], bidx[nv])) {
        best[nv] = rs[c];
        bidx[nv] = rj[c];
      }
      const int64_t v = v0 + c;
      if (v < n) {
        part_s[(int64_t)split * n + v] = best[nv];
        part_j[(int64_t)split * n + v] = bidx[nv];
      }
    }
  }
}

template <int MODE>
void launch_lowp(int precision, const void *Dq, const float *dscale, const void *Zq, int d, int64_t d_pad, int64_t n,
                 int Kq, int splits, float *part_s, int *part_j, LowpCollect col, hipStream_t s) {
  const int ntiles = (int)(d_pad / Q_BA);
  const int nvt = (int)((n + Q_BV - 1) / Q_BV);
  const int tiles_per_split = (ntiles + splits - 1) / splits;
  const int nvt8 = (nvt + 7) / 8 * 8;
  const int64_t blocks = (int64_t)nvt8 * splits;
  if (blocks <= 0) return;
  const bool fp8 = precision == MRF_FP8;
  const int row_bytes = fp8 ? Kq : 2 * Kq;
  if (fp8)
    hipLaunchKernelGGL((k_score_lowp<true, MODE>), dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const uint8_t *>(Dq), dscale, static_cast<const uint8_t *>(Zq), d, ntiles, n, nvt,
                       row_bytes, splits, tiles_per_split, part_s, part_j, col);
  else
    hipLaunchKernelGGL((k_score_lowp<false, MODE>), dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const uint8_t *>(Dq), nullptr, static_cast<const uint8_t *>(Zq), d, ntiles, n, nvt,
                       row_bytes, splits, tiles_per_split, part_s, part_j, col);
}

void launch_score_lowp(int precision, const void *Dq, const float *dscale, const void *Zq, int d, int64_t d_pad,
                       int64_t n, int Kq, int splits, float *part_s, int *part_j, hipStream_t s) {
  launch_lowp<SC_TOP1>(precision, Dq, dscale, Zq, d, d_pad, n, Kq, splits, part_s, part_j, LowpCollect{}, s);
}

void launch_collect_lowp(int precision, const void *Dq, const float *dscale, const void *Zq, int d, int64_t d_pad,
                         int64_t n, int Kq, int splits, const float *thr, unsigned int *count, int32_t *cand, int ccap,
                         hipStream_t s) {
  launch_lowp<SC_COLLECT>(precision, Dq, dscale, Zq, d, d_pad, n, Kq, splits, nullptr, nullptr,
                          LowpCollect{thr, count, cand, ccap}, s);
}

}  // namespace mrf
