// Exhaustive matched filter in split BF16 on gfx950: scores
// s_vj = <Z_v, Dhat_j> ~ hi.hi + hi.lo + lo.hi (v_mfma_f32_32x32x16_bf16,
// FP32 accumulation) with the per-voxel argmax fused in the epilogue (lowest
// index among equal scores).  Operand rows are the split rows of k_split_x3:
// Kx/32 chunks [hi 32 | lo 32].
//
// Block tile: 256 atoms x X_BV voxels (X_BV = 128 or 256), X_WAVES waves in a
// X_WAVES/2 x 2 arrangement, each owning 256/(X_WAVES/2) atoms x X_BV/2 voxels as MFMA tiles
// (atoms are the A rows, voxels the B columns, so a lane folds the running
// maximum of one voxel column per tile).
// One 32-element chunk per stage, double-buffered in LDS (rows of 72 BF16:
// the chunk plus 8 of padding).
#include "k_split.h"
#include "k_topk.h"
#include "mrf_internal.h"

namespace mrf {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

#ifndef MRF_X3_LD
#define MRF_X3_LD 72
#endif
constexpr int X_BA = 256, X_BV = kX3VoxTile, X_LD = MRF_X3_LD;  // LDS row pitch in BF16 (a tuning constant)
constexpr int X_NV = X_BV / 64;  // 32-voxel tiles per wave
// waves per block (8 or 16, a tuning constant) in X_WAVES / 2 atom-row groups x
// 2 voxel-column groups
#ifndef MRF_X3_WAVES
#define MRF_X3_WAVES 16
#endif
constexpr int X_WAVES = MRF_X3_WAVES, X_NT = 64 * X_WAVES;
constexpr int X_WA = X_WAVES / 2;            // atom-row groups
constexpr int X_AROWS = X_BA / X_WA;         // atom rows per wave
constexpr int X_MA = X_AROWS / 32;           // 32-atom tiles per wave
constexpr int X_LSTEP = X_NT / 8;            // rows per loader pass (8 pieces of 16 B per row)
constexpr int X_LA = X_BA / X_LSTEP, X_LZ = X_BV / X_LSTEP;
static_assert(X_MA >= 1 && X_LA >= 1 && X_LZ >= 1, "block shape");
constexpr int X_STAGE = (X_BA + X_BV) * X_LD;  // BF16 elements per stage buffer

__device__ __forceinline__ bool xbetter(float s1, int j1, float s0, int j0) {
  return (s1 > s0) || (s1 == s0 && j1 >= 0 && (j0 < 0 || j1 < j0));
}

// MODE SC_TOP1: per-voxel argmax per atom split; SC_TOPK: the kCertK best
// (score, atom) pairs per atom split [splits][pstride][kCertK] among the atoms
// within cw ||Z_v|| + wabs of the running maximum when scored; SC_COLLECT:
// every atom whose score reaches the voxel's line thr[i] appended to
// cand[i][0..ccap) (count[i] counts them all), voxel rows through rowmap.
struct CollectX3 {
  const int32_t *rowmap;
  const float *thr;
  unsigned int *count;
  int32_t *cand;
  int ccap;
};

template <int MODE>
__global__ __launch_bounds__(X_NT, 1) void k_score_x3(const uint16_t *__restrict__ Dx, const uint16_t *__restrict__ Zx,
                                                     int d, int ntiles_total, int64_t n, int nvt, int Kx,
                                                     int splits, int tiles_per_split, float *__restrict__ part_s,
                                                     int *__restrict__ part_j, const unsigned int *__restrict__ dcnt,
                                                     int64_t pstride, const float *__restrict__ znorm, float cw,
                                                     float wabs, CollectX3 col) {
  // Work item w -> (voxel tile, atom split); all splits of a voxel tile on one
  // XCD (item w on XCD w % 8).  Launched by the host (dcnt null): one item per
  // block, n voxels.  With the voxel count on the device (dcnt): n is only the
  // capacity, the tiles and splits follow from the count, and a grid of a
  // multiple of 8 blocks loops over the items (block b keeps XCD b % 8).
  int64_t nvox = n;
  int nvt_w = nvt, nsplit = splits, tps = tiles_per_split;
  if (dcnt) {
    nvox = min(n, (int64_t)*dcnt);
    nvt_w = (int)((nvox + X_BV - 1) / X_BV);
    // a rescan spreads its few voxel tiles over more splits (about 2,048
    // items); the fallback's split count is the one its merge recomputes
    nsplit = MODE == SC_COLLECT ? max(1, min(ntiles_total, min(256, (2048 + (nvt_w + 7) / 8 * 8 - 1) /
                                                                        max(8, (nvt_w + 7) / 8 * 8))))
                                : x3_device_splits(nvt_w, ntiles_total);
    tps = (ntiles_total + nsplit - 1) / nsplit;
  }
  const int64_t nwork = (int64_t)((nvt_w + 7) / 8 * 8) * nsplit;

  __shared__ __attribute__((aligned(16))) uint16_t S[2 * X_STAGE];
  __shared__ float rs[X_WA][X_BV];
  __shared__ int rj[X_WA][X_BV];
  // SC_TOPK: the waves' lists [X_WA][kCertK][X_BV] go through the stage buffers
  static_assert(X_WA * kCertK * X_BV * 8 <= 2 * X_STAGE * 2, "LDS exchange of the candidate lists");

  for (int64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int xcd = (int)(w & 7);
    const int64_t local = w >> 3;
    const int split = (int)(local % nsplit);
    const int vt = (int)((local / nsplit) * 8 + xcd);
    if (vt >= nvt_w) continue;
    const int tb = split * tps;
    const int te = min(tb + tps, ntiles_total);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wa = wave >> 1, wv = wave & 1;  // atom rows wa*X_AROWS.., voxel columns wv*X_BV/2..
    const int h = lane >> 5, l32 = lane & 31;
    const int64_t v0 = (int64_t)vt * X_BV;
    const int nkc = Kx / 32;
    const int nq = te > tb ? (te - tb) * nkc : 0;
    const int64_t row = 2 * (int64_t)Kx;  // elements per split row

    // loader: 8 pieces of 16 B per stage row; piece = tid % 8, rows tid/8 + X_LSTEP i
    const int lr = tid >> 3, piece = tid & 7;
    const int lc = (piece >> 2) * 32 + (piece & 3) * 8;  // column within [hi 32 | lo 32]
    uint4 ra[X_LA], rz[X_LZ];
    // voxel rows of this thread's loader rows (through the row map in
    // SC_COLLECT; rows past the count read the first listed row, unused)
    const uint16_t *zrow[X_LZ];
    #pragma unroll
    for (int i = 0; i < X_LZ; ++i) {
      int64_t r = v0 + lr + X_LSTEP * i;
      if (MODE == SC_COLLECT) r = col.rowmap[r < nvox ? r : 0];
      zrow[i] = Zx + r * row + lc;
    }
    auto gload = [&](int q) {
      const int tile = tb + q / nkc, kc = q - (q / nkc) * nkc;
      const uint16_t *a = Dx + (int64_t)(tile * X_BA + lr) * row + kc * 64 + lc;
      #pragma unroll
      for (int i = 0; i < X_LA; ++i) ra[i] = *reinterpret_cast<const uint4 *>(a + (int64_t)(X_LSTEP * i) * row);
      #pragma unroll
      for (int i = 0; i < X_LZ; ++i) rz[i] = *reinterpret_cast<const uint4 *>(zrow[i] + kc * 64);
    };
    auto sstore = [&](int buf) {
      uint16_t *B = S + buf * X_STAGE;
      #pragma unroll
      for (int i = 0; i < X_LA; ++i) *reinterpret_cast<uint4 *>(B + (lr + X_LSTEP * i) * X_LD + lc) = ra[i];
      #pragma unroll
      for (int i = 0; i < X_LZ; ++i)
        *reinterpret_cast<uint4 *>(B + (X_BA + lr + X_LSTEP * i) * X_LD + lc) = rz[i];
    };

    f32x16 acc[X_MA][X_NV];
    #pragma unroll
    for (int a = 0; a < X_MA; ++a)
      #pragma unroll
      for (int b = 0; b < X_NV; ++b)
        #pragma unroll
        for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;
    float best[X_NV];
    int bidx[X_NV];
    float ls[X_NV][kCertK];
    int lj[X_NV][kCertK];
    float vthr[X_NV], win[X_NV];  // SC_TOPK: insertion bar and window; SC_COLLECT: the line
    #pragma unroll
    for (int b = 0; b < X_NV; ++b) {
      best[b] = -INFINITY;
      bidx[b] = -1;
      vthr[b] = MODE == SC_TOPK ? -INFINITY : INFINITY;
      win[b] = 0.f;
      const int64_t v = v0 + wv * (X_BV / 2) + b * 32 + l32;
      if (MODE == SC_TOPK) {
        topk_clear(ls[b], lj[b]);
        if (v < nvox) win[b] = cw * fmaxf(znorm[v], 0.f) + wabs;
      }
      if (MODE == SC_COLLECT && v < nvox) vthr[b] = col.thr[v];
    }

    if (nq > 0) {
      gload(0);
      sstore(0);
    }
    __syncthreads();
    for (int q = 0; q < nq; ++q) {
      const int buf = q & 1;
      if (q + 1 < nq) gload(q + 1);
      const __bf16 *B = reinterpret_cast<const __bf16 *>(S) + buf * X_STAGE;
      #pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        bf16x8 ahi[X_MA], alo[X_MA], zhi[X_NV], zlo[X_NV];
        #pragma unroll
        for (int ma = 0; ma < X_MA; ++ma) {
          const __bf16 *p = B + (wa * X_AROWS + ma * 32 + l32) * X_LD + ks * 16 + h * 8;
          ahi[ma] = *reinterpret_cast<const bf16x8 *>(p);
          alo[ma] = *reinterpret_cast<const bf16x8 *>(p + 32);
        }
        #pragma unroll
        for (int nv = 0; nv < X_NV; ++nv) {
          const __bf16 *p = B + (X_BA + wv * (X_BV / 2) + nv * 32 + l32) * X_LD + ks * 16 + h * 8;
          zhi[nv] = *reinterpret_cast<const bf16x8 *>(p);
          zlo[nv] = *reinterpret_cast<const bf16x8 *>(p + 32);
        }
        #pragma unroll
        for (int ma = 0; ma < X_MA; ++ma)
          #pragma unroll
          for (int nv = 0; nv < X_NV; ++nv) {
            acc[ma][nv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[ma], zhi[nv], acc[ma][nv], 0, 0, 0);
            acc[ma][nv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi[ma], zlo[nv], acc[ma][nv], 0, 0, 0);
            acc[ma][nv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo[ma], zhi[nv], acc[ma][nv], 0, 0, 0);
          }
      }
      const int kc = q % nkc;
      if (kc == nkc - 1) {
        // fold this atom tile: 32 atom rows per voxel column and tile
        const int abase = (tb + q / nkc) * X_BA + wa * X_AROWS;
        #pragma unroll
        for (int nv = 0; nv < X_NV; ++nv)
          #pragma unroll
          for (int ma = 0; ma < X_MA; ++ma)
            #pragma unroll
            for (int i = 0; i < 16; ++i) {
              const int j = abase + ma * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
              const float sc = acc[ma][nv][i];
              if (MODE == SC_TOPK) {
                if (j < d && sc > vthr[nv]) {
                  topk_push_ordered(ls[nv], lj[nv], sc, j);
                  vthr[nv] = fmaxf(ls[nv][kCertK - 1], ls[nv][0] - win[nv]);
                }
              } else if (MODE == SC_COLLECT) {
                const int64_t v = v0 + wv * (X_BV / 2) + nv * 32 + l32;
                if (j < d && v < nvox && sc >= vthr[nv]) {
                  const unsigned int pos = atomicAdd(&col.count[v], 1u);
                  if ((int)pos < col.ccap) col.cand[v * col.ccap + pos] = j;
                }
              } else if (j < d && sc > best[nv]) {  // atoms in increasing order: '>' keeps the lowest index
                best[nv] = sc;
                bidx[nv] = j;
              }
            }
        #pragma unroll
        for (int a = 0; a < X_MA; ++a)
          #pragma unroll
          for (int b = 0; b < X_NV; ++b)
            #pragma unroll
            for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;
      }
      if (q + 1 < nq) sstore(buf ^ 1);
      __syncthreads();
    }
    if (MODE == SC_COLLECT) continue;  // the candidates are already written
    if (MODE == SC_TOPK) {
      // the two half-waves, then the X_WA atom-row waves' lists through LDS
      float *ps = reinterpret_cast<float *>(S);
      int *pj = reinterpret_cast<int *>(S) + X_WA * kCertK * X_BV;
      #pragma unroll
      for (int nv = 0; nv < X_NV; ++nv) {
        topk_merge_xor(ls[nv], lj[nv], 32);
        if (h == 0) {
          const int c = wv * (X_BV / 2) + nv * 32 + l32;
          #pragma unroll
          for (int i = 0; i < kCertK; ++i) {
            ps[(wa * kCertK + i) * X_BV + c] = ls[nv][i];
            pj[(wa * kCertK + i) * X_BV + c] = lj[nv][i];
          }
        }
      }
      __syncthreads();
      if (tid < X_BV) {
        float ms[kCertK];
        int mj[kCertK];
        #pragma unroll
        for (int i = 0; i < kCertK; ++i) {
          ms[i] = ps[i * X_BV + tid];
          mj[i] = pj[i * X_BV + tid];
        }
        for (int w = 1; w < X_WA; ++w)
          #pragma unroll
          for (int i = 0; i < kCertK; ++i) topk_push(ms, mj, ps[(w * kCertK + i) * X_BV + tid], pj[(w * kCertK + i) * X_BV + tid]);
        const int64_t v = v0 + tid;
        if (v < nvox) {
          float *os = part_s + ((int64_t)split * pstride + v) * kCertK;
          int *oj = part_j + ((int64_t)split * pstride + v) * kCertK;
          #pragma unroll
          for (int i = 0; i < kCertK; ++i) {
            os[i] = ms[i];
            oj[i] = mj[i];
          }
        }
      }
      __syncthreads();  // the next item reuses the LDS buffers
      continue;
    }
    // the two half-waves, then the X_WA atom-row waves of each voxel column
    #pragma unroll
    for (int nv = 0; nv < X_NV; ++nv) {
      const float ps = __shfl_xor(best[nv], 32, 64);
      const int pj = __shfl_xor(bidx[nv], 32, 64);
      if (xbetter(ps, pj, best[nv], bidx[nv])) {
        best[nv] = ps;
        bidx[nv] = pj;
      }
      if (h == 0) {
        rs[wa][wv * (X_BV / 2) + nv * 32 + l32] = best[nv];
        rj[wa][wv * (X_BV / 2) + nv * 32 + l32] = bidx[nv];
      }
    }
    __syncthreads();
    if (tid < X_BV) {
      float bs = rs[0][tid];
      int bj = rj[0][tid];
      for (int w = 1; w < X_WA; ++w)
        if (xbetter(rs[w][tid], rj[w][tid], bs, bj)) {
          bs = rs[w][tid];
          bj = rj[w][tid];
        }
      const int64_t v = v0 + tid;
      if (v < nvox) {
        part_s[(int64_t)split * pstride + v] = bs;
        part_j[(int64_t)split * pstride + v] = bj;
      }
    }
    __syncthreads();  // the next item reuses the LDS buffers and the reduction arrays
  }
}

// Dx: split atoms [d_pad][2 Kx] (d_pad a multiple of 256); Zx: split voxels
// [n_pad][2 Kx] (n_pad a multiple of X_BV, zero rows beyond n).
void launch_score_x3(const uint16_t *Dx, const uint16_t *Zx, int d, int64_t d_pad, int64_t n, int64_t n_pad,
                     int Kx, int splits, float *part_s, int *part_j, hipStream_t s, bool topk, const float *znorm,
                     float cw, float wabs) {
  const int ntiles = (int)(d_pad / X_BA);
  const int nvt = (int)(n_pad / X_BV);
  const int tps = (ntiles + splits - 1) / splits;
  const int64_t nvt8 = (nvt + 7) / 8 * 8;
  const int64_t blocks = nvt8 * splits;
  if (topk)
    hipLaunchKernelGGL(k_score_x3<SC_TOPK>, dim3((unsigned)blocks), dim3(X_NT), 0, s, Dx, Zx, d, ntiles, n, nvt, Kx,
                       splits, tps, part_s, part_j, nullptr, n, znorm, cw, wabs, CollectX3{});
  else
    hipLaunchKernelGGL(k_score_x3<SC_TOP1>, dim3((unsigned)blocks), dim3(X_NT), 0, s, Dx, Zx, d, ntiles, n, nvt, Kx,
                       splits, tps, part_s, part_j, nullptr, n, nullptr, 0.f, 0.f, CollectX3{});
}

void launch_score_x3_dev(const uint16_t *Dx, const uint16_t *Zx, int d, int64_t d_pad, int64_t cap,
                         const unsigned int *dcnt, int Kx, float *part_s, int *part_j, hipStream_t s) {
  if (cap <= 0) return;
  const int ntiles = (int)(d_pad / X_BA);
  // one block per CU of the 256, each looping over the work items
  hipLaunchKernelGGL(k_score_x3<SC_TOP1>, dim3(256), dim3(X_NT), 0, s, Dx, Zx, d, ntiles, cap, 0, Kx, 1, ntiles,
                     part_s, part_j, dcnt, cap, nullptr, 0.f, 0.f, CollectX3{});
}

void launch_collect_x3_dev(const uint16_t *Dx, const uint16_t *Zx, const int32_t *rows, int d, int64_t d_pad,
                           int64_t cap, const unsigned int *dcnt, int Kx, const float *thr, unsigned int *count,
                           int32_t *cand, int ccap, hipStream_t s) {
  if (cap <= 0) return;
  const int ntiles = (int)(d_pad / X_BA);
  hipLaunchKernelGGL(k_score_x3<SC_COLLECT>, dim3(256), dim3(X_NT), 0, s, Dx, Zx, d, ntiles, cap, 0, Kx, 1, ntiles,
                     nullptr, nullptr, dcnt, cap, nullptr, 0.f, 0.f, CollectX3{rows, thr, count, cand, ccap});
}

}  // namespace mrf
