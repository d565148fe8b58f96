// Exhaustive matched-filter scoring of BF16 rows on the matrix cores of gfx950
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation) with the per-voxel epilogues
// of the reduced-precision filter fused (eq. exactP): the maximum, or every
// atom at or above a per-voxel line.
//
// Block tile: 256 atoms x 256 voxels, MRF_MX_WA x MRF_MX_WV waves, each
// owning a (256 / WA) x (256 / WV) sub-tile of MFMA 32x32 tiles (atoms are the
// A rows, voxels the B columns, so a lane folds one voxel column per tile and
// atoms reach it in increasing order).  Every stage is 128 bytes (64 BF16) of
// each of the 512 rows, double-buffered in LDS with a 144-byte pitch.  Work items are
// (voxel tile, atom split) pairs; the splits of a voxel tile run on one XCD
// (item w on XCD w % 8), so its blocks share the voxel tile and, across the
// voxel tiles in flight, the atom tiles through that XCD's L2.
#include "k_topk.h"
#include "mrf_internal.h"

namespace mrf {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
// staging registers are native vectors: a struct type (uint4) is copied
// through private memory, which serialises every load on its own wait
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// wave grid (atom-row groups x voxel-column groups; tuning constants)
// (4 x 4 = 16 waves of 64 x 64 measured best: 31.8 ms per 65,536 x 100,800 x
// 1,000 against 33.1-33.7 ms for 2 x 4, 4 x 2 and 8 x 2)
#ifndef MRF_MX_WA
#define MRF_MX_WA 4
#endif
#ifndef MRF_MX_WV
#define MRF_MX_WV 4
#endif
constexpr int M_BA = 256, M_BV = 256;
constexpr int M_WA = MRF_MX_WA, M_WV = MRF_MX_WV, M_NT = 64 * M_WA * M_WV;
constexpr int M_LD = 72;                       // LDS row pitch in BF16 (128 bytes + 16 of padding)
constexpr int M_STAGE = (M_BA + M_BV) * M_LD;  // BF16 per stage buffer
constexpr int M_AROWS = M_BA / M_WA, M_VCOLS = M_BV / M_WV;  // per wave
constexpr int M_MA = M_AROWS / 32;             // 32-atom MFMA tiles per wave
constexpr int M_NV = M_VCOLS / 32;             // 32-voxel MFMA tiles per wave
constexpr int M_LROWS = M_NT / 8;              // rows per loader pass (8 pieces of 16 B per row)
constexpr int M_LA = M_BA / M_LROWS, M_LZ = M_BV / M_LROWS;
static_assert(M_MA >= 1 && M_NV >= 1 && M_LA >= 1 && M_LZ >= 1, "block shape");
static_assert(2 * M_STAGE * 2 <= 160 * 1024, "LDS");

}  // namespace

struct MxArgs {
  const uint16_t *D;       // atom rows, pitch `row` BF16 (d_pad rows, zero padded)
  const uint16_t *Z;       // voxel rows, same pitch (rows up to the voxel-tile multiple readable)
  int64_t row;             // row pitch in BF16
  int nstage;              // 128-byte stages per row
  int d, ntiles;           // atoms; 256-atom tiles
  int64_t n;               // voxels (device count: the capacity)
  int splits, tps;         // atom splits and 256-atom tiles per split
  float *part_s;           // SC_TOP1 [splits][pstride]
  int *part_j;
  int64_t pstride;
  const float *thr;        // SC_COLLECT: per-voxel line
  unsigned int *count;
  int32_t *cand;
  int ccap;
};

template <int MODE>
__global__ __launch_bounds__(M_NT, 1) void k_score_mx(MxArgs g) {
  const int64_t nvox = g.n;
  const int nsplit = g.splits, tps = g.tps;
  const int nvt = (int)((nvox + M_BV - 1) / M_BV);
  const int64_t nwork = (int64_t)((nvt + 7) / 8 * 8) * nsplit;

  __shared__ __attribute__((aligned(16))) uint16_t S[2 * M_STAGE];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wa = wave / M_WV, wv = wave % M_WV;
  const int h = lane >> 5, l32 = lane & 31;
  const int lr = tid >> 3, lc = (tid & 7) * 8;  // loader row, BF16 column of the 16-byte piece

  for (int64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int xcd = (int)(w & 7);
    const int64_t local = w >> 3;
    const int split = (int)(local % nsplit);
    const int vt = (int)((local / nsplit) * 8 + xcd);
    if (vt >= nvt) continue;
    const int tb = split * tps;
    const int te = min(tb + tps, g.ntiles);
    const int64_t v0 = (int64_t)vt * M_BV;
    const int nq = te > tb ? (te - tb) * g.nstage : 0;

    const uint16_t *zrow[M_LZ];
#pragma unroll
    for (int i = 0; i < M_LZ; ++i) {
      int64_t r = v0 + lr + M_LROWS * i;
      zrow[i] = g.Z + r * g.row + lc;
    }
    u32x4 ra[M_LA], rz[M_LZ];
    auto gload = [&](int q) {
      const int tile = tb + q / g.nstage, st = q - (q / g.nstage) * g.nstage;
      const uint16_t *a = g.D + (int64_t)(tile * M_BA + lr) * g.row + st * 64 + lc;
#pragma unroll
      for (int i = 0; i < M_LA; ++i) ra[i] = *reinterpret_cast<const u32x4 *>(a + (int64_t)(M_LROWS * i) * g.row);
#pragma unroll
      for (int i = 0; i < M_LZ; ++i) rz[i] = *reinterpret_cast<const u32x4 *>(zrow[i] + st * 64);
    };
    auto sstore = [&](int buf) {
      uint16_t *B = S + buf * M_STAGE;
#pragma unroll
      for (int i = 0; i < M_LA; ++i) *reinterpret_cast<u32x4 *>(B + (lr + M_LROWS * i) * M_LD + lc) = ra[i];
#pragma unroll
      for (int i = 0; i < M_LZ; ++i) *reinterpret_cast<u32x4 *>(B + (M_BA + lr + M_LROWS * i) * M_LD + lc) = rz[i];
    };

    f32x16 acc[M_MA][M_NV];
#pragma unroll
    for (int a = 0; a < M_MA; ++a)
#pragma unroll
      for (int b = 0; b < M_NV; ++b)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;
    float best[M_NV], vthr[M_NV];
    int bidx[M_NV];
#pragma unroll
    for (int b = 0; b < M_NV; ++b) {
      best[b] = -INFINITY;
      bidx[b] = -1;
      vthr[b] = INFINITY;
      const int64_t v = v0 + wv * M_VCOLS + b * 32 + l32;
      if (MODE == SC_COLLECT && v < nvox) vthr[b] = g.thr[v];
    }

    if (nq > 0) {
      gload(0);
      sstore(0);
    }
    __syncthreads();
    for (int q = 0; q < nq; ++q) {
      const int buf = q & 1;
      if (q + 1 < nq) gload(q + 1);
      const __bf16 *B = reinterpret_cast<const __bf16 *>(S) + buf * M_STAGE;
      const __bf16 *Ab = B + (wa * M_AROWS + l32) * M_LD + h * 8;
      const __bf16 *Zb = B + (M_BA + wv * M_VCOLS + l32) * M_LD + h * 8;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        bf16x8 zf[M_NV];
#pragma unroll
        for (int nv = 0; nv < M_NV; ++nv) zf[nv] = *reinterpret_cast<const bf16x8 *>(Zb + nv * 32 * M_LD + ks * 16);
#pragma unroll
        for (int ma = 0; ma < M_MA; ++ma) {
          const bf16x8 af = *reinterpret_cast<const bf16x8 *>(Ab + ma * 32 * M_LD + ks * 16);
#pragma unroll
          for (int nv = 0; nv < M_NV; ++nv)
            acc[ma][nv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, zf[nv], acc[ma][nv], 0, 0, 0);
        }
      }
      const int st = q % g.nstage;
      if (st == g.nstage - 1) {
        // fold this atom tile: 64 atom rows per voxel column and lane
        const int abase = (tb + q / g.nstage) * M_BA + wa * M_AROWS;
#pragma unroll
        for (int nv = 0; nv < M_NV; ++nv) {
          const int64_t v = v0 + wv * M_VCOLS + nv * 32 + l32;
#pragma unroll
          for (int ma = 0; ma < M_MA; ++ma)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
              const int j = abase + ma * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
              const float sc = acc[ma][nv][i];
              if (MODE == SC_TOP1) {
                if (j < g.d && sc > best[nv]) {  // atoms in increasing order: '>' keeps the lowest index
                  best[nv] = sc;
                  bidx[nv] = j;
                }
              } else if (j < g.d && v < nvox && sc >= vthr[nv]) {
                const unsigned int pos = atomicAdd(&g.count[v], 1u);
                if ((int)pos < g.ccap) g.cand[v * g.ccap + pos] = j;
              }
            }
        }
#pragma unroll
        for (int a = 0; a < M_MA; ++a)
#pragma unroll
          for (int b = 0; b < M_NV; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;
      }
      if (q + 1 < nq) sstore(buf ^ 1);
      __syncthreads();
    }
    if (MODE == SC_COLLECT) continue;  // the candidates are already written

    // the two half-waves, then the M_WA atom-row groups of the block through LDS
    {
      float *ps = reinterpret_cast<float *>(S);
      int *pj = reinterpret_cast<int *>(S) + M_WA * M_BV;
#pragma unroll
      for (int nv = 0; nv < M_NV; ++nv) {
        const float os = __shfl_xor(best[nv], 32, 64);
        const int oj = __shfl_xor(bidx[nv], 32, 64);
        if (rank_before(os, oj, best[nv], bidx[nv])) {
          best[nv] = os;
          bidx[nv] = oj;
        }
        if (wa > 0 && h == 0) {
          ps[wa * M_BV + wv * M_VCOLS + nv * 32 + l32] = best[nv];
          pj[wa * M_BV + wv * M_VCOLS + nv * 32 + l32] = bidx[nv];
        }
      }
      __syncthreads();
      if (wa == 0 && h == 0) {
#pragma unroll
        for (int nv = 0; nv < M_NV; ++nv) {
          const int c = wv * M_VCOLS + nv * 32 + l32;
          for (int g2 = 1; g2 < M_WA; ++g2)  // atom groups in increasing order
            if (rank_before(ps[g2 * M_BV + c], pj[g2 * M_BV + c], best[nv], bidx[nv])) {
              best[nv] = ps[g2 * M_BV + c];
              bidx[nv] = pj[g2 * M_BV + c];
            }
          const int64_t v = v0 + c;
          if (v < nvox) {
            g.part_s[(int64_t)split * g.pstride + v] = best[nv];
            g.part_j[(int64_t)split * g.pstride + v] = bidx[nv];
          }
        }
      }
    }
    __syncthreads();  // the next item reuses the LDS buffers
  }
}

namespace {

MxArgs mx_args(const uint16_t *D, const uint16_t *Z, int Kq, int d, int64_t d_pad, int64_t n) {
  MxArgs a{};
  a.D = D;
  a.Z = Z;
  a.row = Kq;
  a.nstage = Kq / 64;
  a.d = d;
  a.ntiles = (int)(d_pad / M_BA);
  a.n = n;
  return a;
}

}  // namespace

int mx_auto_splits(int64_t d_pad, int64_t n) {
  const int64_t nvt = (n + M_BV - 1) / M_BV;
  const int64_t nvt8 = (nvt + 7) / 8 * 8;
  const int64_t ntiles = d_pad / M_BA;
  // 16 splits per voxel tile (measured: 31.8 ms against 33.0 with 8 and 35.1
  // with 4 at 65,536 x 100,800), more to fill the chip for few voxels
  int64_t s = std::max<int64_t>(16, (512 + nvt8 - 1) / nvt8);
  s = std::min<int64_t>(s, std::min<int64_t>(ntiles, 256));
  return (int)std::max<int64_t>(s, 1);
}

void launch_score_mx(const uint16_t *D, const uint16_t *Z, int Kq, int d, int64_t d_pad, int64_t n, int splits,
                     float *part_s, int *part_j, hipStream_t s) {
  MxArgs a = mx_args(D, Z, Kq, d, d_pad, n);
  a.splits = splits;
  a.tps = (a.ntiles + splits - 1) / splits;
  a.part_s = part_s;
  a.part_j = part_j;
  a.pstride = n;
  const int64_t nvt = (n + M_BV - 1) / M_BV;
  const int64_t blocks = (nvt + 7) / 8 * 8 * splits;
  if (blocks > 0) hipLaunchKernelGGL(k_score_mx<SC_TOP1>, dim3((unsigned)blocks), dim3(M_NT), 0, s, a);
}

void launch_collect_mx(const uint16_t *D, const uint16_t *Z, int Kq, int d, int64_t d_pad, int64_t n, int splits,
                       const float *thr, unsigned int *count, int32_t *cand, int ccap, hipStream_t s) {
  MxArgs a = mx_args(D, Z, Kq, d, d_pad, n);
  a.splits = splits;
  a.tps = (a.ntiles + splits - 1) / splits;
  a.thr = thr;
  a.count = count;
  a.cand = cand;
  a.ccap = ccap;
  const int64_t nvt = (n + M_BV - 1) / M_BV;
  const int64_t blocks = (nvt + 7) / 8 * 8 * splits;
  if (blocks > 0) hipLaunchKernelGGL(k_score_mx<SC_COLLECT>, dim3((unsigned)blocks), dim3(M_NT), 0, s, a);
}

}  // namespace mrf
