// Exhaustive matched-filter scoring on the matrix cores of gfx950, FP32
// accumulation, with the per-voxel epilogues of the filter fused (eq.
// exactP).  Three row encodings:
//   BF16: v_mfma_f32_32x32x16_bf16, 8 values of a row per lane and k-step;
//   FP8 E4M3: v_mfma_scale_f32_32x32x64_f8f6f4 with unit block scales, 32
//     values per lane and k-step; an atom's score is the E4M3 product times
//     the atom's row scale (the voxel's scale, common to all its scores, is
//     left out: lines are given in the same unit);
//   split BF16: rows of k_split_x3 (per 32 values a 128-byte chunk
//     [hi 32 | lo 32]); a score is hi.hi + hi.lo + lo.hi, three
//     v_mfma_f32_32x32x16_bf16 per k-step.
// Epilogues: the per-voxel maximum (SC_TOP1), the kCertK best within a window
// of the running maximum (SC_TOPK, the exactness certificate's lists), or
// every atom at or above a per-voxel line (SC_COLLECT).
//
// Block tile: 256 atoms x 256 voxels, MRF_MX_WA x MRF_MX_WV waves, each
// owning a (256 / WA) x (256 / WV) sub-tile of MFMA 32x32 tiles (atoms are the
// A rows, voxels the B columns, so a lane folds one voxel column per tile and
// atoms reach it in increasing order).  A stage is 128 bytes of each of the
// 512 rows, double-buffered in LDS.  Stages go straight from global memory to
// LDS (buffer_load_dwordx4 ... lds: a wave's 64 lanes write 16 bytes each at
// the wave's LDS base + 16 x lane, i.e. eight 128-byte rows), with the eight
// 16-byte chunks of row r stored at slot chunk ^ s(r), s(r) = (r / 2 % 8) ^
// 4 (r % 2): the 16 lanes of one LDS access reading one chunk of 16
// consecutive rows hit 16 distinct 16-byte bank groups (and any 8 of them
// 8 distinct slots of a 128-byte line).  Work items are (voxel
// tile, atom split) pairs; the splits of a voxel tile run on one XCD (item w
// on XCD w % 8), so its blocks share the voxel tile and, across the voxel
// tiles in flight, the atom tiles through that XCD's L2.
#include "k_split.h"
#include "k_topk.h"
#include "mrf_internal.h"

#include <type_traits>

namespace mrf {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

enum { E_BF16 = 0, E_FP8 = 1, E_X3 = 2 };

// wave grid (atom-row groups x voxel-column groups; tuning constants)
// (8 waves of 128 atoms x 64 voxels: BF16 12.5 ms per 65,536 x 100,800 x
// 1,000, against 12.4 for 64 x 128 and 12.9 for 16 waves of 64 x 64; the FP8
// and split forms need 128 x 64 to keep their operands in registers)
#ifndef MRF_MX_WA
#define MRF_MX_WA 2
#endif
#ifndef MRF_MX_WV
#define MRF_MX_WV 4
#endif
constexpr int M_BA = 256, M_BV = 256;
constexpr int M_WA = MRF_MX_WA, M_WV = MRF_MX_WV, M_NT = 64 * M_WA * M_WV;
constexpr int M_ROWB = 128;                            // bytes of a row per stage
constexpr int M_STAGE = (M_BA + M_BV) * M_ROWB;        // bytes per stage buffer
constexpr int M_AROWS = M_BA / M_WA, M_VCOLS = M_BV / M_WV;  // per wave
constexpr int M_MA = M_AROWS / 32;                     // 32-atom MFMA tiles per wave
constexpr int M_NV = M_VCOLS / 32;                     // 32-voxel MFMA tiles per wave
constexpr int M_NW = M_NT / 64;                        // waves
constexpr int M_DI = (M_BA + M_BV) / 8 / M_NW;         // 8-row loads per wave and stage
constexpr int M_DIA = M_BA / 8 / M_NW;                 // of which atom rows
constexpr int M_DIZ = M_DI - M_DIA;
static_assert(M_MA >= 1 && M_NV >= 1, "block shape");
static_assert(M_DI * M_NW * 8 == M_BA + M_BV && (M_BA / 8) % M_NW == 0 && M_NW % 2 == 0, "loader shape");
static_assert(2 * M_STAGE + 2 * M_BA * 4 <= 160 * 1024, "LDS");
static_assert(M_BV == kX3VoxTile, "split-BF16 voxel tiles (gathered rows, device-side splits)");
static_assert(M_WA * kCertK * M_BV * 8 <= 2 * M_STAGE, "LDS exchange of the candidate lists");

// byte offset of the 16-byte chunk c in stage row r (only r % 16 matters)
__device__ __forceinline__ int chunk_at(int c, int r) { return (c ^ ((r >> 1) & 7) ^ ((r & 1) << 2)) * 16; }

}  // namespace

struct MxArgs {
  const uint8_t *D;        // atom rows, pitch `row` bytes (d_pad rows, zero padded)
  const uint8_t *Z;        // voxel rows, same pitch (rows up to the voxel-tile multiple readable)
  const float *dscale;     // FP8: the atoms' row scales
  int64_t row;             // row pitch in bytes
  int nstage;              // 128-byte stages per row
  int d, ntiles;           // atoms; 256-atom tiles
  int64_t n;               // voxels (with dcnt: the capacity)
  const unsigned int *dcnt;  // voxel count on the device (null: n)
  int splits, tps;         // atom splits and 256-atom tiles per split (dcnt: chosen on the device)
  float *part_s;           // SC_TOP1 [splits][pstride], SC_TOPK [splits][pstride][kCertK]
  int *part_j;
  int64_t pstride;
  const float *znorm;      // SC_TOPK: window cw ||Z_v|| + wabs
  float cw, wabs;
  const int32_t *rowmap;   // SC_COLLECT, split rows: voxel i is row rowmap[i] of Z
  const float *thr;        // SC_COLLECT: per-voxel line
  unsigned int *count;
  int32_t *cand;
  int ccap;
};

template <int E, int MODE>
__global__ __launch_bounds__(M_NT, 1) void k_score_mx(MxArgs g) {
  constexpr bool F8 = E == E_FP8, X3 = E == E_X3;
  constexpr bool RMAP = X3 && MODE == SC_COLLECT;
  // work items; with the voxel count on the device the tiles and splits
  // follow from it and the grid loops over the items
  int64_t nvox = g.n;
  int nsplit = g.splits, tps = g.tps;
  int nvt = (int)((nvox + M_BV - 1) / M_BV);
  if (g.dcnt) {
    nvox = min(g.n, (int64_t)*g.dcnt);
    nvt = (int)((nvox + M_BV - 1) / M_BV);
    const int nvt8 = (nvt + 7) / 8 * 8;
    // a rescan spreads its few voxel tiles over more splits (about 2,048
    // items); the fallback's split count is the one its merge recomputes
    nsplit = MODE == SC_COLLECT ? max(1, min(g.ntiles, min(256, (2048 + nvt8 - 1) / max(8, nvt8))))
                                : x3_device_splits(nvt, g.ntiles);
    tps = (g.ntiles + nsplit - 1) / nsplit;
  }
  const int64_t nwork = (int64_t)((nvt + 7) / 8 * 8) * nsplit;

  // two stage buffers, then (FP8) the atom scales of two tiles by tile parity
  __shared__ __attribute__((aligned(16))) uint8_t S[2 * M_STAGE + (F8 ? 2 * M_BA * 4 : 0)];
  float(*SCL)[M_BA] = reinterpret_cast<float(*)[M_BA]>(S + 2 * M_STAGE);

  // the wave index made wave-uniform for the compiler (scalar branches on it)
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wa = wave / M_WV, wv = wave % M_WV;
  const int h = lane >> 5, l32 = lane & 31, rm = l32 & 15;  // every row this lane reads is rm modulo 16
  // loader: load i of wave w covers stage rows R = (i M_NW + w) 8 + lane / 8
  // (atom rows below M_BA, then voxel rows: M_NW divides M_BA / 8), R % 16 =
  // 8 (w % 2) + lane / 8 as M_NW is even; the lane fetches the chunk that
  // belongs in its slot lane % 8
  const int drow = lane >> 3, dchunk = chunk_at(lane & 7, 8 * (wave & 1) + drow);

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

    // loads i < M_DIA fetch atom rows, the rest voxel rows; row R of load i is
    // i M_NW 8 rows after the wave's first, a uniform step (voxel rows of a
    // rescan through the row map; rows past the count read the first listed row)
    const uint8_t *zr[RMAP ? M_DIZ : 1];
#pragma unroll
    for (int i = 0; i < (RMAP ? M_DIZ : 1); ++i) {
      int64_t r = v0 + i * M_NW * 8 + wave * 8 + drow;
      if (RMAP) r = g.rowmap[r < nvox ? r : 0];
      zr[i] = g.Z + r * g.row + dchunk;
    }
    // The stage loads go through buffer resources (buffer_load_dwordx4 ...
    // lds) built per stage on the tile's first row, with 32-bit lane offsets
    // inside the tile: unlike the flat-segment form, these leave the LDS
    // counter in order, so the waits for the fragment reads below stay
    // partial while a stage's loads are in flight.  A rescan's voxel rows
    // (through the row map, anywhere in Z) keep the flat form.
    const uint32_t lrow = (uint32_t)((wave * 8 + drow) * g.row + dchunk);
    const uint32_t lstep = (uint32_t)(M_NW * 8 * g.row);
    auto dload = [&](int q, int buf) {
      const int tq = q / g.nstage;
      const int64_t soff = (q - tq * g.nstage) * M_ROWB;
      const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(g.D + (int64_t)(tb + tq) * M_BA * g.row + soff), 0, (int)(M_BA * g.row), 0x00020000);
      const __amdgpu_buffer_rsrc_t rz =
          __builtin_amdgcn_make_buffer_rsrc((void *)(g.Z + v0 * g.row + soff), 0, (int)(M_BV * g.row), 0x00020000);
#pragma unroll
      for (int i = 0; i < M_DI; ++i) {
        lds_void *dst = (lds_void *)(S + buf * M_STAGE + (i * M_NW + wave) * 8 * M_ROWB);
        if (i < M_DIA)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, dst, 16, lrow + i * lstep, 0, 0, 0);
        else if constexpr (RMAP)
          __builtin_amdgcn_global_load_lds((const void *)(zr[RMAP ? i - M_DIA : 0] + soff), dst, 16, 0, 0);
        else
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rz, dst, 16, lrow + (i - M_DIA) * lstep, 0, 0, 0);
      }
      // FP8: wave 0 loads a tile's 256 atom scales with its first stage, into
      // the LDS slot of the tile's parity (that slot's previous tile was
      // folded before an earlier barrier; the fold of this one follows the
      // stage-end wait and barrier)
      if (F8 && wave == 0 && q == tq * g.nstage) {
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void *)(g.dscale + (int64_t)(tb + tq) * M_BA), 0, M_BA * 4, 0x00020000);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void *)&SCL[(tb + tq) & 1][0], 16, lane * 16, 0, 0, 0);
      }
    };

    f32x16 acc[M_MA][M_NV];
#pragma unroll
    for (int a = 0; a < M_MA; ++a)
#pragma unroll
      for (int b = 0; b < M_NV; ++b)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;
    float best[M_NV], vthr[M_NV], win[M_NV];  // SC_TOPK: insertion bar and window; SC_COLLECT: the line
    int bidx[M_NV];
    float ls[MODE == SC_TOPK ? M_NV : 1][kCertK];
    int lj[MODE == SC_TOPK ? M_NV : 1][kCertK];
#pragma unroll
    for (int b = 0; b < M_NV; ++b) {
      best[b] = -INFINITY;
      bidx[b] = -1;
      vthr[b] = MODE == SC_TOPK ? -INFINITY : INFINITY;
      win[b] = 0.f;
      const int64_t v = v0 + wv * M_VCOLS + b * 32 + l32;
      if constexpr (MODE == SC_TOPK) {
        topk_clear(ls[b], lj[b]);
        if (v < nvox) win[b] = g.cw * fmaxf(g.znorm[v], 0.f) + g.wabs;
      }
      if (MODE == SC_COLLECT && v < nvox) vthr[b] = g.thr[v];
    }

    if (nq > 0) {
      dload(0, 0);
      __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
    for (int q = 0; q < nq; ++q) {
      const int buf = q & 1;
      if (q + 1 < nq) dload(q + 1, buf ^ 1);  // every wave finished reading that buffer before the last barrier
      const uint8_t *B = S + buf * M_STAGE;
      const uint8_t *Ab = B + (wa * M_AROWS + l32) * M_ROWB;
      const uint8_t *Zb = B + (M_BA + wv * M_VCOLS + l32) * M_ROWB;
      // The fragments of the next group of products are read from LDS before
      // the products of the current group issue (scheduling barriers keep
      // the compiler from sinking the reads next to their use), so a wave's
      // LDS latency overlaps its own MFMAs.  A wave raises its priority while
      // it issues products, so that the two waves of a SIMD alternate the
      // matrix pipe and their reads rather than both waiting on LDS at once.
      if constexpr (F8) {
        // two k-steps of 64: the lane supplies 32 bytes (chunks 4 ks + 2 h,
        // + 1); groups (ks, ma), A fragments one group ahead, voxel
        // fragments one k-step ahead
        i32x8 zf[2][M_NV], af[2];
        auto rd2 = [&](const uint8_t *base, int ks) {
          const u32x4 x0 = *reinterpret_cast<const u32x4 *>(base + chunk_at(4 * ks + 2 * h, rm));
          const u32x4 x1 = *reinterpret_cast<const u32x4 *>(base + chunk_at(4 * ks + 2 * h + 1, rm));
          return i32x8{(int)x0.x, (int)x0.y, (int)x0.z, (int)x0.w, (int)x1.x, (int)x1.y, (int)x1.z, (int)x1.w};
        };
        auto rdz = [&](int ks) {
#pragma unroll
          for (int nv = 0; nv < M_NV; ++nv) zf[ks & 1][nv] = rd2(Zb + nv * 32 * M_ROWB, ks);
        };
        rdz(0);
        af[0] = rd2(Ab, 0);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
          for (int ma = 0; ma < M_MA; ++ma) {
            const int gi = ks * M_MA + ma;
            if (ma + 1 < M_MA) {
              af[(gi + 1) & 1] = rd2(Ab + (ma + 1) * 32 * M_ROWB, ks);
            } else if (ks + 1 < 2) {
              rdz(ks + 1);
              af[(gi + 1) & 1] = rd2(Ab, ks + 1);
            }
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int nv = 0; nv < M_NV; ++nv)
              acc[ma][nv] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af[gi & 1], zf[ks & 1][nv], acc[ma][nv], 0,
                                                                            0, 0, 0x7F, 0, 0x7F);
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_setprio(0);
          }
      } else if constexpr (X3) {
        // two k-steps of 16: the lane supplies 8 values of each plane (hi
        // chunk 2 ks + h, lo chunk 4 + 2 ks + h); groups (ks, ma), A
        // fragments one group ahead, voxel fragments one k-step ahead
        bf16x8 zh[2][M_NV], zl[2][M_NV], ah[2], al[2];
        auto rdz = [&](int ks) {
          const int oh = chunk_at(2 * ks + h, rm), ol = chunk_at(4 + 2 * ks + h, rm);
#pragma unroll
          for (int nv = 0; nv < M_NV; ++nv) {
            zh[ks & 1][nv] = *reinterpret_cast<const bf16x8 *>(Zb + nv * 32 * M_ROWB + oh);
            zl[ks & 1][nv] = *reinterpret_cast<const bf16x8 *>(Zb + nv * 32 * M_ROWB + ol);
          }
        };
        auto rda = [&](int ks, int ma, int sl) {
          ah[sl] = *reinterpret_cast<const bf16x8 *>(Ab + ma * 32 * M_ROWB + chunk_at(2 * ks + h, rm));
          al[sl] = *reinterpret_cast<const bf16x8 *>(Ab + ma * 32 * M_ROWB + chunk_at(4 + 2 * ks + h, rm));
        };
        rdz(0);
        rda(0, 0, 0);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
          for (int ma = 0; ma < M_MA; ++ma) {
            const int gi = ks * M_MA + ma, sl = gi & 1, zs = ks & 1;
            if (ma + 1 < M_MA) {
              rda(ks, ma + 1, (gi + 1) & 1);
            } else if (ks + 1 < 2) {
              rdz(ks + 1);
              rda(ks + 1, 0, (gi + 1) & 1);
            }
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int nv = 0; nv < M_NV; ++nv) {
              acc[ma][nv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[sl], zh[zs][nv], acc[ma][nv], 0, 0, 0);
              acc[ma][nv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[sl], zl[zs][nv], acc[ma][nv], 0, 0, 0);
              acc[ma][nv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[sl], zh[zs][nv], acc[ma][nv], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_setprio(0);
          }
      } else {
        // four k-steps of 16: the lane supplies 8 BF16 (chunk 2 ks + h); all
        // fragments one k-step ahead
        bf16x8 zf[2][M_NV], af[2][M_MA];
        auto rd = [&](int ks) {
          const int ko = chunk_at(2 * ks + h, rm);
#pragma unroll
          for (int nv = 0; nv < M_NV; ++nv)
            zf[ks & 1][nv] = *reinterpret_cast<const bf16x8 *>(Zb + nv * 32 * M_ROWB + ko);
#pragma unroll
          for (int ma = 0; ma < M_MA; ++ma)
            af[ks & 1][ma] = *reinterpret_cast<const bf16x8 *>(Ab + ma * 32 * M_ROWB + ko);
        };
        rd(0);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          if (ks + 1 < 4) rd(ks + 1);
          __builtin_amdgcn_sched_barrier(0);
          __builtin_amdgcn_s_setprio(1);
#pragma unroll
          for (int ma = 0; ma < M_MA; ++ma)
#pragma unroll
            for (int nv = 0; nv < M_NV; ++nv)
              acc[ma][nv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[ks & 1][ma], zf[ks & 1][nv], acc[ma][nv], 0,
                                                                    0, 0);
          __builtin_amdgcn_sched_barrier(0);
          __builtin_amdgcn_s_setprio(0);
        }
      }
      const int st = q % g.nstage;
      if (st == g.nstage - 1) {
        // fold this atom tile: M_AROWS atom rows per voxel column and lane,
        // row jb + ro with ro = 32 ma + 8 (i / 4) + i % 4.  jb is made opaque
        // here so that the compiler forms the row numbers at the fold instead
        // of keeping all 64 live across the stage loop, where the products
        // need the registers for their fragments
        const int tile = tb + q / g.nstage;
        const int abase = tile * M_BA + wa * M_AROWS;
        int jb = abase + 4 * h;
        asm volatile("" : "+v"(jb));
        const bool full = abase + M_AROWS <= g.d;  // no padding rows in this wave's rows
        const float *sclh = &SCL[F8 ? (tile & 1) : 0][(F8 ? wa * M_AROWS : 0) + 4 * h];
#pragma unroll
        for (int nv = 0; nv < M_NV; ++nv) {
          if constexpr (MODE == SC_TOP1) {
            // the tile's maximum with its position p = 16 ma + i (a constant
            // per candidate), then one compare with the running maximum:
            // atoms in increasing order, '>' keeps the lowest index
            float tbv = -INFINITY;
            int tp = 0;
            auto scan = [&](auto chk) {
#pragma unroll
              for (int ma = 0; ma < M_MA; ++ma)
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                  const int ro = ma * 32 + 8 * (i >> 2) + (i & 3);
                  float sc = F8 ? acc[ma][nv][i] * sclh[ro] : acc[ma][nv][i];
                  if (decltype(chk)::value && jb + ro >= g.d) sc = -INFINITY;
                  if (sc > tbv) {
                    tbv = sc;
                    tp = ma * 16 + i;
                  }
                }
            };
            if (full)
              scan(std::false_type{});
            else
              scan(std::true_type{});
            if (tbv > best[nv]) {
              best[nv] = tbv;
              bidx[nv] = jb + (tp >> 4) * 32 + 8 * ((tp >> 2) & 3) + (tp & 3);
            }
          } else {
            const int64_t v = v0 + wv * M_VCOLS + nv * 32 + l32;
#pragma unroll
            for (int ma = 0; ma < M_MA; ++ma)
              // the list insertion is long and rare: one copy per tile of the
              // accumulators, its element picked by the (uniform) loop index
#pragma unroll(MODE == SC_TOPK ? 1 : 16)
              for (int i = 0; i < 16; ++i) {
                const int ro = ma * 32 + 8 * (i >> 2) + (i & 3);
                const int j = jb + ro;
                const float sc = F8 ? acc[ma][nv][i] * sclh[ro] : acc[ma][nv][i];
                if constexpr (MODE == SC_TOPK) {
                  if (j < g.d && sc > vthr[nv]) {
                    topk_push_ordered(ls[nv], lj[nv], sc, j);
                    vthr[nv] = fmaxf(ls[nv][kCertK - 1], ls[nv][0] - win[nv]);
                  }
                } else {
                  if (j < g.d && v < nvox && sc >= vthr[nv]) {
                    const unsigned int pos = atomicAdd(&g.count[v], 1u);
                    if ((int)pos < g.ccap) g.cand[v * g.ccap + pos] = j;
                  }
                }
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
      __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of the next stage are in LDS
      __syncthreads();
    }
    if (MODE == SC_COLLECT) continue;  // the candidates are already written

    if constexpr (MODE == SC_TOPK) {
      // the two half-waves, then the M_WA atom-row groups' lists through LDS
      float *ps = reinterpret_cast<float *>(S);
      int *pj = reinterpret_cast<int *>(S) + M_WA * kCertK * M_BV;
#pragma unroll
      for (int nv = 0; nv < M_NV; ++nv) {
        topk_merge_xor(ls[nv], lj[nv], 32);
        if (h == 0) {
          const int c = wv * M_VCOLS + nv * 32 + l32;
#pragma unroll
          for (int i = 0; i < kCertK; ++i) {
            ps[(wa * kCertK + i) * M_BV + c] = ls[nv][i];
            pj[(wa * kCertK + i) * M_BV + c] = lj[nv][i];
          }
        }
      }
      __syncthreads();
      if (tid < M_BV) {
        float ms[kCertK];
        int mj[kCertK];
#pragma unroll
        for (int i = 0; i < kCertK; ++i) {
          ms[i] = ps[i * M_BV + tid];
          mj[i] = pj[i * M_BV + tid];
        }
        for (int w2 = 1; w2 < M_WA; ++w2)
#pragma unroll
          for (int i = 0; i < kCertK; ++i)
            topk_push(ms, mj, ps[(w2 * kCertK + i) * M_BV + tid], pj[(w2 * kCertK + i) * M_BV + tid]);
        const int64_t v = v0 + tid;
        if (v < nvox) {
          float *os = g.part_s + ((int64_t)split * g.pstride + v) * kCertK;
          int *oj = g.part_j + ((int64_t)split * g.pstride + v) * kCertK;
#pragma unroll
          for (int i = 0; i < kCertK; ++i) {
            os[i] = ms[i];
            oj[i] = mj[i];
          }
        }
      }
    } else {
      // the two half-waves, then the M_WA atom-row groups of the block through LDS
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

MxArgs mx_args(int e, const void *D, const void *Z, int row_bytes, int d, int64_t d_pad, int64_t n, int splits) {
  MxArgs a{};
  a.D = static_cast<const uint8_t *>(D);
  a.Z = static_cast<const uint8_t *>(Z);
  a.row = row_bytes;
  a.nstage = row_bytes / M_ROWB;
  a.d = d;
  a.ntiles = (int)(d_pad / M_BA);
  a.n = n;
  a.splits = splits;
  a.tps = (a.ntiles + splits - 1) / splits;
  a.pstride = n;
  (void)e;
  return a;
}

template <int E, int MODE>
void launch_mx(const MxArgs &a, int64_t blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL((k_score_mx<E, MODE>), dim3((unsigned)blocks), dim3(M_NT), 0, s, a);
}

// one block per work item (voxel tiles rounded to whole XCD rounds)
int64_t item_blocks(const MxArgs &a) { return ((a.n + M_BV - 1) / M_BV + 7) / 8 * 8 * a.splits; }

}  // namespace

int mx_auto_splits(int64_t d_pad, int64_t n) {
  const int64_t nvt = (n + M_BV - 1) / M_BV;
  const int64_t nvt8 = (nvt + 7) / 8 * 8;
  const int64_t ntiles = d_pad / M_BA;
  // 8 splits per voxel tile (measured: 12.4 ms against 12.6 with 16 at
  // 65,536 x 100,800, BF16), more to fill the chip for few voxels
  int64_t s = std::max<int64_t>(8, (512 + nvt8 - 1) / nvt8);
  s = std::min<int64_t>(s, std::min<int64_t>(ntiles, 256));
  return (int)std::max<int64_t>(s, 1);
}

void launch_score_mx(bool fp8, const void *D, const float *dscale, const void *Z, int Kq, int d, int64_t d_pad,
                     int64_t n, int splits, float *part_s, int *part_j, hipStream_t s) {
  MxArgs a = mx_args(fp8 ? E_FP8 : E_BF16, D, Z, Kq * (fp8 ? 1 : 2), d, d_pad, n, splits);
  a.dscale = dscale;
  a.part_s = part_s;
  a.part_j = part_j;
  if (fp8)
    launch_mx<E_FP8, SC_TOP1>(a, item_blocks(a), s);
  else
    launch_mx<E_BF16, SC_TOP1>(a, item_blocks(a), s);
}

void launch_collect_mx(bool fp8, const void *D, const float *dscale, const void *Z, int Kq, int d, int64_t d_pad,
                       int64_t n, int splits, const float *thr, unsigned int *count, int32_t *cand, int ccap,
                       hipStream_t s) {
  MxArgs a = mx_args(fp8 ? E_FP8 : E_BF16, D, Z, Kq * (fp8 ? 1 : 2), d, d_pad, n, splits);
  a.dscale = dscale;
  a.thr = thr;
  a.count = count;
  a.cand = cand;
  a.ccap = ccap;
  if (fp8)
    launch_mx<E_FP8, SC_COLLECT>(a, item_blocks(a), s);
  else
    launch_mx<E_BF16, SC_COLLECT>(a, item_blocks(a), s);
}

// Dx: split atoms [d_pad][2 Kx] (d_pad a multiple of 256); Zx: split voxels
// [n_pad][2 Kx] (n_pad a multiple of 256, zero rows beyond n).
void launch_score_x3(const uint16_t *Dx, const uint16_t *Zx, int d, int64_t d_pad, int64_t n, int64_t n_pad,
                     int Kx, int splits, float *part_s, int *part_j, hipStream_t s, bool topk, const float *znorm,
                     float cw, float wabs) {
  (void)n_pad;
  MxArgs a = mx_args(E_X3, Dx, Zx, 4 * Kx, d, d_pad, n, splits);
  a.part_s = part_s;
  a.part_j = part_j;
  a.znorm = znorm;
  a.cw = cw;
  a.wabs = wabs;
  if (topk)
    launch_mx<E_X3, SC_TOPK>(a, item_blocks(a), s);
  else
    launch_mx<E_X3, SC_TOP1>(a, item_blocks(a), s);
}

// device-sized forms: one block per CU of the 256, each looping over the items
void launch_score_x3_dev(const uint16_t *Dx, const uint16_t *Zx, int d, int64_t d_pad, int64_t cap,
                         const unsigned int *dcnt, int Kx, float *part_s, int *part_j, hipStream_t s) {
  if (cap <= 0) return;
  MxArgs a = mx_args(E_X3, Dx, Zx, 4 * Kx, d, d_pad, cap, 1);
  a.dcnt = dcnt;
  a.part_s = part_s;
  a.part_j = part_j;
  launch_mx<E_X3, SC_TOP1>(a, 256, s);
}

void launch_collect_x3_dev(const uint16_t *Dx, const uint16_t *Zx, const int32_t *rows, int d, int64_t d_pad,
                           int64_t cap, const unsigned int *dcnt, int Kx, const float *thr, unsigned int *count,
                           int32_t *cand, int ccap, hipStream_t s) {
  if (cap <= 0) return;
  MxArgs a = mx_args(E_X3, Dx, Zx, 4 * Kx, d, d_pad, cap, 1);
  a.dcnt = dcnt;
  a.rowmap = rows;
  a.thr = thr;
  a.count = count;
  a.cand = cand;
  a.ccap = ccap;
  launch_mx<E_X3, SC_COLLECT>(a, 256, s);
}

}  // namespace mrf
