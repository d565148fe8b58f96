// Exact local matched filter around proposed grid cells (gfx950).
//
// Voxels are grouped by a coarse cell key (counting sort), so a block of 64
// consecutive voxels has neighbouring proposals.  The block scores its voxels
// against every atom of the bounding box of their boxes (gathered rows,
// FP32 MFMA 32x32x2 as in the exhaustive kernel) and keeps, per voxel, the
// best atom inside that voxel's own box (strict '>' over atoms in increasing
// index order: the lowest index wins ties).  Companion kernels flag voxels
// whose best atom sits on an interior box face (re-centring) or whose
// normalised correlation is below the fallback threshold, compact those
// lists, and gather / scatter rows for the exhaustive fallback.
#include <algorithm>
#include <cfloat>

#include "k_split.h"
#include "mrf_internal.h"

namespace mrf {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// grouping
// ---------------------------------------------------------------------------
// A list length on the device (dcnt, may be null) bounds the host's cnt, which
// then only sizes the grid.
__device__ __forceinline__ int64_t list_len(int64_t cnt, const unsigned int *dcnt) {
  return dcnt ? min(cnt, (int64_t)*dcnt) : cnt;
}

// coarse cell of voxel v: its cell's index per parameter (clamped to the
// grid) shifted down by `shift`, mixed in row-major order
__device__ __forceinline__ int coarse_key_of(int v, const int32_t *__restrict__ cells, int P, int shift,
                                             const GridDims &g) {
  int key = 0;
  for (int p = 0; p < P; ++p) {
    const int cd = ((g.dims[p] - 1) >> shift) + 1;
    int c = cells[(int64_t)v * P + p];
    c = c < 0 ? 0 : (c >= g.dims[p] ? g.dims[p] - 1 : c);
    key = key * cd + (c >> shift);
  }
  return key;
}

__global__ void k_coarse_keys(const int32_t *__restrict__ list, int64_t cnt, const unsigned int *__restrict__ dcnt,
                              const int32_t *__restrict__ cells, int P, int shift,
                              GridDims g, int32_t *__restrict__ keys,
                              unsigned int *__restrict__ hist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= list_len(cnt, dcnt)) return;
  const int key = coarse_key_of(list[i], cells, P, shift, g);
  keys[i] = key;
  atomicAdd(&hist[key], 1u);
}

// Block-aggregated forms for nkeys <= kGroupLds: a block counts its voxels
// per key in LDS and makes one global atomic per key present in it, instead of
// one per voxel (the voxels of a key all hit one address).
constexpr int kGroupLds = 4096;
__global__ __launch_bounds__(256) void k_coarse_keys_lds(const int32_t *__restrict__ list, int64_t cnt,
                                                         const unsigned int *__restrict__ dcnt,
                                                         const int32_t *__restrict__ cells, int P, int shift,
                                                         GridDims g, int32_t *__restrict__ keys,
                                                         unsigned int *__restrict__ hist, int nkeys) {
  __shared__ unsigned int h[kGroupLds];
  for (int k = threadIdx.x; k < nkeys; k += 256) h[k] = 0u;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < list_len(cnt, dcnt)) {
    const int key = coarse_key_of(list[i], cells, P, shift, g);
    keys[i] = key;
    atomicAdd(&h[key], 1u);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nkeys; k += 256)
    if (h[k]) atomicAdd(&hist[k], h[k]);
}

__global__ __launch_bounds__(256) void k_group_scatter_lds(const int32_t *__restrict__ list,
                                                           const int32_t *__restrict__ keys, int64_t cnt,
                                                           const unsigned int *__restrict__ dcnt,
                                                           unsigned int *__restrict__ cursor,
                                                           int32_t *__restrict__ out, int nkeys) {
  __shared__ unsigned int h[kGroupLds];  // the block's count per key, then its first position
  for (int k = threadIdx.x; k < nkeys; k += 256) h[k] = 0u;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool valid = i < list_len(cnt, dcnt);
  int key = 0;
  unsigned int rank = 0;
  if (valid) {
    key = keys[i];
    rank = atomicAdd(&h[key], 1u);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nkeys; k += 256)
    if (h[k]) h[k] = atomicAdd(&cursor[k], h[k]);
  __syncthreads();
  if (valid) out[h[key] + rank] = list[i];
}

// Exclusive scans of hist[0..nkeys) (one block): off[k] (the first sorted
// position of key k), cursor[k] = off[k] (consumed by the scatter), and
// toff[k] = the first tile of key k, where key k owns ceil(hist[k] / 64)
// tiles; toff[nkeys] = the number of tiles.  Thread t sums its own run of
// consecutive keys, one block-wide scan of the 1,024 run sums gives each run's
// start, and the thread writes its run's prefixes.
// Up to kScanLds keys go through LDS: coalesced loads, each thread's run
// prefixes kept in LDS, and coalesced writes of the outputs.
constexpr int kScanLds = 16384;
__global__ __launch_bounds__(1024) void k_scan(const unsigned int *__restrict__ hist, int nkeys,
                                               unsigned int *__restrict__ off,
                                               unsigned int *__restrict__ cursor,
                                               unsigned int *__restrict__ toff) {
  __shared__ unsigned int buf[1024], tbuf[1024];
  __shared__ unsigned int hl[kScanLds], th[kScanLds];  // within-run prefixes (keys, tiles)
  __shared__ unsigned int ttotal;
  const int t = threadIdx.x;
  const int per = (nkeys + 1023) / 1024;
  const int b = min(t * per, nkeys), e = min(b + per, nkeys);
  const bool staged = nkeys <= kScanLds;
  unsigned int sum = 0, tsum = 0;
  if (staged) {
    // four loads in flight per thread: one memory round trip per four keys
    for (int i0 = t; i0 < nkeys; i0 += 4096) {
      unsigned int x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = i0 + 1024 * u < nkeys ? hist[i0 + 1024 * u] : 0u;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + 1024 * u < nkeys) hl[i0 + 1024 * u] = x[u];
    }
    __syncthreads();
    for (int i = b; i < e; ++i) {
      const unsigned int x = hl[i];
      hl[i] = sum;
      th[i] = tsum;
      sum += x;
      tsum += (x + 63u) / 64u;
    }
  } else {
    for (int i = b; i < e; ++i) {
      const unsigned int x = hist[i];
      sum += x;
      tsum += (x + 63u) / 64u;
    }
  }
  buf[t] = sum;
  tbuf[t] = tsum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan of the run sums
    const unsigned int y = t >= o ? buf[t - o] : 0u;
    const unsigned int ty = t >= o ? tbuf[t - o] : 0u;
    __syncthreads();
    buf[t] += y;
    tbuf[t] += ty;
    __syncthreads();
  }
  unsigned int run = buf[t] - sum, trun = tbuf[t] - tsum;  // this run's starts
  if (t == 1023) ttotal = tbuf[1023];
  if (staged) {
    __syncthreads();
    buf[t] = run;
    tbuf[t] = trun;
    __syncthreads();
    for (int i = t; i < nkeys; i += 1024) {
      const int r = i / per;
      const unsigned int o = buf[r] + hl[i];
      off[i] = o;
      cursor[i] = o;
      toff[i] = tbuf[r] + th[i];
    }
  } else {
    for (int i = b; i < e; ++i) {
      const unsigned int x = hist[i];
      off[i] = run;
      cursor[i] = run;
      toff[i] = trun;
      run += x;
      trun += (x + 63u) / 64u;
    }
  }
  __syncthreads();
  if (t == 0) toff[nkeys] = ttotal;
}

__global__ void k_group_scatter(const int32_t *__restrict__ list, const int32_t *__restrict__ keys,
                                int64_t cnt, const unsigned int *__restrict__ dcnt,
                                unsigned int *__restrict__ cursor, int32_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= list_len(cnt, dcnt)) return;
  const unsigned int pos = atomicAdd(&cursor[keys[i]], 1u);
  out[pos] = list[i];
}

int coarse_key_count(const GridDims &g, int P, int shift) {
  int64_t k = 1;
  for (int p = 0; p < P; ++p) k *= ((g.dims[p] - 1) >> shift) + 1;
  return (int)k;
}

void launch_group(const int32_t *list, int64_t cnt, const int32_t *cells, int P, int shift,
                  const GridDims &g, int32_t *keys, GroupBufs gb, int32_t *out, hipStream_t s,
                  const unsigned int *dcnt, bool hist_cleared) {
  if (cnt <= 0) return;
  const int nkeys = coarse_key_count(g, P, shift);
  if (!hist_cleared) launch_zero(gb.hist, (int64_t)nkeys * 4, s);
  const unsigned blocks = (unsigned)((cnt + 255) / 256);
  const bool lds = nkeys <= kGroupLds;
  if (lds)
    hipLaunchKernelGGL(k_coarse_keys_lds, dim3(blocks), dim3(256), 0, s, list, cnt, dcnt, cells, P, shift, g,
                       keys, gb.hist, nkeys);
  else
    hipLaunchKernelGGL(k_coarse_keys, dim3(blocks), dim3(256), 0, s, list, cnt, dcnt, cells, P, shift, g,
                       keys, gb.hist);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, gb.hist, nkeys, gb.off, gb.cursor, gb.toff);
  if (lds)
    hipLaunchKernelGGL(k_group_scatter_lds, dim3(blocks), dim3(256), 0, s, list, keys, cnt, dcnt, gb.cursor, out,
                       nkeys);
  else
    hipLaunchKernelGGL(k_group_scatter, dim3(blocks), dim3(256), 0, s, list, keys, cnt, dcnt, gb.cursor, out);
}

// ---------------------------------------------------------------------------
// local scoring
// ---------------------------------------------------------------------------
constexpr int LS_BA = 128, LS_BV = 64;
#ifndef MRF_LS_RUN
#define MRF_LS_RUN 4
#endif
constexpr unsigned int LS_RUN = MRF_LS_RUN;  // consecutive tiles per XCD run (a tuning constant)
// FP32 operands: K chunks of 16, LDS rows of 20 floats.  Split-BF16 operands:
// K stages of LS_XC chunks of 32, LDS rows of LS_XC x [hi 32 | lo 32] + pad 8 BF16.
constexpr int LS_BK32 = 16, LS_LD32 = 20;
constexpr int LS_XC = 1;                            // 32-element chunks per stage
constexpr int LS_BKX = 32 * LS_XC, LS_LDX = 64 * LS_XC + 8;
static_assert(LS_BKX == kX3Stage, "split rows are padded to one stage");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bool lbetter(float s1, int j1, float s0, int j0) {
  return (s1 > s0) || (s1 == s0 && j1 >= 0 && (j0 < 0 || j1 < j0));
}


// Split FP32 rows [rows][Kp] into BF16 hi = RNE(x), lo = RNE(x - hi),
// stored per row as Kx/32 chunks [hi 32 | lo 32] (one 128-byte line per
// chunk, so a K-step of 32 reads whole lines); columns Kp..Kx-1 are zero.
__global__ void k_split_x3(const float *__restrict__ src, int Kp, int64_t rows, int Kx,
                           uint16_t *__restrict__ dst) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one group of 4 columns
  const int64_t per_row = Kx / 4;
  if (q >= rows * per_row) return;
  const int64_t row = q / per_row;
  const int k = (int)(q - row * per_row) * 4;
  float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
  if (k < Kp) x = *reinterpret_cast<const float4 *>(src + row * Kp + k);
  const float xs[4] = {x.x, x.y, x.z, x.w};
  uint16_t hi[4], lo[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) split_bf16(xs[i], hi[i], lo[i]);
  uint16_t *d = dst + row * 2 * Kx + (k >> 5) * 64 + (k & 31);
  *reinterpret_cast<uint2 *>(d) = make_uint2(hi[0] | ((uint32_t)hi[1] << 16), hi[2] | ((uint32_t)hi[3] << 16));
  *reinterpret_cast<uint2 *>(d + 32) =
      make_uint2(lo[0] | ((uint32_t)lo[1] << 16), lo[2] | ((uint32_t)lo[3] << 16));
}

// Chunked split rows -> [rows][hi K | lo K] (for export).
__global__ void k_unsplit_x3(const uint16_t *__restrict__ src, int64_t rows, int Kx, int K,
                             uint16_t *__restrict__ dst) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= rows * K) return;
  const int64_t row = q / K;
  const int k = (int)(q - row * K);
  const uint16_t *r = src + row * 2 * Kx + (k >> 5) * 64 + (k & 31);
  dst[row * 2 * K + k] = r[0];
  dst[row * 2 * K + K + k] = r[32];
}

void launch_unsplit_x3(const uint16_t *src, int64_t rows, int Kx, int K, uint16_t *dst, hipStream_t s) {
  if (rows <= 0) return;
  const int64_t work = rows * K;
  hipLaunchKernelGGL(k_unsplit_x3, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, src, rows, Kx, K, dst);
}

void launch_split_x3(const float *src, int Kp, int64_t rows, int Kx, uint16_t *dst, hipStream_t s) {
  if (rows <= 0) return;
  const int64_t work = rows * (Kx / 4);
  hipLaunchKernelGGL(k_split_x3, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, src, Kp, rows, Kx, dst);
}

// (score, atom) -> 64-bit key ordered as (score, then lower atom): the score
// bits mapped to an order-preserving unsigned integer in the high half,
// 0xFFFFFFFF - atom in the low half.  Key 0 means no candidate.
__device__ __forceinline__ unsigned long long pack_best(float s, int j) {
  unsigned int u = __float_as_uint(s);
  u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((unsigned long long)u << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned int)j);
}

// (score, atom) of a best key; -inf / -1 for key 0 (no candidate)
__device__ __forceinline__ void unpack_best(unsigned long long k, float &s, int32_t &j) {
  if (k == 0ull) {
    s = -INFINITY;
    j = -1;
    return;
  }
  const unsigned int u = (unsigned int)(k >> 32);
  s = __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
  j = (int32_t)(0xFFFFFFFFu - (unsigned int)(k & 0xFFFFFFFFull));
}

// mode 0: keys of the listed voxels (all voxels if list is null) set to 0;
// mode 1: keys unpacked into best_s / best_j (-inf / -1 for key 0).
__global__ void k_best_keys(const int32_t *__restrict__ list, int64_t cnt, const unsigned int *__restrict__ dcnt,
                            unsigned long long *__restrict__ keys, float *__restrict__ best_s,
                            int32_t *__restrict__ best_j, int mode) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= list_len(cnt, dcnt)) return;
  const int64_t v = list ? list[i] : i;
  if (mode == 0) {
    keys[v] = 0ull;
    return;
  }
  float bs;
  int32_t bj;
  unpack_best(keys[v], bs, bj);
  best_s[v] = bs;
  best_j[v] = bj;
}

void launch_best_keys(const int32_t *list, int64_t cnt, unsigned long long *keys, float *best_s, int32_t *best_j,
                      int mode, hipStream_t s, const unsigned int *dcnt) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(k_best_keys, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, list, cnt, dcnt, keys,
                     best_s, best_j, mode);
}

// X3 = false: FP32 rows (pitch Kp), v_mfma_f32_32x32x2f32.
// X3 = true: split-BF16 rows of chunks [hi 32 | lo 32] (pitch 2 Kx), three v_mfma_f32_32x32x16_bf16
// per step (hi.hi + hi.lo + lo.hi) accumulated in FP32.
// COLLECT: instead of each voxel's best, every atom of its box whose score
// reaches the voxel's line col.thr[v] is appended to col.cand[v][0..ccap)
// (col.count[v] counts them all): the candidates of the certified local search.
template <bool X3, bool COLLECT>
__global__ __launch_bounds__(256, X3 ? 3 : 2) void k_local_score(
    const void *__restrict__ Dv, const void *__restrict__ Zv, int pitch,
    const int32_t *__restrict__ order, GroupBufs gb, int nkeys, const int32_t *__restrict__ cells,
    int P, GridDims g, int r, int max_at, unsigned long long *__restrict__ bestkey,
    unsigned long long *__restrict__ work, unsigned long long *__restrict__ boxsum, LocalCollect col) {
  constexpr int BK = X3 ? LS_BKX : LS_BK32;
  constexpr int A_ELEMS = X3 ? LS_BA * LS_LDX : LS_BA * LS_LD32;  // per buffer, in operand units
  constexpr int Z_ELEMS = X3 ? LS_BV * LS_LDX : LS_BV * LS_LD32;
  constexpr int EB = X3 ? 2 : 4;  // bytes per element
  // LDS buffers: FP32 double-buffers its stages; split BF16 (twice the bytes
  // per stage) keeps one buffer, so that more blocks share a CU
#ifndef MRF_LS_X3_NBUF
#define MRF_LS_X3_NBUF 1
#endif
  constexpr int NBUF = X3 ? MRF_LS_X3_NBUF : 2;
  __shared__ __attribute__((aligned(16))) unsigned char smem[NBUF * (A_ELEMS + Z_ELEMS) * EB];
  __shared__ int vid[LS_BV];
  __shared__ int vlo[LS_BV][4], vhi[LS_BV][4];
  __shared__ int blo[4], bdim[4];
  __shared__ unsigned int bmag[4];  // floor(2^32 / bdim) for the multiply-high division
  __shared__ int acoord[LS_BA][4];
  __shared__ int aj[LS_BA];
  __shared__ float red_s[4][LS_BV];
  __shared__ int red_j[4][LS_BV];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  // block = (voxel tile T, atom tile `at` of the tile's bounding box).  Tile T
  // belongs to the key k with toff[k] <= T < toff[k+1]; its voxels are sorted
  // positions off[k] + 64 (T - toff[k]) .. (at most 64, never beyond key k)
  // Workgroups are dealt to the 8 XCDs round-robin (block b on XCD b % 8).
  // Block b = x + 8 j takes the q-th tile of XCD x, q = j / max_at, and its
  // atom tile j % max_at, so all atom tiles of a tile run on one XCD one after
  // the other (its voxel rows stay in that L2).
#ifndef MRF_LS_XCD_SLAB
#define MRF_LS_XCD_SLAB 0
#endif
  // The block's work item w = blockIdx.x (the mapping below), written as a
  // function of w whose early exits return (measured 2 % faster than the
  // same code inline, with two VGPRs fewer).
  auto item = [&](unsigned int w) {
  const unsigned int xcd = w & 7u, jx = w >> 3;
  const unsigned int q = jx / (unsigned)max_at;
  const int at = (int)(jx % (unsigned)max_at);
#if MRF_LS_XCD_SLAB
  // XCD x owns the x-th eighth of the tiles in key order (a slab of the
  // slowest parameter's coarse cells), so the tiles resident on one XCD at a
  // time are neighbouring cells whose bounding boxes share atom rows
  const unsigned int ntile = gb.toff[nkeys];
  const unsigned int per = (ntile + 7u) / 8u;
  const unsigned int T = xcd * per + q;
  if (q >= per || T >= ntile) return;
#else
  // XCD x owns runs of LS_RUN consecutive tiles (runs x, x + 8, ...)
  const unsigned int T = ((q / LS_RUN) * 8u + xcd) * LS_RUN + q % LS_RUN;
  if (T >= gb.toff[nkeys]) return;
#endif
  int lo_k = 0, hi_k = nkeys - 1;
  while (lo_k < hi_k) {
    const int mid = (lo_k + hi_k + 1) >> 1;
    if (gb.toff[mid] <= T) lo_k = mid; else hi_k = mid - 1;
  }
  const int key = lo_k;
  const int64_t v0 = (int64_t)gb.off[key] + 64ll * (T - gb.toff[key]);
  const int64_t vend = (int64_t)gb.off[key] + gb.hist[key];
  // voxels and their clipped boxes (wave 0, one lane per voxel slot); the
  // bounding box and the box volumes by wave reductions
  if (tid < LS_BV) {
    const int64_t i = v0 + tid;
    const int v = i < vend ? order[i] : -1;
    vid[tid] = v;
    unsigned long long vol = v >= 0 ? 1ull : 0ull;
    for (int p = 0; p < 4; ++p) {
      int lo = 1, hi = 0;  // empty box for padding lanes / unused parameters
      if (v >= 0 && p < P) {
        // cells clamped to the grid (as the coarse key is): the tile's
        // bounding box then spans at most 2^shift + 2r cells per parameter
        const int c = min(max(cells[(int64_t)v * P + p], 0), g.dims[p] - 1);
        lo = max(c - r, 0);
        hi = min(c + r, g.dims[p] - 1);
        vol *= (unsigned long long)(hi - lo + 1);
      } else if (p >= P) {
        lo = 0;
        hi = 0;
      }
      vlo[tid][p] = lo;
      vhi[tid][p] = hi;
      int mlo = v >= 0 ? lo : (1 << 30), mhi = v >= 0 ? hi : -1;
      for (int o = 32; o > 0; o >>= 1) {
        mlo = min(mlo, __shfl_xor(mlo, o, 64));
        mhi = max(mhi, __shfl_xor(mhi, o, 64));
      }
      if (tid == 0) {
        if (p >= P || mhi < mlo) {
          mlo = 0;
          mhi = 0;
        }
        blo[p] = mlo;
        bdim[p] = mhi - mlo + 1;
        const unsigned long long m = 0x100000000ull / (unsigned long long)(mhi - mlo + 1);
        bmag[p] = m > 0xFFFFFFFFull ? 0xFFFFFFFFu : (unsigned int)m;
      }
    }
    if (boxsum && at == 0) {
      for (int o = 32; o > 0; o >>= 1) vol += __shfl_xor(vol, o, 64);
      if (tid == 0) atomicAdd(boxsum, vol);
    }
  }
  __syncthreads();
  int64_t natoms = 1;
  for (int p = 0; p < P; ++p) natoms *= bdim[p];
  const int ntiles = (int)((natoms + LS_BA - 1) / LS_BA);
  if (at >= ntiles) return;  // block-uniform: bdim is shared
  const int nkc = pitch / BK;
  const int nq = nkc;
  if (tid == 0 && work) atomicAdd(work, (unsigned long long)LS_BA);

  // bounding-box element e -> dictionary index (-1 beyond the box) and its
  // grid coordinates; natoms < 2^31, and floor(e * m / 2^32) with
  // m = floor(2^32 / d) is the quotient or one less, fixed by one correction
  struct AtomPos {
    int j;
    int c[4];
  };
  auto atom_of = [&](int e) -> AtomPos {
    AtomPos a{-1, {0, 0, 0, 0}};
    if ((int64_t)e >= natoms) return a;
    unsigned int rem = (unsigned int)e;
#pragma unroll
    for (int p = 3; p >= 0; --p) {
      if (p < P) {
        const unsigned int d = (unsigned int)bdim[p];
        unsigned int q = __umulhi(rem, bmag[p]);
        unsigned int rr = rem - q * d;
        if (rr >= d) {
          ++q;
          rr -= d;
        }
        a.c[p] = blo[p] + (int)rr;
        rem = q;
      }
    }
    int j = 0;
#pragma unroll
    for (int p = 0; p < 4; ++p)
      if (p < P) j = j * g.dims[p] + a.c[p];
    a.j = j;
    return a;
  };

  // Loader.  FP32: atom rows lr and lr + 64, voxel row lr; 4 floats at lc.
  // X3: a stage row is LS_XC chunks [hi 32 | lo 32] = 8 LS_XC pieces of 16 B;
  // piece = tid % (8 LS_XC) picks the chunk (piece / 8), the plane
  // (piece / 4 % 2) and the 8-element slice (piece % 4); atom rows
  // tid / (8 LS_XC) + ASTEP i, voxel rows likewise.
  constexpr int PPR = 8 * LS_XC;  // X3 pieces per stage row
  const int piece = tid % PPR;
  const int lr = X3 ? (tid / PPR) : (tid >> 2);
  const int lc = X3 ? (piece >> 3) * 64 + ((piece >> 2) & 1) * 32 + (piece & 3) * 8 : (tid & 3) * 4;  // LDS column
  const int gc = lc;                                             // offset in the stage's row segment
  constexpr int KSTRIDE = X3 ? 2 * LS_BKX : LS_BK32;             // row elements per stage
  constexpr int ASTEP = X3 ? 256 / PPR : 64, ZSTEP = X3 ? 256 / PPR : 32;
  constexpr int NA = X3 ? LS_BA / ASTEP : 2, NZ = X3 ? LS_BV / ZSTEP : 1;
  constexpr int LD = X3 ? LS_LDX : LS_LD32;
  constexpr int RSTRIDE = X3 ? 2 : 1;  // row pitch in units of `pitch`
  int ja[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) ja[i] = -1;
  int zv[NZ];
#pragma unroll
  for (int i = 0; i < NZ; ++i) {
    const int row = lr + ZSTEP * i;
    zv[i] = row < LS_BV ? vid[row] : -1;
  }
  uint4 ra[NA], rz[NZ];
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  typedef const __attribute__((address_space(1))) u32x4 *gptr;
  const int64_t rowb = (int64_t)RSTRIDE * pitch * EB;  // bytes per operand row
  const unsigned char *Db = static_cast<const unsigned char *>(Dv);
  const unsigned char *Zb = static_cast<const unsigned char *>(Zv);
  // rows outside the tile load row 0 (always valid) and are zeroed after the
  // load, so every load is unconditional
  auto gload = [&](int q) {
    const int t = at, kc = q;
    if (kc == 0) {
#pragma unroll
      for (int i = 0; i < NA; ++i) ja[i] = atom_of(t * LS_BA + lr + ASTEP * i).j;
    }
    const int64_t kb = ((int64_t)kc * KSTRIDE + gc) * EB;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const u32x4 x = *(gptr)(Db + (int64_t)max(ja[i], 0) * rowb + kb);
      ra[i] = ja[i] >= 0 ? make_uint4(x.x, x.y, x.z, x.w) : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int i = 0; i < NZ; ++i) {
      const u32x4 x = *(gptr)(Zb + (int64_t)max(zv[i], 0) * rowb + kb);
      rz[i] = zv[i] >= 0 ? make_uint4(x.x, x.y, x.z, x.w) : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto sstore = [&](int buf) {
    unsigned char *As = smem + (size_t)buf * A_ELEMS * EB;
    unsigned char *Zs = smem + (size_t)(NBUF * A_ELEMS + buf * Z_ELEMS) * EB;
#pragma unroll
    for (int i = 0; i < NA; ++i)
      *reinterpret_cast<uint4 *>(As + ((lr + ASTEP * i) * LD + lc) * EB) = ra[i];
#pragma unroll
    for (int i = 0; i < NZ; ++i) {
      const int row = lr + ZSTEP * i;
      if (row < LS_BV) *reinterpret_cast<uint4 *>(Zs + (row * LD + lc) * EB) = rz[i];
    }
  };

  f32x16 acc[2];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[b][i] = 0.f;
  float best[2] = {-INFINITY, -INFINITY};
  int bidx[2] = {-1, -1};

  if (nq > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  for (int q = 0; q < nq; ++q) {
    const int buf = NBUF == 2 ? (q & 1) : 0;
    const int t = at, kc = q;
    if (kc == 0 && tid < LS_BA) {
      const AtomPos a = atom_of(t * LS_BA + tid);
      aj[tid] = a.j;
      acoord[tid][0] = a.c[0];
      acoord[tid][1] = a.c[1];
      acoord[tid][2] = a.c[2];
      acoord[tid][3] = a.c[3];
    }
    if (q + 1 < nq) gload(q + 1);
    if constexpr (X3) {
      const __bf16 *As = reinterpret_cast<const __bf16 *>(smem) + (size_t)buf * A_ELEMS;
      const __bf16 *Zs = reinterpret_cast<const __bf16 *>(smem) + (size_t)(NBUF * A_ELEMS + buf * Z_ELEMS);
#pragma unroll
      for (int ks = 0; ks < 2 * LS_XC; ++ks) {
        const int ko = (ks >> 1) * 64 + (ks & 1) * 16 + h * 8;  // hi of chunk ks/2, half ks%2
        const __bf16 *ar = As + (wave * 32 + l32) * LS_LDX + ko;
        const bf16x8 ahi = *reinterpret_cast<const bf16x8 *>(ar);
        const bf16x8 alo = *reinterpret_cast<const bf16x8 *>(ar + 32);
#pragma unroll
        for (int nv = 0; nv < 2; ++nv) {
          const __bf16 *zr = Zs + (nv * 32 + l32) * LS_LDX + ko;
          const bf16x8 zhi = *reinterpret_cast<const bf16x8 *>(zr);
          const bf16x8 zlo = *reinterpret_cast<const bf16x8 *>(zr + 32);
          acc[nv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, zhi, acc[nv], 0, 0, 0);
          acc[nv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, zlo, acc[nv], 0, 0, 0);
          acc[nv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, zhi, acc[nv], 0, 0, 0);
        }
      }
    } else {
      const float *As = reinterpret_cast<const float *>(smem) + (size_t)buf * A_ELEMS;
      const float *Zs = reinterpret_cast<const float *>(smem) + (size_t)(NBUF * A_ELEMS + buf * Z_ELEMS);
      float af[8], zf[2][8];
      {
        const float *src = As + (wave * 32 + l32) * LS_LD32 + h * 8;
        const float4 x0 = *reinterpret_cast<const float4 *>(src);
        const float4 x1 = *reinterpret_cast<const float4 *>(src + 4);
        af[0] = x0.x; af[1] = x0.y; af[2] = x0.z; af[3] = x0.w;
        af[4] = x1.x; af[5] = x1.y; af[6] = x1.z; af[7] = x1.w;
      }
#pragma unroll
      for (int nv = 0; nv < 2; ++nv) {
        const float *src = Zs + (nv * 32 + l32) * LS_LD32 + h * 8;
        const float4 x0 = *reinterpret_cast<const float4 *>(src);
        const float4 x1 = *reinterpret_cast<const float4 *>(src + 4);
        zf[nv][0] = x0.x; zf[nv][1] = x0.y; zf[nv][2] = x0.z; zf[nv][3] = x0.w;
        zf[nv][4] = x1.x; zf[nv][5] = x1.y; zf[nv][6] = x1.z; zf[nv][7] = x1.w;
      }
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int nv = 0; nv < 2; ++nv)
          acc[nv] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[s], zf[nv][s], acc[nv], 0, 0, 0);
    }
    if (kc == nkc - 1) {
      if (nkc == 1) __syncthreads();  // aj / acoord written this iteration
#pragma unroll
      for (int nv = 0; nv < 2; ++nv) {
        const int c = nv * 32 + l32;
        int lo[4], hi[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          lo[p] = vlo[c][p];
          hi[p] = vhi[c][p];
        }
        const int vv = COLLECT ? vid[c] : -1;
        const float line = (COLLECT && vv >= 0) ? col.thr[vv] : INFINITY;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int row = wave * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
          const int j = aj[row];
          const float sc = acc[nv][i];
          bool in = j >= 0;
#pragma unroll
          for (int p = 0; p < 4; ++p) in = in && acoord[row][p] >= lo[p] && acoord[row][p] <= hi[p];
          if constexpr (COLLECT) {
            if (in && sc >= line) {
              const unsigned int pos = atomicAdd(&col.count[vv], 1u);
              if ((int)pos < col.ccap) col.cand[(int64_t)vv * col.ccap + pos] = j;
            }
          } else if (in && sc > best[nv]) {
            best[nv] = sc;
            bidx[nv] = j;
          }
        }
      }
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[b][i] = 0.f;
    }
    if (NBUF == 1) __syncthreads();  // every wave is done with the single buffer
    if (q + 1 < nq) sstore(NBUF == 2 ? buf ^ 1 : 0);
    __syncthreads();
  }
  if constexpr (COLLECT) return;  // the candidates are already written
#pragma unroll
  for (int nv = 0; nv < 2; ++nv) {
    const float ps = __shfl_xor(best[nv], 32, 64);
    const int pj = __shfl_xor(bidx[nv], 32, 64);
    if (lbetter(ps, pj, best[nv], bidx[nv])) {
      best[nv] = ps;
      bidx[nv] = pj;
    }
    if (h == 0) {
      red_s[wave][nv * 32 + l32] = best[nv];
      red_j[wave][nv * 32 + l32] = bidx[nv];
    }
  }
  __syncthreads();
  if (tid < LS_BV) {
    float bs = red_s[0][tid];
    int bj = red_j[0][tid];
    for (int w = 1; w < 4; ++w)
      if (lbetter(red_s[w][tid], red_j[w][tid], bs, bj)) {
        bs = red_s[w][tid];
        bj = red_j[w][tid];
      }
    const int v = vid[tid];
    if (v >= 0 && bj >= 0) atomicMax(&bestkey[v], pack_best(bs, bj));
  }
  };
  item(blockIdx.x);
}

void launch_local_score(const void *D, const void *Zp, int pitch, bool x3, const int32_t *order, int64_t cnt,
                        GroupBufs gb, int nkeys, const int32_t *cells, int P, const GridDims &g, int r, int shift,
                        unsigned long long *bestkey, unsigned long long *work, unsigned long long *boxsum,
                        hipStream_t s, const LocalCollect *collect) {
  if (cnt <= 0) return;
  // tiles = sum_k ceil(hist[k]/64) <= ceil(cnt/64) + min(nkeys, cnt); a tile's
  // voxels share a coarse cell, so its bounding box spans at most 2^shift + 2r
  // cells per parameter: max_at atom tiles; surplus blocks exit at once
  const int64_t tiles = (cnt + LS_BV - 1) / LS_BV + std::min<int64_t>(nkeys, cnt);
  int64_t bbox = 1;
  for (int p = 0; p < P; ++p) bbox *= std::min<int64_t>(g.dims[p], (1 << shift) + 2 * (int64_t)r);
  const int max_at = (int)((bbox + LS_BA - 1) / LS_BA);
  const int64_t blocks = (tiles + 8 * LS_RUN - 1) / (8 * LS_RUN) * (8 * LS_RUN) * max_at;  // whole runs on all XCDs
  const LocalCollect lc = collect ? *collect : LocalCollect{};
  if (x3 && collect)
    hipLaunchKernelGGL((k_local_score<true, true>), dim3((unsigned)blocks), dim3(256), 0, s, D, Zp, pitch, order, gb,
                       nkeys, cells, P, g, r, max_at, bestkey, work, boxsum, lc);
  else if (x3)
    hipLaunchKernelGGL((k_local_score<true, false>), dim3((unsigned)blocks), dim3(256), 0, s, D, Zp, pitch, order,
                       gb, nkeys, cells, P, g, r, max_at, bestkey, work, boxsum, lc);
  else if (collect)
    hipLaunchKernelGGL((k_local_score<false, true>), dim3((unsigned)blocks), dim3(256), 0, s, D, Zp, pitch, order,
                       gb, nkeys, cells, P, g, r, max_at, bestkey, work, boxsum, lc);
  else
    hipLaunchKernelGGL((k_local_score<false, false>), dim3((unsigned)blocks), dim3(256), 0, s, D, Zp, pitch, order,
                       gb, nkeys, cells, P, g, r, max_at, bestkey, work, boxsum, lc);
}

// Non-expansive safeguard of the inexact projection: the previous iterate's
// atom (the warm index) competes with the local search's best under the same
// order (score, then lower index).  One wave per voxel, FP32 dot product in a
// fixed order.
__global__ __launch_bounds__(256) void k_warm_best(const int32_t *__restrict__ warm, int64_t n, int d,
                                                   const float *__restrict__ Zp, const float *__restrict__ Dhat,
                                                   int Kp, const float *__restrict__ znorm,
                                                   float *__restrict__ best_s, int32_t *__restrict__ best_j) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= n) return;
  const int w = warm[v];
  if (w < 0 || w >= d || !(znorm[v] > 0.f)) return;
  const float4 *z = reinterpret_cast<const float4 *>(Zp + v * Kp);
  const float4 *a = reinterpret_cast<const float4 *>(Dhat + (int64_t)w * Kp);
  float acc = 0.f;
  for (int k = lane; k < Kp / 4; k += 64) {
    const float4 x = z[k], y = a[k];
    acc = fmaf(x.x, y.x, acc);
    acc = fmaf(x.y, y.y, acc);
    acc = fmaf(x.z, y.z, acc);
    acc = fmaf(x.w, y.w, acc);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0 && lbetter(acc, w, best_s[v], best_j[v])) {
    best_s[v] = acc;
    best_j[v] = w;
  }
}

void launch_warm_best(const int32_t *warm, int64_t n, int d, const float *Zp, const float *Dhat, int Kp,
                      const float *znorm, float *best_s, int32_t *best_j, hipStream_t s) {
  if (n <= 0 || !warm) return;
  hipLaunchKernelGGL(k_warm_best, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, warm, n, d, Zp, Dhat, Kp, znorm,
                     best_s, best_j);
}

// ---------------------------------------------------------------------------
// re-centring and fallback selection
// ---------------------------------------------------------------------------
// For listed voxels: if the best atom lies on a box face that is not a grid
// edge, append the voxel to `recentre` and move its cell to the best atom.
// The best atom is best_j[v], or read from the voxel's best key where best_j
// is null (the keys then hold the current answers).
__global__ void k_face(const int32_t *__restrict__ list, int64_t cnt, const unsigned int *__restrict__ dcnt,
                       const int32_t *__restrict__ best_j, int32_t *__restrict__ cells, int P, GridDims g, int r,
                       int32_t *__restrict__ out, unsigned int *__restrict__ count,
                       unsigned long long *__restrict__ bkey, unsigned int *__restrict__ zero, int nzero) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nzero) zero[i] = 0u;
  if (i >= list_len(cnt, dcnt)) return;
  const int v = list[i];
  int j;
  if (best_j) {
    j = best_j[v];
  } else {
    float bs;
    unpack_best(bkey[v], bs, j);
  }
  if (j < 0) return;
  int sub[4];
  for (int p = P - 1; p >= 0; --p) {
    sub[p] = j % g.dims[p];
    j /= g.dims[p];
  }
  bool face = false;
  for (int p = 0; p < P; ++p) {
    const int c = cells[(int64_t)v * P + p];
    face = face || (sub[p] == c - r && sub[p] > 0) || (sub[p] == c + r && sub[p] < g.dims[p] - 1);
  }
  if (!face) return;
  for (int p = 0; p < P; ++p) cells[(int64_t)v * P + p] = sub[p];
  if (bkey) bkey[v] = 0ull;  // its best key is searched again around the new cell
  out[atomicAdd(count, 1u)] = v;
}

void launch_face(const int32_t *list, int64_t cnt, const int32_t *best_j, int32_t *cells, int P,
                 const GridDims &g, int r, int32_t *out, unsigned int *count, hipStream_t s,
                 const unsigned int *dcnt, unsigned long long *bkey, unsigned int *zero, int nzero) {
  const int64_t m = std::max<int64_t>(cnt, nzero);
  if (m <= 0) return;
  hipLaunchKernelGGL(k_face, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, list, cnt, dcnt, best_j,
                     cells, P, g, r, out, count, bkey, zero, nzero);
}

// Voxels with a finite, non-zero norm whose normalised correlation is below
// the threshold (or with no candidate) go to the exhaustive fallback list.
__device__ __forceinline__ bool needs_fallback(float bs, int32_t bj, float zn, float thr) {
  if (!(zn > 0.f)) return false;
  const float corr = bs / zn;
  return bj < 0 || !(corr >= thr);
}

__global__ void k_select_fallback(int64_t n, const float *__restrict__ best_s,
                                  const int32_t *__restrict__ best_j, const float *__restrict__ znorm,
                                  float thr, int32_t *__restrict__ out, unsigned int *__restrict__ count) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (needs_fallback(best_s[v], best_j[v], znorm[v], thr)) out[atomicAdd(count, 1u)] = (int32_t)v;
}

// Every voxel's best key unpacked (k_best_keys, mode 1, over all voxels) and,
// in the same pass, the fallback selection of k_select_fallback.
// With fin.idx, a voxel that does not fall back is finished here as well.
__global__ void k_best_select(int64_t n, const unsigned long long *__restrict__ keys, float *__restrict__ best_s,
                              int32_t *__restrict__ best_j, const float *__restrict__ znorm, float thr,
                              int32_t *__restrict__ out, unsigned int *__restrict__ count, FinishArgs fin) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  float bs;
  int32_t bj;
  unpack_best(keys[v], bs, bj);
  best_s[v] = bs;
  best_j[v] = bj;
  if (needs_fallback(bs, bj, znorm[v], thr))
    out[atomicAdd(count, 1u)] = (int32_t)v;
  else if (fin.idx)
    finish_single(v, bs, bj, fin);
}

void launch_best_select(int64_t n, const unsigned long long *keys, float *best_s, int32_t *best_j,
                        const float *znorm, float thr, int32_t *out, unsigned int *count, hipStream_t s,
                        const FinishArgs *fin) {
  if (n <= 0) return;
  const FinishArgs f = fin ? *fin : FinishArgs{};
  hipLaunchKernelGGL(k_best_select, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, keys, best_s, best_j,
                     znorm, thr, out, count, f);
}

void launch_select_fallback(int64_t n, const float *best_s, const int32_t *best_j, const float *znorm,
                            float thr, int32_t *out, unsigned int *count, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_select_fallback, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, best_s,
                     best_j, znorm, thr, out, count);
}

// rows[i] = Zp[list[i]] (zero rows up to cnt_pad)
__global__ void k_gather_rows(const float *__restrict__ Zp, int Kp, const int32_t *__restrict__ list,
                              int64_t cnt, int64_t cnt_pad, float *__restrict__ out) {
  const int64_t i = blockIdx.x;
  if (i >= cnt_pad) return;
  const float4 *src = i < cnt ? reinterpret_cast<const float4 *>(Zp + (int64_t)list[i] * Kp) : nullptr;
  float4 *dst = reinterpret_cast<float4 *>(out + i * Kp);
  for (int k = threadIdx.x; k < Kp / 4; k += blockDim.x)
    dst[k] = src ? src[k] : make_float4(0.f, 0.f, 0.f, 0.f);
}

void launch_gather_rows(const float *Zp, int Kp, const int32_t *list, int64_t cnt, int64_t cnt_pad,
                        float *out, hipStream_t s) {
  if (cnt_pad <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)cnt_pad), dim3(256), 0, s, Zp, Kp, list, cnt,
                     cnt_pad, out);
}

// Rows list[i] of Zp (pitch Kp floats) into out[i] for i < the device count,
// zero rows up to the next whole voxel tile of the split-BF16 filter; a
// grid-stride loop, so the grid does not depend on the count.
__global__ void k_gather_rows_dev(const float *__restrict__ Zp, int Kp, const int32_t *__restrict__ list,
                                  int64_t cap, const unsigned int *__restrict__ dcnt, float *__restrict__ out,
                                  unsigned long long *__restrict__ total) {
  const int64_t c = min(cap, (int64_t)*dcnt);
  if (total && blockIdx.x == 0 && threadIdx.x == 0) *total += *dcnt;
  const int64_t rows = (c + kX3VoxTile - 1) / kX3VoxTile * kX3VoxTile;
  for (int64_t i = blockIdx.x; i < rows; i += gridDim.x) {
    const float4 *src = i < c ? reinterpret_cast<const float4 *>(Zp + (int64_t)list[i] * Kp) : nullptr;
    float4 *dst = reinterpret_cast<float4 *>(out + i * Kp);
    for (int k = threadIdx.x; k < Kp / 4; k += blockDim.x)
      dst[k] = src ? src[k] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

void launch_gather_rows_dev(const float *Zp, int Kp, const int32_t *list, int64_t cap, const unsigned int *dcnt,
                            float *out, hipStream_t s, unsigned long long *total) {
  if (cap <= 0) return;
  hipLaunchKernelGGL(k_gather_rows_dev, dim3(1024), dim3(256), 0, s, Zp, Kp, list, cap, dcnt, out, total);
}

// total += *count (one thread)
__global__ void k_add_count(unsigned long long *__restrict__ total, const unsigned int *__restrict__ count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *total += *count;
}

void launch_add_count(unsigned long long *total, const unsigned int *count, hipStream_t s) {
  hipLaunchKernelGGL(k_add_count, dim3(1), dim3(64), 0, s, total, count);
}

// best[list[i]] = merged exhaustive result i (splits merged in order).  With
// a device count (dcnt), cnt is the capacity and the split count and part
// stride are those of the device-sized split-BF16 filter (ntiles atom tiles).
__global__ void k_scatter_best(const int32_t *__restrict__ list, int64_t cnt,
                               const float *__restrict__ part_s, const int *__restrict__ part_j,
                               int splits, float *__restrict__ best_s, int32_t *__restrict__ best_j,
                               const unsigned int *__restrict__ dcnt, int ntiles, FinishArgs fin) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c = cnt;
  const int64_t stride = cnt;
  if (dcnt) {
    c = min(cnt, (int64_t)*dcnt);
    splits = x3_device_splits((int)((c + kX3VoxTile - 1) / kX3VoxTile), ntiles);
  }
  if (i >= c) return;
  float bs = -INFINITY;
  int bj = -1;
  for (int s = 0; s < splits; ++s) {
    const float ps = part_s[(int64_t)s * stride + i];
    const int pj = part_j[(int64_t)s * stride + i];
    if (pj >= 0 && lbetter(ps, pj, bs, bj)) {
      bs = ps;
      bj = pj;
    }
  }
  const int v = list[i];
  best_s[v] = bs;
  best_j[v] = bj;
  if (fin.idx) finish_single(v, bs, bj, fin);
}

void launch_scatter_best(const int32_t *list, int64_t cnt, const float *part_s, const int *part_j,
                         int splits, float *best_s, int32_t *best_j, hipStream_t s, const unsigned int *dcnt,
                         int ntiles, const FinishArgs *fin) {
  if (cnt <= 0) return;
  const FinishArgs f = fin ? *fin : FinishArgs{};
  hipLaunchKernelGGL(k_scatter_best, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, list, cnt,
                     part_s, part_j, splits, best_s, best_j, dcnt, ntiles, f);
}

// Start of a learned call (learned_prep_at for every thread).
__global__ void k_learned_prep(LearnedPrep p, int64_t n) {
  learned_prep_at((int64_t)blockIdx.x * blockDim.x + threadIdx.x, p, n);
}

void launch_learned_prep(const LearnedPrep &p, int64_t n, hipStream_t s) {
  const int64_t m = std::max<int64_t>(n, std::max(p.nz, p.nz2));
  if (m > 0) hipLaunchKernelGGL(k_learned_prep, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, p, n);
}

__global__ void k_iota(int32_t *x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = (int32_t)i;
}

void launch_iota(int32_t *x, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n);
}

}  // namespace mrf

namespace mrf {

__global__ void k_mark(const int32_t *__restrict__ list, int64_t cnt, const unsigned int *__restrict__ dcnt,
                       int32_t *__restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < list_len(cnt, dcnt)) flags[list[i]] = 1;
}

void launch_mark(const int32_t *list, int64_t cnt, int32_t *flags, hipStream_t s, const unsigned int *dcnt) {
  if (cnt > 0)
    hipLaunchKernelGGL(k_mark, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, list, cnt, dcnt, flags);
}

}  // namespace mrf
