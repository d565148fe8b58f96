// Matched-filter kernels for gfx950: voxel packing, exhaustive FP32 MFMA
// scoring with a fused argmax, split merge + rescaling (eq. exactP,
// eq. exactPs), and the write of gamma_v D_j* back into image layout.
#include <cfloat>

#include "k_split.h"
#include "k_finish.h"
#include "k_topk.h"
#include "mrf_internal.h"

namespace mrf {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// packing
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum_f64(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// One wave per voxel row (voxel-major input [n][L] complex64).  Zp may be
// null when only the split-BF16 rows are wanted.
__global__ __launch_bounds__(256) void k_pack_voxel_major(const float2 *__restrict__ Z, int64_t n,
                                                          int64_t n_pad, int L, int real_atoms,
                                                          int Kp, float *__restrict__ Zp,
                                                          float *__restrict__ znorm,
                                                          unsigned long long *counters,
                                                          const float2 *__restrict__ vphase,
                                                          uint16_t *__restrict__ zx3, int Kx,
                                                          float *__restrict__ inv) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= n_pad) return;
  float *row = Zp ? Zp + v * Kp : nullptr;
  uint16_t *xrow = zx3 ? zx3 + v * 2 * Kx : nullptr;
  const int K = real_atoms ? L : 2 * L;
  if (v >= n) {
    if (row)
      for (int k = lane; k < Kp; k += 64) row[k] = 0.f;
    if (xrow)
      for (int k = lane; k < 2 * Kx; k += 64) xrow[k] = 0;
    return;
  }
  const float2 *z = Z + v * (int64_t)L;
  const float2 e = vphase ? vphase[v] : make_float2(1.f, 0.f);  // rotate by conj(e)
  double acc = 0.0;
  for (int t = lane; t < L; t += 64) {
    const float2 z0 = z[t];
    const float2 a = vphase ? make_float2(e.x * z0.x + e.y * z0.y, e.x * z0.y - e.y * z0.x) : z0;
    acc += (double)a.x * a.x + (double)a.y * a.y;
    if (row) {
      if (real_atoms) {
        row[t] = a.x;
      } else {
        row[2 * t] = a.x;
        row[2 * t + 1] = a.y;
      }
    }
    if (xrow) {  // split BF16 row, fused
      if (real_atoms) {
        uint16_t h, l;
        split_bf16(a.x, h, l);
        xrow[split_off(t)] = h;
        xrow[split_off(t) + 32] = l;
      } else {
        uint16_t h0, l0, h1, l1;
        split_bf16(a.x, h0, l0);
        split_bf16(a.y, h1, l1);
        const int64_t o = split_off(2 * t);
        *reinterpret_cast<uint32_t *>(xrow + o) = h0 | ((uint32_t)h1 << 16);
        *reinterpret_cast<uint32_t *>(xrow + o + 32) = l0 | ((uint32_t)l1 << 16);
      }
    }
  }
  if (row)
    for (int k = K + lane; k < Kp; k += 64) row[k] = 0.f;
  if (xrow)
    for (int k = K + lane; k < Kx; k += 64) {
      xrow[split_off(k)] = 0;
      xrow[split_off(k) + 32] = 0;
    }
  acc = wave_sum_f64(acc);
  if (lane == 0) {
    const bool fin = isfinite(acc);
    const float zn = fin ? (float)sqrt(acc) : -1.f;
    znorm[v] = zn;
    if (inv) inv[v] = zn > 0.f ? 1.f / zn : 0.f;  // as k_inv_norm
    if (counters) {  // counted only where the caller reads the counts
      if (!fin) atomicAdd(&counters[1], 1ull);
      else if (acc == 0.0) atomicAdd(&counters[0], 1ull);
    }
  }
}

// The same with two complex values per lane and step, for even L and a
// 16-byte aligned Z: 16-byte loads and FP32 stores, 8-byte split stores.
__global__ __launch_bounds__(256) void k_pack_voxel_major2(const float2 *__restrict__ Z, int64_t n,
                                                           int64_t n_pad, int L, int real_atoms,
                                                           int Kp, float *__restrict__ Zp,
                                                           float *__restrict__ znorm,
                                                           unsigned long long *counters,
                                                           const float2 *__restrict__ vphase,
                                                           uint16_t *__restrict__ zx3, int Kx,
                                                           float *__restrict__ inv) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= n_pad) return;
  float *row = Zp ? Zp + v * Kp : nullptr;
  uint16_t *xrow = zx3 ? zx3 + v * 2 * Kx : nullptr;
  const int K = real_atoms ? L : 2 * L;
  if (v >= n) {
    if (row)
      for (int k = lane; k < Kp; k += 64) row[k] = 0.f;
    if (xrow)
      for (int k = lane; k < 2 * Kx; k += 64) xrow[k] = 0;
    return;
  }
  const float4 *z = reinterpret_cast<const float4 *>(Z + v * (int64_t)L);
  const float2 e = vphase ? vphase[v] : make_float2(1.f, 0.f);  // rotate by conj(e)
  double acc = 0.0;
  for (int u = lane; u < L / 2; u += 64) {  // complex values 2u and 2u + 1
    const float4 q = z[u];
    float2 a0 = make_float2(q.x, q.y), a1 = make_float2(q.z, q.w);
    if (vphase) {
      a0 = make_float2(e.x * q.x + e.y * q.y, e.x * q.y - e.y * q.x);
      a1 = make_float2(e.x * q.z + e.y * q.w, e.x * q.w - e.y * q.z);
    }
    acc += (double)a0.x * a0.x + (double)a0.y * a0.y;
    acc += (double)a1.x * a1.x + (double)a1.y * a1.y;
    if (real_atoms) {
      if (row) *reinterpret_cast<float2 *>(row + 2 * u) = make_float2(a0.x, a1.x);
      if (xrow) {  // columns 2u, 2u + 1 share a 32-column chunk
        uint16_t h0, l0, h1, l1;
        split_bf16(a0.x, h0, l0);
        split_bf16(a1.x, h1, l1);
        const int64_t o = split_off(2 * u);
        *reinterpret_cast<uint32_t *>(xrow + o) = h0 | ((uint32_t)h1 << 16);
        *reinterpret_cast<uint32_t *>(xrow + o + 32) = l0 | ((uint32_t)l1 << 16);
      }
    } else {
      if (row) *reinterpret_cast<float4 *>(row + 4 * u) = make_float4(a0.x, a0.y, a1.x, a1.y);
      if (xrow) {  // columns 4u .. 4u + 3 share a 32-column chunk
        uint16_t h[4], l[4];
        split_bf16(a0.x, h[0], l[0]);
        split_bf16(a0.y, h[1], l[1]);
        split_bf16(a1.x, h[2], l[2]);
        split_bf16(a1.y, h[3], l[3]);
        const int64_t o = split_off(4 * u);
        *reinterpret_cast<uint2 *>(xrow + o) =
            make_uint2(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16));
        *reinterpret_cast<uint2 *>(xrow + o + 32) =
            make_uint2(l[0] | ((uint32_t)l[1] << 16), l[2] | ((uint32_t)l[3] << 16));
      }
    }
  }
  if (row)
    for (int k = K + lane; k < Kp; k += 64) row[k] = 0.f;
  if (xrow)
    for (int k = K + lane; k < Kx; k += 64) {
      xrow[split_off(k)] = 0;
      xrow[split_off(k) + 32] = 0;
    }
  acc = wave_sum_f64(acc);
  if (lane == 0) {
    const bool fin = isfinite(acc);
    const float zn = fin ? (float)sqrt(acc) : -1.f;
    znorm[v] = zn;
    if (inv) inv[v] = zn > 0.f ? 1.f / zn : 0.f;  // as k_inv_norm
    if (counters) {  // counted only where the caller reads the counts
      if (!fin) atomicAdd(&counters[1], 1ull);
      else if (acc == 0.0) atomicAdd(&counters[0], 1ull);
    }
  }
}

// 64 voxels per block; frame tiles of 16 staged in LDS for the transpose.
template <bool HAS_G>
__global__ __launch_bounds__(256) void k_pack_frame_major(const float2 *__restrict__ X,
                                                          const float2 *__restrict__ G, float mu,
                                                          int64_t n, int64_t n_pad, int64_t npix,
                                                          int L, int real_atoms, int Kp,
                                                          float *__restrict__ Zp,
                                                          float *__restrict__ znorm,
                                                          unsigned long long *counters,
                                                          const float2 *__restrict__ vphase,
                                                          uint16_t *__restrict__ zx3, int Kx) {
  __shared__ float2 tile[16][65];
  __shared__ double red[4][64];
  const int tid = threadIdx.x;
  const int vi = tid & 63, fi = tid >> 6;
  const int64_t v0 = (int64_t)blockIdx.x * 64;
  const int64_t v = v0 + vi;
  const bool valid = v < n;
  const int64_t sl = valid ? v / npix : 0;
  const int64_t p = valid ? v - sl * npix : 0;
  const float2 ev = (vphase && valid) ? vphase[v] : make_float2(1.f, 0.f);  // rotate by conj(ev)
  double acc = 0.0;
  // writer mapping: 4 threads per voxel row, each 4 frames
  const int wv = tid >> 2, wp = tid & 3;
  const int64_t vw = v0 + wv;
  for (int t0 = 0; t0 < L; t0 += 16) {
#pragma unroll
    for (int f = fi; f < 16; f += 4) {
      const int t = t0 + f;
      float2 z = make_float2(0.f, 0.f);
      if (valid && t < L) {
        const int64_t e = (sl * L + t) * npix + p;
        z = X[e];
        if (HAS_G) {
          const float2 g = G[e];
          z.x = z.x - mu * g.x;
          z.y = z.y - mu * g.y;
        }
        if (vphase) z = make_float2(ev.x * z.x + ev.y * z.y, ev.x * z.y - ev.y * z.x);
        acc += (double)z.x * z.x + (double)z.y * z.y;
      }
      tile[f][vi] = z;
    }
    __syncthreads();
    if (vw < n_pad) {
      float *row = Zp + vw * Kp;
      uint16_t *xrow = zx3 ? zx3 + vw * 2 * Kx : nullptr;
      if (real_atoms) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int t = t0 + wp * 4 + q;
          if (t < L) {
            const float x = tile[wp * 4 + q][wv].x;
            row[t] = x;
            if (xrow) {
              uint16_t h, l;
              split_bf16(x, h, l);
              xrow[split_off(t)] = h;
              xrow[split_off(t) + 32] = l;
            }
          }
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int t = t0 + wp * 4 + q;
          if (t < L) {
            const float2 z = tile[wp * 4 + q][wv];
            *reinterpret_cast<float2 *>(row + 2 * t) = z;
            if (xrow) {
              uint16_t h0, l0, h1, l1;
              split_bf16(z.x, h0, l0);
              split_bf16(z.y, h1, l1);
              const int64_t o = split_off(2 * t);
              *reinterpret_cast<uint32_t *>(xrow + o) = h0 | ((uint32_t)h1 << 16);
              *reinterpret_cast<uint32_t *>(xrow + o + 32) = l0 | ((uint32_t)l1 << 16);
            }
          }
        }
      }
    }
    __syncthreads();
  }
  // zero the padding columns
  const int K = real_atoms ? L : 2 * L;
  if (vw < n_pad) {
    float *row = Zp + vw * Kp;
    for (int k = K + wp; k < Kp; k += 4) row[k] = 0.f;
    if (zx3) {
      uint16_t *xrow = zx3 + vw * 2 * Kx;
      for (int k = K + wp; k < Kx; k += 4) {
        xrow[split_off(k)] = 0;
        xrow[split_off(k) + 32] = 0;
      }
    }
  }
  red[fi][vi] = acc;
  __syncthreads();
  if (fi == 0 && valid) {
    const double s = red[0][vi] + red[1][vi] + red[2][vi] + red[3][vi];
    const bool fin = isfinite(s);
    znorm[v] = fin ? (float)sqrt(s) : -1.f;
    if (counters) {  // counted only where the caller reads the counts
      if (!fin) atomicAdd(&counters[1], 1ull);
      else if (s == 0.0) atomicAdd(&counters[0], 1ull);
    }
  }
}

void launch_pack_voxel_major(const float2 *Z, int64_t n, int64_t n_pad, int L, int real_atoms,
                             int Kp, float *Zp, float *znorm, unsigned long long *counters,
                             hipStream_t s, const float2 *vphase, uint16_t *zx3, int Kx, float *inv) {
  const int64_t blocks = (n_pad + 3) / 4;
  if (L % 2 == 0 && (reinterpret_cast<uintptr_t>(Z) & 15) == 0 && Kp % 4 == 0)
    hipLaunchKernelGGL(k_pack_voxel_major2, dim3((unsigned)blocks), dim3(256), 0, s, Z, n, n_pad, L,
                       real_atoms, Kp, Zp, znorm, counters, vphase, zx3, Kx, inv);
  else
    hipLaunchKernelGGL(k_pack_voxel_major, dim3((unsigned)blocks), dim3(256), 0, s, Z, n, n_pad, L,
                       real_atoms, Kp, Zp, znorm, counters, vphase, zx3, Kx, inv);
}

void launch_pack_frame_major(const float2 *X, const float2 *G, float mu, int64_t n, int64_t n_pad,
                             int64_t npix, int L, int real_atoms, int Kp, float *Zp, float *znorm,
                             unsigned long long *counters, hipStream_t s, const float2 *vphase, uint16_t *zx3,
                             int Kx) {
  const int64_t blocks = (n_pad + 63) / 64;
  if (G)
    hipLaunchKernelGGL(k_pack_frame_major<true>, dim3((unsigned)blocks), dim3(256), 0, s, X, G,
                       mu, n, n_pad, npix, L, real_atoms, Kp, Zp, znorm, counters, vphase, zx3, Kx);
  else
    hipLaunchKernelGGL(k_pack_frame_major<false>, dim3((unsigned)blocks), dim3(256), 0, s, X,
                       nullptr, 0.f, n, n_pad, npix, L, real_atoms, Kp, Zp, znorm, counters, vphase, zx3, Kx);
}

// ---------------------------------------------------------------------------
// exhaustive FP32 scoring with a fused per-voxel epilogue
// ---------------------------------------------------------------------------
// Block tile: 128 atoms x 128 voxels, K chunks of 16, double-buffered LDS.
// Four waves in a 2 x 2 arrangement, each owning 64 atoms x 64 voxels as
// 2 x 2 MFMA 32x32x2 tiles.  Atoms are the MFMA rows (A operand) and voxels
// the columns (B operand), so each lane accumulates one voxel column and 16
// atom rows per tile, and atoms reach a lane in increasing index order.
// Epilogues (per voxel column, folded once per atom tile):
//   SC_TOP1    the running maximum in registers (a strict '>' keeps the
//              lowest index among equal scores);
//   SC_TOPK    the kCertK best (score, atom) pairs among those within
//              W_v = cw ||Z_v|| + wabs of the running maximum when they
//              arrive (W_v > twice the scores' error bound, so every atom the
//              exactness certificate needs is kept; the window makes
//              insertions rare);
//   SC_COLLECT every atom whose score reaches the voxel's threshold is
//              appended to its candidate list (the certificate's rescan).
// Work items (voxel tile, atom split) are dealt so all splits of a voxel tile
// share an XCD (blocks are dealt to the 8 XCDs round-robin) and its L2.  With
// the voxel count on the device (dcnt) a grid of a multiple of 8 blocks loops
// over the items the count implies.
constexpr int F_BA = 128, F_BV = 128, F_BK = 16, F_LDK = 20;

__device__ __forceinline__ bool better(float s1, int j1, float s0, int j0) {
  // (s1, j1) beats (s0, j0): higher score, or equal score with a lower valid index
  return (s1 > s0) || (s1 == s0 && j1 >= 0 && (j0 < 0 || j1 < j0));
}

// Atom splits of the FP32 filter for a device-side voxel count: about 2,048
// work items, at most 256 splits and one split per 128-atom tile (a rescan of
// a few voxel tiles still spreads over the whole chip).
__device__ __forceinline__ int f32_device_splits(int nvt, int ntiles) {
  const int nvt8 = (nvt + 7) / 8 * 8;
  const int s = nvt8 > 0 ? (2048 + nvt8 - 1) / nvt8 : 1;
  return max(1, min(s, min(ntiles, 256)));
}

struct CollectArgs {
  const float *thr;     // [cap] per-voxel threshold
  unsigned int *count;  // [cap] candidates found (may exceed ccap)
  int32_t *cand;        // [cap][ccap] atom indices, unordered
  int ccap;
};

template <int MODE>
__global__ __launch_bounds__(256, 2) void k_score_f32(const float *__restrict__ D,
                                                      const float *__restrict__ Zp, int d,
                                                      int ntiles_total, int64_t n, int nvt,
                                                      int Kp, int splits, int tiles_per_split,
                                                      float *__restrict__ part_s,
                                                      int *__restrict__ part_j, int64_t pstride,
                                                      const unsigned int *__restrict__ dcnt,
                                                      const int32_t *__restrict__ rowmap,
                                                      CollectArgs col, const float *__restrict__ znorm,
                                                      float cw, float wabs) {
  int64_t nvox = n;
  int nvt_w = nvt, nsplit = splits, tps = tiles_per_split;
  if (dcnt) {
    nvox = min(n, (int64_t)*dcnt);
    nvt_w = (int)((nvox + F_BV - 1) / F_BV);
    nsplit = f32_device_splits(nvt_w, ntiles_total);
    tps = (ntiles_total + nsplit - 1) / nsplit;
  }
  const int64_t nwork = (int64_t)((nvt_w + 7) / 8 * 8) * nsplit;

  __shared__ float As[2][F_BA][F_LDK];
  __shared__ float Zs[2][F_BV][F_LDK];

  for (int64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int xcd = (int)(w & 7);
    const int64_t local = w >> 3;
    const int split = (int)(local % nsplit);
    const int vt = (int)((local / nsplit) * 8 + xcd);
    if (vt >= nvt_w) continue;
    const int tb = split * tps;
    const int te = min(tb + tps, ntiles_total);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wa = wave >> 1, wv = wave & 1;
    const int h = lane >> 5, l32 = lane & 31;
    const int64_t v0 = (int64_t)vt * F_BV;
    const int nkc = Kp / F_BK;
    const int nq = te > tb ? (te - tb) * nkc : 0;

    const int lr = tid >> 2, lc = (tid & 3) * 4;
    // voxel rows of this thread's two loader rows: through the row map when
    // given (rows past the count read the first listed row; their results
    // are discarded)
    int64_t zr0 = v0 + lr, zr1 = v0 + lr + 64;
    if (rowmap) {
      zr0 = rowmap[zr0 < nvox ? zr0 : 0];
      zr1 = rowmap[zr1 < nvox ? zr1 : 0];
    }
    const float *zp0 = Zp + zr0 * Kp + lc, *zp1 = Zp + zr1 * Kp + lc;
    float4 ra0, ra1, rz0, rz1;
    auto gload = [&](int q) {
      const int tile = tb + q / nkc, kc = q - (q / nkc) * nkc;
      const float *a = D + (int64_t)(tile * F_BA + lr) * Kp + kc * F_BK + lc;
      ra0 = *reinterpret_cast<const float4 *>(a);
      ra1 = *reinterpret_cast<const float4 *>(a + (int64_t)64 * Kp);
      rz0 = *reinterpret_cast<const float4 *>(zp0 + kc * F_BK);
      rz1 = *reinterpret_cast<const float4 *>(zp1 + kc * F_BK);
    };
    auto sstore = [&](int buf) {
      *reinterpret_cast<float4 *>(&As[buf][lr][lc]) = ra0;
      *reinterpret_cast<float4 *>(&As[buf][lr + 64][lc]) = ra1;
      *reinterpret_cast<float4 *>(&Zs[buf][lr][lc]) = rz0;
      *reinterpret_cast<float4 *>(&Zs[buf][lr + 64][lc]) = rz1;
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
    float ls[2][kCertK];
    int lj[2][kCertK];
    float vthr[2] = {INFINITY, INFINITY};  // SC_COLLECT: the line; SC_TOPK: the insertion bar
    float win[2] = {0.f, 0.f};
    if (MODE == SC_TOPK) {
      topk_clear(ls[0], lj[0]);
      topk_clear(ls[1], lj[1]);
#pragma unroll
      for (int nv = 0; nv < 2; ++nv) {
        const int64_t v = v0 + wv * 64 + nv * 32 + l32;
        win[nv] = v < nvox ? cw * fmaxf(znorm[v], 0.f) + wabs : 0.f;
        vthr[nv] = -INFINITY;
      }
    }
    if (MODE == SC_COLLECT) {
#pragma unroll
      for (int nv = 0; nv < 2; ++nv) {
        const int64_t v = v0 + wv * 64 + nv * 32 + l32;
        if (v < nvox) vthr[nv] = col.thr[v];
      }
    }

    if (nq > 0) {
      gload(0);
      sstore(0);
    }
    __syncthreads();
    for (int q = 0; q < nq; ++q) {
      const int buf = q & 1;
      if (q + 1 < nq) gload(q + 1);
      float af[2][8], zf[2][8];
#pragma unroll
      for (int ma = 0; ma < 2; ++ma) {
        const float *src = &As[buf][wa * 64 + ma * 32 + l32][h * 8];
        const float4 x0 = *reinterpret_cast<const float4 *>(src);
        const float4 x1 = *reinterpret_cast<const float4 *>(src + 4);
        af[ma][0] = x0.x; af[ma][1] = x0.y; af[ma][2] = x0.z; af[ma][3] = x0.w;
        af[ma][4] = x1.x; af[ma][5] = x1.y; af[ma][6] = x1.z; af[ma][7] = x1.w;
      }
#pragma unroll
      for (int nv = 0; nv < 2; ++nv) {
        const float *src = &Zs[buf][wv * 64 + nv * 32 + l32][h * 8];
        const float4 x0 = *reinterpret_cast<const float4 *>(src);
        const float4 x1 = *reinterpret_cast<const float4 *>(src + 4);
        zf[nv][0] = x0.x; zf[nv][1] = x0.y; zf[nv][2] = x0.z; zf[nv][3] = x0.w;
        zf[nv][4] = x1.x; zf[nv][5] = x1.y; zf[nv][6] = x1.z; zf[nv][7] = x1.w;
      }
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int ma = 0; ma < 2; ++ma)
#pragma unroll
          for (int nv = 0; nv < 2; ++nv)
            acc[ma][nv] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[ma][s], zf[nv][s], acc[ma][nv], 0, 0, 0);

      const int kc = q % nkc;
      if (kc == nkc - 1) {
        // epilogue of one atom tile: 32 atom rows per voxel column
        const int abase = (tb + q / nkc) * F_BA + wa * 64;
#pragma unroll
        for (int nv = 0; nv < 2; ++nv) {
#pragma unroll
          for (int ma = 0; ma < 2; ++ma) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
              const int j = abase + ma * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
              const float sc = acc[ma][nv][i];
              if (MODE == SC_TOP1) {
                if (j < d && sc > best[nv]) {  // NaN never wins
                  best[nv] = sc;
                  bidx[nv] = j;
                }
              } else if (MODE == SC_TOPK) {
                if (j < d && sc > vthr[nv]) {
                  topk_push_ordered(ls[nv], lj[nv], sc, j);
                  vthr[nv] = fmaxf(ls[nv][kCertK - 1], ls[nv][0] - win[nv]);
                }
              } else {
                const int64_t v = v0 + wv * 64 + nv * 32 + l32;
                if (j < d && v < nvox && sc >= vthr[nv]) {
                  const unsigned int pos = atomicAdd(&col.count[v], 1u);
                  if ((int)pos < col.ccap) col.cand[v * col.ccap + pos] = j;
                }
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
    if (MODE == SC_COLLECT) continue;  // the candidates are already written

    // combine the two half-waves (rows 4h..4h+3 of each 8-row group), then
    // the two atom halves of the block (wa = 0, 1) through LDS
    if (MODE == SC_TOP1) {
#pragma unroll
      for (int nv = 0; nv < 2; ++nv) {
        const float ps = __shfl_xor(best[nv], 32, 64);
        const int pj = __shfl_xor(bidx[nv], 32, 64);
        if (better(ps, pj, best[nv], bidx[nv])) {
          best[nv] = ps;
          bidx[nv] = pj;
        }
      }
      float *rs = &As[0][0][0];
      int *rj = reinterpret_cast<int *>(&Zs[0][0][0]);
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
          const float ps = rs[c];
          const int pj = rj[c];
          // equal scores resolve to the lower atom index
          if (better(ps, pj, best[nv], bidx[nv])) {
            best[nv] = ps;
            bidx[nv] = pj;
          }
          const int64_t v = v0 + c;
          if (v < nvox) {
            part_s[(int64_t)split * pstride + v] = best[nv];
            part_j[(int64_t)split * pstride + v] = bidx[nv];
          }
        }
      }
    } else {
#pragma unroll
      for (int nv = 0; nv < 2; ++nv) topk_merge_xor(ls[nv], lj[nv], 32);
      // 128 voxel columns x kCertK pairs fit in the stage buffers
      float *rs = &As[0][0][0];
      int *rj = reinterpret_cast<int *>(&Zs[0][0][0]);
      static_assert(F_BV * kCertK <= 2 * F_BA * F_LDK, "LDS exchange");
      if (wa == 1 && h == 0) {
#pragma unroll
        for (int nv = 0; nv < 2; ++nv) {
          const int c = wv * 64 + nv * 32 + l32;
#pragma unroll
          for (int i = 0; i < kCertK; ++i) {
            rs[i * F_BV + c] = ls[nv][i];
            rj[i * F_BV + c] = lj[nv][i];
          }
        }
      }
      __syncthreads();
      if (wa == 0 && h == 0) {
#pragma unroll
        for (int nv = 0; nv < 2; ++nv) {
          const int c = wv * 64 + nv * 32 + l32;
#pragma unroll
          for (int i = 0; i < kCertK; ++i) topk_push(ls[nv], lj[nv], rs[i * F_BV + c], rj[i * F_BV + c]);
          const int64_t v = v0 + c;
          if (v < nvox) {
            float *os = part_s + ((int64_t)split * pstride + v) * kCertK;
            int *oj = part_j + ((int64_t)split * pstride + v) * kCertK;
#pragma unroll
            for (int i = 0; i < kCertK; ++i) {
              os[i] = ls[nv][i];
              oj[i] = lj[nv][i];
            }
          }
        }
      }
    }
    __syncthreads();  // the next item reuses the LDS buffers
  }
}

void launch_score_f32(const float *D, const float *Zp, int d, int64_t d_pad, int64_t n,
                      int64_t n_pad, int Kp, int splits, float *part_s, int *part_j,
                      hipStream_t s, bool topk, const float *znorm, float cw, float wabs) {
  const int ntiles = (int)(d_pad / F_BA);
  const int nvt = (int)((n + F_BV - 1) / F_BV);
  (void)n_pad;
  const int tiles_per_split = (ntiles + splits - 1) / splits;
  const int nvt8 = (nvt + 7) / 8 * 8;
  const int64_t blocks = (int64_t)nvt8 * splits;
  if (blocks <= 0) return;
  if (topk)
    hipLaunchKernelGGL(k_score_f32<SC_TOPK>, dim3((unsigned)blocks), dim3(256), 0, s, D, Zp, d, ntiles, n,
                       nvt, Kp, splits, tiles_per_split, part_s, part_j, n, nullptr, nullptr, CollectArgs{},
                       znorm, cw, wabs);
  else
    hipLaunchKernelGGL(k_score_f32<SC_TOP1>, dim3((unsigned)blocks), dim3(256), 0, s, D, Zp, d, ntiles, n,
                       nvt, Kp, splits, tiles_per_split, part_s, part_j, n, nullptr, nullptr, CollectArgs{},
                       nullptr, 0.f, 0.f);
}

void launch_collect_f32_dev(const float *D, const float *Zp, const int32_t *rows, int d, int64_t d_pad,
                            int64_t cap, const unsigned int *dcnt, int Kp, const float *thr, unsigned int *count,
                            int32_t *cand, int ccap, hipStream_t s) {
  if (cap <= 0) return;
  const int ntiles = (int)(d_pad / F_BA);
  // two blocks per CU, each looping over the work items of the device count
  hipLaunchKernelGGL(k_score_f32<SC_COLLECT>, dim3(512), dim3(256), 0, s, D, Zp, d, ntiles, cap, 0, Kp, 1,
                     ntiles, nullptr, nullptr, cap, dcnt, rows, CollectArgs{thr, count, cand, ccap}, nullptr, 0.f,
                     0.f);
}

// ---------------------------------------------------------------------------
// merge + rescale + look-up
// ---------------------------------------------------------------------------
__global__ void k_merge_argmax(const float *__restrict__ part_s, const int *__restrict__ part_j,
                               int splits, int64_t n, int d, const float *znorm, const int32_t *warm,
                               const float *inv_norm, const float *params, int nparam,
                               int32_t *idx, float *pd, float *corr, float *params_out,
                               float *gamma_hat) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  float bs = -INFINITY;
  int bj = -1;
  for (int s = 0; s < splits; ++s) {
    const float ps = part_s[(int64_t)s * n + v];
    const int pj = part_j[(int64_t)s * n + v];
    if (pj >= 0 && better(ps, pj, bs, bj)) {
      bs = ps;
      bj = pj;
    }
  }
  finish_voxel(v, bs, bj, d, znorm, warm, inv_norm, params, nparam, idx, pd, corr, params_out,
               gamma_hat);
}

void launch_merge_argmax(const float *part_s, const int *part_j, int splits, int64_t n, int d,
                         const float *znorm, const int32_t *warm, const float *inv_norm,
                         const float *params, int nparam, int32_t *idx, float *pd, float *corr,
                         float *params_out, float *gamma_hat, hipStream_t s) {
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_merge_argmax, dim3((unsigned)blocks), dim3(256), 0, s, part_s, part_j,
                     splits, n, d, znorm, warm, inv_norm, params, nparam, idx, pd, corr,
                     params_out, gamma_hat);
}

// ---------------------------------------------------------------------------
// X = gamma_hat * Dhat_idx
// ---------------------------------------------------------------------------
template <bool FRAME, bool DELTA>
__global__ __launch_bounds__(256) void k_write_x(const int32_t *__restrict__ idx,
                                                 const float *__restrict__ gamma_hat,
                                                 const float *__restrict__ D, int Kp,
                                                 int real_atoms, int64_t n, int L, int64_t npix,
                                                 float2 *__restrict__ X,
                                                 const float2 *__restrict__ X_prev,
                                                 float2 *__restrict__ dX, double *part,
                                                 const float2 *__restrict__ vphase) {
  __shared__ double red[256];
  const int64_t total = n * L;
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    int64_t v;
    int t;
    if (FRAME) {
      const int64_t pair = e / npix;  // s*L + t
      const int64_t p = e - pair * npix;
      const int64_t sl = pair / L;
      t = (int)(pair - sl * L);
      v = sl * npix + p;
    } else {
      v = e / L;
      t = (int)(e - v * L);
    }
    const int j = idx[v];
    float2 x = make_float2(0.f, 0.f);
    if (j >= 0) {
      const float g = gamma_hat[v];
      const float *a = D + (int64_t)j * Kp;
      if (real_atoms) {
        x.x = g * a[t];
      } else {
        const float2 c = *reinterpret_cast<const float2 *>(a + 2 * t);
        x.x = g * c.x;
        x.y = g * c.y;
      }
      if (vphase) {  // phase-aligned projection: X_v = gamma e^{i theta_v} Dhat^a_j
        const float2 ph = vphase[v];
        x = make_float2(ph.x * x.x - ph.y * x.y, ph.x * x.y + ph.y * x.x);
      }
    }
    X[e] = x;
    if (DELTA) {
      const float2 xp = X_prev[e];
      const float2 dd = make_float2(x.x - xp.x, x.y - xp.y);
      dX[e] = dd;
      acc += (double)dd.x * dd.x + (double)dd.y * dd.y;
    }
  }
  if (DELTA) {
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
  }
}

void launch_write_x(const int32_t *idx, const float *gamma_hat, const float *D, int Kp,
                    int real_atoms, int64_t n, int L, int frame_major, int64_t npix, float2 *X,
                    const float2 *X_prev, float2 *dX, double *part, int *nblocks_out,
                    hipStream_t s, const float2 *vphase) {
  const int64_t total = n * (int64_t)L;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (nblocks_out) *nblocks_out = (int)blocks;
  if (frame_major) {
    if (X_prev)
      hipLaunchKernelGGL((k_write_x<true, true>), dim3((unsigned)blocks), dim3(256), 0, s, idx,
                         gamma_hat, D, Kp, real_atoms, n, L, npix, X, X_prev, dX, part, vphase);
    else
      hipLaunchKernelGGL((k_write_x<true, false>), dim3((unsigned)blocks), dim3(256), 0, s, idx,
                         gamma_hat, D, Kp, real_atoms, n, L, npix, X, nullptr, nullptr, nullptr, vphase);
  } else {
    hipLaunchKernelGGL((k_write_x<false, false>), dim3((unsigned)blocks), dim3(256), 0, s, idx,
                       gamma_hat, D, Kp, real_atoms, n, L, npix, X, nullptr, nullptr, nullptr, vphase);
  }
}

}  // namespace mrf

namespace mrf {

__global__ void k_lookup(const int32_t *__restrict__ idx, const float *__restrict__ params,
                         int nparam, int64_t n, float *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nparam) return;
  const int64_t v = e / nparam;
  const int p = (int)(e - v * nparam);
  const int j = idx[v];
  out[e] = j >= 0 ? params[(int64_t)j * nparam + p] : 0.f;
}

void launch_lookup(const int32_t *idx, const float *params, int nparam, int64_t n,
                   float *params_out, hipStream_t s) {
  const int64_t total = n * nparam;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_lookup, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, idx,
                     params, nparam, n, params_out);
}

__global__ void k_scale_f32(float *x, int64_t count, float a) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256)
    x[i] *= a;
}

void launch_scale_f32(float *x, int64_t count, float a, hipStream_t s) {
  int64_t blocks = (count + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks > 0) hipLaunchKernelGGL(k_scale_f32, dim3((unsigned)blocks), dim3(256), 0, s, x, count, a);
}

}  // namespace mrf
