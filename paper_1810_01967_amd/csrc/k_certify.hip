// Exactness certificate of the exhaustive matched filter (eq. exactP).
//
// The scoring kernels compute every score in a fast arithmetic (FP32 or split
// BF16 on the matrix cores) whose error is bounded by |s_hat - s| <= E_v =
// c * ||Z_v|| for every atom (c from the arithmetic and K; the host derives
// it), where s = <Z_v, Dhat_j> is the exact score over the FP32 normalised
// atoms.  Each voxel arrives with the kCertK best (s_hat, j) pairs.  Here:
//   1. the first pair is rescored exactly (FP64: every product of two FP32
//      values is exact in FP64, the sum of K of them is within ~K 2^-53);
//   2. with b the best exact score so far, any atom that could beat or tie b
//      has s_hat >= b - E_v, so every listed pair above that line is rescored
//      too (the list is sorted, so the first one below it ends the loop);
//   3. if the whole list lies above the line, atoms beyond it may as well:
//      the voxel is queued for a rescan, which collects every atom with an
//      FP32 score >= b - E32_v and rescores all of them exactly; a voxel with
//      more candidates than the list holds is scanned exactly over all atoms.
// The answer is the lowest index among the exactly highest scores: the exact
// argmax of eq. exactP over the FP32 normalised atoms, whatever the rounding
// of the fast pass.
#include <algorithm>
#include <cfloat>

#include "k_topk.h"
#include "mrf_internal.h"

namespace mrf {

namespace {

__device__ __forceinline__ double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Exact (FP64) <z, a> over K FP32 values; every lane returns the same value
// (fixed reduction order).  Rows are 16-byte aligned and zero from K up to
// their pitch (a multiple of 16), so the lanes read 16-byte pieces up to K
// rounded to 4: every product of two FP32 values is exact in FP64, and the
// loads of a lane are independent of its two running sums.
__device__ __forceinline__ double dot64(const float *__restrict__ z, const float *__restrict__ a, int K, int lane) {
  const int K4 = (K + 3) & ~3;
  double acc0 = 0.0, acc1 = 0.0;
#pragma unroll 4
  for (int k = 4 * lane; k < K4; k += 256) {
    const float4 x = *reinterpret_cast<const float4 *>(z + k);
    const float4 y = *reinterpret_cast<const float4 *>(a + k);
    acc0 = fma((double)x.x, (double)y.x, acc0);
    acc1 = fma((double)x.y, (double)y.y, acc1);
    acc0 = fma((double)x.z, (double)y.z, acc0);
    acc1 = fma((double)x.w, (double)y.w, acc1);
  }
  return wave_sum(acc0 + acc1);
}

// Adds each thread's x to *dst with one global atomic per block (every
// thread of the block calls it): one atomic per voxel on a single counter
// serialises at its L2 channel.
__device__ __forceinline__ void block_add(unsigned long long *dst, unsigned long long x) {
  __shared__ unsigned long long acc;
  if (threadIdx.x == 0) acc = 0ull;
  __syncthreads();
  if (x) atomicAdd(&acc, x);
  __syncthreads();
  if (threadIdx.x == 0 && acc) atomicAdd(dst, acc);
}

__device__ __forceinline__ bool exact_better(double s1, int j1, double s0, int j0) {
  return s1 > s0 || (s1 == s0 && j1 < j0);
}

// Rescale and look up (eq. exactPs) as the merge kernels do: gamma_hat =
// max(score, 0), PD = gamma_hat / ||D_j||, corr = score / ||Z_v||; a zero
// voxel keeps its warm atom (else atom 0), a non-finite one gets index -1.
__device__ __forceinline__ void finish(int64_t v, float sc, int j, int d, const CertOut &o) {
  const float zn = o.znorm[v];
  float g = 0.f, c = 0.f;
  if (zn < 0.f || j < 0) {
    j = -1;
  } else if (zn == 0.f) {
    j = o.warm ? o.warm[v] : 0;
    if (j < 0 || j >= d) j = 0;
  } else {
    g = fmaxf(sc, 0.f);
    c = sc / zn;
  }
  o.idx[v] = j;
  if (o.pd) o.pd[v] = j >= 0 ? g * o.inv_norm[j] : 0.f;
  if (o.corr) o.corr[v] = c;
  o.gamma_hat[v] = g;
  if (o.params_out)
    for (int p = 0; p < o.nparam; ++p)
      o.params_out[v * o.nparam + p] = j >= 0 ? o.params[(int64_t)j * o.nparam + p] : 0.f;
}

}  // namespace

// One wave per voxel.
__global__ __launch_bounds__(256) void k_certify(const float *__restrict__ part_s, const int *__restrict__ part_j,
                                                 int splits, int64_t pstride, int64_t n, int d,
                                                 const float *__restrict__ Zp, const float *__restrict__ D, int Kp,
                                                 int K, float cE, float cE32, float eabs, CertOut o, CertQueue q) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  unsigned long long counted = 0;
  do {
    if (v >= n) break;
    float ls[kCertK];
    int lj[kCertK];
    topk_clear(ls, lj);
    for (int sp = 0; sp < splits; ++sp) {
      const float *cs = part_s + ((int64_t)sp * pstride + v) * kCertK;
      const int *cj = part_j + ((int64_t)sp * pstride + v) * kCertK;
#pragma unroll
      for (int i = 0; i < kCertK; ++i) topk_push(ls, lj, cs[i], cj[i]);
    }
    const float zn = o.znorm[v];
    if (!(zn > 0.f) || lj[0] < 0) {  // zero or non-finite voxel: nothing to certify
      if (lane == 0) finish(v, ls[0], lj[0], d, o);
      break;
    }
    const float *z = Zp + v * Kp;
    const double E = (double)cE * zn + eabs;
    double bs = dot64(z, D + (int64_t)lj[0] * Kp, K, lane);
    int bj = lj[0];
    int rescored = 1;
    bool full = true;  // every listed pair lies on or above the line
#pragma unroll
    for (int c = 1; c < kCertK; ++c) {
      if (lj[c] < 0 || (double)ls[c] < bs - E) {
        full = false;
        break;
      }
      const double sc = dot64(z, D + (int64_t)lj[c] * Kp, K, lane);
      ++rescored;
      if (exact_better(sc, lj[c], bs, bj)) {
        bs = sc;
        bj = lj[c];
      }
    }
    if (full && (double)ls[kCertK - 1] < bs - E) full = false;  // the line rose above the last pair
    if (lane == 0) {
      finish(v, (float)bs, bj, d, o);
      counted = (unsigned long long)rescored;
      if (full) {
        const unsigned int pos = atomicAdd(q.count, 1u);
        q.list[pos] = (int32_t)v;
        q.ccount[pos] = 0u;
        // the rescan's line in FP32 scores (rounded down); b itself lies on or above it
        const double line = bs - ((double)cE32 * zn + eabs);
        float t = (float)line;
        if ((double)t > line) t = nextafterf(t, -INFINITY);
        q.thr[pos] = t;
      }
    }
  } while (false);
  block_add(q.rescored, counted);
}

void launch_certify(const float *part_s, const int *part_j, int splits, int64_t pstride, int64_t n, int d,
                    const float *Zp, const float *D, int Kp, int K, float cE, float cE32, float eabs,
                    const CertOut &o, const CertQueue &q, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_certify, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, part_s, part_j, splits, pstride, n,
                     d, Zp, D, Kp, K, cE, cE32, eabs, o, q);
}

// One wave per queued voxel (the queue's length on the device): exact
// rescore of every collected candidate; voxels whose candidates overflowed
// the list go to the full scan.
__global__ __launch_bounds__(256) void k_rescore_collected(const float *__restrict__ Zp, const float *__restrict__ D,
                                                           int Kp, int K, int d, int64_t cap, CertQueue q,
                                                           const int32_t *__restrict__ cand, int ccap, CertOut o) {
  const int lane = threadIdx.x & 63;
  const int64_t nq = min(cap, (int64_t)*q.count);
  unsigned long long counted = 0;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < nq; i += (int64_t)gridDim.x * 4) {
    const int64_t v = q.list[i];
    const unsigned int c = q.ccount[i];
    if ((int)c > ccap) {
      if (lane == 0) {
        const unsigned int pos = atomicAdd(q.scan_count, 1u);
        q.scan_list[pos] = (int32_t)v;
      }
      continue;
    }
    const float *z = Zp + v * Kp;
    double bs = -DBL_MAX;
    int bj = INT32_MAX;
    for (unsigned int t = 0; t < c; ++t) {
      const int j = cand[i * ccap + t];
      const double sc = dot64(z, D + (int64_t)j * Kp, K, lane);
      if (exact_better(sc, j, bs, bj)) {
        bs = sc;
        bj = j;
      }
    }
    if (lane == 0) {
      counted += c;
      if (c > 0) finish(v, (float)bs, bj, d, o);
    }
  }
  block_add(q.rescored, counted);
}

void launch_rescore_collected(const float *Zp, const float *D, int Kp, int K, int d, int64_t cap, const CertQueue &q,
                              const int32_t *cand, int ccap, const CertOut &o, hipStream_t s) {
  if (cap <= 0) return;
  hipLaunchKernelGGL(k_rescore_collected, dim3(1024), dim3(256), 0, s, Zp, D, Kp, K, d, cap, q, cand, ccap, o);
}

// One block per voxel of the scan list: exact scores of all atoms (four
// waves, atom j on wave j % 4), best per wave, then across the waves.
__global__ __launch_bounds__(256) void k_scan_exact(const float *__restrict__ Zp, const float *__restrict__ D, int Kp,
                                                    int K, int d, int64_t cap, CertQueue q, CertOut o) {
  __shared__ double ws[4];
  __shared__ int wj[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nq = min(cap, (int64_t)*q.scan_count);
  for (int64_t i = blockIdx.x; i < nq; i += gridDim.x) {
    const int64_t v = q.scan_list[i];
    const float *z = Zp + v * Kp;
    double bs = -DBL_MAX;
    int bj = INT32_MAX;
    for (int j = wave; j < d; j += 4) {
      const double sc = dot64(z, D + (int64_t)j * Kp, K, lane);
      if (exact_better(sc, j, bs, bj)) {
        bs = sc;
        bj = j;
      }
    }
    if (lane == 0) {
      ws[wave] = bs;
      wj[wave] = bj;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < 4; ++w)
        if (exact_better(ws[w], wj[w], bs, bj)) {
          bs = ws[w];
          bj = wj[w];
        }
      atomicAdd(q.rescored, (unsigned long long)d);
      finish(v, (float)bs, bj, d, o);
    }
    __syncthreads();
  }
}

// Reduced-precision passes (BF16 / FP8).  One wave per voxel: merge the
// pass's split maxima, rescore the best atom exactly (b), finish the voxel
// with it, and (certified) write the voxel's line for the collect pass.
// With q_v the decoded voxel row and r_j the atoms' decoded rows, the pass's
// score (times the voxel's FP8 scale) differs from the exact one by at most
//   E_v = (gq ||q_v|| + ||z_v - q_v||) max_j ||r_j|| + ||z_v|| max_j ||d_j - r_j||
// (the products' quantisation errors by Cauchy-Schwarz, gq = gamma_{K+1}
// the FP32 accumulation and scale multiply), so every atom that could beat or
// tie b scores at least (b - E_v) / scale_v in the pass's unit.
__global__ __launch_bounds__(256) void k_lowp_line(const float *__restrict__ part_s, const int *__restrict__ part_j,
                                                   int splits, int64_t n, int d, const float *__restrict__ Zp,
                                                   const float *__restrict__ D, int Kp, int K,
                                                   const double2 *__restrict__ qnorm, const float *__restrict__ zscale,
                                                   double gq, double Nq, double Ne, double eabs, CertOut o,
                                                   float *__restrict__ thr, unsigned int *__restrict__ ccount,
                                                   double *__restrict__ bex, int certify) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= n) return;
  float bs = -INFINITY;
  int bj = -1;
  for (int sp = 0; sp < splits; ++sp) {
    const float ps = part_s[(int64_t)sp * n + v];
    const int pj = part_j[(int64_t)sp * n + v];
    if (rank_before(ps, pj, bs, bj)) {
      bs = ps;
      bj = pj;
    }
  }
  const float zn = o.znorm[v];
  if (!(zn > 0.f) || bj < 0) {  // zero or non-finite voxel
    if (lane == 0) {
      finish(v, 0.f, bj, d, o);
      if (certify) {
        thr[v] = INFINITY;
        ccount[v] = 0u;
      }
    }
    return;
  }
  const double b = dot64(Zp + v * Kp, D + (int64_t)bj * Kp, K, lane);
  if (lane == 0) {
    finish(v, (float)b, bj, d, o);
    if (certify) {
      const double2 qn = qnorm[v];
      const double E = 1.01 * ((gq * qn.x + qn.y) * Nq + (double)zn * Ne) + eabs;
      const double sc = zscale ? (double)zscale[v] : 1.0;
      const double line = (b - E) / sc;
      float t = (float)line;
      if ((double)t > line) t = nextafterf(t, -INFINITY);
      thr[v] = t;
      ccount[v] = 0u;
      bex[v] = b;
    }
  }
}

void launch_lowp_line(const float *part_s, const int *part_j, int splits, int64_t n, int d, const float *Zp,
                      const float *D, int Kp, int K, const double2 *qnorm, const float *zscale, double gq, double Nq,
                      double Ne, double eabs, const CertOut &o, float *thr, unsigned int *ccount, double *bex,
                      int certify, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_lowp_line, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, part_s, part_j, splits, n, d, Zp,
                     D, Kp, K, qnorm, zscale, gq, Nq, Ne, eabs, o, thr, ccount, bex, certify);
}

// One wave per voxel: exact rescore of the reduced-precision pass's collected
// candidates; a voxel with more than ccap of them is queued for the FP32
// rescan with the FP32 line b - (cE32 ||Z_v|| + eabs).
__global__ __launch_bounds__(256) void k_rescore_lowp(const float *__restrict__ Zp, const float *__restrict__ D, int Kp,
                                                      int K, int d, int64_t n, const unsigned int *__restrict__ ccount,
                                                      const int32_t *__restrict__ cand, int ccap,
                                                      const double *__restrict__ bex, float cE32, float eabs,
                                                      CertOut o, CertQueue q) {
  const int lane = threadIdx.x & 63;
  unsigned long long counted = 0;
  for (int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); v < n; v += (int64_t)gridDim.x * 4) {
    const unsigned int c = ccount[v];
    if (c == 0) continue;  // zero or non-finite voxel, finished already
    if ((int)c > ccap) {
      if (lane == 0) {
        const unsigned int pos = atomicAdd(q.count, 1u);
        q.list[pos] = (int32_t)v;
        q.ccount[pos] = 0u;
        const double line = bex[v] - ((double)cE32 * o.znorm[v] + eabs);
        float t = (float)line;
        if ((double)t > line) t = nextafterf(t, -INFINITY);
        q.thr[pos] = t;
      }
      continue;
    }
    const float *z = Zp + v * Kp;
    double bs = -DBL_MAX;
    int bj = INT32_MAX;
    for (unsigned int t = 0; t < c; ++t) {
      const int j = cand[v * ccap + t];
      const double sc = dot64(z, D + (int64_t)j * Kp, K, lane);
      if (exact_better(sc, j, bs, bj)) {
        bs = sc;
        bj = j;
      }
    }
    if (lane == 0) {
      counted += c;
      finish(v, (float)bs, bj, d, o);
    }
  }
  block_add(q.rescored, counted);
}

void launch_rescore_lowp(const float *Zp, const float *D, int Kp, int K, int d, int64_t n, const unsigned int *ccount,
                         const int32_t *cand, int ccap, const double *bex, float cE32, float eabs, const CertOut &o,
                         const CertQueue &q, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 3) / 4, 4096);
  hipLaunchKernelGGL(k_rescore_lowp, dim3((unsigned)blocks), dim3(256), 0, s, Zp, D, Kp, K, d, n, ccount, cand, ccap,
                     bex, cE32, eabs, o, q);
}

// Certified local search (the learned path's answer made exact within its
// box).  With b the exact score of the local search's answer, every box atom
// that could beat or tie b scores at least b - E_v in the local pass (E_v its
// error bound), so the collect pass gathers them and they are rescored
// exactly here; the warm atom (outside the box in general) is rescored too.
// Exhaustive fallbacks go to the FP32 rescan of the exhaustive certificate.
__device__ __forceinline__ void queue_rescan(int64_t v, double b, float cE32, float eabs, const CertOut &o,
                                             const CertQueue &q) {
  const unsigned int pos = atomicAdd(q.count, 1u);
  q.list[pos] = (int32_t)v;
  q.ccount[pos] = 0u;
  const double line = b - ((double)cE32 * o.znorm[v] + eabs);
  float t = (float)line;
  if ((double)t > line) t = nextafterf(t, -INFINITY);
  q.thr[pos] = t;
}

__global__ __launch_bounds__(256) void k_local_line(const float *__restrict__ best_s,
                                                    const int32_t *__restrict__ best_j,
                                                    const int32_t *__restrict__ fbflag, int64_t n, int d,
                                                    const float *__restrict__ Zp, const float *__restrict__ D, int Kp,
                                                    int K, float cE, float cE32, float eabs, CertOut o,
                                                    float *__restrict__ thr, unsigned int *__restrict__ ccount,
                                                    double *__restrict__ bex, int32_t *__restrict__ bjx,
                                                    CertQueue q) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int bj = v < n ? best_j[v] : -1;
  const float zn = v < n ? o.znorm[v] : 0.f;
  const bool live = v < n && zn > 0.f && bj >= 0 && bj < d;
  if (v < n && !live && lane == 0) {  // zero or non-finite voxel: nothing to certify
    finish(v, best_s[v], bj, d, o);
    thr[v] = INFINITY;
    ccount[v] = 0u;
    bex[v] = 0.0;
    bjx[v] = -1;
  }
  block_add(q.rescored, live && lane == 0 ? 1ull : 0ull);
  if (!live) return;
  const double b = dot64(Zp + v * Kp, D + (int64_t)bj * Kp, K, lane);
  if (lane == 0) {
    finish(v, (float)b, bj, d, o);
    ccount[v] = 0u;
    bex[v] = b;
    bjx[v] = bj;
    if (fbflag && fbflag[v]) {
      thr[v] = INFINITY;  // no box: the exhaustive certificate's rescan
      queue_rescan(v, b, cE32, eabs, o, q);
    } else {
      const double line = b - ((double)cE * zn + eabs);
      float t = (float)line;
      if ((double)t > line) t = nextafterf(t, -INFINITY);
      thr[v] = t;
    }
  }
}

void launch_local_line(const float *best_s, const int32_t *best_j, const int32_t *fbflag, int64_t n, int d,
                       const float *Zp, const float *D, int Kp, int K, float cE, float cE32, float eabs,
                       const CertOut &o, float *thr, unsigned int *ccount, double *bex, int32_t *bjx,
                       const CertQueue &q, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_local_line, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, best_s, best_j, fbflag, n, d, Zp,
                     D, Kp, K, cE, cE32, eabs, o, thr, ccount, bex, bjx, q);
}

__global__ __launch_bounds__(256) void k_rescore_local(const float *__restrict__ Zp, const float *__restrict__ D,
                                                       int Kp, int K, int d, int64_t n,
                                                       const unsigned int *__restrict__ ccount,
                                                       const int32_t *__restrict__ cand, int ccap,
                                                       const double *__restrict__ bex, const int32_t *__restrict__ bjx,
                                                       const int32_t *__restrict__ warm,
                                                       const int32_t *__restrict__ fbflag, float cE32, float eabs,
                                                       CertOut o, CertQueue q) {
  const int lane = threadIdx.x & 63;
  unsigned long long counted = 0;
  for (int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); v < n; v += (int64_t)gridDim.x * 4) {
    int bj = bjx[v];
    if (bj < 0 || (fbflag && fbflag[v])) continue;  // finished already, or in the rescan queue
    double bs = bex[v];
    const unsigned int c = ccount[v];
    if ((int)c > ccap) {
      if (lane == 0) queue_rescan(v, bs, cE32, eabs, o, q);
      continue;
    }
    const float *z = Zp + v * Kp;
    const int w = warm ? warm[v] : -1;
    unsigned int rescored = 0;
    for (unsigned int t = 0; t <= c; ++t) {
      const int j = t < c ? cand[v * ccap + t] : w;
      if (j < 0 || j >= d || j == bjx[v]) continue;
      const double sc = dot64(z, D + (int64_t)j * Kp, K, lane);
      ++rescored;
      if (exact_better(sc, j, bs, bj)) {
        bs = sc;
        bj = j;
      }
    }
    if (lane == 0) {
      counted += rescored;
      if (bj != bjx[v]) finish(v, (float)bs, bj, d, o);
    }
  }
  block_add(q.rescored, counted);
}

void launch_rescore_local(const float *Zp, const float *D, int Kp, int K, int d, int64_t n,
                          const unsigned int *ccount, const int32_t *cand, int ccap, const double *bex,
                          const int32_t *bjx, const int32_t *warm, const int32_t *fbflag, float cE32, float eabs,
                          const CertOut &o, const CertQueue &q, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 3) / 4, 4096);
  hipLaunchKernelGGL(k_rescore_local, dim3((unsigned)blocks), dim3(256), 0, s, Zp, D, Kp, K, d, n, ccount, cand,
                     ccap, bex, bjx, warm, fbflag, cE32, eabs, o, q);
}

void launch_scan_exact(const float *Zp, const float *D, int Kp, int K, int d, int64_t cap, const CertQueue &q,
                       const CertOut &o, hipStream_t s) {
  if (cap <= 0) return;
  hipLaunchKernelGGL(k_scan_exact, dim3(256), dim3(256), 0, s, Zp, D, Kp, K, d, cap, q, o);
}

}  // namespace mrf
