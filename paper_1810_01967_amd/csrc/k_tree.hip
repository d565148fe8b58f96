// Cover-tree (1+eps)-approximate nearest-neighbour search (Algorithm 1) for
// a batch of queries on gfx950, level-synchronous: one launch per tree
// level, one wavefront per query.  The wave computes the FP32 distances
// ||p - x_c|| of a query's children one at a time with coalesced row reads
// (self-children reuse their parent's distance), reduces the argmin (ties:
// lower atom) and compacts the refined
// candidate set Q_{i+1} = {q : ||p - q|| <= d_min + maxdist(q)} with ballots.
// Queries whose candidate set outgrows the per-query capacity are flagged
// for the exhaustive filter.
#include <cfloat>

#include "mrf_internal.h"

namespace mrf {

__device__ __forceinline__ float lane_dist(const float *__restrict__ p, const float *__restrict__ x, int K4,
                                           float inv) {
  const float4 *p4 = reinterpret_cast<const float4 *>(p);
  const float4 *x4 = reinterpret_cast<const float4 *>(x);
  float s = 0.f;
  for (int k = 0; k < K4; ++k) {
    const float4 a = p4[k], b = x4[k];
    const float d0 = a.x * inv - b.x, d1 = a.y * inv - b.y, d2 = a.z * inv - b.z, d3 = a.w * inv - b.w;
    s = fmaf(d0, d0, s);
    s = fmaf(d1, d1, s);
    s = fmaf(d2, d2, s);
    s = fmaf(d3, d3, s);
  }
  return sqrtf(s);
}

// Cooperative distance: the wave splits the row into float4 slices (lane,
// lane + 64, ...); ps holds this lane's slices of the query times 1/||Z||.
constexpr int TQ = kTreeMaxK / 256;  // float4 slices per lane held in registers
__device__ __forceinline__ float wave_dist(const float4 (&ps)[TQ], const float *__restrict__ x, int K4, int lane) {
  const float4 *x4 = reinterpret_cast<const float4 *>(x);
  float s = 0.f;
#pragma unroll
  for (int q = 0; q < TQ; ++q) {
    const int k = lane + 64 * q;
    if (k < K4) {
      const float4 b = x4[k];
      const float d0 = ps[q].x - b.x, d1 = ps[q].y - b.y, d2 = ps[q].z - b.z, d3 = ps[q].w - b.w;
      s = fmaf(d0, d0, s);
      s = fmaf(d1, d1, s);
      s = fmaf(d2, d2, s);
      s = fmaf(d3, d3, s);
    }
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  return sqrtf(s);
}

__device__ __forceinline__ void wave_argmin(float &d, int &node) {
  for (int o = 32; o > 0; o >>= 1) {
    const float od = __shfl_xor(d, o, 64);
    const int on = __shfl_xor(node, o, 64);
    if (od < d || (od == d && on < node)) {
      d = od;
      node = on;
    }
  }
}

// Start of the search: q_c = warm start (or the root), d_min = ||p - q_c||,
// Q_0 = {root}.  Queries with a zero or non-finite norm are not searched.
__global__ __launch_bounds__(256) void k_tree_init(TreeDev t, const float *__restrict__ Zp, int Kp,
                                                   const float *__restrict__ znorm, const int32_t *warm,
                                                   int64_t n, TreeState st) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= n) return;
  const float zn = znorm[v];
  if (!(zn > 0.f) || !isfinite(zn)) {
    if (lane == 0) {
      st.active[v] = 0;
      st.qc[v] = 0;
      st.cnt[v] = 0;
      st.flags[v] = 0;
    }
    return;
  }
  const float inv = 1.f / zn;
  const float *p = Zp + v * Kp;
  int qc = 0;
  if (warm) {
    const int j = warm[v];
    qc = (j >= 0 && j < t.d) ? t.uniq_of[j] : 0;
  }
  // lane 0: distance to q_c, lane 1: distance to the root
  float dl = 0.f;
  if (lane < 2) {
    const int u = lane == 0 ? qc : t.node[0];
    dl = lane_dist(p, t.dhat + (int64_t)t.rep[u] * Kp, Kp / 4, inv);
  }
  const float dqc = __shfl(dl, 0, 64), droot = __shfl(dl, 1, 64);
  if (lane == 0) {
    st.active[v] = 1;
    st.qc[v] = qc;
    st.dmin[v] = dqc;
    st.flags[v] = 0;
    st.cnt[v] = 1;
    st.Qe[v * st.cap] = 0;
    st.Qd[v * st.cap] = droot;
    atomicAdd(st.evals, (unsigned long long)((warm && qc != t.node[0]) ? 2 : 1));
  }
}

// One level of Algorithm 1 for every active query; reads Q_i from (Qe, Qd)
// and writes Q_{i+1} into (Qe2, Qd2).
__global__ __launch_bounds__(256) void k_tree_level(TreeDev t, const float *__restrict__ Zp, int Kp,
                                                    const float *__restrict__ znorm, int64_t n, int level,
                                                    float inv_eps, TreeState st, int32_t *__restrict__ Qe2,
                                                    float *__restrict__ Qd2) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= n) return;
  if (!st.active[v]) return;
  float dmin = st.dmin[v];
  int qc = st.qc[v];
  // loop condition of Algorithm 1 (1/eps = inf for eps = 0)
  const float bound = t.sigma * exp2f((float)(1 - level)) * (1.f + inv_eps);
  const int cnt = st.cnt[v];
  if (!(level < t.imax && bound > dmin) || cnt == 0) {
    if (lane == 0) st.active[v] = 0;
    return;
  }
  const float inv = 1.f / znorm[v];
  const float *p = Zp + v * Kp;
  const int32_t *Qe = st.Qe + v * st.cap;
  const float *Qd = st.Qd + v * st.cap;
  int32_t *Oe = Qe2 + v * st.cap;
  float *Od = Qd2 + v * st.cap;
  float4 ps[TQ];
  {
    const float4 *p4 = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const int k = lane + 64 * q;
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
      if (k < Kp / 4) {
        a = p4[k];
        a.x *= inv;
        a.y *= inv;
        a.z *= inv;
        a.w *= inv;
      }
      ps[q] = a;
    }
  }
  int out = 0;
  bool overflow = false;
  unsigned long long evals = 0;
  for (int q = 0; q < cnt; ++q) {
    const int e = Qe[q];
    const float dq = Qd[q];
    const int cb = t.child_begin[e], ce = t.child_end[e];
    for (int c0 = cb; c0 < ce; c0 += 64) {
      const int c = c0 + lane;
      const int nc = min(64, ce - c0);
      int node = 0x7fffffff;
      bool self = false;
      if (c < ce) {
        node = t.node[c];
        self = t.is_self[c] != 0;
      }
      // distances of the chunk's children, one child per wave-wide pass
      float dc = INFINITY;
      for (int k = 0; k < nc; ++k) {
        const int nk = __shfl(node, k, 64);
        const bool sk = __shfl((int)self, k, 64) != 0;
        float dk;
        if (sk) {
          dk = dq;
        } else {
          dk = wave_dist(ps, t.dhat + (int64_t)t.rep[nk] * Kp, Kp / 4, lane);
          ++evals;
        }
        if (lane == k) dc = dk;
      }
      float bd = dc;
      int bn = node;
      wave_argmin(bd, bn);
      if (bd < dmin) {
        dmin = bd;
        qc = bn;
      }
      // provisional refinement with the running d_min (final filter below)
      const bool keep = c < ce && dc <= dmin + t.maxdist[c];
      const unsigned long long m = __ballot(keep);
      const int pos = out + __popcll(m & ((1ull << lane) - 1ull));
      if (keep) {
        if (pos < st.cap) {
          Oe[pos] = c;
          Od[pos] = dc;
        }
      }
      out += __popcll(m);
      if (out > st.cap) overflow = true;
    }
  }
  // final refinement with the level's d_min, compacted in place
  int kept = 0;
  const int total = out < st.cap ? out : st.cap;
  for (int b = 0; b < total; b += 64) {
    const int i = b + lane;
    int e = 0;
    float dc = 0.f;
    bool keep = false;
    if (i < total) {
      e = Oe[i];
      dc = Od[i];
      keep = dc <= dmin + t.maxdist[e];
    }
    const unsigned long long m = __ballot(keep);
    const int pos = kept + __popcll(m & ((1ull << lane) - 1ull));
    // pos <= i: compaction never overwrites an unread entry of a later chunk
    if (keep) {
      Oe[pos] = e;
      Od[pos] = dc;
    }
    kept += __popcll(m);
  }
  if (lane == 0) {
    st.dmin[v] = dmin;
    st.qc[v] = qc;
    st.cnt[v] = kept;
    if (overflow) {
      st.flags[v] = 1;
      st.active[v] = 0;
    }
    atomicAdd(st.evals, evals);
  }
}

// best_s[v] = Re<Z_v, Dhat_j> and best_j[v] = j for the found atom (flagged
// and unsearched voxels get index -1 / the warm handling of the merge).
__global__ __launch_bounds__(256) void k_tree_finish(TreeDev t, const float *__restrict__ Zp, int Kp, int K,
                                                     const float *__restrict__ znorm, int64_t n, TreeState st,
                                                     float *__restrict__ best_s, int32_t *__restrict__ best_j) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= n) return;
  const float zn = znorm[v];
  const int j = t.rep[st.qc[v]];
  float acc = 0.f;
  if (zn > 0.f && isfinite(zn)) {
    const float *z = Zp + v * Kp;
    const float *a = t.dhat + (int64_t)j * Kp;
    for (int k = lane; k < K; k += 64) acc = fmaf(z[k], a[k], acc);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  }
  if (lane == 0) {
    best_s[v] = acc;
    best_j[v] = j;
  }
}

__global__ void k_tree_select(const TreeState st, int64_t n, int32_t *__restrict__ out,
                              unsigned int *__restrict__ count) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && st.flags[v]) out[atomicAdd(count, 1u)] = (int32_t)v;
}

// Queries of a subset (the learned path's fallback list): norms and warm
// atoms (the local search's best, clamped to the dictionary) gathered.
__global__ void k_gather_queries(const int32_t *__restrict__ list, int64_t cnt, const float *__restrict__ znorm,
                                 const int32_t *__restrict__ best_j, int d, float *__restrict__ qnorm,
                                 int32_t *__restrict__ qwarm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int v = list[i];
  qnorm[i] = znorm[v];
  const int j = best_j[v];
  qwarm[i] = (j >= 0 && j < d) ? j : 0;
}

void launch_gather_queries(const int32_t *list, int64_t cnt, const float *znorm, const int32_t *best_j, int d,
                           float *qnorm, int32_t *qwarm, hipStream_t s) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(k_gather_queries, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, list, cnt, znorm,
                     best_j, d, qnorm, qwarm);
}

void launch_tree_init(const TreeDev &t, const float *Zp, int Kp, const float *znorm, const int32_t *warm,
                      int64_t n, const TreeState &st, hipStream_t s) {
  hipLaunchKernelGGL(k_tree_init, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, t, Zp, Kp, znorm, warm, n, st);
}

void launch_tree_level(const TreeDev &t, const float *Zp, int Kp, const float *znorm, int64_t n, int level,
                       float inv_eps, const TreeState &st, int32_t *Qe2, float *Qd2, hipStream_t s) {
  hipLaunchKernelGGL(k_tree_level, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, t, Zp, Kp, znorm, n, level,
                     inv_eps, st, Qe2, Qd2);
}

void launch_tree_finish(const TreeDev &t, const float *Zp, int Kp, int K, const float *znorm, int64_t n,
                        const TreeState &st, float *best_s, int32_t *best_j, hipStream_t s) {
  hipLaunchKernelGGL(k_tree_finish, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, t, Zp, Kp, K, znorm, n, st,
                     best_s, best_j);
}

void launch_tree_select(const TreeState &st, int64_t n, int32_t *out, unsigned int *count, hipStream_t s) {
  hipLaunchKernelGGL(k_tree_select, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, st, n, out, count);
}

}  // namespace mrf
