// Host-side helpers shared by the C-ABI translation units: error reporting,
// device buffers that grow on demand, and the handle structures.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "covertree.h"
#include "mrf_internal.h"

namespace mrf {

std::string &last_error();
mrf_status fail(mrf_status st, const char *fmt, ...);

#define HIP_TRY(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return ::mrf::fail(MRF_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_CHECK(what)                                                                   \
  do {                                                                                       \
    hipError_t e_ = hipGetLastError();                                                       \
    if (e_ != hipSuccess) return ::mrf::fail(MRF_E_HIP, "%s launch failed: %s", what, hipGetErrorString(e_)); \
  } while (0)

#define TRY(expr)                    \
  do {                               \
    mrf_status st_ = (expr);         \
    if (st_ != MRF_OK) return st_;   \
  } while (0)

struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  template <class T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

mrf_status grow(DevBuf &b, size_t bytes);

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr, c = nullptr, d = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (c) (void)hipEventDestroy(c);
    if (d) (void)hipEventDestroy(d);
  }
};

// SplitMix64 finaliser (Steele, Lea, Flood 2014), host copy used to derive
// the counter-generator keys of the training-data stream.
inline uint64_t mix64_host(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace mrf

struct mrf_dict_s;
namespace mrf {
mrf_status check_learned(const mrf_dict_s *D, const mrf_match_opts *o, bool need_net);
mrf_status match_exhaustive(mrf_dict_s *D, const mrf_match_opts *o, int64_t n, const int32_t *warm,
                            int32_t *idx, float *pd, float *corr, float *params_out, hipStream_t s,
                            hipEvent_t ev_s0, hipEvent_t ev_s1, int *splits_used);
mrf_status match_learned(mrf_dict_s *D, const mrf_match_opts *o, int64_t n, const int32_t *warm,
                         int32_t *idx, float *pd, float *corr, float *params_out, int32_t *cells_in,
                         int32_t *fallback_out, mrf_match_stats *st, hipStream_t s);
mrf_status match_core(mrf_dict_s *D, const mrf_match_opts *o, int64_t n, const int32_t *warm,
                      int32_t *idx, float *pd, float *corr, float *params_out, hipStream_t s,
                      hipEvent_t ev_s0, hipEvent_t ev_s1, int *splits_used, mrf_match_stats *st);
// want_fp32 = false leaves out the FP32 rows of a voxel-major packing that
// writes the split rows (see learned_split_rows_only); want_counts: the zero
// and non-finite rows counted into D->counters (read back for statistics)
mrf_status pack_voxels(mrf_dict_s *D, const void *Z, int32_t z_layout, int64_t slice_voxels,
                       int64_t n, hipStream_t s, bool want_x3 = false, bool want_fp32 = true,
                       bool want_counts = true);
// True when a learned match reads the voxels only as split-BF16 rows: split
// BF16 scoring, no warm start, no cover-tree fallback, and (unless the
// caller gives the cells) a network whose BF16 form reads the split rows.
bool learned_split_rows_only(const mrf_dict_s *D, const mrf_match_opts *o, const int32_t *warm, bool cells_given);
mrf_status check_opts(const mrf_dict_s *D, const mrf_match_opts *o);
int auto_splits(const mrf_dict_s *D, int64_t n);
// Exactness certificate of the exhaustive filter on caller-given buffers
// (counters 64 bytes; list, thr, ccount, scan [n]; cand [n][kCertCap]).
struct CertBufs {
  unsigned int *counters;
  int32_t *list;
  float *thr;
  unsigned int *ccount;
  int32_t *scan;
  int32_t *cand;
};
size_t cert_bytes(int64_t n);
float cert_coeff(int precision, int K);
float cert_window(float cE);
mrf_status certify_run(mrf_dict_s *D, const CertBufs &b, const float *zp, const float *znorm, const uint16_t *zx3,
                       float *gamma, const float *part_s, const int *part_j, int64_t n, int splits, int precision,
                       const int32_t *warm, int32_t *idx, float *pd, float *corr, float *params_out, hipStream_t s);
mrf_status match_tree(mrf_dict_s *D, const mrf_match_opts *o, int64_t n, const int32_t *warm,
                      int32_t *idx, float *pd, float *corr, float *params_out, mrf_match_stats *st,
                      hipStream_t s);
mrf_status upload_tree(mrf_dict_s *D, const double *Xnorm);
// Algorithm 1 for n query rows Q (pitch Kp, norms qnorm, warm-start atoms or
// NULL) into out_s / out_j (scores as the merge expects); queries whose
// candidate set overflows the capacity go to the exhaustive FP32 filter
// (work buffers ovf, rows, ps, pj; their count into *n_overflow).
mrf_status tree_search(mrf_dict_s *D, const float *Q, const float *qnorm, const int32_t *warm, int64_t n,
                       float eps, int cap, float *out_s, int32_t *out_j, DevBuf &ovf, DevBuf &rows, DevBuf &ps,
                       DevBuf &pj, int64_t *n_overflow, hipStream_t s);
mrf_status ensure_x3(mrf_dict_s *D, hipStream_t s);
// device counter of the learned path's fallback voxels: created zeroed / read (syncs s)
mrf_status fallback_total_buf(mrf_dict_s *D, hipStream_t s);
mrf_status read_fallback_total(mrf_dict_s *D, hipStream_t s, int64_t *out);
int auto_splits_x3(const mrf_dict_s *D, int64_t n);
bool net_bf16_ok(const mrf_net_s *net, int64_t K, int64_t ldx);
mrf_status net_forward_bf16(mrf_net_s *net, const float *X, int64_t ldx, int64_t K, int64_t B,
                            const float *rowscale, float *Y, uint16_t *h1, hipStream_t s);
}  // namespace mrf

struct mrf_dict_s {
  int device = 0;
  int d = 0, L = 0, nparam = 0, is_complex = 0, K = 0, Kp = 0, Kq = 0;
  int Kx = 0;  // split-BF16 row: Kx/32 chunks [hi 32 | lo 32]; K rounded up to 32
  int64_t d_pad = 0;
  uint32_t flags = 0;
  std::vector<int32_t> grid_dims;
  std::vector<double> params_host;              // d x nparam
  std::vector<std::vector<double>> axes_host;   // grid axis values (if grid_dims)
  mrf::DevBuf dhat, inv_norm, params, dbf16, dfp8, fp8_scale;
  mrf::DevBuf dx3;                              // split-BF16 atoms [d_pad][Kx/32][hi 32 | lo 32] (built on first use)
  mrf::DevBuf axes, aoff, dims;                 // device copies of the grid axes
  int64_t bytes = 0;
  mrf::DevBuf fbtot;  // device u64: voxels sent to the fallback by the learned path (all calls)
  // workspace (grows lazily)
  mrf::DevBuf zp, znorm, gamma, counters, part_s, part_j, zq, zscale, cand_s, cand_j, zx3;
  // exactness certificate: counters (u32 queue, u32 scan, u64 rescored), queue
  // (list, thr, candidate counts), scan list, candidates [n][kCertCap]
  mrf::DevBuf cert, cert_list, cert_thr, cert_ccount, cert_scan, cert_cand;
  // reduced-precision certificate: per voxel the decoded row norms, line, exact
  // best score, candidate count and candidates [n][kLowpCap]
  mrf::DevBuf lp_qn, lp_thr, lp_b, lp_count, lp_cand;
  // certified local search: per-voxel line, candidate count and list, exact
  // score and index of the local answer, exhaustive-fallback flags
  mrf::DevBuf lc_thr, lc_count, lc_cand, lc_bex, lc_bjx, lc_fb;
  // max over the atoms of ||r_j|| and ||d_j - r_j|| for the BF16 and FP8 copies r_j
  double qn_bf16[2] = {0.0, 0.0}, qn_fp8[2] = {0.0, 0.0};
  bool cert_used = false;  // the last exhaustive match ran the certificate
  bool zx3_fresh = false;  // zx3 holds the split rows of the current packing (written by the pack)
  bool zp_fresh = false;   // zp holds the FP32 rows of the current packing
  bool inv_fresh = false;  // inv holds 1/znorm of the current packing (written by the pack)
  mrf::DevBuf kbuf, gbuf, xbuf, rbuf, abuf, red, scal, idxbuf, pdbuf;
  // temporal subspace (a compressed dictionary: atoms V^H Dhat_j of L = s frames)
  int Lfull = 0;                    // frames of the uncompressed dictionary, 0 if not compressed
  mrf::DevBuf Vs;                   // V, FP32 complex [Lfull][L]
  std::vector<double> V_host, lam;  // V (FP64 complex [Lfull][L], interleaved) and its eigenvalues
  mrf::DevBuf kfull;                // full-frame k-space of the compressed adjoint
  mrf::DevBuf cbuf;                 // per-coil images (coil maps)
  mrf::DevBuf nbuf, nbuf2;          // oversampled grids of the non-uniform FFT
  mrf::DevBuf xfull;                // full-frame images of a compressed iterate (non-uniform FFT)
  // phase alignment (complex PD): first principal direction u [L] (FP32
  // complex), per-atom alignment factors f_j [d] (aligned atom = f_j Dhat_j),
  // per-voxel factors e^{i theta_v} of the last packing
  int align = 0;
  mrf::DevBuf u1, afac, vphase;
  mrf::DevBuf inv, h1, h2, yout, cells, best_s, best_j, bestkey, list_a, list_b, list_c, keys, hist, off, cnt, rows;
  // cover tree (host copy for export, device arrays for the traversal)
  bool has_tree = false;
  mrf::HostTree tree;
  int64_t tree_entries = 0;
  mrf::DevBuf t_node, t_rep, t_uniq, t_cb, t_ce, t_md, t_self;
  mrf::DevBuf ts_active, ts_qc, ts_cnt, ts_flags, ts_dmin, ts_Qe0, ts_Qe1, ts_Qd0, ts_Qd1, ts_evals;
  mrf::DevBuf fb_rows, fb_norm, fb_warm, fb_s, fb_j;  // learned-path fallback through the cover tree
  double *host_scal = nullptr;  // pinned readback of reduced scalars
  ~mrf_dict_s() {
    if (host_scal) (void)hipHostFree(host_scal);
  }
};

struct mrf_nufft_s {
  int nx = 0, ny = 0, L = 0, nslices = 0, W = 7;
  float beta = 0.f;
  int64_t M = 0;
  mrf::DevBuf off, coords, bperm, boff, dy, dx;
};

struct mrf_net_s {
  int I = 0, H = 0, P = 0;
  int64_t nw = 0;
  int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  mrf::DevBuf w, g, m, v;
  float mean[8] = {0}, stdv[8] = {1, 1, 1, 1, 1, 1, 1, 1};
  int logm[8] = {0};
  bool has_std = false;
  mrf::DevBuf dstd;   // device: mean[8], std[8], logm[8] (as int)
  int64_t t = 0;      // Adam step count
  // per-batch workspace
  mrf::DevBuf a1, hb1, a2, hb2, y, dy, da, db, X, T, red, scal;
  mrf::DevBuf gpart;  // split-K partial sums of the weight gradients
  mrf::DevBuf wb;     // BF16 copies of W1 [H][round_up(I, 32)] and W2 [H][H] for inference
  uint64_t wver = 1;  // bumped by every write of w
  uint64_t wbver = 0; // the w version wb was made from
  double *host_scal = nullptr;
  ~mrf_net_s() {
    if (host_scal) (void)hipHostFree(host_scal);
  }
};
