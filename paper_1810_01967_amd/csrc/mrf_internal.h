// Internal declarations shared by the host library and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/mrf.h"
#include "k_finish.h"

namespace mrf {

// Row pitches: FP32 rows are padded to a multiple of 16 elements (the FP32
// scoring kernel's K chunk), reduced-precision rows to a multiple of 128
// (the FP8 MFMA K step; also a multiple of the BF16 one).
constexpr int kPitchF32 = 16;
// Longest padded FP32 row the cover-tree traversal keeps in registers
// (64 lanes x 8 float4 slices).
constexpr int kTreeMaxK = 2048;
// Elements per plane of one split-BF16 local-search stage; split rows are
// padded to a multiple of it.
constexpr int kX3Stage = 32;
constexpr int kPitchLP = 128;
// Largest temporal subspace dimension of a compressed dictionary (the V row
// of one frame is staged in LDS by the compressed sampler).
constexpr int kMaxSubspace = 512;
// Bin size (oversampled-grid cells per dimension) of the non-uniform FFT's
// sample sorting, shared by the plan builder and the spreading kernel.
constexpr int kNufftBin = 8;
// Atom / voxel row counts are padded to multiples of 256 so every tiling of
// the scoring kernels reads inside the allocation.
constexpr int kRowPad = 256;
// voxels per tile of the split-BF16 exhaustive filter (the matrix-core
// kernel's voxel tile; gathered fallback rows are padded to it)
#ifndef MRF_X3_BV
#define MRF_X3_BV 256
#endif
constexpr int kX3VoxTile = MRF_X3_BV;
// K per stage of the BF16 network kernels (32 or 64; a tuning constant); the
// first layer's BF16 weight rows are padded to a multiple of it
#ifndef MRF_MLP_BK
#define MRF_MLP_BK 32
#endif
constexpr int kMlpBK = MRF_MLP_BK;
static_assert(kRowPad % kX3VoxTile == 0, "voxel rows are padded to whole tiles");

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------- matched filter
// Pack voxel rows into the padded FP32 contraction layout [n_pad][Kp]:
// complex atoms -> interleaved (re, im) rows of length 2L; real atoms -> Re(Z)
// rows of length L.  znorm[v] = ||Z_v|| (complex norm, FP64 accumulation),
// -1 for a non-finite row.  counters (may be null: not counted)[0] += zero rows,
// counters[1] += non-finite.
// Frame-major input: Zf[s][L][npix]; with G != nullptr the packed value is
// X - mu*G (the gradient update of eq. blip), G in the same layout as X.
// vphase (optional, [n]): unit factors e^{i theta_v}; each voxel is packed
// rotated by conj(vphase[v]) (phase-aligned projection).  zx3 (optional):
// also the split-BF16 rows [n_pad][2 Kx] of the packed rows (the encoding of
// k_split_x3, zero beyond K and for rows n..n_pad).  inv (optional, [n]):
// 1/znorm (0 for zero or non-finite rows), the network's row scale.
void launch_pack_voxel_major(const float2 *Z, int64_t n, int64_t n_pad, int L, int real_atoms,
                             int Kp, float *Zp, float *znorm, unsigned long long *counters,
                             hipStream_t s, const float2 *vphase = nullptr, uint16_t *zx3 = nullptr, int Kx = 0,
                             float *inv = nullptr);
void launch_pack_frame_major(const float2 *X, const float2 *G, float mu, int64_t n, int64_t n_pad,
                             int64_t npix, int L, int real_atoms, int Kp, float *Zp, float *znorm,
                             unsigned long long *counters, hipStream_t s, const float2 *vphase = nullptr,
                             uint16_t *zx3 = nullptr, int Kx = 0);
// Phase alignment: vphase[v] = c_v/|c_v| with c_v = u^H Z_v accumulated in
// FP64 ((1, 0) where c_v is 0 or not finite); Z voxel-major [n][L], or
// frame-major X - mu G (G may be null) over slices of npix voxels.
void launch_voxel_phase(const float2 *Z, int64_t n, int L, const float2 *u, float2 *vphase, hipStream_t s);
void launch_voxel_phase_frames(const float2 *X, const float2 *G, float mu, int64_t n, int64_t npix, int L,
                               const float2 *u, float2 *vphase, hipStream_t s);
// out[v] = arg(vphase[v] * afac[idx[v]]) (0 where idx < 0): the phase of the complex PD.
void launch_pd_phase(const int32_t *idx, const float2 *vphase, const float2 *afac, int64_t n, float *out,
                     hipStream_t s);

// Exhaustive FP32 scoring with fused per-voxel argmax.  D: [d_pad][Kp] FP32
// normalised atoms; Zp: [n_pad][Kp].  Writes per-split (score, index) partials
// [splits][n]; with topk, the kCertK best pairs per split and voxel
// [splits][n][kCertK] (best first, empty slots (-inf, -1)) among the atoms
// within cw znorm[v] + wabs of the voxel's running maximum when scored.
void launch_score_f32(const float *D, const float *Zp, int d, int64_t d_pad, int64_t n,
                      int64_t n_pad, int Kp, int splits, float *part_s, int *part_j,
                      hipStream_t s, bool topk = false, const float *znorm = nullptr, float cw = 0.f,
                      float wabs = 0.f);
// The same filter over the voxel rows Zp[rows[i]] for i < *dcnt (<= cap),
// collecting every atom j with score >= thr[i] into cand[i][0..ccap)
// (count[i] = number found, which may exceed ccap; counts zeroed by the
// caller).
void launch_collect_f32_dev(const float *D, const float *Zp, const int32_t *rows, int d, int64_t d_pad,
                            int64_t cap, const unsigned int *dcnt, int Kp, const float *thr, unsigned int *count,
                            int32_t *cand, int ccap, hipStream_t s);

// Merge the per-split partial argmax, then rescale (eq. exactPs) and look up.
// gamma_hat[v] = max(score,0) is the multiplier of the normalised atom.
void launch_merge_argmax(const float *part_s, const int *part_j, int splits, int64_t n, int d,
                         const float *znorm, const int32_t *warm, const float *inv_norm,
                         const float *params, int nparam, int32_t *idx, float *pd, float *corr,
                         float *params_out, float *gamma_hat, hipStream_t s);
// Exactness certificate of the exhaustive filter (k_certify.hip).  Outputs
// and look-ups of the rescaling step, as the merge kernels take them.
struct CertOut {
  const float *znorm;
  const int32_t *warm;
  const float *inv_norm;
  const float *params;
  int nparam;
  int32_t *idx;
  float *pd;
  float *corr;
  float *params_out;
  float *gamma_hat;
};
// Voxels queued for the rescan (list/thr, count on the device), those whose
// rescan overflowed the candidate list (scan_list), and the number of exact
// rescores (statistics).  Capacity n each.
struct CertQueue {
  unsigned int *count;
  int32_t *list;
  float *thr;
  unsigned int *ccount;  // per queued voxel: candidates the rescan found (zeroed when queued)
  unsigned int *scan_count;
  int32_t *scan_list;
  unsigned long long *rescored;
};
constexpr int kCertCap = 64;  // candidates per rescanned voxel
// absolute slack of the scoring passes' error bound (flushed subnormal
// products) and of the candidate lists' window
constexpr float kCertAbs = 1e-30f;
constexpr float kCertWinAbs = 3e-30f;
// Merge the per-split lists [splits][pstride][kCertK], rescore exactly, finish
// each voxel and queue the uncertified ones; E_v = cE ||Z_v|| + eabs bounds the
// scoring pass's error, cE32 ||Z_v|| + eabs that of the FP32 rescan.
void launch_certify(const float *part_s, const int *part_j, int splits, int64_t pstride, int64_t n, int d,
                    const float *Zp, const float *D, int Kp, int K, float cE, float cE32, float eabs,
                    const CertOut &o, const CertQueue &q, hipStream_t s);
void launch_rescore_collected(const float *Zp, const float *D, int Kp, int K, int d, int64_t cap, const CertQueue &q,
                              const int32_t *cand, int ccap, const CertOut &o, hipStream_t s);
void launch_scan_exact(const float *Zp, const float *D, int Kp, int K, int d, int64_t cap, const CertQueue &q,
                       const CertOut &o, hipStream_t s);
// Reduced-precision passes: merge the split maxima, rescore the best exactly,
// finish every voxel and (certify) write its line thr[v] (in the pass's unit)
// and exact best score bex[v], zeroing ccount[v] (see k_certify.hip).
void launch_lowp_line(const float *part_s, const int *part_j, int splits, int64_t n, int d, const float *Zp,
                      const float *D, int Kp, int K, const double2 *qnorm, const float *zscale, double gq, double Nq,
                      double Ne, double eabs, const CertOut &o, float *thr, unsigned int *ccount, double *bex,
                      int certify, hipStream_t s);
// Exact rescore of the collected candidates of every voxel; overflowing voxels
// (> ccap) are queued in q for the FP32 rescan.
void launch_rescore_lowp(const float *Zp, const float *D, int Kp, int K, int d, int64_t n, const unsigned int *ccount,
                         const int32_t *cand, int ccap, const double *bex, float cE32, float eabs, const CertOut &o,
                         const CertQueue &q, hipStream_t s);
// Certified local search.  One wave per voxel: the exact (FP64) score b of
// the local search's answer best_j[v] (box maximum, the warm atom or the
// exhaustive fallback's), the voxel finished with it; voxels flagged in
// fbflag (exhaustive fallbacks) go to the FP32 rescan queue with the line
// b - (cE32 ||Z_v|| + eabs), the others get the line thr[v] = b - (cE ||Z_v||
// + eabs) in the local pass's scores (every box atom that could beat or tie b
// reaches it) and ccount[v] = 0; bex / bjx keep (b, best_j).
void launch_local_line(const float *best_s, const int32_t *best_j, const int32_t *fbflag, int64_t n, int d,
                       const float *Zp, const float *D, int Kp, int K, float cE, float cE32, float eabs,
                       const CertOut &o, float *thr, unsigned int *ccount, double *bex, int32_t *bjx,
                       const CertQueue &q, hipStream_t s);
// One wave per voxel: exact rescore of the box candidates the collect pass
// found (and of the warm atom), starting from (bex, bjx); a voxel with more
// than ccap candidates goes to the FP32 rescan queue.
void launch_rescore_local(const float *Zp, const float *D, int Kp, int K, int d, int64_t n,
                          const unsigned int *ccount, const int32_t *cand, int ccap, const double *bex,
                          const int32_t *bjx, const int32_t *warm, const int32_t *fbflag, float cE32, float eabs,
                          const CertOut &o, const CertQueue &q, hipStream_t s);
constexpr int kLowpCap = 256;  // candidates per voxel of a reduced-precision collect pass

// X_v = gamma_hat_v * Dhat_{idx_v} (zero where idx < 0), written voxel-major
// [n][L] or frame-major [S][L][npix].  With X_prev != nullptr (frame-major only)
// also writes dX = X_new - X_prev into dX and per-block FP64 partial sums of
// |dX|^2 into part (grid-sized).
void launch_write_x(const int32_t *idx, const float *gamma_hat, const float *D, int Kp,
                    int real_atoms, int64_t n, int L, int frame_major, int64_t npix,
                    float2 *X, const float2 *X_prev, float2 *dX, double *part, int *nblocks_out,
                    hipStream_t s, const float2 *vphase = nullptr);

// BF16 / FP8 row encoders (see mrf_quantize_rows); norms (optional): per row
// (||q||, ||x - q||) of the decoded row q, in FP64.
void launch_quantize_rows(const float *in, int64_t rows, int K, int64_t in_pitch, int precision,
                          void *out, int64_t out_pitch, float *scales, hipStream_t s, double2 *norms = nullptr);

// ---------------------------------------------------------------- Fourier operator
// In-place unitary 2-D DFT of `nimg` frames of ny x nx complex64 (forward:
// exp(-2 pi i k.r/N), inverse: conjugate), each 1-D pass scaled by 1/sqrt(N).
void launch_fft2(float2 *data, int64_t nimg, int ny, int nx, int inverse, hipStream_t s);
// Sampling with c coils: the images are [S][c][L][npix] and the virtual
// pairs pv = (slice * c + coil) * L + frame share the CSR pattern of pair
// slice * L + frame; sample arrays (Y, R, A) are coil-major [c][M] while
// the weights w [M] are shared by all coils (c = 1: the single-coil case).
// R[i] = K[pv image][idx[i]] - Y[i] (Y may be null); part[pv] = sum_i w_i |R_i|^2
// over the samples of virtual pair pv (w = 1 when dcf is null).
// Sample ranges are clamped to [0, M) and indices outside [0, npix) read as
// zero (scatter: are skipped), so malformed patterns cannot address outside
// the buffers.
void launch_sample(const float2 *K, int64_t npix, const int64_t *off, const int32_t *sidx,
                   const float2 *Y, const float *w, float2 *R, double *part, int nvpairs,
                   int64_t M, int L, int ncoil, hipStream_t s);
// K zero-filled (total complex elements), then K[pv image][idx[i]] = w_i R_i (w = 1 when null).
void launch_scatter(const float2 *R, const float *w, const int64_t *off, const int32_t *sidx,
                    float2 *K, int64_t npix, int nvpairs, int64_t total, int64_t M, int L, int ncoil,
                    hipStream_t s);
// part_a[pv] = sum w|A|^2 and part_ra[pv] = sum w|R + A|^2 per virtual pair; optionally R += A.
void launch_step_norms(const float2 *R, const float2 *A, const float *w, const int64_t *off,
                       int nvpairs, int64_t M, int L, int ncoil, double *part_a, double *part_ra,
                       float2 *R_update, hipStream_t s);
// Coil sensitivities maps [S][c][npix]: out [S][c][F][npix] = S_q X_f, and
// G [S][F][npix] = sum_q conj(S_q) Gc [S][c][F][npix] (coils in order).
void launch_coil_expand(const float2 *X, const float2 *maps, int S, int ncoil, int F, int64_t npix, float2 *out,
                        hipStream_t s);
void launch_coil_combine(const float2 *Gc, const float2 *maps, int S, int ncoil, int F, int64_t npix, float2 *G,
                         hipStream_t s);
// Non-uniform FFT (gridding on the 2x oversampled grid, kernel width W,
// "exponential of semicircle" parameter beta).  pad: images [nimg][ny][nx]
// -> fine grids [nimg][2ny][2nx] (centred, times the deapodisation dy dx);
// crop: the reverse; interp: samples of every virtual pair from its fine
// grid (V non-null: from the sdim compressed fine grids of its (slice,
// coil)); spread: the adjoint of interp into [nvpairs][2ny][2nx] (samples
// of each pair sorted by 8 x 8 fine-cell bins: bperm [M], boff
// [npairs][nbins + 1] offsets within the pair).
void launch_nufft_pad(const float2 *X, int64_t nimg, int ny, int nx, const float *dy, const float *dx, float2 *out,
                      hipStream_t s);
void launch_nufft_crop(const float2 *K, int64_t nimg, int ny, int nx, const float *dy, const float *dx, float2 *X,
                       hipStream_t s);
void launch_nufft_interp(const float2 *K, int ny, int nx, int W, float beta, const int64_t *off,
                         const float2 *coords, const float2 *Y, const float *w, float2 *R, double *part,
                         int nvpairs, int64_t M, int L, int ncoil, const float2 *V, int sdim, hipStream_t s);
void launch_nufft_spread(const float2 *R, const float *w, const int64_t *off, const float2 *coords,
                         const int32_t *bperm, const int32_t *boff, int ny, int nx, int W, float beta, int64_t M,
                         int L, int ncoil, int64_t nvpairs, float2 *out, hipStream_t s);

// Temporal subspace (V: FP32 complex [L][sdim], frame-major rows).
// out[r][t] = row r of the FP32 normalised atoms widened to FP64 complex.
void launch_widen(const float *dhat, int Kp, int is_complex, int64_t rows, int L, double2 *out, hipStream_t s);
// As launch_sample, with the pair image formed from the sdim compressed
// k-space images of its (slice, coil), Kc [S][c][sdim][npix]: sum_k V[t, k] Kc_k.
void launch_sample_sub(const float2 *Kc, int64_t npix, int L, int sdim, const float2 *V, const int64_t *off,
                       const int32_t *sidx, const float2 *Y, const float *w, float2 *R, double *part, int nvpairs,
                       int64_t M, int ncoil, hipStream_t s);
// X [S][L][npix] = per pixel sum_k V[t, k] Xc [S][sdim][npix].
void launch_expand_frames(const float2 *Xc, int64_t npix, int S, int L, int sdim, const float2 *V, float2 *X,
                          hipStream_t s);
// Kc [S][sdim][npix] = per pixel sum_t conj(V[t, k]) Kfull [S][L][npix]
// (S counts virtual slices: slice x coil).
void launch_compress_frames(const float2 *Kfull, int64_t npix, int S, int L, int sdim, const float2 *V, float2 *Kc,
                            hipStream_t s);
// part[p] = sum w|A|^2 and part2[p] = sum w|R + A|^2 per pair; optionally R += A.
void launch_step_norms(const float2 *R, const float2 *A, const float *w, const int64_t *off,
                       int npairs, int64_t M, double *part_a, double *part_ra, float2 *R_update,
                       hipStream_t s);
// out[0] = sum of part[0..count) in a fixed order (one block).
void launch_reduce_sum(const double *part, int64_t count, double *out, hipStream_t s);
// y = x * a (complex64, elementwise), used by the kappa rescaling.
void launch_scale(float2 *x, int64_t count, float a, hipStream_t s);
void launch_zero(void *p, int64_t bytes, hipStream_t s);

}  // namespace mrf

namespace mrf {
// params_out[v][p] = params[idx[v]][p] (0 where idx < 0).
void launch_lookup(const int32_t *idx, const float *params, int nparam, int64_t n,
                   float *params_out, hipStream_t s);
// pd[v] *= a, gamma_hat[v] *= a (kappa rescaling of the first iterate).
void launch_scale_f32(float *x, int64_t count, float a, hipStream_t s);
// Per-block FP64 partial sums of |x_i|^2 (at most 1024 blocks) into part.
void launch_norm2(const float2 *x, int64_t count, double *part, int *nblocks_out, hipStream_t s);
}  // namespace mrf

namespace mrf {
// ---------------------------------------------------------------- learned proposal
enum { GEMM_STORE = 0, GEMM_GELU = 1, GEMM_GELU_GRAD = 2 };
struct GemmEpi {
  int kind = GEMM_STORE;
  const float *bias = nullptr;     // [N], added after the row scale
  const float *rowscale = nullptr; // [M] multiplier of the accumulated sum
  float *pre = nullptr;            // GEMM_GELU: pre-activation written here (ld = ldc)
  const float *gpre = nullptr;     // GEMM_GELU_GRAD: C = acc * gelu'(gpre) (ld = ldc)
};
// C[m][n] = epi(sum_k A(m,k) B(n,k)); A(m,k) = A[m*lda+k] if a_kcontig else
// A[k*lda+m]; B likewise.  Row-major C with leading dimension ldc.
void launch_gemm(int M, int N, int K, const float *A, int64_t lda, bool a_kcontig, const float *B,
                 int64_t ldb, bool b_kcontig, float *C, int64_t ldc, const GemmEpi &epi,
                 hipStream_t s);
// C[M][N] (ldc = N) = sum_k A(m,k) B(n,k) with K split over `splits` blocks
// whose partial sums (workspace part, splits * M * N floats) are added in order.
void launch_gemm_splitk(int M, int N, int K, const float *A, int64_t lda, bool a_kcontig, const float *B,
                        int64_t ldb, bool b_kcontig, float *C, int splits, float *part, hipStream_t s);
void launch_mse(const float *y, const float *t, int64_t count, float scale, float *dy, double *part,
                int *nblocks, hipStream_t s);
void launch_colsum(const float *x, int rows, int cols, float *out, hipStream_t s);
void launch_adam(float *w, const float *g, float *m, float *v, int64_t count, float lr, float b1,
                 float b2, float eps, int64_t t, hipStream_t s);
void launch_inv_norm(const float *znorm, int64_t n, float *inv, hipStream_t s);
void launch_noisy_batch(const float *Dhat, int Kp, int L, int real_atoms, int d, const float *params,
                        int nparam, const float *mean, const float *stdv, const int *logm,
                        uint64_t key_atom, uint64_t key_snr, uint64_t key_noise, int64_t offset,
                        int64_t B, float snr_lo, float snr_hi, float *X, int ldx, float *T,
                        int32_t *atom_out, hipStream_t s);
// Start of a learned call: list[i] = i and keys[i] = 0 for i < n, the first
// nz words of z and nz2 words of z2 set to zero (counters, histogram).
struct LearnedPrep {
  int32_t *list;
  unsigned long long *keys;
  unsigned int *z;
  int nz;
  unsigned int *z2;
  int nz2;
};
__device__ __forceinline__ void learned_prep_at(int64_t i, const LearnedPrep &p, int64_t n) {
  if (i < n) {
    p.list[i] = (int32_t)i;
    p.keys[i] = 0ull;
  }
  if (i < p.nz) p.z[i] = 0u;
  if (i < p.nz2) p.z2[i] = 0u;
}
// prep (optional): that initialisation folded into the same launch.
void launch_cells(const float *Y, int64_t n, int P, const float *mean, const float *stdv,
                  const int *logm, const float *axes, const int *aoff, const int *dims, int32_t *cells,
                  hipStream_t s, const LearnedPrep *prep = nullptr);

// ---------------------------------------------------------------- local search
struct GridDims {
  int dims[4];
};
// Counting-sort buffers of the voxel grouping: per coarse key its count
// (hist), first sorted position (off), scatter cursor, and first tile
// (toff, nkeys + 1 entries: toff[nkeys] = number of tiles).
struct GroupBufs {
  unsigned int *hist, *off, *cursor, *toff;
};
int coarse_key_count(const GridDims &g, int P, int shift);
// dcnt (device, may be null) in the list kernels below: the list's length on
// the device, bounded by cnt, which then only sizes the grid.
void launch_group(const int32_t *list, int64_t cnt, const int32_t *cells, int P, int shift,
                  const GridDims &g, int32_t *keys, GroupBufs gb, int32_t *out, hipStream_t s,
                  const unsigned int *dcnt = nullptr, bool hist_cleared = false);
// Local search over the grouped list: one block per tile of <= 64 voxels of
// one coarse key.  x3 = false: FP32 rows of pitch `pitch`; x3 = true:
// split-BF16 rows of pitch/32 chunks [hi 32 | lo 32].
// One block per (tile, atom tile of the tile's bounding box); per-voxel
// maxima merge into `bestkey` by atomicMax on (score, lower atom) keys (zero
// them first, unpack after with launch_best_keys).
// Candidates of the certified local search: every atom of a voxel's box whose
// score reaches thr[v] goes to cand[v][0..ccap) (count[v] counts them all;
// zeroed by the caller).
struct LocalCollect {
  const float *thr;
  unsigned int *count;
  int32_t *cand;
  int ccap;
};
void launch_local_score(const void *D, const void *Zp, int pitch, bool x3, const int32_t *order, int64_t cnt,
                        GroupBufs gb, int nkeys, const int32_t *cells, int P, const GridDims &g, int r, int shift,
                        unsigned long long *bestkey, unsigned long long *work, unsigned long long *boxsum,
                        hipStream_t s, const LocalCollect *collect = nullptr);
// mode 0: zero the keys of the listed voxels (all if list is null); mode 1:
// unpack them into best_s / best_j (-inf / -1 where no candidate).
void launch_best_keys(const int32_t *list, int64_t cnt, unsigned long long *keys, float *best_s, int32_t *best_j,
                      int mode, hipStream_t s, const unsigned int *dcnt = nullptr);
// Exhaustive split-BF16 scoring with fused argmax per atom split (Dx split
// atoms [d_pad][2 Kx], Zx split voxels [n_pad][2 Kx]); merged by
// launch_merge_argmax like the FP32 filter.
// With topk: the kCertK best pairs per split and voxel, as launch_score_f32.
void launch_score_x3(const uint16_t *Dx, const uint16_t *Zx, int d, int64_t d_pad, int64_t n, int64_t n_pad,
                     int Kx, int splits, float *part_s, int *part_j, hipStream_t s, bool topk = false,
                     const float *znorm = nullptr, float cw = 0.f, float wabs = 0.f);
// BF16 / FP8 matrix-core scoring (k_score_mx.hip): atoms D [d_pad][Kq], voxels
// Z [round_up(n, 256)][Kq] (BF16 or E4M3 values; FP8 atom scores are scaled by
// dscale[j]); per split and voxel the best (score, atom) [splits][n] (lowest
// atom on equal scores), or every atom with score >= thr[v] collected into
// cand[v][0..ccap) (count[v] counts them all; zeroed by the caller).
int mx_auto_splits(int64_t d_pad, int64_t n);
void launch_score_mx(bool fp8, const void *D, const float *dscale, const void *Z, int Kq, int d, int64_t d_pad,
                     int64_t n, int splits, float *part_s, int *part_j, hipStream_t s);
void launch_collect_mx(bool fp8, const void *D, const float *dscale, const void *Z, int Kq, int d, int64_t d_pad,
                       int64_t n, int splits, const float *thr, unsigned int *count, int32_t *cand, int ccap,
                       hipStream_t s);
// The split-BF16 filter over the split rows Zx[rows[i]] for i < *dcnt (<= cap),
// collecting atoms as launch_collect_f32_dev.
void launch_collect_x3_dev(const uint16_t *Dx, const uint16_t *Zx, const int32_t *rows, int d, int64_t d_pad,
                           int64_t cap, const unsigned int *dcnt, int Kx, const float *thr, unsigned int *count,
                           int32_t *cand, int ccap, hipStream_t s);
// The same filter over the first *dcnt (<= cap) rows of Zx ([round_up(cap,
// 128)][2 Kx]), the count read on the device: one block per CU loops over the
// (voxel tile, atom split) items; partial results at part[split * cap + i].
void launch_score_x3_dev(const uint16_t *Dx, const uint16_t *Zx, int d, int64_t d_pad, int64_t cap,
                         const unsigned int *dcnt, int Kx, float *part_s, int *part_j, hipStream_t s);
// BF16 inference of a hidden-256 network (layer 1 writes BF16 H1 [B][256],
// layer 2 fuses the output layer into Y [B][P]).
void launch_to_bf16(const float *src, int rows, int cols, int64_t lds, uint16_t *dst, int ldd, hipStream_t s);
void launch_mlp_bf16(int64_t B, const float *X, int64_t ldx, int K, int Kx, const float *rowscale,
                     const uint16_t *W1b, const float *b1, uint16_t *H1, const uint16_t *W2b, const float *b2,
                     const float *W3, const float *b3, int P, float *Y, hipStream_t s);
// The same network with layer 1 reading the high parts of split-BF16 rows Xs
// (pitch ldxs elements, Kx columns, Kx a multiple of the K stage) and
// applying rowscale to its accumulator.
void launch_mlp_bf16_split(int64_t B, const uint16_t *Xs, int64_t ldxs, int Kx, const float *rowscale,
                           const uint16_t *W1b, const float *b1, uint16_t *H1, const uint16_t *W2b, const float *b2,
                           const float *W3, const float *b3, int P, float *Y, hipStream_t s);
// FP32 rows [rows][Kp] -> split-BF16 rows of Kx/32 chunks [hi 32 | lo 32]
// (hi = RNE(x), lo = RNE(x - hi), zero beyond Kp); and back to [rows][hi K | lo K].
void launch_split_x3(const float *src, int Kp, int64_t rows, int Kx, uint16_t *dst, hipStream_t s);
void launch_unsplit_x3(const uint16_t *src, int64_t rows, int Kx, int K, uint16_t *dst, hipStream_t s);
// best <- the warm atom where it scores higher (ties: lower index).
void launch_warm_best(const int32_t *warm, int64_t n, int d, const float *Zp, const float *Dhat, int Kp,
                      const float *znorm, float *best_s, int32_t *best_j, hipStream_t s);
// Also resets the best key of each voxel it lists (bkey, may be null) and
// clears zero[0..nzero) (the next grouping's histogram).  With best_j null
// the best atoms are read from bkey (then required).
void launch_face(const int32_t *list, int64_t cnt, const int32_t *best_j, int32_t *cells, int P,
                 const GridDims &g, int r, int32_t *out, unsigned int *count, hipStream_t s,
                 const unsigned int *dcnt = nullptr, unsigned long long *bkey = nullptr,
                 unsigned int *zero = nullptr, int nzero = 0);
void launch_select_fallback(int64_t n, const float *best_s, const int32_t *best_j, const float *znorm,
                            float thr, int32_t *out, unsigned int *count, hipStream_t s);
// launch_best_keys (mode 1, every voxel) and launch_select_fallback in one
// pass; with fin, the voxels that do not fall back are also finished
// (finish_single; the fallbacks are finished by launch_scatter_best).
void launch_best_select(int64_t n, const unsigned long long *keys, float *best_s, int32_t *best_j,
                        const float *znorm, float thr, int32_t *out, unsigned int *count, hipStream_t s,
                        const FinishArgs *fin = nullptr);
void launch_gather_rows(const float *Zp, int Kp, const int32_t *list, int64_t cnt, int64_t cnt_pad,
                        float *out, hipStream_t s);
// rows list[i] for i < *dcnt (<= cap), zero rows up to the next multiple of
// 128; total (device, may be null) += *dcnt
void launch_gather_rows_dev(const float *Zp, int Kp, const int32_t *list, int64_t cap, const unsigned int *dcnt,
                            float *out, hipStream_t s, unsigned long long *total = nullptr);
void launch_learned_prep(const LearnedPrep &p, int64_t n, hipStream_t s);
void launch_add_count(unsigned long long *total, const unsigned int *count, hipStream_t s);
// With dcnt: cnt is the capacity (also the part stride) and the splits are
// those launch_score_x3_dev chose for the device count (ntiles = d_pad / 256).
// fin (optional): each listed voxel also finished (finish_single) from its
// merged best, in place of a later merge pass.
void launch_scatter_best(const int32_t *list, int64_t cnt, const float *part_s, const int *part_j,
                         int splits, float *best_s, int32_t *best_j, hipStream_t s,
                         const unsigned int *dcnt = nullptr, int ntiles = 0, const FinishArgs *fin = nullptr);
void launch_iota(int32_t *x, int64_t n, hipStream_t s);
}  // namespace mrf

namespace mrf {
// ---------------------------------------------------------------- cover tree
struct TreeDev {
  const float *dhat;          // FP32 normalised atoms [d_pad][Kp]
  const int32_t *node;        // per entry: unique atom
  const int32_t *rep;         // unique atom -> dictionary row
  const int32_t *uniq_of;     // dictionary row -> unique atom
  const int32_t *child_begin, *child_end;
  const float *maxdist;
  const uint8_t *is_self;
  int d;
  float sigma;
  int imax;
};
struct TreeState {
  int32_t *active, *qc, *cnt, *flags;
  float *dmin;
  int32_t *Qe;   // current candidate entries [n][cap]
  float *Qd;     // their distances
  int cap;
  unsigned long long *evals;
};
void launch_tree_init(const TreeDev &t, const float *Zp, int Kp, const float *znorm, const int32_t *warm,
                      int64_t n, const TreeState &st, hipStream_t s);
void launch_tree_level(const TreeDev &t, const float *Zp, int Kp, const float *znorm, int64_t n, int level,
                       float inv_eps, const TreeState &st, int32_t *Qe2, float *Qd2, hipStream_t s);
void launch_tree_finish(const TreeDev &t, const float *Zp, int Kp, int K, const float *znorm, int64_t n,
                        const TreeState &st, float *best_s, int32_t *best_j, hipStream_t s);
void launch_tree_select(const TreeState &st, int64_t n, int32_t *out, unsigned int *count, hipStream_t s);
// qnorm[i] = znorm[list[i]], qwarm[i] = best_j[list[i]] (0 if outside [0, d)).
void launch_gather_queries(const int32_t *list, int64_t cnt, const float *znorm, const int32_t *best_j, int d,
                           float *qnorm, int32_t *qwarm, hipStream_t s);
}  // namespace mrf
