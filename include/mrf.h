/*
 * mrf.h - C ABI of the MI355X matched-filter / projected-gradient library.
 *
 * The library computes, on one AMD Instinct MI355X (gfx950), the hot path
 * of iterative MRF reconstruction by projected gradient (BLIP, and the
 * inexact variants of CoverBLIP; Golbabaee, Chen, Wiaux, Davies, "CoverBLIP:
 * accelerated and scalable iterative matched-filtering for Magnetic Resonance
 * Fingerprint reconstruction"):
 *
 *     X^{k+1} = P_cone(D)( X^k - mu_k A^H W (A X^k - Y) )          (eq. blip, eq. blip_dcf)
 *
 * with A = P_Omega F S (eq. forward: per-frame unitary 2-D DFT on a Cartesian
 * grid or a non-uniform Fourier transform for spiral readouts, k-space
 * subsampling, optional coil sensitivities S) and P_cone(D) the per-voxel
 * matched filter (eq. exactP / exactPs): nearest normalised atom, then the
 * proton density gamma_v = max(Re<Z_v, D_j*>/||D_j*||^2, 0) — exhaustive,
 * by a learned proposal with an exact local search, or by the cover tree;
 * optionally in the temporal subspace of the dictionary (eq. CS1) and with
 * a complex proton density by phase alignment.
 *
 * Conventions (apply to every entry point):
 *  - Every call returns mrf_status; MRF_OK is 0 and errors are negative.  No
 *    C++ exception or abort crosses the ABI.  mrf_last_error() returns a
 *    thread-local message describing the last failing call of this thread.
 *  - Pointers documented DEVICE are device (HBM) addresses owned by the
 *    caller; HOST pointers are host memory owned by the caller.  The library
 *    owns only its handles (mrf_dict) and the workspace they hold.
 *  - Complex data is complex64: interleaved (re, im) float pairs.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *    and calls return without waiting, except where a stats pointer is
 *    given (then the call synchronises the stream to fill it) and the
 *    solver (which reads three scalars back per step-size trial).
 *  - Arguments are validated before anything is enqueued; a call that fails
 *    validation (MRF_E_INVAL) has no side effect.
 *  - A handle may be used by one host thread at a time.  Concurrent calls on
 *    one handle race on its workspace.
 */
#ifndef MRF_H
#define MRF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *mrf_stream; /* hipStream_t */

typedef enum {
  MRF_OK = 0,
  MRF_E_INVAL = -1,       /* bad argument: null pointer, bad size, bad enum */
  MRF_E_NOMEM = -2,       /* device allocation failed */
  MRF_E_HIP = -3,         /* a HIP runtime call failed (message has the HIP error) */
  MRF_E_UNSUPPORTED = -4, /* valid request the library does not implement */
  MRF_E_NUMERIC = -5,     /* non-finite input detected (only reported when stats are requested) */
  MRF_E_NOCONV = -6       /* step size not accepted within max_shrinks (solver) */
} mrf_status;

/* Thread-local description of the last error ("" if none). */
const char *mrf_last_error(void);
/* Library version string. */
const char *mrf_version(void);

/* ------------------------------------------------------------------------ */
/* Dictionary                                                                */
/* ------------------------------------------------------------------------ */
/* The fingerprint dictionary D = {D_j} of eq. fingerprints with its look-up
 * table of parameters.  The build normalises every atom in FP64 and keeps on
 * the device: FP32 normalised atoms, 1/||D_j|| (FP32, from FP64), the
 * parameter table (FP32) and, if asked, BF16 and FP8-E4M3 copies (the FP8
 * copy with one FP32 scale per atom). */
typedef struct mrf_dict_s *mrf_dict;

enum {
  MRF_STORE_BF16 = 1u << 1,     /* also keep a BF16 copy (precision MRF_BF16) */
  MRF_STORE_FP8 = 1u << 2,      /* also keep an FP8-E4M3 copy (precision MRF_FP8) */
  MRF_BUILD_COVERTREE = 1u << 3 /* build the cover tree of the normalised atoms (MRF_COVERTREE);
                                   real rows of at most 2048 values (L <= 1024 complex),
                                   else MRF_E_UNSUPPORTED */
};
enum { MRF_F64 = 0, MRF_F32 = 1 }; /* element type of host atom arrays */

typedef struct {
  int32_t d;          /* number of atoms, >= 1 */
  int32_t L;          /* frames per atom (temporal length), >= 1 */
  int32_t nparam;     /* parameters per atom (e.g. T1, T2[, B1], df), 1..8 */
  int32_t is_complex; /* 1: complex atoms (d x L complex); 0: real atoms (d x L) */
  const void *atoms;  /* HOST, row-major d x L (x2 interleaved if complex) */
  int32_t atoms_dtype;/* MRF_F64 or MRF_F32 */
  const double *params;     /* HOST d x nparam, the look-up table Theta_j */
  const int32_t *grid_dims; /* HOST nparam sizes when atoms are the row-major
                               product grid of the parameters (last fastest),
                               else NULL */
  uint32_t flags;           /* MRF_STORE_* */
} mrf_dict_desc;

/* Upload and normalise a dictionary (eq. fingerprints; atoms normalised as
 * the search of eq. exactP requires).  An atom of zero or non-finite norm,
 * or a non-finite parameter, is rejected (MRF_E_INVAL) before any device
 * call.  On success *out is a new handle; the host arrays may be
 * freed after the call returns (the upload completes before return). */
mrf_status mrf_dict_build(const mrf_dict_desc *desc, mrf_stream stream, mrf_dict *out);
/* Release the handle and all device memory it owns (NULL is accepted). */
mrf_status mrf_dict_destroy(mrf_dict D);

typedef struct {
  int32_t d, L, nparam, is_complex;
  int32_t K;       /* real contraction length: 2L (complex) or L (real) */
  int32_t Kp;      /* padded row pitch (elements) of the FP32 atom copy */
  int32_t Kq;      /* padded row pitch (elements) of the BF16 / FP8 copies */
  uint32_t flags;
  int64_t device_bytes; /* device memory held by the handle (excl. workspace) */
  int32_t L_full;       /* compressed dictionary (mrf_dict_compress): frames of the
                           uncompressed atoms, else 0 */
  int32_t phase_aligned; /* 1 for a phase-aligned dictionary (mrf_dict_align) */
} mrf_dict_info;
mrf_status mrf_dict_query(mrf_dict D, mrf_dict_info *info);

/* Copy the device's normalised atoms (precision MRF_FP32: float [d][K],
 * MRF_BF16: uint16 [d][K], MRF_FP8: uint8 [d][K], MRF_BF16X3: uint16
 * [d][2K] = hi K then lo K per row) into DEVICE memory `dst`
 * (row pitch K elements, 2K for MRF_BF16X3), and for MRF_FP8 the per-atom scales into DEVICE
 * `scales` [d] (else ignored).  For checks against an independent encoder. */
mrf_status mrf_dict_copy_atoms(mrf_dict D, int32_t precision, void *dst, float *scales,
                               mrf_stream stream);

/* Temporal subspace compression (Section "Dimension-reduced subspace
 * matched-filtering", eq. CS1 and the compressed updates eq. gradupdate,
 * eq. gradcompression).  From a dictionary of L frames, builds a new handle
 * *out whose atoms are Dtilde_j = V^H Dhat_j (s complex frames, normalised
 * again in FP64 as mrf_dict_build does, same parameters and grid), where V
 * (L x s, orthonormal columns) holds the s dominant eigenvectors of
 * sum_j Dhat_j Dhat_j^H over the FP32 normalised atoms of D widened to
 * FP64, in decreasing eigenvalue order, each multiplied by the unit phase
 * that makes its entry of largest magnitude (the lowest row among equal
 * magnitudes) real and positive.  The Gram matrix, its eigenvectors and the
 * compressed atoms are computed on the device in FP64 (rocBLAS zherk and
 * zgemm, rocSOLVER zheevd); the handle keeps V (FP64 on the host, FP32 on
 * the device).  `flags` are the MRF_STORE_* / MRF_BUILD_COVERTREE flags of
 * the new handle.
 *
 * With a compressed handle, mrf_match projects compressed voxels (s
 * frames) and mrf_ipg_step / mrf_ipg_solve take images of s compressed
 * frames per slice with an operator of L frames: the forward model is
 * A(V X~) and the gradient V^H A^H W (A V X~ - Y); the step rule uses the
 * compressed norm ||X~' - X~||^2 (equal to the full one, V having
 * orthonormal columns).  The call synchronises `stream`.  Errors:
 * MRF_E_INVAL (null handle, s outside 1..min(L, 512), unknown flags, a
 * compressed atom of zero norm), MRF_E_UNSUPPORTED (D already compressed),
 * MRF_E_NUMERIC (eigensolver failure), MRF_E_NOMEM, MRF_E_HIP. */
mrf_status mrf_dict_compress(mrf_dict D, int32_t s, uint32_t flags, mrf_stream stream, mrf_dict *out);
/* Phase alignment for a complex proton density (Section "CoverBLIP
 * algorithm", the phase-alignment paragraph).  Builds a new handle *out of
 * aligned atoms f_j Dhat_j: with u the first principal direction of D (the
 * dominant eigenvector of sum_j Dhat_j Dhat_j^H with the phase convention
 * of mrf_dict_compress; for a compressed D the first compressed coordinate)
 * and c_j = u^H Dhat_j, f_j = conj(c_j)/|c_j| for complex atoms and the sign
 * of Re c_j for real atoms (which stay real); f_j = 1 where c_j = 0.  Every
 * matcher and the projected-gradient entry points then run the aligned
 * projection: theta_v = angle(u^H Z_v), the search on Z_v e^{-i theta_v}
 * against the aligned atoms, gamma_v as in eq. exactPs and
 * X_v = gamma_v e^{i theta_v} f_j* Dhat_j*, i.e. the complex PD
 * rho_v = gamma_v e^{i theta_v} f_j* (pd reports |rho_v| = gamma_v; its
 * phase through mrf_match_opts.pd_phase).  A compressed D keeps its V.
 * `flags` are the MRF_STORE_* / MRF_BUILD_COVERTREE flags of the new handle.
 * Synchronises `stream`.  Errors: MRF_E_INVAL (null handle, unknown flags),
 * MRF_E_UNSUPPORTED (D already aligned), MRF_E_NUMERIC, MRF_E_NOMEM,
 * MRF_E_HIP. */
mrf_status mrf_dict_align(mrf_dict D, uint32_t flags, mrf_stream stream, mrf_dict *out);
/* V of a compressed handle into HOST `V` [L_full][s] complex (interleaved
 * FP64 pairs, row t = frame t) and its eigenvalues into HOST `lam` [s]
 * (descending); either may be NULL.  MRF_E_INVAL if C is not compressed. */
mrf_status mrf_dict_subspace(mrf_dict C, double *V, double *lam);

/* Cover tree (Section "Cover trees"), built at mrf_dict_build with
 * MRF_BUILD_COVERTREE on the host in FP64 over the normalised atoms, exactly
 * equal atoms merged into the lowest index: greedy nested nets (root atom 0,
 * sigma = max_j ||D_0 - D_j||; level i+1 keeps S_i and adds, scanning atoms
 * in increasing index, every atom farther than sigma 2^-(i+1) from all nodes
 * already in S_{i+1}; a new node's parent is its nearest node of S_i, ties to
 * the lower index), with the exact maxdist of every (level, node). */
typedef struct {
  int32_t unique_atoms;   /* atoms after merging exact duplicates */
  int32_t imax;           /* deepest level */
  int64_t entries;        /* (level, node) pairs stored for the traversal */
  double sigma;           /* root coverage radius */
} mrf_tree_info;
mrf_status mrf_dict_tree_info(mrf_dict D, mrf_tree_info *info);
/* HOST arrays of unique_atoms entries: rep (lowest dictionary index of each
 * unique atom), ins_level (level at which it became a node), parent (its
 * parent, a unique index, -1 for the root); maxdist HOST [entries] in the
 * order level-major, nodes ascending within a level (or NULL). */
mrf_status mrf_dict_tree_export(mrf_dict D, int32_t *rep, int32_t *ins_level, int32_t *parent,
                                float *maxdist);

/* ------------------------------------------------------------------------ */
/* Matched filter P_cone(D) (eq. exactP, eq. exactPs)                         */
/* ------------------------------------------------------------------------ */
enum {
  MRF_EXHAUSTIVE = 0, /* every atom scored (eq. exactP) */
  MRF_LEARNED = 1,    /* network proposal + exact local search + fallback: the cover tree
                         (eps >= 0, warm-started at the local best) when the dictionary
                         holds one, else (or with eps < 0) the exhaustive filter */
  MRF_COVERTREE = 2   /* cover-tree (1+eps)-ANNS (Algorithm 1) on Z_v/||Z_v||, warm-started */
};
enum {
  MRF_FP32 = 0,
  MRF_BF16 = 1,
  MRF_FP8 = 2,
  MRF_BF16X3 = 3 /* split BF16: x = hi + lo (both BF16, hi = RNE(x), lo = RNE(x - hi)) and
                    <z, a> ~ hi.hi + hi.lo + lo.hi on BF16 MFMA with FP32 accumulation;
                    per-term error <= 3 * 2^-16 |z_k a_k|, i.e. scores within
                    4.6e-5 ||Z|| of exact, typically ~1e-7 (close to FP32) */
};
enum { MRF_VOXEL_MAJOR = 0, MRF_FRAME_MAJOR = 1 };

typedef struct mrf_net_s *mrf_net; /* learned proposal network (see below) */

typedef struct {
  int32_t method;      /* MRF_EXHAUSTIVE or MRF_LEARNED */
  int32_t precision;   /* exhaustive scoring arithmetic: MRF_FP32, MRF_BF16X3, MRF_BF16 or
                          MRF_FP8 (FP32 accumulation on the matrix cores).  Certified (see
                          no_certificate) every precision returns the exact argmax; the
                          reduced-precision ones (BF16, FP8 with per-row scales) first take
                          each voxel's maximum, then collect every atom whose score lies
                          within the derived quantisation bound of the exactly rescored
                          best (at most 256 per voxel, else the FP32 rescan) and rescore
                          them exactly.  MRF_LEARNED: local search and exhaustive fallback
                          in MRF_FP32 or MRF_BF16X3. */
  int32_t topk;        /* unused (0..8 accepted) */
  int32_t atom_splits; /* 0 = automatic; else number of atom ranges scored in parallel */
  mrf_net net;         /* MRF_LEARNED: trained network (input length = the dictionary's K) */
  int32_t box_radius;  /* MRF_LEARNED: half-width of the local box per parameter (0 = 3) */
  float fallback_corr; /* MRF_LEARNED: fallback search below this normalised
                          correlation (0 = 0.98; negative disables the fallback) */
  int32_t recentre;    /* MRF_LEARNED: re-centre rounds when the best atom lies on an
                          interior face of the box (0 = none) */
  float eps;           /* MRF_COVERTREE: search inaccuracy eps >= 0 (Definition 3.1;
                          0 = exact).  MRF_LEARNED with a dictionary holding a tree:
                          eps >= 0 sends the fallback voxels to the cover tree with this
                          eps, eps < 0 to the exhaustive filter; NaN and +inf are errors */
  int32_t tree_capacity; /* MRF_COVERTREE and the tree fallback: candidate-set capacity per
                            query (0 = 1024); queries that outgrow it use the exhaustive filter */
  float *pd_phase;       /* DEVICE float [n] or NULL, mrf_match only: the phase (radians) of
                            the complex PD rho_v on the normalised atom Dhat_j* with a
                            phase-aligned dictionary (mrf_dict_align), 0 otherwise; the
                            projected-gradient entry points ignore it (their X carries it) */
  int32_t no_certificate; /* MRF_EXHAUSTIVE.  0 (default): the exact argmax of eq. exactP over
                            the FP32 normalised atoms, certified.  MRF_FP32 / MRF_BF16X3: the
                            scoring pass keeps each voxel's 8 best atoms (among those within
                            twice its derived error bound of the running maximum), rescored
                            exactly (FP64) while they lie within the bound of the best exact
                            score; voxels whose 8 all lie within it are rescanned (every atom
                            within the bound collected and rescored exactly, or, past 64 such
                            atoms, all atoms rescored).  MRF_BF16 / MRF_FP8: as described at
                            `precision`.  1: the scoring arithmetic's own argmax, uncertified
                            (its rounding can pick an atom whose exact score is below the
                            maximum by up to that bound); PD and corr come from the exact
                            score of the returned atom for BF16 / FP8. */
  int32_t certify_local;  /* MRF_LEARNED.  0 (default): the local search's own argmax over the
                            box (and the warm atom), in the arithmetic of `precision`.  1: that
                            argmax made exact (eq. exactP restricted to the box): the answer's
                            exact (FP64) score b is computed, a second pass over the boxes
                            collects every atom whose score reaches b minus the pass's error
                            bound, and those (and the warm atom) are rescored exactly; a voxel
                            with more than 64 such atoms, and every exhaustive fallback, takes
                            the exhaustive certificate's rescan.  Needs the voxels' FP32 rows
                            (packed whenever it is set). */
} mrf_match_opts;

typedef struct {
  int64_t n;             /* voxels processed */
  int64_t zero_voxels;   /* voxels with ||Z_v|| = 0 */
  int64_t nonfinite;     /* voxels with a NaN/Inf entry (idx = -1 for them) */
  float ms;              /* device time of the call (hipEvents on `stream`) */
  float score_ms;        /* device time of the candidate-scoring kernel alone
                            (MRF_LEARNED: the first local-search scoring kernel) */
  int32_t splits;        /* atom ranges the scoring kernel used */
  int64_t fallbacks;     /* MRF_LEARNED: voxels sent to the fallback search */
  int64_t recentred;     /* MRF_LEARNED: box re-centrings performed */
  int64_t local_atoms;   /* MRF_LEARNED: atom rows scored by the local search (incl. padding) */
  float proposal_ms;     /* MRF_LEARNED: device time of the network and cell mapping */
  float fallback_ms;     /* MRF_LEARNED: device time of the fallback search */
  float search_ms;       /* MRF_LEARNED / MRF_COVERTREE: device time of the search stage */
  int64_t distance_evals;/* MRF_COVERTREE, and MRF_LEARNED with the tree fallback: distances
                            computed by the tree search (self-children excluded) */
  int32_t tree_levels;   /* MRF_COVERTREE: level launches */
  int64_t first_box_atoms; /* MRF_LEARNED: sum over the voxels of the first local-search
                              launch of their clipped box sizes (2 K flops each) */
  int64_t cert_rescored;   /* certified exhaustive filter: atoms rescored exactly */
  int64_t cert_rescanned;  /* ... voxels rescanned (all 8 listed atoms within the bound) */
  int64_t cert_scanned;    /* ... voxels whose rescan exceeded 64 candidates (all atoms rescored) */
} mrf_match_stats;

/* Project n voxels onto cone(D).
 *   Z        DEVICE complex64.  z_layout MRF_VOXEL_MAJOR: [n][L];
 *            MRF_FRAME_MAJOR: [n/slice_voxels][L][slice_voxels] (frame images
 *            of consecutive slices), slice_voxels must divide n.
 *   warm_idx DEVICE int32 [n] or NULL: Algorithm 2's previous estimate: the
 *            index reported for voxels with ||Z_v|| = 0, and the cover tree's
 *            warm start q_c; NULL -> 0 (the root).
 *   idx      DEVICE int32 [n]: j* (lowest index among equal scores); -1 for
 *            non-finite voxels.
 *   pd       DEVICE float [n] or NULL: gamma_v of eq. exactPs.
 *   corr     DEVICE float [n] or NULL: Re<Z_v, D_j*>/(||D_j*|| ||Z_v||) (0 if Z_v = 0).
 *   X_out    DEVICE complex64, same layout as Z, or NULL: gamma_v D_j*.
 *   params_out DEVICE float [n][nparam] or NULL: Theta_{j*} (look-up table).
 * For real atoms the contraction uses Re(Z_v) and ||Z_v|| is the complex norm.
 * Returns MRF_E_UNSUPPORTED for a precision whose copy was not stored. */
mrf_status mrf_match(mrf_dict D, const mrf_match_opts *opts, int64_t n, const void *Z,
                     int32_t z_layout, int64_t slice_voxels, const int32_t *warm_idx,
                     int32_t *idx, float *pd, float *corr, void *X_out, float *params_out,
                     mrf_match_stats *stats, mrf_stream stream);

/* mrf_match for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation):
 * the exhaustive MRF_FP32 filter (certified unless opts->no_certificate),
 * with every intermediate in a fixed 32 MiB device workspace that the
 * library holds per device until the process ends; the arguments are
 * mrf_match's without the statistics.  opts NULL or method MRF_EXHAUSTIVE
 * with precision MRF_FP32 (else MRF_E_UNSUPPORTED); the dictionary's device
 * must be current (else MRF_E_INVAL).  A call whose workspace would exceed
 * 32 MiB (n_pad*Kp*4 bytes of packed voxels, n_pad = n rounded up to 256,
 * plus per voxel 64 to 512 bytes of candidate lists and 276 of the
 * certificate: about 6,000 voxels at L = 500 complex) fails with
 * MRF_E_INVAL before any device work.  Calls share the workspace: calls that
 * overlap on one device race; results are complete when the stream reaches
 * the call's end.  No hipMalloc, hipFree or allocating library call is made. */
mrf_status mrf_match_noalloc(mrf_dict D, const mrf_match_opts *opts, int64_t n, const void *Z,
                             int32_t z_layout, int64_t slice_voxels, const int32_t *warm_idx,
                             int32_t *idx, float *pd, float *corr, void *X_out, float *params_out,
                             mrf_stream stream);

/* Local matched filter around given proposals (the search stage of
 * MRF_LEARNED): for voxel v the candidates are the atoms of the box
 * prod_p [cells[v][p] - r, cells[v][p] + r] clipped to the grid (the
 * dictionary must have grid_dims, nparam <= 4); the answer is the exact
 * matched filter over that box (lowest index on ties), with opts->recentre
 * re-centring rounds and the exhaustive FP32 filter as fallback below
 * opts->fallback_corr.  cells: DEVICE int32 [n][nparam] (modified in place
 * by re-centring); fallback: DEVICE int32 [n] or NULL (1 where the fallback
 * decided).  Other arguments as mrf_match; opts->net is ignored. */
mrf_status mrf_match_local(mrf_dict D, const mrf_match_opts *opts, int64_t n, const void *Z,
                           int32_t z_layout, int64_t slice_voxels, int32_t *cells,
                           const int32_t *warm_idx, int32_t *idx, float *pd, float *corr,
                           int32_t *fallback, void *X_out, float *params_out,
                           mrf_match_stats *stats, mrf_stream stream);

/* ------------------------------------------------------------------------ */
/* Learned proposal network                                                   */
/* ------------------------------------------------------------------------ */
/* A multilayer perceptron x -> 256 -> 256 -> nout with exact GELU, mapping a
 * voxel's normalised signature x = Z_v/||Z_v|| (in the dictionary's
 * contraction layout: interleaved re/im, or the real part for real atoms) to
 * standardised parameters u_p = (f_p(theta_p) - mean_p)/std_p (f_p = ln for
 * positive wide-range parameters).  Weights are FP32 on the device, stored
 * [out][in] in one array: W1[H][I], b1[H], W2[H][H], b2[H], W3[P][H], b3[P].
 * The network only proposes a grid cell; the local search decides. */
mrf_status mrf_net_create(int32_t in_dim, int32_t hidden, int32_t nout, uint64_t seed, mrf_net *out);
mrf_status mrf_net_destroy(mrf_net net);
/* Number of FP32 parameters (the length of the arrays below). */
mrf_status mrf_net_size(mrf_net net, int64_t *count);
/* HOST arrays of `count` floats (must equal mrf_net_size). */
mrf_status mrf_net_set_params(mrf_net net, const float *host, int64_t count);
mrf_status mrf_net_get_params(mrf_net net, float *host, int64_t count);
mrf_status mrf_net_get_grads(mrf_net net, float *host, int64_t count);
/* Target standardisation (HOST arrays of nout): mean, std (> 0), log_mask. */
mrf_status mrf_net_set_standardisation(mrf_net net, const float *mean, const float *stdv,
                                       const int32_t *log_mask);
mrf_status mrf_net_get_standardisation(mrf_net net, float *mean, float *stdv, int32_t *log_mask);
/* Y = net(X): X DEVICE [B][in_dim], Y DEVICE [B][nout] (standardised). */
mrf_status mrf_net_forward(mrf_net net, const float *X, int64_t B, float *Y, mrf_stream stream);
/* The inference form MRF_LEARNED uses for its proposal (hidden width 256,
 * in_dim a multiple of 8, else MRF_E_UNSUPPORTED): X, W1 and W2 rounded to
 * BF16 (nearest, ties to even), products accumulated in FP32, the first
 * hidden layer rounded to BF16 after its GELU, the second kept in FP32, the
 * output layer in FP32.  Inside mrf_match with MRF_FP32 scoring the network
 * reads X = Z_v/||Z_v||, rounded after the scale; with MRF_BF16X3 scoring it
 * reads the BF16 high parts of the split voxel rows, RNE(Z_v), and divides
 * its first layer's FP32 accumulator by ||Z_v|| (the same network, the input
 * rounded before the scale; the proposals differ by rounding only).  Same
 * arguments as mrf_net_forward. */
mrf_status mrf_net_forward_bf16(mrf_net net, const float *X, int64_t B, float *Y, mrf_stream stream);
/* Mean-squared loss against T (DEVICE [B][nout]) and its gradients (kept in
 * the net; mrf_net_get_grads reads them).  loss (HOST, may be NULL) forces a
 * stream synchronisation. */
mrf_status mrf_net_loss_grad(mrf_net net, const float *X, const float *T, int64_t B, double *loss,
                             mrf_stream stream);
/* One Adam update (Kingma and Ba) with the stored gradients. */
mrf_status mrf_net_adam(mrf_net net, float lr, float beta1, float beta2, float eps,
                        mrf_stream stream);
/* Noisy training examples generated on the device from the dictionary:
 * sample s (global index offset + s) takes atom j ~ U{0..d-1}, SNR ~
 * U(snr_lo, snr_hi) dB and circular complex Gaussian noise, each draw a
 * counter-based SplitMix64 value keyed by `seed`; X DEVICE [B][K] rows as the
 * network input, T DEVICE [B][nout] standardised targets (or NULL), atom
 * DEVICE [B] (or NULL). */
mrf_status mrf_net_noisy_batch(mrf_net net, mrf_dict D, uint64_t seed, int64_t offset, int64_t B,
                               float snr_lo, float snr_hi, float *X, float *T, int32_t *atom,
                               mrf_stream stream);
typedef struct {
  int64_t samples;     /* training-set size (noisy atoms), e.g. 2,000,000 */
  int32_t batch;       /* e.g. 4096 */
  int32_t epochs;      /* passes over the training set */
  float lr;            /* Adam learning rate (cosine-decayed to lr_min) */
  float lr_min;
  float snr_lo, snr_hi;/* dB */
  uint64_t seed;
} mrf_train_opts;
typedef struct {
  int32_t steps;
  double first_loss, last_loss;  /* mean loss over the first / last 16 steps */
  float ms;
} mrf_train_stats;
/* Train on noisy atoms of D (standardisation set from D's parameter table
 * if not set).  Synchronises `stream`. */
mrf_status mrf_net_train(mrf_net net, mrf_dict D, const mrf_train_opts *opts,
                         mrf_train_stats *stats, mrf_stream stream);

/* ------------------------------------------------------------------------ */
/* Forward model A = P_Omega F S (eq. forward)                                */
/* ------------------------------------------------------------------------ */
/* Images are frame-major [nslices][L][ny][nx] complex64.  F is the unitary
 * 2-D DFT of each frame, k-space in unshifted FFT order.  The sampling
 * pattern is CSR over (slice, frame) pairs p = s*L + t: the samples of pair p
 * are the flat k-space indices samp_idx[samp_off[p] .. samp_off[p+1]) (ky*nx+kx),
 * which must be distinct within a pair.  dcf (optional) holds the positive
 * weights w of the weighted least squares of eq. blip_dcf, one per sample.
 * S: with ncoils = 0, S = I (one coil whose sensitivity is absorbed in X);
 * with ncoils = c >= 1, S maps each frame to its c copies multiplied pixel-wise
 * by the coil sensitivity maps smaps (the same maps for every frame), and
 * the pattern of each (slice, frame) samples every coil.  Sample arrays
 * (Y, R) then hold c*M values, coil-major ([c][M]); the dcf weights apply
 * to every coil. */
/* Non-Cartesian sampling (Section "In-vivo data with variable-density
 * spiral acquisition": F in eq. forward is a non-uniform Fourier transform).
 * A plan holds the trajectory of nslices*L (slice, frame) pairs: the
 * samples of pair p are coords[samp_off[p] .. samp_off[p+1]), each (ky, kx)
 * in cycles per pixel (|ky|, |kx| <= 1024; the transform is 1-periodic in
 * them).  The operator it defines is the non-uniform DFT
 *     y(k) = (ny nx)^(-1/2) sum_{ry<ny, rx<nx} X[ry][rx] exp(-2 pi i (ky ry + kx rx)),
 * which at grid frequencies (kappa_y/ny, kappa_x/nx) is the unitary DFT of
 * the Cartesian operator.  It is computed by gridding on the 2x
 * oversampled grid with the "exponential of semicircle" kernel of `width`
 * fine cells (4..8, 0 = 7; relative error about 10^-(width-1)) and a
 * deterministic gather for the adjoint.  samp_off and coords are HOST
 * arrays copied by the call.  Errors: MRF_E_INVAL (sizes, offsets not
 * running from 0 to nsamples, coordinates not finite or beyond 1024),
 * MRF_E_NOMEM,
 * MRF_E_HIP. */
typedef struct mrf_nufft_s *mrf_nufft;
mrf_status mrf_nufft_create(int32_t nx, int32_t ny, int32_t L, int32_t nslices, int64_t nsamples,
                            const int64_t *samp_off, const float *coords, int32_t width, mrf_nufft *out);
mrf_status mrf_nufft_destroy(mrf_nufft plan);

typedef struct {
  int32_t nx, ny;          /* powers of two, 16..256 */
  int32_t L, nslices;      /* >= 1 */
  int64_t nsamples;        /* M = samp_off[nslices*L] (per coil) */
  const int64_t *samp_off; /* DEVICE [nslices*L + 1] */
  const int32_t *samp_idx; /* DEVICE [M], each in [0, ny*nx) */
  const float *dcf;        /* DEVICE [M] or NULL (w = 1) */
  int32_t ncoils;          /* 0: S = I; c in 1..64: coil maps below */
  int32_t reserved;        /* 0 */
  const void *smaps;       /* DEVICE complex64 [nslices][c][ny][nx] (ncoils >= 1), else ignored */
  mrf_nufft nufft;         /* NULL: Cartesian samples at samp_idx; else the non-Cartesian plan
                              (same nx, ny, L, nslices, nsamples; samp_off must hold the plan's
                              offsets on the device; samp_idx is ignored) */
} mrf_op;

/* R = A X - Y  (Y NULL: R = A X), samples in CSR order (coil-major with
 * coils), DEVICE complex64 [max(ncoils,1) * M].
 * If wnorm2 is non-NULL it receives ||R||_W^2 (stream synchronised). */
mrf_status mrf_op_forward(const mrf_op *A, const void *X, const void *Y, void *R,
                          double *wnorm2, mrf_stream stream);
/* G = A^H diag(w) R (apply_dcf != 0) or A^H R, DEVICE complex64 images
 * (with coils: sum_q conj(S_q) F^H P_Omega^T R_q). */
mrf_status mrf_op_adjoint(const mrf_op *A, const void *R, int32_t apply_dcf, void *G,
                          mrf_stream stream);

/* ------------------------------------------------------------------------ */
/* Projected gradient                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
  double dx2;    /* ||X_out - X_in||^2 */
  double adx2;   /* ||A(X_out - X_in)||_W^2 */
  double f_in;   /* ||A X_in - Y||_W^2 */
  double f_out;  /* ||A X_out - Y||_W^2 */
  float ms;      /* device time of the step */
  int64_t distance_evals; /* cover-tree projection (MRF_COVERTREE, or the tree fallback of
                             MRF_LEARNED): distances computed by the tree search */
} mrf_step_stats;

/* One step of eq. blip / eq. blip_dcf at a fixed step size mu:
 *   Z = X_in - mu A^H W (A X_in - Y);  X_out = P_cone(D)(Z).
 * Y DEVICE complex64 [max(ncoils,1) * M] (coil-major); X_in, X_out DEVICE
 * frame-major images (distinct); idx_in DEVICE int32 [n] or NULL (warm index for zero voxels); idx_out,
 * pd DEVICE [n] (pd may be NULL).  stats (HOST, may be NULL) receives the
 * quantities of the step-size rule (eq. steprule) and the objectives.
 * The images have D's frame count: A->L for an uncompressed D; for a
 * compressed D (mrf_dict_compress, A->L equal to its L_full) they hold the
 * s compressed frames X~ and the step is eq. gradupdate: A X means
 * A(V X~), the gradient is V^H A^H W (A V X~ - Y) and dx2 is the compressed
 * norm.  MRF_E_INVAL if A->L differs from D's (uncompressed) frames. */
mrf_status mrf_ipg_step(mrf_dict D, const mrf_op *A, const void *Y, const void *X_in,
                        void *X_out, const int32_t *idx_in, int32_t *idx_out, float *pd,
                        float mu, const mrf_match_opts *opts, mrf_step_stats *stats,
                        mrf_stream stream);

typedef struct {
  float mu0;           /* initial step size of every iteration (Algorithm 2) */
  float zeta;          /* shrink factor > 1 (eq. steprule rule), e.g. 2 */
  int32_t adaptive;    /* 1: shrink until mu < ||dX||^2/||A dX||_W^2; 0: fixed mu */
  int32_t max_iter;    /* accepted iterations, >= 1 (the paper uses 50) */
  double rel_tol;      /* stop when (f_k - f_{k+1})/f_k < rel_tol; 0 disables */
  int32_t max_shrinks; /* MRF_E_NOCONV after this many shrinks in one iteration */
  int32_t kappa;       /* 1: rescale X^1 and mu by ||Y||/||A X^1|| after iteration 1 */
  mrf_match_opts match;
} mrf_solve_opts;

typedef struct {
  int32_t iters;          /* accepted iterations */
  int32_t total_shrinks;  /* step-size shrinks over all iterations */
  int32_t cap;            /* capacity of the HOST arrays below (0 if all NULL) */
  double *f;              /* HOST [cap] or NULL: objective after each iteration */
  float *mu;              /* HOST [cap] or NULL: accepted step size */
  int32_t *shrinks;       /* HOST [cap] or NULL: shrinks per iteration */
  double f0;              /* objective of the initial X */
  float ms;               /* device time of the whole solve */
  int64_t fallbacks;      /* MRF_LEARNED: voxels sent to the fallback search, summed
                             over every projection of the solve (step-size trials included) */
  int64_t distance_evals; /* cover-tree projections: tree distances computed, summed over
                             every projection of the solve (step-size trials included) */
} mrf_solve_stats;

/* Algorithm 2 with the exact projection: X (DEVICE frame-major, D's frame
 * count as in mrf_ipg_step: compressed frames for a compressed D) holds X^0 on
 * entry (zero it for the paper's initialisation) and the reconstruction on
 * return; idx, pd DEVICE [n]; params_out DEVICE [n][nparam] or NULL (the
 * look-up table applied to the final indices).  Synchronises `stream`. */
mrf_status mrf_ipg_solve(mrf_dict D, const mrf_op *A, const void *Y,
                         const mrf_solve_opts *opts, void *X, int32_t *idx, float *pd,
                         float *params_out, mrf_solve_stats *stats, mrf_stream stream);

/* ------------------------------------------------------------------------ */
/* Reduced-precision encodings                                                */
/* ------------------------------------------------------------------------ */
/* Encode `rows` FP32 rows of length K (DEVICE, row pitch in_pitch elements)
 * to BF16 (round to nearest even; out uint16, pitch out_pitch) or to
 * FP8-E4M3 with a per-row FP32 scale amax/448 (out uint8 codes of x/scale,
 * round to nearest even, saturating; scales DEVICE [rows]).  Padding columns
 * K..out_pitch are written as zero. */
mrf_status mrf_quantize_rows(const float *in, int64_t rows, int32_t K, int64_t in_pitch,
                             int32_t precision, void *out, int64_t out_pitch, float *scales,
                             mrf_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* MRF_H */
