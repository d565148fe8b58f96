// Host side of the C ABI: argument validation, dictionary handles and their
// workspace, and the projected-gradient control loop (Algorithm 2 with the
// step-size rule eq. steprule).  All device work is enqueued on the caller's
// stream through the launchers of the kernel files.
#include <algorithm>
#include <cmath>
#include <memory>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "host_common.h"
#include "k_topk.h"

using namespace mrf;

namespace mrf {

std::string &last_error() {
  static thread_local std::string e;
  return e;
}

mrf_status fail(mrf_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error() = buf;
  return st;
}

mrf_status grow(DevBuf &b, size_t bytes) {
  if (bytes <= b.cap) return MRF_OK;
  if (b.p) {
    (void)hipDeviceSynchronize();
    (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
  }
  const size_t want = bytes < 256 ? 256 : bytes;
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(MRF_E_NOMEM, "device allocation of %zu bytes failed: %s", want,
                hipGetErrorString(e));
  }
  b.cap = want;
  return MRF_OK;
}

}  // namespace mrf

extern "C" const char *mrf_last_error(void) { return last_error().c_str(); }
extern "C" const char *mrf_version(void) { return "mrf-mi355x 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// dictionary
// ---------------------------------------------------------------------------
extern "C" mrf_status mrf_dict_build(const mrf_dict_desc *desc, mrf_stream stream,
                                     mrf_dict *out) {
  last_error().clear();
  if (!desc || !out) return fail(MRF_E_INVAL, "mrf_dict_build: null desc or out");
  *out = nullptr;
  const mrf_dict_desc &q = *desc;
  if (q.d < 1 || q.L < 1) return fail(MRF_E_INVAL, "mrf_dict_build: d=%d L=%d must be >= 1", q.d, q.L);
  if (q.nparam < 1 || q.nparam > 8) return fail(MRF_E_INVAL, "mrf_dict_build: nparam=%d not in 1..8", q.nparam);
  if (q.is_complex != 0 && q.is_complex != 1) return fail(MRF_E_INVAL, "mrf_dict_build: is_complex must be 0 or 1");
  if (!q.atoms || !q.params) return fail(MRF_E_INVAL, "mrf_dict_build: null atoms or params");
  if (q.atoms_dtype != MRF_F64 && q.atoms_dtype != MRF_F32) return fail(MRF_E_INVAL, "mrf_dict_build: bad atoms_dtype");
  if (q.flags & ~(uint32_t)(MRF_STORE_BF16 | MRF_STORE_FP8 | MRF_BUILD_COVERTREE))
    return fail(MRF_E_INVAL, "mrf_dict_build: unknown flags 0x%x", q.flags);
  const int64_t K = (int64_t)(q.is_complex ? 2 : 1) * q.L;
  if (K > (1 << 20)) return fail(MRF_E_INVAL, "mrf_dict_build: L too large");
  if (q.grid_dims) {
    int64_t prod = 1;
    for (int p = 0; p < q.nparam; ++p) {
      if (q.grid_dims[p] < 1) return fail(MRF_E_INVAL, "mrf_dict_build: grid_dims[%d] < 1", p);
      prod *= q.grid_dims[p];
    }
    if (prod != q.d) return fail(MRF_E_INVAL, "mrf_dict_build: grid_dims product %lld != d %d", (long long)prod, q.d);
  }
  // atom norms in FP64 first: a zero or non-finite atom is rejected before
  // any device call
  std::vector<double> anorm((size_t)q.d);
  for (int64_t j = 0; j < q.d; ++j) {
    double nrm2 = 0.0;
    if (q.atoms_dtype == MRF_F64) {
      const double *a = static_cast<const double *>(q.atoms) + j * K;
      for (int64_t k = 0; k < K; ++k) nrm2 += a[k] * a[k];
    } else {
      const float *a = static_cast<const float *>(q.atoms) + j * K;
      for (int64_t k = 0; k < K; ++k) nrm2 += (double)a[k] * a[k];
    }
    if (!(nrm2 > 0.0) || !std::isfinite(nrm2))
      return fail(MRF_E_INVAL, "mrf_dict_build: atom %lld has zero or non-finite norm", (long long)j);
    anorm[(size_t)j] = std::sqrt(nrm2);
  }
  for (int64_t i = 0; i < (int64_t)q.d * q.nparam; ++i)
    if (!std::isfinite(q.params[i])) return fail(MRF_E_INVAL, "mrf_dict_build: non-finite parameter %lld", (long long)i);
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto *D = new mrf_dict_s();
  std::unique_ptr<mrf_dict_s> guard(D);
  HIP_TRY(hipGetDevice(&D->device));
  D->d = q.d;
  D->L = q.L;
  D->nparam = q.nparam;
  D->is_complex = q.is_complex;
  D->K = (int)K;
  D->Kp = (int)round_up(K, kPitchF32);
  D->Kx = (int)round_up(K, kX3Stage);
  D->Kq = (int)round_up(K, kPitchLP);
  D->d_pad = round_up(q.d, kRowPad);
  D->flags = q.flags;
  if (q.grid_dims) D->grid_dims.assign(q.grid_dims, q.grid_dims + q.nparam);

  TRY(grow(D->dhat, (size_t)D->d_pad * D->Kp * sizeof(float)));
  TRY(grow(D->inv_norm, (size_t)q.d * sizeof(float)));
  TRY(grow(D->params, (size_t)q.d * q.nparam * sizeof(float)));
  // normalise in FP64 on the host, upload FP32 rows in chunks
  const int64_t chunk = 8192;
  std::vector<float> stage((size_t)chunk * D->Kp);
  std::vector<float> inv((size_t)q.d);
  const bool tree = (q.flags & MRF_BUILD_COVERTREE) != 0;
  if (tree && D->Kp > kTreeMaxK)
    return fail(MRF_E_UNSUPPORTED, "mrf_dict_build: cover tree supports rows of at most %d reals", kTreeMaxK);
  std::vector<double> xnorm;  // FP64 normalised rows for the cover tree
  if (tree) xnorm.resize((size_t)q.d * K);
  for (int64_t r0 = 0; r0 < D->d_pad; r0 += chunk) {
    const int64_t r1 = std::min<int64_t>(r0 + chunk, D->d_pad);
    std::fill(stage.begin(), stage.end(), 0.f);
    for (int64_t j = r0; j < r1; ++j) {
      if (j >= q.d) continue;
      const double nrm = anorm[(size_t)j];
      if (q.atoms_dtype == MRF_F64) {
        const double *a = static_cast<const double *>(q.atoms) + j * K;
        for (int64_t k = 0; k < K; ++k) stage[(size_t)(j - r0) * D->Kp + k] = (float)(a[k] / nrm);
        if (tree)
          for (int64_t k = 0; k < K; ++k) xnorm[(size_t)(j * K + k)] = a[k] / nrm;
        inv[(size_t)j] = (float)(1.0 / nrm);
      } else {
        const float *a = static_cast<const float *>(q.atoms) + j * K;
        for (int64_t k = 0; k < K; ++k) stage[(size_t)(j - r0) * D->Kp + k] = (float)((double)a[k] / nrm);
        if (tree)
          for (int64_t k = 0; k < K; ++k) xnorm[(size_t)(j * K + k)] = (double)a[k] / nrm;
        inv[(size_t)j] = (float)(1.0 / nrm);
      }
    }
    HIP_TRY(hipMemcpy(D->dhat.as<float>() + r0 * D->Kp, stage.data(),
                      (size_t)(r1 - r0) * D->Kp * sizeof(float), hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMemcpy(D->inv_norm.p, inv.data(), inv.size() * sizeof(float), hipMemcpyHostToDevice));
  std::vector<float> pf((size_t)q.d * q.nparam);
  for (size_t i = 0; i < pf.size(); ++i) pf[i] = (float)q.params[i];
  D->params_host.assign(q.params, q.params + (size_t)q.d * q.nparam);
  if (q.grid_dims) {
    // axis p value i: the parameter p of the atom with sub-index i on axis p, 0 elsewhere
    std::vector<float> ax;
    std::vector<int32_t> aoff, dims;
    D->axes_host.resize(q.nparam);
    for (int p = 0; p < q.nparam; ++p) {
      int64_t stride = 1;
      for (int r = p + 1; r < q.nparam; ++r) stride *= q.grid_dims[r];
      aoff.push_back((int32_t)ax.size());
      dims.push_back(q.grid_dims[p]);
      for (int i = 0; i < q.grid_dims[p]; ++i) {
        const double v = q.params[(size_t)(i * stride) * q.nparam + p];
        D->axes_host[p].push_back(v);
        ax.push_back((float)v);
      }
    }
    TRY(grow(D->axes, ax.size() * 4));
    TRY(grow(D->aoff, aoff.size() * 4));
    TRY(grow(D->dims, dims.size() * 4));
    HIP_TRY(hipMemcpy(D->axes.p, ax.data(), ax.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(D->aoff.p, aoff.data(), aoff.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(D->dims.p, dims.data(), dims.size() * 4, hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMemcpy(D->params.p, pf.data(), pf.size() * sizeof(float), hipMemcpyHostToDevice));
  D->bytes = (int64_t)(D->dhat.cap + D->inv_norm.cap + D->params.cap);
  // reduced-precision copies, with the largest decoded-row and quantisation
  // error norms over the atoms (the certificate's per-dictionary constants)
  DevBuf qn;
  std::vector<double> qnh;
  auto qmax = [&](double *out) -> mrf_status {
    qnh.resize((size_t)2 * q.d);
    HIP_TRY(hipMemcpyAsync(qnh.data(), qn.p, qnh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    out[0] = out[1] = 0.0;
    for (int64_t j = 0; j < q.d; ++j) {
      out[0] = std::max(out[0], qnh[(size_t)2 * j]);
      out[1] = std::max(out[1], qnh[(size_t)2 * j + 1]);
    }
    return MRF_OK;
  };
  if (q.flags & (MRF_STORE_BF16 | MRF_STORE_FP8)) TRY(grow(qn, (size_t)D->d_pad * 16));
  if (q.flags & MRF_STORE_BF16) {
    TRY(grow(D->dbf16, (size_t)D->d_pad * D->Kq * 2));
    launch_quantize_rows(D->dhat.as<float>(), D->d_pad, D->K, D->Kp, MRF_BF16, D->dbf16.p, D->Kq,
                         nullptr, s, qn.as<double2>());
    LAUNCH_CHECK("quantize_rows(bf16)");
    TRY(qmax(D->qn_bf16));
    D->bytes += (int64_t)D->dbf16.cap;
  }
  if (q.flags & MRF_STORE_FP8) {
    TRY(grow(D->dfp8, (size_t)D->d_pad * D->Kq));
    TRY(grow(D->fp8_scale, (size_t)D->d_pad * sizeof(float)));
    launch_quantize_rows(D->dhat.as<float>(), D->d_pad, D->K, D->Kp, MRF_FP8, D->dfp8.p, D->Kq,
                         D->fp8_scale.as<float>(), s, qn.as<double2>());
    LAUNCH_CHECK("quantize_rows(fp8)");
    TRY(qmax(D->qn_fp8));
    D->bytes += (int64_t)(D->dfp8.cap + D->fp8_scale.cap);
  }
  if (tree) TRY(upload_tree(D, xnorm.data()));
  HIP_TRY(hipHostMalloc((void **)&D->host_scal, 16 * sizeof(double), hipHostMallocDefault));
  HIP_TRY(hipStreamSynchronize(s));
  *out = guard.release();
  return MRF_OK;
}

extern "C" mrf_status mrf_dict_destroy(mrf_dict D) {
  last_error().clear();
  if (!D) return MRF_OK;
  (void)hipDeviceSynchronize();
  delete D;
  return MRF_OK;
}

extern "C" mrf_status mrf_dict_query(mrf_dict D, mrf_dict_info *info) {
  last_error().clear();
  if (!D || !info) return fail(MRF_E_INVAL, "mrf_dict_query: null argument");
  info->d = D->d;
  info->L = D->L;
  info->nparam = D->nparam;
  info->is_complex = D->is_complex;
  info->K = D->K;
  info->Kp = D->Kp;
  info->Kq = D->Kq;
  info->flags = D->flags;
  info->device_bytes = D->bytes;
  info->L_full = D->Lfull;
  info->phase_aligned = D->align;
  return MRF_OK;
}

extern "C" mrf_status mrf_dict_copy_atoms(mrf_dict D, int32_t precision, void *dst, float *scales,
                                          mrf_stream stream) {
  last_error().clear();
  if (!D || !dst) return fail(MRF_E_INVAL, "mrf_dict_copy_atoms: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (precision == MRF_FP32) {
    HIP_TRY(hipMemcpy2DAsync(dst, (size_t)D->K * 4, D->dhat.p, (size_t)D->Kp * 4, (size_t)D->K * 4,
                             D->d, hipMemcpyDeviceToDevice, s));
  } else if (precision == MRF_BF16) {
    if (!D->dbf16.p) return fail(MRF_E_UNSUPPORTED, "mrf_dict_copy_atoms: no BF16 copy stored");
    HIP_TRY(hipMemcpy2DAsync(dst, (size_t)D->K * 2, D->dbf16.p, (size_t)D->Kq * 2,
                             (size_t)D->K * 2, D->d, hipMemcpyDeviceToDevice, s));
  } else if (precision == MRF_FP8) {
    if (!D->dfp8.p) return fail(MRF_E_UNSUPPORTED, "mrf_dict_copy_atoms: no FP8 copy stored");
    if (!scales) return fail(MRF_E_INVAL, "mrf_dict_copy_atoms: FP8 needs scales");
    HIP_TRY(hipMemcpy2DAsync(dst, (size_t)D->K, D->dfp8.p, (size_t)D->Kq, (size_t)D->K, D->d,
                             hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(scales, D->fp8_scale.p, (size_t)D->d * 4, hipMemcpyDeviceToDevice, s));
  } else if (precision == MRF_BF16X3) {
    TRY(ensure_x3(D, s));
    launch_unsplit_x3(D->dx3.as<uint16_t>(), D->d, D->Kx, D->K, static_cast<uint16_t *>(dst), s);
    LAUNCH_CHECK("copy split atoms");
  } else {
    return fail(MRF_E_INVAL, "mrf_dict_copy_atoms: bad precision %d", precision);
  }
  return MRF_OK;
}

// ---------------------------------------------------------------------------
// matched filter
// ---------------------------------------------------------------------------
namespace mrf {

mrf_status check_opts(const mrf_dict_s *D, const mrf_match_opts *o) {
  if (!o) return MRF_OK;
  if (o->method != MRF_EXHAUSTIVE && o->method != MRF_LEARNED && o->method != MRF_COVERTREE)
    return fail(MRF_E_INVAL, "unknown method %d", o->method);
  if (o->method == MRF_LEARNED) TRY(check_learned(D, o, true));
  if (o->method == MRF_COVERTREE) {
    if (!D->has_tree) return fail(MRF_E_UNSUPPORTED, "MRF_COVERTREE needs MRF_BUILD_COVERTREE at build");
    if (!(o->eps >= 0.f) || !std::isfinite(o->eps)) return fail(MRF_E_INVAL, "eps must be >= 0");
    if (o->tree_capacity < 0 || o->tree_capacity > (1 << 16)) return fail(MRF_E_INVAL, "bad tree_capacity");
    if (D->Kp % 4 != 0) return fail(MRF_E_INVAL, "internal pitch");
  }
  if (o->precision < MRF_FP32 || o->precision > MRF_BF16X3) return fail(MRF_E_INVAL, "bad precision %d", o->precision);
  if (o->method == MRF_LEARNED && o->precision != MRF_FP32 && o->precision != MRF_BF16X3)
    return fail(MRF_E_INVAL, "MRF_LEARNED scores in MRF_FP32 or MRF_BF16X3");
  if (o->topk < 0 || o->topk > 8) return fail(MRF_E_INVAL, "topk %d not in 0..8", o->topk);
  if (o->atom_splits < 0) return fail(MRF_E_INVAL, "atom_splits must be >= 0");
  if (o->precision == MRF_BF16 && !D->dbf16.p) return fail(MRF_E_UNSUPPORTED, "BF16 scoring needs MRF_STORE_BF16 at build");
  if (o->precision == MRF_FP8 && !D->dfp8.p) return fail(MRF_E_UNSUPPORTED, "FP8 scoring needs MRF_STORE_FP8 at build");
  return MRF_OK;
}

int auto_splits(const mrf_dict_s *D, int64_t n) {
  const int64_t nvt = (n + 127) / 128;
  const int64_t nvt8 = (nvt + 7) / 8 * 8;
  const int64_t ntiles = D->d_pad / 128;
  int64_t s = (1024 + nvt8 - 1) / nvt8;
  if (s < 1) s = 1;
  if (s > ntiles) s = ntiles;
  if (s > 64) s = 64;
  return (int)s;
}

// Atom splits of the split-BF16 filter (256-atom tiles, kX3VoxTile-voxel
// tiles): about 1,024 blocks.
int auto_splits_x3(const mrf_dict_s *D, int64_t n) {
  const int64_t nvt = round_up(n, kRowPad) / kX3VoxTile;
  const int64_t nvt8 = (nvt + 7) / 8 * 8;
  const int64_t ntiles = D->d_pad / 256;
  int64_t s = (1024 + nvt8 - 1) / nvt8;
  if (s < 1) s = 1;
  if (s > ntiles) s = ntiles;
  if (s > 64) s = 64;
  return (int)s;
}

// Error bound of a scoring pass, |s_hat - s| <= c ||Z_v|| + kCertAbs for every
// atom, with s the exact score over the FP32 normalised atoms (unit norm up to
// 2^-24 per element) and Z_v the packed FP32 row.  Each product and addition of
// the matrix-core accumulation is taken to round with relative error at most
// u = 2^-24 in any order of evaluation, so a sum of N terms is within
// gamma_N = N u / (1 - N u) of exact times the sum of their magnitudes (the
// standard bound of recursive or blocked summation), here at most ||Z_v||.
//   FP32: K products of the exact operands, gamma_K.
//   split BF16: z = hi + lo + e with |e| <= 2^-16 |z| (both operands), the
//     dropped lo.lo term at most 2^-16 (1 + 2^-8)^2 |z a|, so the three exact
//     BF16 products per element miss z a by at most 3.008 2^-16 |z a|; their
//     3K-term FP32 sum adds gamma_3K times at most 1.016 sum |z a|.
// The factor 1.01 covers the FP32 rounding of ||Z_v|| and of the unit norm;
// kCertAbs covers flushed subnormal products.
double gamma_n(double N) {
  const double u = 0x1p-24;
  return N * u / (1.0 - N * u);
}
float cert_coeff(int precision, int K) {
  if (precision == MRF_BF16X3) return (float)(1.01 * (3.02 * 0x1p-16 + 1.016 * gamma_n(3.0 * K)));
  return (float)(1.01 * gamma_n((double)K));
}

// Window of the scoring passes' candidate lists: more than twice the bound.
float cert_window(float cE) { return 2.02f * cE; }

// Certified finish of the exhaustive filter from the per-split lists of the
// scoring pass in `precision` (MRF_FP32 or MRF_BF16X3, whose arithmetic also
// rescans; see k_certify.hip), on the buffers in b (capacity n each).
mrf_status certify_run(mrf_dict_s *D, const CertBufs &b, const float *zp, const float *znorm, const uint16_t *zx3,
                       float *gamma, const float *part_s, const int *part_j, int64_t n, int splits, int precision,
                       const int32_t *warm, int32_t *idx, float *pd, float *corr, float *params_out, hipStream_t s) {
  const float cE = cert_coeff(precision, D->K);
  launch_zero(b.counters, 64, s);
  LAUNCH_CHECK("certificate counters");
  CertQueue q{b.counters, b.list, b.thr, b.ccount, b.counters + 1, b.scan,
              reinterpret_cast<unsigned long long *>(b.counters + 2)};
  CertOut out{znorm, warm, D->inv_norm.as<float>(), D->params.as<float>(), D->nparam, idx, pd, corr, params_out,
              gamma};
  launch_certify(part_s, part_j, splits, n, n, D->d, zp, D->dhat.as<float>(), D->Kp, D->K, cE, cE, kCertAbs, out, q,
                 s);
  LAUNCH_CHECK("certify");
  if (precision == MRF_BF16X3)
    launch_collect_x3_dev(D->dx3.as<uint16_t>(), zx3, q.list, D->d, D->d_pad, n, q.count, D->Kx, q.thr, q.ccount,
                          b.cand, kCertCap, s);
  else
    launch_collect_f32_dev(D->dhat.as<float>(), zp, q.list, D->d, D->d_pad, n, q.count, D->Kp, q.thr, q.ccount,
                           b.cand, kCertCap, s);
  LAUNCH_CHECK("certificate rescan");
  launch_rescore_collected(zp, D->dhat.as<float>(), D->Kp, D->K, D->d, n, q, b.cand, kCertCap, out, s);
  LAUNCH_CHECK("certificate rescore");
  launch_scan_exact(zp, D->dhat.as<float>(), D->Kp, D->K, D->d, n, q, out, s);
  LAUNCH_CHECK("certificate scan");
  return MRF_OK;
}

size_t cert_bytes(int64_t n) { return 64 + (size_t)n * (4 * 5 + 4 * kCertCap); }

// The same on the handle's workspace (grown to n).
mrf_status certify_exhaustive(mrf_dict_s *D, int64_t n, int splits, int precision, const int32_t *warm, int32_t *idx,
                              float *pd, float *corr, float *params_out, hipStream_t s) {
  TRY(grow(D->cert, 64));
  TRY(grow(D->cert_list, (size_t)n * 4));
  TRY(grow(D->cert_thr, (size_t)n * 4));
  TRY(grow(D->cert_ccount, (size_t)n * 4));
  TRY(grow(D->cert_scan, (size_t)n * 4));
  TRY(grow(D->cert_cand, (size_t)n * kCertCap * 4));
  CertBufs b{D->cert.as<unsigned int>(), D->cert_list.as<int32_t>(), D->cert_thr.as<float>(),
             D->cert_ccount.as<unsigned int>(), D->cert_scan.as<int32_t>(), D->cert_cand.as<int32_t>()};
  TRY(certify_run(D, b, D->zp.as<float>(), D->znorm.as<float>(), D->zx3.as<uint16_t>(), D->gamma.as<float>(),
                  D->part_s.as<float>(), D->part_j.as<int>(), n, splits, precision, warm, idx, pd, corr, params_out,
                  s));
  D->cert_used = true;
  return MRF_OK;
}

// Score + merge on already packed voxels (ws zp/znorm filled for n rows).
mrf_status match_exhaustive(mrf_dict_s *D, const mrf_match_opts *o, int64_t n, const int32_t *warm,
                            int32_t *idx, float *pd, float *corr, float *params_out, hipStream_t s,
                            hipEvent_t ev_s0, hipEvent_t ev_s1, int *splits_used) {
  const int precision = o ? o->precision : MRF_FP32;
  const bool certify = !(o && o->no_certificate);
  const size_t lw = certify ? kCertK : 1;  // list length per split and voxel
  D->cert_used = false;
  int splits = (o && o->atom_splits > 0) ? o->atom_splits : auto_splits(D, n);
  const int64_t ntiles = D->d_pad / 128;
  if (splits > ntiles) splits = (int)ntiles;
  const int64_t n_pad = round_up(n, kRowPad);
  TRY(grow(D->gamma, (size_t)n * 4));
  if (splits_used) *splits_used = splits;
  if (precision == MRF_BF16X3) {
    // split BF16: voxel rows split per call, atom rows once per dictionary
    TRY(ensure_x3(D, s));
    int xs = (o && o->atom_splits > 0) ? o->atom_splits : auto_splits_x3(D, n);
    xs = (int)std::min<int64_t>(xs, D->d_pad / 256);
    if (splits_used) *splits_used = xs;
    TRY(grow(D->zx3, (size_t)n_pad * 2 * D->Kx * 2));
    TRY(grow(D->part_s, (size_t)xs * n * 4 * lw));
    TRY(grow(D->part_j, (size_t)xs * n * 4 * lw));
    if (ev_s0) HIP_TRY(hipEventRecord(ev_s0, s));
    if (!D->zx3_fresh) launch_split_x3(D->zp.as<float>(), D->Kp, n_pad, D->Kx, D->zx3.as<uint16_t>(), s);
    const float cw = cert_window(cert_coeff(MRF_BF16X3, D->K));
    launch_score_x3(D->dx3.as<uint16_t>(), D->zx3.as<uint16_t>(), D->d, D->d_pad, n, n_pad, D->Kx, xs,
                    D->part_s.as<float>(), D->part_j.as<int>(), s, certify, D->znorm.as<float>(), cw, kCertWinAbs);
    LAUNCH_CHECK("score_x3");
    if (ev_s1) HIP_TRY(hipEventRecord(ev_s1, s));
    if (certify) return certify_exhaustive(D, n, xs, MRF_BF16X3, warm, idx, pd, corr, params_out, s);
    launch_merge_argmax(D->part_s.as<float>(), D->part_j.as<int>(), xs, n, D->d, D->znorm.as<float>(), warm,
                        D->inv_norm.as<float>(), D->params.as<float>(), D->nparam, idx, pd, corr, params_out,
                        D->gamma.as<float>(), s);
    LAUNCH_CHECK("merge_argmax");
    return MRF_OK;
  }
  if (precision == MRF_FP32) {
    TRY(grow(D->part_s, (size_t)splits * n * 4 * lw));
    TRY(grow(D->part_j, (size_t)splits * n * 4 * lw));
    if (ev_s0) HIP_TRY(hipEventRecord(ev_s0, s));
    launch_score_f32(D->dhat.as<float>(), D->zp.as<float>(), D->d, D->d_pad, n, n_pad, D->Kp,
                     splits, D->part_s.as<float>(), D->part_j.as<int>(), s, certify, D->znorm.as<float>(),
                     cert_window(cert_coeff(MRF_FP32, D->K)), kCertWinAbs);
    LAUNCH_CHECK("score_f32");
    if (ev_s1) HIP_TRY(hipEventRecord(ev_s1, s));
    if (certify) return certify_exhaustive(D, n, splits, MRF_FP32, warm, idx, pd, corr, params_out, s);
    launch_merge_argmax(D->part_s.as<float>(), D->part_j.as<int>(), splits, n, D->d,
                        D->znorm.as<float>(), warm, D->inv_norm.as<float>(),
                        D->params.as<float>(), D->nparam, idx, pd, corr, params_out,
                        D->gamma.as<float>(), s);
    LAUNCH_CHECK("merge_argmax");
    return MRF_OK;
  }
  // BF16 / FP8: the pass's per-voxel maximum, rescored exactly; certified,
  // a second pass collects every atom at or above the voxel's line, all of
  // them rescored exactly (an overflowing voxel goes to the FP32 rescan)
  const bool fp8 = precision == MRF_FP8;
  TRY(grow(D->zq, (size_t)n_pad * D->Kq * (fp8 ? 1 : 2)));
  if (fp8) TRY(grow(D->zscale, (size_t)n_pad * 4));
  TRY(grow(D->lp_qn, (size_t)n_pad * 16));
  launch_quantize_rows(D->zp.as<float>(), n_pad, D->K, D->Kp, precision, D->zq.p, D->Kq,
                       fp8 ? D->zscale.as<float>() : nullptr, s, certify ? D->lp_qn.as<double2>() : nullptr);
  LAUNCH_CHECK("quantize_rows");
  // 256 x 256 matrix-core tiles
  if (!(o && o->atom_splits > 0)) splits = mx_auto_splits(D->d_pad, n);
  splits = (int)std::min<int64_t>(splits, D->d_pad / 256);
  if (splits_used) *splits_used = splits;
  TRY(grow(D->part_s, (size_t)splits * n * 4));
  TRY(grow(D->part_j, (size_t)splits * n * 4));
  const void *Dq = fp8 ? D->dfp8.p : D->dbf16.p;
  const float *dsc = fp8 ? D->fp8_scale.as<float>() : nullptr;
  if (ev_s0) HIP_TRY(hipEventRecord(ev_s0, s));
  launch_score_mx(fp8, Dq, dsc, D->zq.p, D->Kq, D->d, D->d_pad, n, splits, D->part_s.as<float>(),
                  D->part_j.as<int>(), s);
  LAUNCH_CHECK("score_lowp");
  if (ev_s1) HIP_TRY(hipEventRecord(ev_s1, s));
  CertOut out{D->znorm.as<float>(), warm, D->inv_norm.as<float>(), D->params.as<float>(), D->nparam, idx, pd, corr,
              params_out, D->gamma.as<float>()};
  const double *qd = fp8 ? D->qn_fp8 : D->qn_bf16;
  if (certify) {
    TRY(grow(D->lp_thr, (size_t)n * 4));
    TRY(grow(D->lp_b, (size_t)n * 8));
    TRY(grow(D->lp_count, (size_t)n * 4));
    TRY(grow(D->lp_cand, (size_t)n * kLowpCap * 4));
  }
  launch_lowp_line(D->part_s.as<float>(), D->part_j.as<int>(), splits, n, D->d, D->zp.as<float>(),
                   D->dhat.as<float>(), D->Kp, D->K, D->lp_qn.as<double2>(), fp8 ? D->zscale.as<float>() : nullptr,
                   gamma_n((double)D->K + 1.0), qd[0], qd[1], kCertAbs, out, D->lp_thr.as<float>(),
                   D->lp_count.as<unsigned int>(), D->lp_b.as<double>(), certify ? 1 : 0, s);
  LAUNCH_CHECK("lowp line");
  if (!certify) return MRF_OK;
  launch_collect_mx(fp8, Dq, dsc, D->zq.p, D->Kq, D->d, D->d_pad, n, splits, D->lp_thr.as<float>(),
                    D->lp_count.as<unsigned int>(), D->lp_cand.as<int32_t>(), kLowpCap, s);
  LAUNCH_CHECK("collect_lowp");
  TRY(grow(D->cert, 64));
  TRY(grow(D->cert_list, (size_t)n * 4));
  TRY(grow(D->cert_thr, (size_t)n * 4));
  TRY(grow(D->cert_ccount, (size_t)n * 4));
  TRY(grow(D->cert_scan, (size_t)n * 4));
  TRY(grow(D->cert_cand, (size_t)n * kCertCap * 4));
  launch_zero(D->cert.p, 64, s);
  unsigned int *cnt = D->cert.as<unsigned int>();
  CertQueue q{cnt, D->cert_list.as<int32_t>(), D->cert_thr.as<float>(), D->cert_ccount.as<unsigned int>(), cnt + 1,
              D->cert_scan.as<int32_t>(), reinterpret_cast<unsigned long long *>(cnt + 2)};
  launch_rescore_lowp(D->zp.as<float>(), D->dhat.as<float>(), D->Kp, D->K, D->d, n, D->lp_count.as<unsigned int>(),
                      D->lp_cand.as<int32_t>(), kLowpCap, D->lp_b.as<double>(), cert_coeff(MRF_FP32, D->K), kCertAbs,
                      out, q, s);
  LAUNCH_CHECK("rescore_lowp");
  launch_collect_f32_dev(D->dhat.as<float>(), D->zp.as<float>(), q.list, D->d, D->d_pad, n, q.count, D->Kp, q.thr,
                         q.ccount, D->cert_cand.as<int32_t>(), kCertCap, s);
  LAUNCH_CHECK("certificate rescan");
  launch_rescore_collected(D->zp.as<float>(), D->dhat.as<float>(), D->Kp, D->K, D->d, n, q,
                           D->cert_cand.as<int32_t>(), kCertCap, out, s);
  LAUNCH_CHECK("certificate rescore");
  launch_scan_exact(D->zp.as<float>(), D->dhat.as<float>(), D->Kp, D->K, D->d, n, q, out, s);
  LAUNCH_CHECK("certificate scan");
  D->cert_used = true;
  return MRF_OK;
}


mrf_status match_core(mrf_dict_s *D, const mrf_match_opts *o, int64_t n, const int32_t *warm,
                      int32_t *idx, float *pd, float *corr, float *params_out, hipStream_t s,
                      hipEvent_t ev_s0, hipEvent_t ev_s1, int *splits_used, mrf_match_stats *st) {
  if (o && o->method == MRF_LEARNED)
    return match_learned(D, o, n, warm, idx, pd, corr, params_out, nullptr, nullptr, st, s);
  if (o && o->method == MRF_COVERTREE) return match_tree(D, o, n, warm, idx, pd, corr, params_out, st, s);
  return match_exhaustive(D, o, n, warm, idx, pd, corr, params_out, s, ev_s0, ev_s1, splits_used);
}

mrf_status pack_voxels(mrf_dict_s *D, const void *Z, int32_t z_layout, int64_t slice_voxels,
                       int64_t n, hipStream_t s, bool want_x3, bool want_fp32, bool want_counts) {
  const int64_t n_pad = round_up(n, kRowPad);
  // the voxel-major packing may leave out the FP32 rows (split rows only);
  // the frame-major one always writes them
  if (!want_x3 || z_layout != MRF_VOXEL_MAJOR) want_fp32 = true;
  if (want_fp32) TRY(grow(D->zp, (size_t)n_pad * D->Kp * 4));
  D->zx3_fresh = false;
  D->zp_fresh = false;
  D->inv_fresh = false;
  uint16_t *zx3 = nullptr;
  if (want_x3) {  // split-BF16 rows written by the packing itself
    TRY(grow(D->zx3, (size_t)n_pad * 2 * D->Kx * 2));
    zx3 = D->zx3.as<uint16_t>();
  }
  TRY(grow(D->znorm, (size_t)n_pad * 4));
  TRY(grow(D->counters, 64));  // [0] zero rows, [1] non-finite rows
  unsigned long long *counters = want_counts ? D->counters.as<unsigned long long>() : nullptr;
  if (counters) launch_zero(counters, 16, s);
  const int real = D->is_complex ? 0 : 1;
  const float2 *vph = nullptr;
  if (D->align) {  // phase-aligned dictionary: voxel phases first, packed rotated
    TRY(grow(D->vphase, (size_t)n * 8));
    if (z_layout == MRF_VOXEL_MAJOR)
      launch_voxel_phase(static_cast<const float2 *>(Z), n, D->L, D->u1.as<float2>(), D->vphase.as<float2>(), s);
    else
      launch_voxel_phase_frames(static_cast<const float2 *>(Z), nullptr, 0.f, n, slice_voxels, D->L,
                                D->u1.as<float2>(), D->vphase.as<float2>(), s);
    LAUNCH_CHECK("voxel phase");
    vph = D->vphase.as<float2>();
  }
  if (z_layout == MRF_VOXEL_MAJOR) {
    // the network's row scale comes with the norms (learned matching reads it)
    TRY(grow(D->inv, (size_t)n * 4));
    launch_pack_voxel_major(static_cast<const float2 *>(Z), n, n_pad, D->L, real, D->Kp,
                            want_fp32 ? D->zp.as<float>() : nullptr, D->znorm.as<float>(), counters, s, vph,
                            zx3, D->Kx, D->inv.as<float>());
  } else
    launch_pack_frame_major(static_cast<const float2 *>(Z), nullptr, 0.f, n, n_pad, slice_voxels,
                            D->L, real, D->Kp, D->zp.as<float>(), D->znorm.as<float>(), counters, s, vph, zx3,
                            D->Kx);
  LAUNCH_CHECK("pack");
  D->zx3_fresh = want_x3;
  D->zp_fresh = want_fp32;
  D->inv_fresh = z_layout == MRF_VOXEL_MAJOR;
  return MRF_OK;
}

}  // namespace mrf

extern "C" mrf_status mrf_match(mrf_dict D, const mrf_match_opts *opts, int64_t n, const void *Z,
                                int32_t z_layout, int64_t slice_voxels, const int32_t *warm_idx,
                                int32_t *idx, float *pd, float *corr, void *X_out,
                                float *params_out, mrf_match_stats *stats, mrf_stream stream) {
  last_error().clear();
  if (!D) return fail(MRF_E_INVAL, "mrf_match: null dictionary");
  TRY(check_opts(D, opts));
  if (n < 0) return fail(MRF_E_INVAL, "mrf_match: n < 0");
  if (n > 0 && (!Z || !idx)) return fail(MRF_E_INVAL, "mrf_match: null Z or idx");
  if (z_layout != MRF_VOXEL_MAJOR && z_layout != MRF_FRAME_MAJOR)
    return fail(MRF_E_INVAL, "mrf_match: bad z_layout %d", z_layout);
  if (z_layout == MRF_FRAME_MAJOR && (slice_voxels < 1 || n % slice_voxels != 0))
    return fail(MRF_E_INVAL, "mrf_match: slice_voxels must divide n for the frame-major layout");
  if (n > ((int64_t)1 << 31) - 1024) return fail(MRF_E_INVAL, "mrf_match: n too large");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (n == 0) return MRF_OK;
  EventPair ev;
  if (stats) {
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    HIP_TRY(hipEventCreate(&ev.c));
    HIP_TRY(hipEventCreate(&ev.d));
    HIP_TRY(hipEventRecord(ev.a, s));
  }
  const int real = D->is_complex ? 0 : 1;
  const bool want_x3 = opts && opts->precision == MRF_BF16X3 && opts->method != MRF_COVERTREE;
  TRY(pack_voxels(D, Z, z_layout, slice_voxels, n, s, want_x3, !learned_split_rows_only(D, opts, warm_idx, false),
                  stats != nullptr));
  int splits_used = 0;
  TRY(match_core(D, opts, n, warm_idx, idx, pd, corr, params_out, s, ev.c, ev.d, &splits_used, stats));
  const float2 *vph = D->align ? D->vphase.as<float2>() : nullptr;
  if (X_out) {
    launch_write_x(idx, D->gamma.as<float>(), D->dhat.as<float>(), D->Kp, real, n, D->L,
                   z_layout == MRF_FRAME_MAJOR, slice_voxels, static_cast<float2 *>(X_out),
                   nullptr, nullptr, nullptr, nullptr, s, vph);
    LAUNCH_CHECK("write_x");
  }
  if (opts && opts->pd_phase) {
    if (vph)
      launch_pd_phase(idx, vph, D->afac.as<float2>(), n, opts->pd_phase, s);
    else
      launch_zero(opts->pd_phase, n * (int64_t)sizeof(float), s);  // real, non-negative PD
    LAUNCH_CHECK("pd phase");
  }
  if (stats) {
    HIP_TRY(hipEventRecord(ev.b, s));
    unsigned long long cnt[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(cnt, D->counters.p, sizeof cnt, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipEventElapsedTime(&stats->ms, ev.a, ev.b));
    if (!opts || opts->method == MRF_EXHAUSTIVE) HIP_TRY(hipEventElapsedTime(&stats->score_ms, ev.c, ev.d));
    if ((!opts || opts->method == MRF_EXHAUSTIVE) && D->cert_used) {
      uint32_t c[4] = {0, 0, 0, 0};
      HIP_TRY(hipMemcpy(c, D->cert.p, sizeof c, hipMemcpyDeviceToHost));
      uint64_t r;
      std::memcpy(&r, c + 2, sizeof r);
      stats->cert_rescored = (int64_t)r;
      stats->cert_rescanned = c[0];
      stats->cert_scanned = c[1];
    }
    stats->splits = splits_used;
    stats->n = n;
    stats->zero_voxels = (int64_t)cnt[0];
    stats->nonfinite = (int64_t)cnt[1];
    if (cnt[1] > 0)
      return fail(MRF_E_NUMERIC, "mrf_match: %llu voxel(s) with non-finite entries", cnt[1]);
  }
  return MRF_OK;
}

// ---------------------------------------------------------------------------
// forward model
// ---------------------------------------------------------------------------
namespace {

bool pow2_in(int x, int lo, int hi) { return x >= lo && x <= hi && (x & (x - 1)) == 0; }

mrf_status check_op(const mrf_op *A) {
  if (!A) return fail(MRF_E_INVAL, "null operator");
  if (!pow2_in(A->nx, 16, 256) || !pow2_in(A->ny, 16, 256))
    return fail(MRF_E_INVAL, "nx=%d ny=%d must be powers of two in 16..256", A->nx, A->ny);
  if (A->L < 1 || A->nslices < 1) return fail(MRF_E_INVAL, "L and nslices must be >= 1");
  if (A->nsamples < 0) return fail(MRF_E_INVAL, "nsamples < 0");
  if (!A->samp_off) return fail(MRF_E_INVAL, "null sampling offsets");
  if (A->nufft) {
    const mrf_nufft_s *P = A->nufft;
    if (P->nx != A->nx || P->ny != A->ny || P->L != A->L || P->nslices != A->nslices || P->M != A->nsamples)
      return fail(MRF_E_INVAL, "operator sizes differ from its non-uniform FFT plan");
  } else if (A->nsamples > 0 && !A->samp_idx) {
    return fail(MRF_E_INVAL, "null sampling arrays");
  }
  if (A->ncoils < 0 || A->ncoils > 64) return fail(MRF_E_INVAL, "ncoils=%d not in 0..64", A->ncoils);
  if (A->ncoils >= 1 && !A->smaps) return fail(MRF_E_INVAL, "ncoils=%d needs smaps", A->ncoils);
  if ((int64_t)A->nslices * std::max(A->ncoils, 1) * A->L > (1 << 30)) return fail(MRF_E_INVAL, "too many frames");
  return MRF_OK;
}

// Sizes of the operator: coils (1 without maps), the maps, the virtual
// (slice, coil, frame) pairs and the coil-major sample count.
struct OpDims {
  int64_t npix;
  int nc;
  const float2 *maps;
  int64_t nvpairs;
  int64_t nsamp;
};
OpDims dims_of(const mrf_op *A) {
  OpDims o;
  o.npix = (int64_t)A->nx * A->ny;
  o.nc = A->ncoils >= 1 ? A->ncoils : 1;
  o.maps = A->ncoils >= 1 ? static_cast<const float2 *>(A->smaps) : nullptr;
  o.nvpairs = (int64_t)A->nslices * o.nc * A->L;
  o.nsamp = (int64_t)o.nc * A->nsamples;
  return o;
}

// Images img [S'][F][npix] (S' = slices x coils; overwritten by the
// Cartesian path) to samples: R = (A img) - Y at every virtual pair, with
// per-pair weighted norms into part.  F = Dsub->L compressed frames when Dsub
// is a compressed dictionary (each sample then combines them with its
// frame's row of V), else A->L.  Cartesian: FFT in place, gather;
// non-Cartesian: pad onto the oversampled grids (ws->nbuf), FFT, interpolate.
mrf_status transform_sample(mrf_dict_s *ws, const mrf_op *A, const OpDims &o, float2 *img, int F,
                            const mrf_dict_s *Dsub, const float2 *Y, float2 *R, double *part, hipStream_t s) {
  const bool sub = Dsub && Dsub->Lfull > 0;
  const int64_t nkimg = (int64_t)A->nslices * o.nc * F;
  const float2 *V = sub ? Dsub->Vs.as<float2>() : nullptr;
  if (A->nufft) {
    const mrf_nufft_s *P = A->nufft;
    TRY(grow(ws->nbuf, (size_t)nkimg * 4 * o.npix * 8));
    launch_nufft_pad(img, nkimg, A->ny, A->nx, P->dy.as<float>(), P->dx.as<float>(), ws->nbuf.as<float2>(), s);
    LAUNCH_CHECK("nufft pad");
    launch_fft2(ws->nbuf.as<float2>(), nkimg, 2 * A->ny, 2 * A->nx, 0, s);
    LAUNCH_CHECK("fft2 (oversampled)");
    launch_nufft_interp(ws->nbuf.as<float2>(), A->ny, A->nx, P->W, P->beta, P->off.as<int64_t>(),
                        P->coords.as<float2>(), Y, A->dcf, R, part, (int)o.nvpairs, A->nsamples, A->L, o.nc, V,
                        sub ? Dsub->L : 1, s);
    LAUNCH_CHECK("nufft interp");
    return MRF_OK;
  }
  launch_fft2(img, nkimg, A->ny, A->nx, 0, s);
  LAUNCH_CHECK("fft2");
  if (sub)
    launch_sample_sub(img, o.npix, A->L, Dsub->L, V, A->samp_off, A->samp_idx, Y, A->dcf, R, part, (int)o.nvpairs,
                      A->nsamples, o.nc, s);
  else
    launch_sample(img, o.npix, A->samp_off, A->samp_idx, Y, A->dcf, R, part, (int)o.nvpairs, A->nsamples, A->L,
                  o.nc, s);
  LAUNCH_CHECK("sample");
  return MRF_OK;
}

// Weighted samples w R to images out [S'][F][npix] (before the coil
// combination): scatter into the zero-filled k-space of every virtual pair
// (non-Cartesian: spread onto its oversampled grid), V^H over the frames for
// a compressed dictionary, inverse transforms (non-Cartesian: then crop and
// deapodise).  Workspace: ws->kfull, ws->nbuf, ws->nbuf2.
mrf_status scatter_transform(mrf_dict_s *ws, const mrf_op *A, const OpDims &o, const float2 *R, const float *w,
                             const mrf_dict_s *Dsub, float2 *out, hipStream_t s) {
  const bool sub = Dsub && Dsub->Lfull > 0;
  const int F = sub ? Dsub->L : A->L;
  const int Sv = A->nslices * o.nc;
  const int64_t nkimg = (int64_t)Sv * F;
  const float2 *V = sub ? Dsub->Vs.as<float2>() : nullptr;
  if (A->nufft) {
    const mrf_nufft_s *P = A->nufft;
    const int64_t plane = 4 * o.npix;
    TRY(grow(ws->nbuf, (size_t)o.nvpairs * plane * 8));
    launch_nufft_spread(R, w, P->off.as<int64_t>(), P->coords.as<float2>(), P->bperm.as<int32_t>(),
                        P->boff.as<int32_t>(), A->ny, A->nx, P->W, P->beta, A->nsamples, A->L, o.nc, o.nvpairs,
                        ws->nbuf.as<float2>(), s);
    LAUNCH_CHECK("nufft spread");
    float2 *grid = ws->nbuf.as<float2>();
    if (sub) {
      TRY(grow(ws->nbuf2, (size_t)nkimg * plane * 8));
      launch_compress_frames(grid, plane, Sv, A->L, Dsub->L, V, ws->nbuf2.as<float2>(), s);
      LAUNCH_CHECK("compress frames");
      grid = ws->nbuf2.as<float2>();
    }
    launch_fft2(grid, nkimg, 2 * A->ny, 2 * A->nx, 1, s);
    LAUNCH_CHECK("ifft2 (oversampled)");
    launch_nufft_crop(grid, nkimg, A->ny, A->nx, P->dy.as<float>(), P->dx.as<float>(), out, s);
    LAUNCH_CHECK("nufft crop");
    return MRF_OK;
  }
  if (sub) {
    TRY(grow(ws->kfull, (size_t)o.nvpairs * o.npix * 8));
    launch_scatter(R, w, A->samp_off, A->samp_idx, ws->kfull.as<float2>(), o.npix, (int)o.nvpairs,
                   o.nvpairs * o.npix, A->nsamples, A->L, o.nc, s);
    LAUNCH_CHECK("scatter");
    launch_compress_frames(ws->kfull.as<float2>(), o.npix, Sv, A->L, Dsub->L, V, out, s);
    LAUNCH_CHECK("compress frames");
  } else {
    launch_scatter(R, w, A->samp_off, A->samp_idx, out, o.npix, (int)o.nvpairs, o.nvpairs * o.npix, A->nsamples,
                   A->L, o.nc, s);
    LAUNCH_CHECK("scatter");
  }
  launch_fft2(out, nkimg, A->ny, A->nx, 1, s);
  LAUNCH_CHECK("ifft2");
  return MRF_OK;
}

// R = A X - Y; partial weighted norms per virtual (slice, coil, frame) pair
// into part[0..nvpairs).  With coil maps the images are first expanded to
// their c weighted copies.  With a temporally compressed dictionary Dsub
// (Lfull > 0) X holds Dsub->L compressed frames per slice (eq. gradcompression).
mrf_status forward_into(mrf_dict_s *ws, const mrf_op *A, const float2 *X, const float2 *Y,
                        float2 *R, double *part, hipStream_t s, const mrf_dict_s *Dsub = nullptr) {
  const OpDims o = dims_of(A);
  const bool sub = Dsub && Dsub->Lfull > 0;
  int F = sub ? Dsub->L : A->L;  // image frames per slice
  const float2 *src = X;
  if (sub && A->nufft) {
    // non-uniform F: the per-sample interpolation dominates, so V acts in the
    // image domain (X = V X~ per pixel) and the transform runs on the L frames
    TRY(grow(ws->xfull, (size_t)A->nslices * A->L * o.npix * 8));
    launch_expand_frames(X, o.npix, A->nslices, A->L, Dsub->L, Dsub->Vs.as<float2>(), ws->xfull.as<float2>(), s);
    LAUNCH_CHECK("expand frames");
    src = ws->xfull.as<float2>();
    F = A->L;
    Dsub = nullptr;
  }
  const int64_t nkimg = (int64_t)A->nslices * o.nc * F;  // images after the coil expansion
  TRY(grow(ws->kbuf, (size_t)nkimg * o.npix * 8));
  if (o.maps) {
    launch_coil_expand(src, o.maps, A->nslices, o.nc, F, o.npix, ws->kbuf.as<float2>(), s);
    LAUNCH_CHECK("coil expand");
  } else {
    HIP_TRY(hipMemcpyAsync(ws->kbuf.p, src, (size_t)nkimg * o.npix * 8, hipMemcpyDeviceToDevice, s));
  }
  return transform_sample(ws, A, o, ws->kbuf.as<float2>(), F, Dsub, Y, R, part, s);
}

// G = A^H diag(w) R, coils combined with conj(S_q).
mrf_status adjoint_into(mrf_dict_s *ws, const mrf_op *A, const float2 *R, const float *w, float2 *G,
                        hipStream_t s, const mrf_dict_s *Dsub = nullptr) {
  const OpDims o = dims_of(A);
  const bool sub = Dsub && Dsub->Lfull > 0;
  if (sub && A->nufft) {  // the full-frame adjoint, then V^H per pixel (see forward_into)
    TRY(grow(ws->xfull, (size_t)A->nslices * A->L * o.npix * 8));
    TRY(adjoint_into(ws, A, R, w, ws->xfull.as<float2>(), s, nullptr));
    launch_compress_frames(ws->xfull.as<float2>(), o.npix, A->nslices, A->L, Dsub->L, Dsub->Vs.as<float2>(), G, s);
    LAUNCH_CHECK("compress frames");
    return MRF_OK;
  }
  const int F = sub ? Dsub->L : A->L;
  const int64_t nkimg = (int64_t)A->nslices * o.nc * F;
  float2 *Gc = G;
  if (o.maps) {
    TRY(grow(ws->cbuf, (size_t)nkimg * o.npix * 8));
    Gc = ws->cbuf.as<float2>();
  }
  TRY(scatter_transform(ws, A, o, R, w, Dsub, Gc, s));
  if (o.maps) {
    launch_coil_combine(Gc, o.maps, A->nslices, o.nc, F, o.npix, G, s);
    LAUNCH_CHECK("coil combine");
  }
  return MRF_OK;
}

// A thread-local scratch handle for the operator-only entry points.
// (never freed: its buffers may outlive the HIP runtime at process exit)
mrf_dict_s &op_scratch() {
  static thread_local mrf_dict_s *ws = new mrf_dict_s();
  return *ws;
}

}  // namespace

extern "C" mrf_status mrf_op_forward(const mrf_op *A, const void *X, const void *Y, void *R,
                                     double *wnorm2, mrf_stream stream) {
  last_error().clear();
  TRY(check_op(A));
  if (!X || !R) return fail(MRF_E_INVAL, "mrf_op_forward: null X or R");
  hipStream_t s = static_cast<hipStream_t>(stream);
  mrf_dict_s &ws = op_scratch();
  const int64_t nvpairs = dims_of(A).nvpairs;
  TRY(grow(ws.red, (size_t)(nvpairs + 8) * 8));
  TRY(forward_into(&ws, A, static_cast<const float2 *>(X), static_cast<const float2 *>(Y),
                   static_cast<float2 *>(R), ws.red.as<double>(), s));
  if (wnorm2) {
    TRY(grow(ws.scal, 64));
    launch_reduce_sum(ws.red.as<double>(), nvpairs, ws.scal.as<double>(), s);
    LAUNCH_CHECK("reduce_sum");
    HIP_TRY(hipMemcpyAsync(wnorm2, ws.scal.p, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return MRF_OK;
}

extern "C" mrf_status mrf_op_adjoint(const mrf_op *A, const void *R, int32_t apply_dcf, void *G,
                                     mrf_stream stream) {
  last_error().clear();
  TRY(check_op(A));
  if (!R || !G) return fail(MRF_E_INVAL, "mrf_op_adjoint: null R or G");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return adjoint_into(&op_scratch(), A, static_cast<const float2 *>(R), apply_dcf ? A->dcf : nullptr,
                      static_cast<float2 *>(G), s);
}

// ---------------------------------------------------------------------------
// projected gradient
// ---------------------------------------------------------------------------
namespace {

mrf_status check_step_args(mrf_dict_s *D, const mrf_op *A, const void *Y) {
  if (!D) return fail(MRF_E_INVAL, "null dictionary");
  TRY(check_op(A));
  const int L = D->Lfull > 0 ? D->Lfull : D->L;
  if (A->L != L) return fail(MRF_E_INVAL, "operator L=%d differs from the dictionary's frames L=%d", A->L, L);
  if (A->nsamples > 0 && !Y) return fail(MRF_E_INVAL, "null Y");
  return MRF_OK;
}

// Given R = A X - Y (workspace rbuf) and G (gbuf): Z = X - mu G, project,
// write X_new (and dX into kbuf), A dX into abuf, and reduce
// scal[0] = ||dX||^2, scal[1] = ||A dX||_W^2, scal[2] = ||R + A dX||_W^2.
mrf_status trial(mrf_dict_s *D, const mrf_op *A, const mrf_match_opts *o, const float2 *X,
                 float mu, const int32_t *warm, float2 *X_new, int32_t *idx, float *pd,
                 float2 *R_update, hipStream_t s) {
  const OpDims od = dims_of(A);
  const int64_t npix = od.npix;
  const int64_t n = (int64_t)A->nslices * npix;
  const int64_t nimg = (int64_t)A->nslices * D->L;   // image frames (compressed frames if Lfull > 0)
  const int64_t nvp = od.nvpairs;                    // sampled (slice, coil, frame) pairs
  const int64_t n_pad = round_up(n, kRowPad);
  const int real = D->is_complex ? 0 : 1;
  TRY(grow(D->zp, (size_t)n_pad * D->Kp * 4));
  TRY(grow(D->znorm, (size_t)n_pad * 4));
  TRY(grow(D->kbuf, (size_t)nimg * npix * 8));
  TRY(grow(D->abuf, (size_t)(od.nsamp > 0 ? od.nsamp : 1) * 8));
  TRY(grow(D->red, (size_t)(8192 + 2 * nvp + 8) * 8));
  TRY(grow(D->scal, 64));
  const float2 *vph = nullptr;
  if (D->align) {  // phase-aligned projection of Z = X - mu G
    TRY(grow(D->vphase, (size_t)n * 8));
    launch_voxel_phase_frames(X, D->gbuf.as<float2>(), mu, n, npix, D->L, D->u1.as<float2>(),
                              D->vphase.as<float2>(), s);
    LAUNCH_CHECK("voxel phase");
    vph = D->vphase.as<float2>();
  }
  const bool want_x3 = o && o->precision == MRF_BF16X3 && o->method != MRF_COVERTREE;
  if (want_x3) TRY(grow(D->zx3, (size_t)n_pad * 2 * D->Kx * 2));
  launch_pack_frame_major(X, D->gbuf.as<float2>(), mu, n, n_pad, npix, D->L, real, D->Kp,
                          D->zp.as<float>(), D->znorm.as<float>(), nullptr, s, vph,
                          want_x3 ? D->zx3.as<uint16_t>() : nullptr, D->Kx);  // row counts not read here
  LAUNCH_CHECK("grad_update_pack");
  D->zx3_fresh = want_x3;
  D->zp_fresh = true;
  D->inv_fresh = false;
  TRY(match_core(D, o, n, warm, idx, pd, nullptr, nullptr, s, nullptr, nullptr, nullptr, nullptr));
  double *red = D->red.as<double>();
  int nb = 0;
  launch_write_x(idx, D->gamma.as<float>(), D->dhat.as<float>(), D->Kp, real, n, D->L, 1, npix,
                 X_new, X, D->kbuf.as<float2>(), red, &nb, s, vph);
  LAUNCH_CHECK("write_x");
  launch_reduce_sum(red, nb, D->scal.as<double>() + 0, s);
  // A dX: dX sits in kbuf (full frames in xfull for a compressed iterate
  // under the non-uniform F, coil copies in cbuf with coil maps)
  float2 *K = D->kbuf.as<float2>();
  int F = D->L;
  const mrf_dict_s *tsub = D;
  if (D->Lfull > 0 && A->nufft) {
    TRY(grow(D->xfull, (size_t)A->nslices * A->L * npix * 8));
    launch_expand_frames(K, npix, A->nslices, A->L, D->L, D->Vs.as<float2>(), D->xfull.as<float2>(), s);
    LAUNCH_CHECK("expand frames(dX)");
    K = D->xfull.as<float2>();
    F = A->L;
    tsub = nullptr;
  }
  if (od.maps) {
    TRY(grow(D->cbuf, (size_t)A->nslices * od.nc * F * npix * 8));
    launch_coil_expand(K, od.maps, A->nslices, od.nc, F, npix, D->cbuf.as<float2>(), s);
    LAUNCH_CHECK("coil expand(dX)");
    K = D->cbuf.as<float2>();
  }
  TRY(transform_sample(D, A, od, K, F, tsub, nullptr, D->abuf.as<float2>(), nullptr, s));
  launch_step_norms(D->rbuf.as<float2>(), D->abuf.as<float2>(), A->dcf, A->samp_off, (int)nvp, A->nsamples,
                    A->L, od.nc, red + 8192, red + 8192 + nvp, R_update, s);
  LAUNCH_CHECK("step_norms");
  launch_reduce_sum(red + 8192, nvp, D->scal.as<double>() + 1, s);
  launch_reduce_sum(red + 8192 + nvp, nvp, D->scal.as<double>() + 2, s);
  LAUNCH_CHECK("reduce_sum");
  return MRF_OK;
}

// R = A X - Y into rbuf, ||R||_W^2 into scal[3]; G = A^H W R into gbuf.
mrf_status residual_and_gradient(mrf_dict_s *D, const mrf_op *A, const float2 *X,
                                 const float2 *Y, bool gradient, hipStream_t s) {
  const OpDims od = dims_of(A);
  const int64_t nimg = (int64_t)A->nslices * D->L;
  TRY(grow(D->rbuf, (size_t)(od.nsamp > 0 ? od.nsamp : 1) * 8));
  TRY(grow(D->gbuf, (size_t)nimg * od.npix * 8));
  TRY(grow(D->red, (size_t)(8192 + 2 * od.nvpairs + 8) * 8));
  TRY(grow(D->scal, 64));
  double *red = D->red.as<double>();
  TRY(forward_into(D, A, X, Y, D->rbuf.as<float2>(), red + 8192, s, D));
  launch_reduce_sum(red + 8192, od.nvpairs, D->scal.as<double>() + 3, s);
  LAUNCH_CHECK("reduce_sum");
  if (gradient) TRY(adjoint_into(D, A, D->rbuf.as<float2>(), A->dcf, D->gbuf.as<float2>(), s, D));
  return MRF_OK;
}

mrf_status read_scalars(mrf_dict_s *D, int count, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(D->host_scal, D->scal.p, (size_t)count * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MRF_OK;
}

}  // namespace

extern "C" mrf_status mrf_ipg_step(mrf_dict D, const mrf_op *A, const void *Y, const void *X_in,
                                   void *X_out, const int32_t *idx_in, int32_t *idx_out,
                                   float *pd, float mu, const mrf_match_opts *opts,
                                   mrf_step_stats *stats, mrf_stream stream) {
  last_error().clear();
  TRY(check_step_args(D, A, Y));
  TRY(check_opts(D, opts));
  if (!X_in || !X_out || !idx_out) return fail(MRF_E_INVAL, "mrf_ipg_step: null X_in, X_out or idx_out");
  if (X_in == X_out) return fail(MRF_E_INVAL, "mrf_ipg_step: X_in and X_out must differ");
  if (!std::isfinite(mu)) return fail(MRF_E_INVAL, "mrf_ipg_step: non-finite mu");
  hipStream_t s = static_cast<hipStream_t>(stream);
  EventPair ev;
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    HIP_TRY(hipEventRecord(ev.a, s));
    TRY(grow(D->ts_evals, 64));
    launch_zero(D->ts_evals.p, 8, s);
  }
  TRY(residual_and_gradient(D, A, static_cast<const float2 *>(X_in), static_cast<const float2 *>(Y),
                            true, s));
  TRY(trial(D, A, opts, static_cast<const float2 *>(X_in), mu, idx_in,
            static_cast<float2 *>(X_out), idx_out, pd, nullptr, s));
  if (stats) {
    HIP_TRY(hipEventRecord(ev.b, s));
    unsigned long long evals = 0;
    HIP_TRY(hipMemcpyAsync(&evals, D->ts_evals.p, 8, hipMemcpyDeviceToHost, s));
    TRY(read_scalars(D, 4, s));
    stats->distance_evals = (int64_t)evals;
    HIP_TRY(hipEventElapsedTime(&stats->ms, ev.a, ev.b));
    stats->dx2 = D->host_scal[0];
    stats->adx2 = D->host_scal[1];
    stats->f_out = D->host_scal[2];
    stats->f_in = D->host_scal[3];
  }
  return MRF_OK;
}

extern "C" mrf_status mrf_ipg_solve(mrf_dict D, const mrf_op *A, const void *Y,
                                    const mrf_solve_opts *o, void *X, int32_t *idx, float *pd,
                                    float *params_out, mrf_solve_stats *stats,
                                    mrf_stream stream) {
  last_error().clear();
  TRY(check_step_args(D, A, Y));
  if (!o) return fail(MRF_E_INVAL, "mrf_ipg_solve: null options");
  TRY(check_opts(D, &o->match));
  if (!X || !idx) return fail(MRF_E_INVAL, "mrf_ipg_solve: null X or idx");
  if (!(o->mu0 > 0.f) || !std::isfinite(o->mu0)) return fail(MRF_E_INVAL, "mrf_ipg_solve: mu0 must be > 0");
  if (o->adaptive && !(o->zeta > 1.f)) return fail(MRF_E_INVAL, "mrf_ipg_solve: zeta must be > 1");
  if (o->max_iter < 1) return fail(MRF_E_INVAL, "mrf_ipg_solve: max_iter must be >= 1");
  if (o->max_shrinks < 0) return fail(MRF_E_INVAL, "mrf_ipg_solve: max_shrinks must be >= 0");
  if (stats && stats->cap < 0) return fail(MRF_E_INVAL, "mrf_ipg_solve: stats->cap < 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t npix = (int64_t)A->nx * A->ny;
  const int64_t n = (int64_t)A->nslices * npix;
  const int64_t nimg = (int64_t)A->nslices * D->L;  // image frames (compressed frames if Lfull > 0)
  const OpDims od = dims_of(A);
  const int64_t nvp = od.nvpairs;                   // sampled (slice, coil, frame) pairs
  const float2 *Yc = static_cast<const float2 *>(Y);
  TRY(grow(D->xbuf, (size_t)nimg * npix * 8));
  TRY(grow(D->idxbuf, (size_t)n * 4));
  TRY(grow(D->pdbuf, (size_t)n * 4));
  EventPair ev;
  HIP_TRY(hipEventCreate(&ev.a));
  HIP_TRY(hipEventCreate(&ev.b));
  HIP_TRY(hipEventRecord(ev.a, s));

  float2 *cur = static_cast<float2 *>(X), *nxt = D->xbuf.as<float2>();
  int32_t *idx_cur = idx, *idx_nxt = D->idxbuf.as<int32_t>();
  float *pd_cur = pd ? pd : D->pdbuf.as<float>();
  float *pd_nxt = D->pdbuf.as<float>();
  TRY(grow(D->gbuf, (size_t)nimg * npix * 8));
  TRY(residual_and_gradient(D, A, cur, Yc, false, s));
  TRY(read_scalars(D, 4, s));
  double f = D->host_scal[3];
  int64_t fallback_start = 0;
  if (stats) TRY(read_fallback_total(D, s, &fallback_start));
  if (stats) {
    stats->iters = 0;
    stats->total_shrinks = 0;
    stats->f0 = f;
    stats->fallbacks = 0;
    stats->distance_evals = 0;
    TRY(grow(D->ts_evals, 64));
    launch_zero(D->ts_evals.p, 8, s);
  }
  bool have_idx = false;
  float mu_init = o->mu0;
  for (int k = 0; k < o->max_iter; ++k) {
    TRY(adjoint_into(D, A, D->rbuf.as<float2>(), A->dcf, D->gbuf.as<float2>(), s, D));
    float mu = mu_init;
    int shrinks = 0;
    double dx2 = 0, adx2 = 0, f_new = 0;
    for (;;) {
      TRY(trial(D, A, &o->match, cur, mu, have_idx ? idx_cur : nullptr, nxt, idx_nxt,
                pd ? pd_nxt : nullptr, nullptr, s));
      TRY(read_scalars(D, 3, s));
      dx2 = D->host_scal[0];
      adx2 = D->host_scal[1];
      f_new = D->host_scal[2];
      const bool accept = !o->adaptive || dx2 == 0.0 || adx2 == 0.0 || (double)mu < dx2 / adx2;
      if (accept) break;
      mu /= o->zeta;
      ++shrinks;
      if (shrinks > o->max_shrinks)
        return fail(MRF_E_NOCONV, "mrf_ipg_solve: step size not accepted after %d shrinks at iteration %d",
                    o->max_shrinks, k);
    }
    // accept: R <- R + A dX (abuf holds A dX), swap iterates
    launch_step_norms(D->rbuf.as<float2>(), D->abuf.as<float2>(), A->dcf, A->samp_off, (int)nvp, A->nsamples,
                      A->L, od.nc, D->red.as<double>() + 8192, D->red.as<double>() + 8192 + nvp,
                      D->rbuf.as<float2>(), s);
    LAUNCH_CHECK("residual update");
    std::swap(cur, nxt);
    std::swap(idx_cur, idx_nxt);
    if (pd) std::swap(pd_cur, pd_nxt);
    have_idx = true;
    if (o->kappa && k == 0) {
      // kappa = ||Y|| / ||A X^1|| (plain norms), then X^1 <- kappa X^1, mu <- kappa mu
      mrf_op A0 = *A;
      A0.dcf = nullptr;
      double *red = D->red.as<double>();
      TRY(forward_into(D, &A0, cur, nullptr, D->abuf.as<float2>(), red + 8192, s, D));
      launch_reduce_sum(red + 8192, nvp, D->scal.as<double>() + 4, s);
      int nb = 0;
      launch_norm2(Yc, od.nsamp, red, &nb, s);
      launch_reduce_sum(red, nb, D->scal.as<double>() + 5, s);
      LAUNCH_CHECK("kappa norms");
      TRY(read_scalars(D, 6, s));
      const double ax2 = D->host_scal[4], y2 = D->host_scal[5];
      const float kap = (ax2 > 0.0) ? (float)std::sqrt(y2 / ax2) : 1.f;
      launch_scale(cur, nimg * npix, kap, s);
      if (pd) launch_scale_f32(pd_cur, n, kap, s);
      LAUNCH_CHECK("kappa scale");
      mu_init *= kap;
      TRY(residual_and_gradient(D, A, cur, Yc, false, s));
      TRY(read_scalars(D, 4, s));
      f_new = D->host_scal[3];
    }
    if (stats) {
      if (k < stats->cap) {
        if (stats->f) stats->f[k] = f_new;
        if (stats->mu) stats->mu[k] = mu;
        if (stats->shrinks) stats->shrinks[k] = shrinks;
      }
      stats->iters = k + 1;
      stats->total_shrinks += shrinks;
      int64_t fallback_now = 0;
      TRY(read_fallback_total(D, s, &fallback_now));
      stats->fallbacks = fallback_now - fallback_start;
      unsigned long long evals = 0;
      HIP_TRY(hipMemcpyAsync(&evals, D->ts_evals.p, 8, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      stats->distance_evals = (int64_t)evals;
    }
    const double f_old = f;
    f = f_new;
    if (dx2 == 0.0) break;
    if (o->rel_tol > 0.0 && f_old > 0.0 && (f_old - f_new) / f_old < o->rel_tol) break;
  }
  // results into the caller's buffers
  if (cur != static_cast<float2 *>(X))
    HIP_TRY(hipMemcpyAsync(X, cur, (size_t)nimg * npix * 8, hipMemcpyDeviceToDevice, s));
  if (idx_cur != idx) HIP_TRY(hipMemcpyAsync(idx, idx_cur, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
  if (pd && pd_cur != pd) HIP_TRY(hipMemcpyAsync(pd, pd_cur, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
  if (params_out) {
    launch_lookup(idx, D->params.as<float>(), D->nparam, n, params_out, s);
    LAUNCH_CHECK("lookup");
  }
  HIP_TRY(hipEventRecord(ev.b, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (stats) HIP_TRY(hipEventElapsedTime(&stats->ms, ev.a, ev.b));
  return MRF_OK;
}

// ---------------------------------------------------------------------------
// encodings
// ---------------------------------------------------------------------------
extern "C" mrf_status mrf_quantize_rows(const float *in, int64_t rows, int32_t K, int64_t in_pitch,
                                        int32_t precision, void *out, int64_t out_pitch,
                                        float *scales, mrf_stream stream) {
  last_error().clear();
  if (!in || !out) return fail(MRF_E_INVAL, "mrf_quantize_rows: null in or out");
  if (rows < 0 || K < 1 || in_pitch < K || out_pitch < K) return fail(MRF_E_INVAL, "mrf_quantize_rows: bad sizes");
  if (precision != MRF_BF16 && precision != MRF_FP8) return fail(MRF_E_INVAL, "mrf_quantize_rows: precision must be BF16 or FP8");
  if (precision == MRF_FP8 && !scales) return fail(MRF_E_INVAL, "mrf_quantize_rows: FP8 needs scales");
  if (rows == 0) return MRF_OK;
  launch_quantize_rows(in, rows, K, in_pitch, precision, out, out_pitch, scales,
                       static_cast<hipStream_t>(stream));
  LAUNCH_CHECK("quantize_rows");
  return MRF_OK;
}
