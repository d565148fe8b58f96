// Temporal subspace compression and phase alignment of a dictionary.
//
// Compression (Section "Dimension-reduced
// subspace matched-filtering", eq. CS1): V_s = the s dominant eigenvectors of
// sum_j Dhat_j Dhat_j^H over the device's FP32 normalised atoms widened to
// FP64, each multiplied by the unit phase that makes its entry of largest
// magnitude (the lowest row among equal magnitudes) real and positive; the
// compressed atoms Dtilde_j = V_s^H Dhat_j become a new dictionary of s
// frames that carries V_s, so that the projected-gradient entry points run
// the compressed iteration of eq. gradupdate / eq. gradcompression.
//
// The Gram matrix (zherk over row chunks), its eigendecomposition (zheevd)
// and the compression (zgemm) run on the device in FP64 through
// rocBLAS / rocSOLVER: a one-off build step, not part of the iteration.
//
// Phase alignment (Section "CoverBLIP algorithm", the phase-alignment
// paragraph): with u the first principal direction (the first compressed
// coordinate for a compressed dictionary), each atom is rotated so that its
// coefficient u^H Dhat_j becomes real non-negative (real atoms: flipped by
// the sign), and the handle keeps u and the factors for the voxel alignment
// of every projection.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <memory>
#include <string>
#include <vector>

#include "host_common.h"

using namespace mrf;

namespace {

struct Blas {
  rocblas_handle h = nullptr;
  ~Blas() {
    if (h) (void)rocblas_destroy_handle(h);
  }
};

#define BLAS_TRY(call)                                                                              \
  do {                                                                                              \
    rocblas_status b_ = (call);                                                                     \
    if (b_ != rocblas_status_success)                                                               \
      return ::mrf::fail(MRF_E_HIP, "%s failed: %s", #call, rocblas_status_to_string(b_));        \
  } while (0)

constexpr int64_t kChunkRows = 32768;

}  // namespace

namespace {

// The s dominant eigenvectors of sum_j Dhat_j Dhat_j^H over D's FP32
// normalised atoms widened to FP64 (column-major L x s in Vcol, row-major
// interleaved [L][s] in Vh, eigenvalues in lam, decreasing), each with the
// phase that makes its largest-magnitude entry real positive.
mrf_status dominant_basis(mrf_dict_s *D, int s_dim, hipStream_t st, rocblas_handle h,
                          std::vector<std::complex<double>> &Vcol, std::vector<double> &Vh,
                          std::vector<double> &lam) {
  const int L = D->L;
  const int64_t d = D->d;
  const int64_t chunk = std::min<int64_t>(kChunkRows, d);
  DevBuf W, G, ev, E, info;
  TRY(grow(W, (size_t)chunk * L * sizeof(double2)));
  TRY(grow(G, (size_t)L * L * sizeof(double2)));
  TRY(grow(ev, (size_t)L * sizeof(double)));
  TRY(grow(E, (size_t)L * sizeof(double)));
  TRY(grow(info, sizeof(rocblas_int)));

  // G = sum_j Dhat_j Dhat_j^H (column-major L x L, lower triangle): the
  // widened rows of a chunk are the columns of an L x rows matrix B, G += B B^H
  for (int64_t r0 = 0; r0 < d; r0 += chunk) {
    const int64_t rows = std::min<int64_t>(chunk, d - r0);
    launch_widen(D->dhat.as<float>() + r0 * D->Kp, D->Kp, D->is_complex, rows, L, W.as<double2>(), st);
    LAUNCH_CHECK("widen");
    if (r0 == 0) HIP_TRY(hipMemsetAsync(G.p, 0, (size_t)L * L * sizeof(double2), st));
    const double one = 1.0, beta = r0 == 0 ? 0.0 : 1.0;
    BLAS_TRY(rocblas_zherk(h, rocblas_fill_lower, rocblas_operation_none, L, (rocblas_int)rows, &one,
                           W.as<rocblas_double_complex>(), L, &beta, G.as<rocblas_double_complex>(), L));
  }
  // sanity: trace(G) = sum_j ||Dhat_j||^2, which is d up to FP32 rounding
  std::vector<std::complex<double>> U((size_t)L * L);
  HIP_TRY(hipMemcpyAsync(U.data(), G.p, U.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double trace = 0.0;
  for (int t = 0; t < L; ++t) trace += U[(size_t)t * L + t].real();
  const std::vector<std::complex<double>> Gh = U;
  if (!(std::fabs(trace - (double)d) <= 1e-4 * (double)d))
    return fail(MRF_E_NUMERIC, "dictionary basis: Gram trace %.9g differs from the atom count %lld", trace,
                (long long)d);
  // Eigendecomposition (ascending eigenvalues, eigenvectors in the columns):
  // QR iteration (zheev) first; each result is checked (all selected columns
  // finite and unit-norm, the leading pairs' residuals ||G u - lambda u||
  // against the Gram matrix on the host), and the divide-and-conquer
  // (zheevd) and Jacobi (zheevj) solvers are tried in turn if it fails.
  std::vector<double> lam_all((size_t)L);
  std::string why;
  auto validate = [&](const char *name) -> bool {
    double lsum = 0.0;
    for (double v : lam_all) lsum += v;
    if (!(std::fabs(lsum - trace) <= 1e-8 * trace)) {
      char b2[200];
      snprintf(b2, sizeof b2, "%s: eigenvalues sum to %.12g, trace %.12g; ", name, lsum, trace);
      why += b2;
      return false;
    }
    for (int k = 0; k < s_dim; ++k) {
      const int c = L - 1 - k;
      const std::complex<double> *u = U.data() + (size_t)c * L;
      double res = 0.0, un = 0.0;
      for (int t = 0; t < L; ++t) un += std::norm(u[t]);
      if (k < 4)
        for (int t = 0; t < L; ++t) {
          std::complex<double> acc = 0.0;
          for (int q = 0; q < L; ++q) {
            const std::complex<double> g = t >= q ? Gh[(size_t)q * L + t] : std::conj(Gh[(size_t)t * L + q]);
            acc += g * u[q];
          }
          res += std::norm(acc - lam_all[(size_t)c] * u[t]);
        }
      if (!(std::fabs(un - 1.0) <= 1e-9) || !(std::sqrt(res) <= 1e-9 * std::max(lam_all[(size_t)(L - 1)], 1.0))) {
        char b2[200];
        snprintf(b2, sizeof b2, "%s: eigenpair %d residual %.3g, |u|^2 %.12g; ", name, k, std::sqrt(res), un);
        why += b2;
        return false;
      }
    }
    return true;
  };
  bool ok = false;
  for (int method = 0; method < 3 && !ok; ++method) {
    HIP_TRY(hipMemcpyAsync(G.p, Gh.data(), Gh.size() * sizeof(double2), hipMemcpyHostToDevice, st));
    rocblas_int inf = 0;
    const char *name = method == 0 ? "zheev" : method == 1 ? "zheevd" : "zheevj";
    if (method == 0) {
      BLAS_TRY(rocsolver_zheev(h, rocblas_evect_original, rocblas_fill_lower, L, G.as<rocblas_double_complex>(),
                               L, ev.as<double>(), E.as<double>(), info.as<rocblas_int>()));
    } else if (method == 1) {
      BLAS_TRY(rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_lower, L,
                                G.as<rocblas_double_complex>(), L, ev.as<double>(), E.as<double>(),
                                info.as<rocblas_int>()));
    } else {
      TRY(grow(E, (size_t)std::max(L, 2) * sizeof(double)));
      BLAS_TRY(rocsolver_zheevj(h, rocblas_esort_ascending, rocblas_evect_original, rocblas_fill_lower, L,
                                G.as<rocblas_double_complex>(), L, 0.0, E.as<double>(), 100,
                                E.as<rocblas_int>() + 2, ev.as<double>(), info.as<rocblas_int>()));
    }
    HIP_TRY(hipMemcpyAsync(U.data(), G.p, U.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(lam_all.data(), ev.p, lam_all.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&inf, info.p, sizeof inf, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (inf != 0) {
      char b2[120];
      snprintf(b2, sizeof b2, "%s: info %d; ", name, (int)inf);
      why += b2;
      continue;
    }
    ok = validate(name);
  }
  if (!ok) return fail(MRF_E_NUMERIC, "dictionary basis: no eigensolver result passed the checks (%s)", why.c_str());

  // eigenvalues ascending -> the s largest in descending order, phase fixed
  Vh.assign((size_t)L * s_dim * 2, 0.0);
  lam.assign((size_t)s_dim, 0.0);
  Vcol.assign((size_t)L * s_dim, 0.0);
  for (int k = 0; k < s_dim; ++k) {
    const int c = L - 1 - k;
    lam[(size_t)k] = lam_all[(size_t)c];
    const std::complex<double> *u = U.data() + (size_t)c * L;
    int imax = 0;
    double mmax = -1.0;
    for (int t = 0; t < L; ++t) {
      const double m = std::abs(u[t]);
      if (m > mmax) {
        mmax = m;
        imax = t;
      }
    }
    const std::complex<double> ph = std::conj(u[imax]) / mmax;
    for (int t = 0; t < L; ++t) {
      std::complex<double> v = u[t] * ph;
      if (t == imax) v = std::complex<double>(std::abs(u[t]), 0.0);
      Vcol[(size_t)k * L + t] = v;
      Vh[((size_t)t * s_dim + k) * 2] = v.real();
      Vh[((size_t)t * s_dim + k) * 2 + 1] = v.imag();
    }
  }

  return MRF_OK;
}

// At [d][s] (interleaved FP64 complex) = V^H Dhat_j for every atom, V the
// column-major L x s matrix Vcol; the first and last rows are checked against
// a host FP64 product.
mrf_status project_rows(mrf_dict_s *D, const std::vector<std::complex<double>> &Vcol, int s_dim, hipStream_t st,
                        rocblas_handle h, std::vector<double> &At) {
  const int L = D->L;
  const int64_t d = D->d;
  const int64_t chunk = std::min<int64_t>(kChunkRows, d);
  DevBuf W, Vc, Out;
  TRY(grow(W, (size_t)chunk * L * sizeof(double2)));
  // Dtilde_j = V^H Dhat_j: (s x L) op C times the L x rows chunk, column-major
  // s x rows = row-major [rows][s]
  TRY(grow(Vc, Vcol.size() * sizeof(double2)));
  TRY(grow(Out, (size_t)chunk * s_dim * sizeof(double2)));
  HIP_TRY(hipMemcpyAsync(Vc.p, Vcol.data(), Vcol.size() * sizeof(double2), hipMemcpyHostToDevice, st));
  At.assign((size_t)d * s_dim * 2, 0.0);
  const rocblas_double_complex one_c(1.0, 0.0), zero_c(0.0, 0.0);
  for (int64_t r0 = 0; r0 < d; r0 += chunk) {
    const int64_t rows = std::min<int64_t>(chunk, d - r0);
    launch_widen(D->dhat.as<float>() + r0 * D->Kp, D->Kp, D->is_complex, rows, L, W.as<double2>(), st);
    LAUNCH_CHECK("widen");
    HIP_TRY(hipMemsetAsync(Out.p, 0, (size_t)rows * s_dim * sizeof(double2), st));
    BLAS_TRY(rocblas_zgemm(h, rocblas_operation_conjugate_transpose, rocblas_operation_none, s_dim,
                           (rocblas_int)rows, L, &one_c, Vc.as<rocblas_double_complex>(), L,
                           W.as<rocblas_double_complex>(), L, &zero_c, Out.as<rocblas_double_complex>(),
                           s_dim));
    HIP_TRY(hipMemcpyAsync(At.data() + (size_t)r0 * s_dim * 2, Out.p, (size_t)rows * s_dim * sizeof(double2),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }

  for (size_t i = 0; i < At.size(); ++i)
    if (!std::isfinite(At[i]))
      return fail(MRF_E_NUMERIC, "dictionary projection: non-finite coordinate at %zu", i);
  // the first and last compressed atoms against a host FP64 product
  for (int64_t j : {(int64_t)0, d - 1}) {
    std::vector<float> row((size_t)D->K);
    HIP_TRY(hipMemcpy(row.data(), D->dhat.as<float>() + j * D->Kp, row.size() * sizeof(float),
                      hipMemcpyDeviceToHost));
    for (int k = 0; k < s_dim; ++k) {
      std::complex<double> acc = 0.0;
      for (int t = 0; t < L; ++t) {
        const std::complex<double> x = D->is_complex ? std::complex<double>(row[2 * t], row[2 * t + 1])
                                                     : std::complex<double>(row[t], 0.0);
        acc += std::conj(Vcol[(size_t)k * L + t]) * x;
      }
      const double *g = At.data() + ((size_t)j * s_dim + k) * 2;
      if (!(std::abs(acc - std::complex<double>(g[0], g[1])) <= 1e-10))
        return fail(MRF_E_NUMERIC, "dictionary projection: atom %lld coordinate %d is (%.9g, %.9g), host (%.9g, %.9g)",
                    (long long)j, k, g[0], g[1], acc.real(), acc.imag());
    }
  }
  return MRF_OK;
}

}  // namespace

extern "C" mrf_status mrf_dict_compress(mrf_dict D, int32_t s_dim, uint32_t flags, mrf_stream stream,
                                        mrf_dict *out) {
  last_error().clear();
  if (!D || !out) return fail(MRF_E_INVAL, "mrf_dict_compress: null argument");
  if (D->Lfull > 0) return fail(MRF_E_UNSUPPORTED, "mrf_dict_compress: dictionary is already compressed");
  if (D->align)
    return fail(MRF_E_UNSUPPORTED, "mrf_dict_compress: compress first, then align (dictionary is phase-aligned)");
  const int L = D->L;
  if (s_dim < 1 || s_dim > L || s_dim > kMaxSubspace)
    return fail(MRF_E_INVAL, "mrf_dict_compress: s=%d not in 1..min(L=%d, %d)", s_dim, L, kMaxSubspace);
  if (flags & ~(uint32_t)(MRF_STORE_BF16 | MRF_STORE_FP8 | MRF_BUILD_COVERTREE))
    return fail(MRF_E_INVAL, "mrf_dict_compress: unknown flags 0x%x", flags);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Blas blas;
  BLAS_TRY(rocblas_create_handle(&blas.h));
  BLAS_TRY(rocblas_set_stream(blas.h, st));
  BLAS_TRY(rocblas_set_pointer_mode(blas.h, rocblas_pointer_mode_host));

  std::vector<std::complex<double>> Vcol;
  std::vector<double> Vh, lam, At;
  TRY(dominant_basis(D, s_dim, st, blas.h, Vcol, Vh, lam));
  TRY(project_rows(D, Vcol, s_dim, st, blas.h, At));
  mrf_dict_desc q{};
  q.d = D->d;
  q.L = s_dim;
  q.nparam = D->nparam;
  q.is_complex = 1;
  q.atoms = At.data();
  q.atoms_dtype = MRF_F64;
  q.params = D->params_host.data();
  q.grid_dims = D->grid_dims.empty() ? nullptr : D->grid_dims.data();
  q.flags = flags;
  mrf_dict C = nullptr;
  TRY(mrf_dict_build(&q, stream, &C));
  std::unique_ptr<mrf_dict_s> guard(C);
  C->Lfull = L;
  C->V_host = std::move(Vh);
  C->lam = std::move(lam);
  std::vector<float> vf(C->V_host.size());
  for (size_t i = 0; i < vf.size(); ++i) vf[i] = (float)C->V_host[i];
  TRY(grow(C->Vs, vf.size() * sizeof(float)));
  HIP_TRY(hipMemcpy(C->Vs.p, vf.data(), vf.size() * sizeof(float), hipMemcpyHostToDevice));
  C->bytes += (int64_t)C->Vs.cap;
  *out = guard.release();
  return MRF_OK;
}

extern "C" mrf_status mrf_dict_align(mrf_dict D, uint32_t flags, mrf_stream stream, mrf_dict *out) {
  last_error().clear();
  if (!D || !out) return fail(MRF_E_INVAL, "mrf_dict_align: null argument");
  if (D->align) return fail(MRF_E_UNSUPPORTED, "mrf_dict_align: dictionary is already phase-aligned");
  if (flags & ~(uint32_t)(MRF_STORE_BF16 | MRF_STORE_FP8 | MRF_BUILD_COVERTREE))
    return fail(MRF_E_INVAL, "mrf_dict_align: unknown flags 0x%x", flags);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int L = D->L;
  const int64_t d = D->d;
  Blas blas;
  BLAS_TRY(rocblas_create_handle(&blas.h));
  BLAS_TRY(rocblas_set_stream(blas.h, st));
  BLAS_TRY(rocblas_set_pointer_mode(blas.h, rocblas_pointer_mode_host));
  // u: the first principal direction (the first compressed coordinate of a
  // compressed dictionary, whose basis starts with it)
  std::vector<std::complex<double>> u;
  if (D->Lfull > 0) {
    u.assign((size_t)L, 0.0);
    u[0] = 1.0;
  } else {
    std::vector<double> Vh, lam;
    TRY(dominant_basis(D, 1, st, blas.h, u, Vh, lam));
  }
  std::vector<double> c;
  TRY(project_rows(D, u, 1, st, blas.h, c));
  // alignment factors f_j and the aligned rows (FP64) of the FP32 normalised atoms
  std::vector<std::complex<double>> f((size_t)d);
  for (int64_t j = 0; j < d; ++j) {
    const std::complex<double> cj(c[2 * j], c[2 * j + 1]);
    const double m = std::abs(cj);
    if (D->is_complex)
      f[(size_t)j] = m > 0.0 ? std::conj(cj) / m : std::complex<double>(1.0, 0.0);
    else
      f[(size_t)j] = cj.real() < 0.0 ? -1.0 : 1.0;
  }
  const int K = D->K;
  std::vector<double> atoms((size_t)d * K);
  {
    const int64_t chunk = 65536;
    std::vector<float> rows((size_t)std::min<int64_t>(chunk, d) * D->Kp);
    for (int64_t r0 = 0; r0 < d; r0 += chunk) {
      const int64_t nr = std::min<int64_t>(chunk, d - r0);
      HIP_TRY(hipMemcpy(rows.data(), D->dhat.as<float>() + r0 * D->Kp, (size_t)nr * D->Kp * sizeof(float),
                        hipMemcpyDeviceToHost));
      for (int64_t r = 0; r < nr; ++r) {
        const float *a = rows.data() + (size_t)r * D->Kp;
        double *o = atoms.data() + (size_t)(r0 + r) * K;
        const std::complex<double> fj = f[(size_t)(r0 + r)];
        if (D->is_complex) {
          for (int t = 0; t < L; ++t) {
            const std::complex<double> x = std::complex<double>(a[2 * t], a[2 * t + 1]) * fj;
            o[2 * t] = x.real();
            o[2 * t + 1] = x.imag();
          }
        } else {
          for (int t = 0; t < L; ++t) o[t] = (double)a[t] * fj.real();
        }
      }
    }
  }
  mrf_dict_desc q{};
  q.d = D->d;
  q.L = L;
  q.nparam = D->nparam;
  q.is_complex = D->is_complex;
  q.atoms = atoms.data();
  q.atoms_dtype = MRF_F64;
  q.params = D->params_host.data();
  q.grid_dims = D->grid_dims.empty() ? nullptr : D->grid_dims.data();
  q.flags = flags;
  mrf_dict C = nullptr;
  TRY(mrf_dict_build(&q, stream, &C));
  std::unique_ptr<mrf_dict_s> guard(C);
  C->align = 1;
  std::vector<float> uf((size_t)L * 2), ff((size_t)d * 2);
  for (int t = 0; t < L; ++t) {
    uf[2 * t] = (float)u[(size_t)t].real();
    uf[2 * t + 1] = (float)u[(size_t)t].imag();
  }
  for (int64_t j = 0; j < d; ++j) {
    ff[2 * j] = (float)f[(size_t)j].real();
    ff[2 * j + 1] = (float)f[(size_t)j].imag();
  }
  TRY(grow(C->u1, uf.size() * sizeof(float)));
  TRY(grow(C->afac, ff.size() * sizeof(float)));
  HIP_TRY(hipMemcpy(C->u1.p, uf.data(), uf.size() * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(C->afac.p, ff.data(), ff.size() * sizeof(float), hipMemcpyHostToDevice));
  C->bytes += (int64_t)(C->u1.cap + C->afac.cap);
  if (D->Lfull > 0) {  // keep the temporal subspace of a compressed dictionary
    C->Lfull = D->Lfull;
    C->V_host = D->V_host;
    C->lam = D->lam;
    TRY(grow(C->Vs, D->V_host.size() * sizeof(float)));
    HIP_TRY(hipMemcpy(C->Vs.p, D->Vs.p, D->V_host.size() * sizeof(float), hipMemcpyDeviceToDevice));
    C->bytes += (int64_t)C->Vs.cap;
  }
  *out = guard.release();
  return MRF_OK;
}

extern "C" mrf_status mrf_dict_subspace(mrf_dict C, double *V, double *lam) {
  last_error().clear();
  if (!C) return fail(MRF_E_INVAL, "mrf_dict_subspace: null dictionary");
  if (C->Lfull <= 0) return fail(MRF_E_INVAL, "mrf_dict_subspace: dictionary is not compressed");
  if (V) std::copy(C->V_host.begin(), C->V_host.end(), V);
  if (lam) std::copy(C->lam.begin(), C->lam.end(), lam);
  return MRF_OK;
}
