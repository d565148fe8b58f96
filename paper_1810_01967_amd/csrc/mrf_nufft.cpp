// Plans of the non-uniform FFT for non-Cartesian sampling (the in-vivo
// spiral setting of eq. forward): the trajectory and its CSR offsets on the
// device, the samples of every (slice, frame) pair sorted into 8 x 8 bins
// of the 2x oversampled grid (for the deterministic gather-spread), and the
// deapodisation factors: sqrt(N/n) / phihat((r - n/2)/N) per dimension, with
// phihat the Fourier transform of the "exponential of semicircle" kernel
// evaluated by composite Simpson quadrature in FP64.
#include <algorithm>
#include <cmath>
#include <memory>
#include <numeric>
#include <vector>

#include "host_common.h"
#include "nufft_host.h"

using namespace mrf;

namespace {

bool pow2_in(int x, int lo, int hi) { return x >= lo && x <= hi && (x & (x - 1)) == 0; }

}  // namespace

extern "C" mrf_status mrf_nufft_create(int32_t nx, int32_t ny, int32_t L, int32_t nslices, int64_t nsamples,
                                       const int64_t *samp_off, const float *coords, int32_t width,
                                       mrf_nufft *out) {
  last_error().clear();
  if (!out || !samp_off || (nsamples > 0 && !coords)) return fail(MRF_E_INVAL, "mrf_nufft_create: null argument");
  if (!pow2_in(nx, 16, 256) || !pow2_in(ny, 16, 256))
    return fail(MRF_E_INVAL, "mrf_nufft_create: nx=%d ny=%d must be powers of two in 16..256", nx, ny);
  if (L < 1 || nslices < 1 || nsamples < 0) return fail(MRF_E_INVAL, "mrf_nufft_create: bad sizes");
  const int W = width == 0 ? 7 : width;
  if (W < 4 || W > 8) return fail(MRF_E_INVAL, "mrf_nufft_create: width %d not in 4..8", W);
  const int64_t npairs = (int64_t)nslices * L;
  if (npairs > (1 << 26)) return fail(MRF_E_INVAL, "mrf_nufft_create: too many frames");
  if (samp_off[0] != 0 || samp_off[npairs] != nsamples)
    return fail(MRF_E_INVAL, "mrf_nufft_create: offsets must run from 0 to nsamples");
  for (int64_t p = 0; p < npairs; ++p)
    if (samp_off[p + 1] < samp_off[p]) return fail(MRF_E_INVAL, "mrf_nufft_create: decreasing offsets at %lld",
                                                   (long long)p);
  if (nsamples > ((int64_t)1 << 31) - 1) return fail(MRF_E_INVAL, "mrf_nufft_create: too many samples");
  for (int64_t i = 0; i < 2 * nsamples; ++i)
    if (!(std::fabs(coords[i]) <= 1024.f))
      return fail(MRF_E_INVAL, "mrf_nufft_create: coordinate %lld is not finite or exceeds 1024 in magnitude",
                  (long long)i);
  auto *P = new mrf_nufft_s();
  std::unique_ptr<mrf_nufft_s> guard(P);
  P->nx = nx;
  P->ny = ny;
  P->L = L;
  P->nslices = nslices;
  P->W = W;
  P->beta = (float)(2.30 * W);
  P->M = nsamples;
  const int Ny = 2 * ny, Nx = 2 * nx;
  // bins: samples of each pair sorted by the bin of their fine position (mod N)
  std::vector<int32_t> bperm, boff;
  nufft_host::bin_samples(samp_off, npairs, coords, Ny, Nx, kNufftBin, bperm, boff);
  std::vector<float> dy((size_t)ny), dx((size_t)nx);
  for (int a = 0; a < ny; ++a)
    dy[(size_t)a] = (float)(std::sqrt(2.0) / nufft_host::phihat((double)(a - ny / 2) / Ny, W, 2.30 * W));
  for (int a = 0; a < nx; ++a)
    dx[(size_t)a] = (float)(std::sqrt(2.0) / nufft_host::phihat((double)(a - nx / 2) / Nx, W, 2.30 * W));
  TRY(grow(P->off, (size_t)(npairs + 1) * 8));
  TRY(grow(P->coords, (size_t)std::max<int64_t>(nsamples, 1) * 8));
  TRY(grow(P->bperm, bperm.size() * 4));
  TRY(grow(P->boff, boff.size() * 4));
  TRY(grow(P->dy, dy.size() * 4));
  TRY(grow(P->dx, dx.size() * 4));
  HIP_TRY(hipMemcpy(P->off.p, samp_off, (size_t)(npairs + 1) * 8, hipMemcpyHostToDevice));
  if (nsamples > 0) HIP_TRY(hipMemcpy(P->coords.p, coords, (size_t)nsamples * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(P->bperm.p, bperm.data(), bperm.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(P->boff.p, boff.data(), boff.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(P->dy.p, dy.data(), dy.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(P->dx.p, dx.data(), dx.size() * 4, hipMemcpyHostToDevice));
  *out = guard.release();
  return MRF_OK;
}

extern "C" mrf_status mrf_nufft_destroy(mrf_nufft plan) {
  last_error().clear();
  if (!plan) return MRF_OK;
  (void)hipDeviceSynchronize();
  delete plan;
  return MRF_OK;
}
