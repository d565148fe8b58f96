// mrf_match_noalloc: the certified (or plain) exhaustive FP32 matched filter
// of mrf_match on a fixed device workspace, for callers that cannot allocate
// device memory (code under stream capture, serving loops).  The workspace is
// the file-scope array below; each device holds its own copy, whose address
// is looked up once per device and used for every call on it.  Calls that
// overlap on one device share (and race on) that memory.
#include <mutex>

#include "host_common.h"
#include "k_topk.h"

namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;  // 32 MiB per device
constexpr int kMaxDevices = 64;
constexpr int kNoAllocMaxSplits = 16;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex scratch_mu;
void *scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (current).
mrf_status scratch_on(int dev, unsigned char **out) {
  if (dev < 0 || dev >= kMaxDevices) return mrf::fail(MRF_E_UNSUPPORTED, "mrf_match_noalloc: device %d", dev);
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return mrf::fail(MRF_E_HIP, "mrf_match_noalloc: no device address for the workspace");
    scratch_dev[dev] = p;
  }
  *out = static_cast<unsigned char *>(scratch_dev[dev]);
  return MRF_OK;
}

// Bump allocator over the workspace (256-byte aligned pieces).
struct Carve {
  unsigned char *base;
  size_t used = 0;
  template <class T>
  T *take(size_t bytes) {
    T *p = reinterpret_cast<T *>(base + used);
    used += (bytes + 255) / 256 * 256;
    return p;
  }
};

}  // namespace

extern "C" mrf_status mrf_match_noalloc(mrf_dict D, const mrf_match_opts *opts, int64_t n, const void *Z,
                                        int32_t z_layout, int64_t slice_voxels, const int32_t *warm_idx,
                                        int32_t *idx, float *pd, float *corr, void *X_out, float *params_out,
                                        mrf_stream stream) {
  using namespace mrf;
  last_error().clear();
  if (!D) return fail(MRF_E_INVAL, "mrf_match_noalloc: null dictionary");
  TRY(check_opts(D, opts));
  if (opts && (opts->method != MRF_EXHAUSTIVE || opts->precision != MRF_FP32))
    return fail(MRF_E_UNSUPPORTED, "mrf_match_noalloc: exhaustive MRF_FP32 only");
  if (n < 0) return fail(MRF_E_INVAL, "mrf_match_noalloc: n < 0");
  if (n > 0 && (!Z || !idx)) return fail(MRF_E_INVAL, "mrf_match_noalloc: null Z or idx");
  if (z_layout != MRF_VOXEL_MAJOR && z_layout != MRF_FRAME_MAJOR)
    return fail(MRF_E_INVAL, "mrf_match_noalloc: bad z_layout %d", z_layout);
  if (z_layout == MRF_FRAME_MAJOR && (slice_voxels < 1 || n % slice_voxels != 0))
    return fail(MRF_E_INVAL, "mrf_match_noalloc: slice_voxels must divide n for the frame-major layout");
  if (n > ((int64_t)1 << 31) - 1024) return fail(MRF_E_INVAL, "mrf_match_noalloc: n too large");
  if (n == 0) return MRF_OK;
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != D->device)
    return fail(MRF_E_INVAL, "mrf_match_noalloc: the dictionary lives on device %d, device %d is current", D->device,
                dev);

  const bool certify = !(opts && opts->no_certificate);
  int splits = (opts && opts->atom_splits > 0) ? opts->atom_splits : std::min(auto_splits(D, n), kNoAllocMaxSplits);
  splits = (int)std::min<int64_t>(splits, D->d_pad / 128);
  const int64_t n_pad = round_up(n, kRowPad);
  const size_t lw = certify ? kCertK : 1;
  // carve the workspace (addresses only), then check it fits before any launch
  unsigned char *base = nullptr;
  TRY(scratch_on(dev, &base));
  Carve c{base};
  float *zp = c.take<float>((size_t)n_pad * D->Kp * 4);
  float *znorm = c.take<float>((size_t)n_pad * 4);
  float *gamma = c.take<float>((size_t)n * 4);
  unsigned long long *counters = c.take<unsigned long long>(64);
  float *part_s = c.take<float>((size_t)splits * n * 4 * lw);
  int *part_j = c.take<int>((size_t)splits * n * 4 * lw);
  float2 *vph = D->align ? c.take<float2>((size_t)n * 8) : nullptr;
  CertBufs b{};
  if (certify) {
    b.counters = c.take<unsigned int>(64);
    b.list = c.take<int32_t>((size_t)n * 4);
    b.thr = c.take<float>((size_t)n * 4);
    b.ccount = c.take<unsigned int>((size_t)n * 4);
    b.scan = c.take<int32_t>((size_t)n * 4);
    b.cand = c.take<int32_t>((size_t)n * kCertCap * 4);
  }
  if (c.used > kScratchBytes)
    return fail(MRF_E_INVAL, "mrf_match_noalloc: %lld voxels need %zu bytes of workspace, more than the %zu of the "
                "fixed workspace", (long long)n, c.used, kScratchBytes);

  hipStream_t s = static_cast<hipStream_t>(stream);
  const int real = D->is_complex ? 0 : 1;
  launch_zero(counters, 64, s);
  if (vph) {
    if (z_layout == MRF_VOXEL_MAJOR)
      launch_voxel_phase(static_cast<const float2 *>(Z), n, D->L, D->u1.as<float2>(), vph, s);
    else
      launch_voxel_phase_frames(static_cast<const float2 *>(Z), nullptr, 0.f, n, slice_voxels, D->L,
                                D->u1.as<float2>(), vph, s);
    LAUNCH_CHECK("voxel phase");
  }
  if (z_layout == MRF_VOXEL_MAJOR)
    launch_pack_voxel_major(static_cast<const float2 *>(Z), n, n_pad, D->L, real, D->Kp, zp, znorm, counters, s,
                            vph);
  else
    launch_pack_frame_major(static_cast<const float2 *>(Z), nullptr, 0.f, n, n_pad, slice_voxels, D->L, real, D->Kp,
                            zp, znorm, counters, s, vph);
  LAUNCH_CHECK("pack");
  launch_score_f32(D->dhat.as<float>(), zp, D->d, D->d_pad, n, n_pad, D->Kp, splits, part_s, part_j, s, certify,
                   znorm, cert_window(cert_coeff(MRF_FP32, D->K)), kCertWinAbs);
  LAUNCH_CHECK("score_f32");
  if (certify) {
    TRY(certify_run(D, b, zp, znorm, nullptr, gamma, part_s, part_j, n, splits, MRF_FP32, warm_idx, idx, pd, corr,
                    params_out, s));
  } else {
    launch_merge_argmax(part_s, part_j, splits, n, D->d, znorm, warm_idx, D->inv_norm.as<float>(),
                        D->params.as<float>(), D->nparam, idx, pd, corr, params_out, gamma, s);
    LAUNCH_CHECK("merge_argmax");
  }
  if (X_out) {
    launch_write_x(idx, gamma, D->dhat.as<float>(), D->Kp, real, n, D->L, z_layout == MRF_FRAME_MAJOR, slice_voxels,
                   static_cast<float2 *>(X_out), nullptr, nullptr, nullptr, nullptr, s, vph);
    LAUNCH_CHECK("write_x");
  }
  if (opts && opts->pd_phase) {
    if (vph)
      launch_pd_phase(idx, vph, D->afac.as<float2>(), n, opts->pd_phase, s);
    else
      launch_zero(opts->pd_phase, n * (int64_t)sizeof(float), s);
    LAUNCH_CHECK("pd phase");
  }
  return MRF_OK;
}
