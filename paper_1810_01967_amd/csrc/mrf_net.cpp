// Host side of the learned-proposal path: network handles, training on
// device-generated noisy atoms, and the proposal -> local search ->
// re-centring -> exhaustive fallback pipeline used by MRF_LEARNED.
#include "host_common.h"

using namespace mrf;

namespace {

mrf_status check_net(const mrf_net_s *net) {
  if (!net) return fail(MRF_E_INVAL, "null network");
  return MRF_OK;
}

// Counter-generator keys of the training stream (SplitMix64 of the seed
// combined with a purpose tag 1, 2, 3).
void train_keys(uint64_t seed, uint64_t *ka, uint64_t *ks, uint64_t *kn) {
  const uint64_t base = seed * 0xD1B54A32D192ED03ull;
  *ka = mix64_host(base + 1);
  *ks = mix64_host(base + 2);
  *kn = mix64_host(base + 3);
}

mrf_status upload_std(mrf_net_s *net) {
  TRY(grow(net->dstd, 24 * 4));
  float buf[24];
  for (int p = 0; p < 8; ++p) {
    buf[p] = net->mean[p];
    buf[8 + p] = net->stdv[p];
    int li = net->logm[p];
    std::memcpy(&buf[16 + p], &li, 4);
  }
  HIP_TRY(hipMemcpy(net->dstd.p, buf, sizeof buf, hipMemcpyHostToDevice));
  return MRF_OK;
}

const float *dmean(const mrf_net_s *n) { return n->dstd.as<float>(); }
const float *dstdv(const mrf_net_s *n) { return n->dstd.as<float>() + 8; }
const int *dlogm(const mrf_net_s *n) { return reinterpret_cast<const int *>(n->dstd.as<float>() + 16); }

// Standardisation from a dictionary's parameter table: ln for parameters
// that are positive with max/min >= 4, identity otherwise.
void std_from_dict(mrf_net_s *net, const mrf_dict_s *D) {
  for (int p = 0; p < net->P; ++p) {
    double mn = 1e300, mx = -1e300;
    for (int j = 0; j < D->d; ++j) {
      const double v = D->params_host[(size_t)j * D->nparam + p];
      mn = std::min(mn, v);
      mx = std::max(mx, v);
    }
    const int lg = (mn > 0.0 && mx / mn >= 4.0) ? 1 : 0;
    double s1 = 0.0, s2 = 0.0;
    for (int j = 0; j < D->d; ++j) {
      double v = D->params_host[(size_t)j * D->nparam + p];
      if (lg) v = std::log(v);
      s1 += v;
      s2 += v * v;
    }
    const double mean = s1 / D->d;
    double var = s2 / D->d - mean * mean;
    if (!(var > 0.0)) var = 1.0;
    net->mean[p] = (float)mean;
    net->stdv[p] = (float)std::sqrt(var);
    net->logm[p] = lg;
  }
  net->has_std = true;
}

mrf_status net_ws(mrf_net_s *net, int64_t B, bool train) {
  TRY(grow(net->hb1, (size_t)B * net->H * 4));
  TRY(grow(net->hb2, (size_t)B * net->H * 4));
  if (train) {
    TRY(grow(net->a1, (size_t)B * net->H * 4));
    TRY(grow(net->a2, (size_t)B * net->H * 4));
    TRY(grow(net->y, (size_t)B * net->P * 4));
    TRY(grow(net->dy, (size_t)B * net->P * 4));
    TRY(grow(net->da, (size_t)B * net->H * 4));
    TRY(grow(net->db, (size_t)B * net->H * 4));
    TRY(grow(net->red, 512 * 8));
    TRY(grow(net->scal, 64));
  }
  return MRF_OK;
}

// X [B][I] (ld ldx) -> Y [B][P]; rowscale (or null) multiplies each row's
// first-layer product (the 1/||Z_v|| of the input normalisation).
mrf_status net_forward_rows(mrf_net_s *net, const float *X, int64_t ldx, int64_t B,
                            const float *rowscale, float *Y, float *h1, float *h2, hipStream_t s) {
  const float *w = net->w.as<float>();
  GemmEpi e1;
  e1.kind = GEMM_GELU;
  e1.bias = w + net->ob1;
  e1.rowscale = rowscale;
  launch_gemm((int)B, net->H, net->I, X, ldx, true, w + net->oW1, net->I, true, h1, net->H, e1, s);
  GemmEpi e2;
  e2.kind = GEMM_GELU;
  e2.bias = w + net->ob2;
  launch_gemm((int)B, net->H, net->H, h1, net->H, true, w + net->oW2, net->H, true, h2, net->H, e2, s);
  GemmEpi e3;
  e3.bias = w + net->ob3;
  launch_gemm((int)B, net->P, net->H, h2, net->H, true, w + net->oW3, net->H, true, Y, net->P, e3, s);
  LAUNCH_CHECK("net forward");
  return MRF_OK;
}

// Loss partial sums into net->red[0..nb), gradients into net->g.
mrf_status net_loss_grad(mrf_net_s *net, const float *X, const float *T, int64_t B, int *nb,
                         hipStream_t s) {
  TRY(net_ws(net, B, true));
  const int H = net->H, P = net->P, I = net->I;
  const float *w = net->w.as<float>();
  float *g = net->g.as<float>();
  GemmEpi e1;
  e1.kind = GEMM_GELU;
  e1.bias = w + net->ob1;
  e1.pre = net->a1.as<float>();
  launch_gemm((int)B, H, I, X, I, true, w + net->oW1, I, true, net->hb1.as<float>(), H, e1, s);
  GemmEpi e2;
  e2.kind = GEMM_GELU;
  e2.bias = w + net->ob2;
  e2.pre = net->a2.as<float>();
  launch_gemm((int)B, H, H, net->hb1.as<float>(), H, true, w + net->oW2, H, true,
              net->hb2.as<float>(), H, e2, s);
  GemmEpi e3;
  e3.bias = w + net->ob3;
  launch_gemm((int)B, P, H, net->hb2.as<float>(), H, true, w + net->oW3, H, true,
              net->y.as<float>(), P, e3, s);
  launch_mse(net->y.as<float>(), T, B * P, (float)(2.0 / ((double)B * P)), net->dy.as<float>(),
             net->red.as<double>(), nb, s);
  // weight gradients: long sums over the batch, split over blocks
  const int ksplit = (int)std::max<int64_t>(1, std::min<int64_t>(16, B / 256));
  TRY(grow(net->gpart, (size_t)ksplit * std::max<int64_t>((int64_t)H * I, (int64_t)H * H) * 4));
  float *gpart = net->gpart.as<float>();
  // dW3[p][h] = sum_b dy[b][p] h2[b][h]
  launch_gemm_splitk(P, H, (int)B, net->dy.as<float>(), P, false, net->hb2.as<float>(), H, false, g + net->oW3,
                     ksplit, gpart, s);
  launch_colsum(net->dy.as<float>(), (int)B, P, g + net->ob3, s);
  // da2 = (dy W3) * gelu'(a2)
  GemmEpi gg2;
  gg2.kind = GEMM_GELU_GRAD;
  gg2.gpre = net->a2.as<float>();
  launch_gemm((int)B, H, P, net->dy.as<float>(), P, true, w + net->oW3, H, false,
              net->da.as<float>(), H, gg2, s);
  launch_gemm_splitk(H, H, (int)B, net->da.as<float>(), H, false, net->hb1.as<float>(), H, false, g + net->oW2,
                     ksplit, gpart, s);
  launch_colsum(net->da.as<float>(), (int)B, H, g + net->ob2, s);
  // da1 = (da2 W2) * gelu'(a1)
  GemmEpi gg1;
  gg1.kind = GEMM_GELU_GRAD;
  gg1.gpre = net->a1.as<float>();
  launch_gemm((int)B, H, H, net->da.as<float>(), H, true, w + net->oW2, H, false,
              net->db.as<float>(), H, gg1, s);
  launch_gemm_splitk(H, I, (int)B, net->db.as<float>(), H, false, X, I, false, g + net->oW1, ksplit, gpart, s);
  launch_colsum(net->db.as<float>(), (int)B, H, g + net->ob1, s);
  LAUNCH_CHECK("net backward");
  return MRF_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
extern "C" mrf_status mrf_net_create(int32_t in_dim, int32_t hidden, int32_t nout, uint64_t seed,
                                     mrf_net *out) {
  last_error().clear();
  if (!out) return fail(MRF_E_INVAL, "mrf_net_create: null out");
  *out = nullptr;
  if (in_dim < 1 || hidden < 1 || hidden > 4096 || nout < 1 || nout > 8)
    return fail(MRF_E_INVAL, "mrf_net_create: bad sizes (in %d hidden %d out %d)", in_dim, hidden, nout);
  auto *net = new mrf_net_s();
  std::unique_ptr<mrf_net_s> guard(net);
  net->I = in_dim;
  net->H = hidden;
  net->P = nout;
  net->oW1 = 0;
  net->ob1 = (int64_t)hidden * in_dim;
  net->oW2 = net->ob1 + hidden;
  net->ob2 = net->oW2 + (int64_t)hidden * hidden;
  net->oW3 = net->ob2 + hidden;
  net->ob3 = net->oW3 + (int64_t)nout * hidden;
  net->nw = net->ob3 + nout;
  TRY(grow(net->w, net->nw * 4));
  TRY(grow(net->g, net->nw * 4));
  TRY(grow(net->m, net->nw * 4));
  TRY(grow(net->v, net->nw * 4));
  // He-normal weights N(0, 2/fan_in) from a counter-based stream, zero biases
  std::vector<float> h((size_t)net->nw, 0.f);
  const uint64_t key = mix64_host(seed * 0xD1B54A32D192ED03ull + 11);
  auto normal = [&](uint64_t i) {
    const double u1 = 1.0 - (double)(mix64_host(key + (2 * i + 1) * 0x9E3779B97F4A7C15ull) >> 11) * 0x1.0p-53;
    const double u2 = (double)(mix64_host(key + (2 * i + 2) * 0x9E3779B97F4A7C15ull) >> 11) * 0x1.0p-53;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
  };
  auto fill = [&](int64_t off, int64_t count, int fan) {
    const double sd = std::sqrt(2.0 / fan);
    for (int64_t i = 0; i < count; ++i) h[(size_t)(off + i)] = (float)(sd * normal((uint64_t)(off + i)));
  };
  fill(net->oW1, (int64_t)hidden * in_dim, in_dim);
  fill(net->oW2, (int64_t)hidden * hidden, hidden);
  fill(net->oW3, (int64_t)nout * hidden, hidden);
  HIP_TRY(hipMemcpy(net->w.p, h.data(), net->nw * 4, hipMemcpyHostToDevice));
  ++net->wver;
  HIP_TRY(hipMemset(net->g.p, 0, net->nw * 4));
  HIP_TRY(hipMemset(net->m.p, 0, net->nw * 4));
  HIP_TRY(hipMemset(net->v.p, 0, net->nw * 4));
  HIP_TRY(hipHostMalloc((void **)&net->host_scal, 16 * sizeof(double), hipHostMallocDefault));
  TRY(upload_std(net));
  *out = guard.release();
  return MRF_OK;
}

extern "C" mrf_status mrf_net_destroy(mrf_net net) {
  last_error().clear();
  if (!net) return MRF_OK;
  (void)hipDeviceSynchronize();
  delete net;
  return MRF_OK;
}

extern "C" mrf_status mrf_net_size(mrf_net net, int64_t *count) {
  last_error().clear();
  TRY(check_net(net));
  if (!count) return fail(MRF_E_INVAL, "mrf_net_size: null count");
  *count = net->nw;
  return MRF_OK;
}

static mrf_status net_copy(mrf_net net, float *host, const float *src_host, int64_t count, DevBuf &dev,
                           bool to_dev) {
  TRY(check_net(net));
  if (count != net->nw) return fail(MRF_E_INVAL, "parameter count %lld != %lld", (long long)count, (long long)net->nw);
  if (to_dev) {
    if (!src_host) return fail(MRF_E_INVAL, "null host array");
    HIP_TRY(hipMemcpy(dev.p, src_host, count * 4, hipMemcpyHostToDevice));
  } else {
    if (!host) return fail(MRF_E_INVAL, "null host array");
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(host, dev.p, count * 4, hipMemcpyDeviceToHost));
  }
  return MRF_OK;
}

extern "C" mrf_status mrf_net_set_params(mrf_net net, const float *host, int64_t count) {
  last_error().clear();
  TRY(net_copy(net, nullptr, host, count, net->w, true));
  ++net->wver;
  return MRF_OK;
}
extern "C" mrf_status mrf_net_get_params(mrf_net net, float *host, int64_t count) {
  last_error().clear();
  return net_copy(net, host, nullptr, count, net->w, false);
}
extern "C" mrf_status mrf_net_get_grads(mrf_net net, float *host, int64_t count) {
  last_error().clear();
  return net_copy(net, host, nullptr, count, net->g, false);
}

extern "C" mrf_status mrf_net_set_standardisation(mrf_net net, const float *mean, const float *stdv,
                                                  const int32_t *log_mask) {
  last_error().clear();
  TRY(check_net(net));
  if (!mean || !stdv || !log_mask) return fail(MRF_E_INVAL, "null standardisation array");
  for (int p = 0; p < net->P; ++p) {
    if (!(stdv[p] > 0.f) || !std::isfinite(mean[p])) return fail(MRF_E_INVAL, "bad standardisation");
    net->mean[p] = mean[p];
    net->stdv[p] = stdv[p];
    net->logm[p] = log_mask[p] ? 1 : 0;
  }
  net->has_std = true;
  return upload_std(net);
}

extern "C" mrf_status mrf_net_get_standardisation(mrf_net net, float *mean, float *stdv,
                                                  int32_t *log_mask) {
  last_error().clear();
  TRY(check_net(net));
  if (!mean || !stdv || !log_mask) return fail(MRF_E_INVAL, "null standardisation array");
  for (int p = 0; p < net->P; ++p) {
    mean[p] = net->mean[p];
    stdv[p] = net->stdv[p];
    log_mask[p] = net->logm[p];
  }
  return MRF_OK;
}

extern "C" mrf_status mrf_net_forward(mrf_net net, const float *X, int64_t B, float *Y,
                                      mrf_stream stream) {
  last_error().clear();
  TRY(check_net(net));
  if (B < 0 || B > (1 << 30)) return fail(MRF_E_INVAL, "mrf_net_forward: bad B");
  if (B == 0) return MRF_OK;
  if (!X || !Y) return fail(MRF_E_INVAL, "mrf_net_forward: null X or Y");
  hipStream_t s = static_cast<hipStream_t>(stream);
  TRY(net_ws(net, B, false));
  return net_forward_rows(net, X, net->I, B, nullptr, Y, net->hb1.as<float>(), net->hb2.as<float>(), s);
}

namespace mrf {

bool net_bf16_ok(const mrf_net_s *net, int64_t K, int64_t ldx) {
  return net->H == 256 && net->P <= 8 && K % 8 == 0 && ldx % 4 == 0 && K <= round_up(net->I, kMlpBK);
}

// The network reads split-BF16 voxel rows of D directly: the BF16 form, and
// W1's padded width within the split rows' columns.
bool net_split_ok(const mrf_net_s *net, const mrf_dict_s *D) {
  return net->H == 256 && net->P <= 8 && net->I == D->K && round_up(net->I, kMlpBK) <= D->Kx;
}

// BF16 copies of W1 ([H][Kx], Kx = I rounded up to the K stage) and W2, made
// once per weight version; the wait lets later calls on any stream use them.
static mrf_status net_bf16_weights(mrf_net_s *net, hipStream_t s, uint16_t **w1b, uint16_t **w2b, int *Kx) {
  const int H = net->H, I = net->I;
  *Kx = (int)round_up(I, kMlpBK);
  TRY(grow(net->wb, ((size_t)H * *Kx + (size_t)H * H) * 2));
  const float *w = net->w.as<float>();
  *w1b = net->wb.as<uint16_t>();
  *w2b = *w1b + (size_t)H * *Kx;
  if (net->wbver != net->wver) {
    launch_to_bf16(w + net->oW1, H, I, I, *w1b, *Kx, s);
    launch_to_bf16(w + net->oW2, H, H, H, *w2b, H, s);
    LAUNCH_CHECK("network weights to bf16");
    HIP_TRY(hipStreamSynchronize(s));
    net->wbver = net->wver;
  }
  return MRF_OK;
}

// X: [B][ldx] FP32 with K readable columns (columns >= I meet zero weights).
mrf_status net_forward_bf16(mrf_net_s *net, const float *X, int64_t ldx, int64_t K, int64_t B,
                            const float *rowscale, float *Y, uint16_t *h1, hipStream_t s) {
  uint16_t *w1b, *w2b;
  int Kx;
  TRY(net_bf16_weights(net, s, &w1b, &w2b, &Kx));
  const float *w = net->w.as<float>();
  launch_mlp_bf16(B, X, ldx, (int)K, Kx, rowscale, w1b, w + net->ob1, h1, w2b, w + net->ob2, w + net->oW3,
                  w + net->ob3, net->P, Y, s);
  LAUNCH_CHECK("net forward (bf16)");
  return MRF_OK;
}

// Xs: split-BF16 rows of D ([B][2 D->Kx]); requires net_split_ok(net, D).
static mrf_status net_forward_bf16_split(mrf_net_s *net, const mrf_dict_s *D, const uint16_t *Xs, int64_t B,
                                         const float *rowscale, float *Y, uint16_t *h1, hipStream_t s) {
  uint16_t *w1b, *w2b;
  int Kx;
  TRY(net_bf16_weights(net, s, &w1b, &w2b, &Kx));
  const float *w = net->w.as<float>();
  launch_mlp_bf16_split(B, Xs, 2 * (int64_t)D->Kx, Kx, rowscale, w1b, w + net->ob1, h1, w2b, w + net->ob2,
                        w + net->oW3, w + net->ob3, net->P, Y, s);
  LAUNCH_CHECK("net forward (bf16, split rows)");
  return MRF_OK;
}

bool learned_split_rows_only(const mrf_dict_s *D, const mrf_match_opts *o, const int32_t *warm, bool cells_given) {
  if (!D || !o || o->method != MRF_LEARNED || o->precision != MRF_BF16X3 || warm) return false;
  if (o->certify_local) return false;  // the certificate rescores on the FP32 rows
  if (D->has_tree && o->eps >= 0.f) return false;  // the cover-tree fallback reads the FP32 rows
  return cells_given || (o->net && net_split_ok(o->net, D));
}

}  // namespace mrf

extern "C" mrf_status mrf_net_forward_bf16(mrf_net net, const float *X, int64_t B, float *Y,
                                           mrf_stream stream) {
  last_error().clear();
  TRY(check_net(net));
  if (B < 0 || B > (1 << 30)) return fail(MRF_E_INVAL, "mrf_net_forward_bf16: bad B");
  if (!net_bf16_ok(net, net->I, net->I))
    return fail(MRF_E_UNSUPPORTED, "mrf_net_forward_bf16: needs hidden width 256 and in_dim a multiple of 8");
  if (B == 0) return MRF_OK;
  if (!X || !Y) return fail(MRF_E_INVAL, "mrf_net_forward_bf16: null X or Y");
  hipStream_t s = static_cast<hipStream_t>(stream);
  TRY(net_ws(net, B, false));
  return net_forward_bf16(net, X, net->I, net->I, B, nullptr, Y, net->hb1.as<uint16_t>(), s);
}

extern "C" mrf_status mrf_net_loss_grad(mrf_net net, const float *X, const float *T, int64_t B,
                                        double *loss, mrf_stream stream) {
  last_error().clear();
  TRY(check_net(net));
  if (B < 1 || B > (1 << 24)) return fail(MRF_E_INVAL, "mrf_net_loss_grad: bad B");
  if (!X || !T) return fail(MRF_E_INVAL, "mrf_net_loss_grad: null X or T");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int nb = 0;
  TRY(net_loss_grad(net, X, T, B, &nb, s));
  if (loss) {
    launch_reduce_sum(net->red.as<double>(), nb, net->scal.as<double>(), s);
    LAUNCH_CHECK("reduce");
    HIP_TRY(hipMemcpyAsync(net->host_scal, net->scal.p, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *loss = net->host_scal[0] / ((double)B * net->P);
  }
  return MRF_OK;
}

extern "C" mrf_status mrf_net_adam(mrf_net net, float lr, float beta1, float beta2, float eps,
                                   mrf_stream stream) {
  last_error().clear();
  TRY(check_net(net));
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f))
    return fail(MRF_E_INVAL, "mrf_net_adam: bad hyper-parameters");
  net->t += 1;
  ++net->wver;
  launch_adam(net->w.as<float>(), net->g.as<float>(), net->m.as<float>(), net->v.as<float>(), net->nw,
              lr, beta1, beta2, eps, net->t, static_cast<hipStream_t>(stream));
  LAUNCH_CHECK("adam");
  return MRF_OK;
}

extern "C" mrf_status mrf_net_noisy_batch(mrf_net net, mrf_dict D, uint64_t seed, int64_t offset,
                                          int64_t B, float snr_lo, float snr_hi, float *X, float *T,
                                          int32_t *atom, mrf_stream stream) {
  last_error().clear();
  TRY(check_net(net));
  if (!D) return fail(MRF_E_INVAL, "null dictionary");
  if (net->I != D->K || net->P != D->nparam)
    return fail(MRF_E_INVAL, "network sizes (%d in, %d out) do not fit the dictionary (K %d, %d params)",
                net->I, net->P, D->K, D->nparam);
  if (B < 0 || offset < 0 || !X) return fail(MRF_E_INVAL, "mrf_net_noisy_batch: bad arguments");
  if (!(snr_hi >= snr_lo)) return fail(MRF_E_INVAL, "mrf_net_noisy_batch: snr_hi < snr_lo");
  if (T && !net->has_std) {
    std_from_dict(net, D);
    TRY(upload_std(net));
  }
  if (B == 0) return MRF_OK;
  uint64_t ka, ks, kn;
  train_keys(seed, &ka, &ks, &kn);
  launch_noisy_batch(D->dhat.as<float>(), D->Kp, D->L, D->is_complex ? 0 : 1, D->d,
                     D->params.as<float>(), D->nparam, dmean(net), dstdv(net), dlogm(net), ka, ks, kn,
                     offset, B, snr_lo, snr_hi, X, D->K, T, atom, static_cast<hipStream_t>(stream));
  LAUNCH_CHECK("noisy_batch");
  return MRF_OK;
}

extern "C" mrf_status mrf_net_train(mrf_net net, mrf_dict D, const mrf_train_opts *o,
                                    mrf_train_stats *st, mrf_stream stream) {
  last_error().clear();
  TRY(check_net(net));
  if (!D || !o) return fail(MRF_E_INVAL, "mrf_net_train: null argument");
  if (net->I != D->K || net->P != D->nparam)
    return fail(MRF_E_INVAL, "network sizes (%d in, %d out) do not fit the dictionary (K %d, %d params)",
                net->I, net->P, D->K, D->nparam);
  if (o->samples < 1 || o->batch < 1 || o->batch > (1 << 20) || o->epochs < 1 || !(o->lr > 0.f) ||
      !(o->lr_min >= 0.f) || !(o->snr_hi >= o->snr_lo))
    return fail(MRF_E_INVAL, "mrf_net_train: bad options");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!net->has_std) {
    std_from_dict(net, D);
    TRY(upload_std(net));
  }
  const int64_t B = o->batch;
  const int64_t per_epoch = std::max<int64_t>(1, o->samples / B);
  const int64_t total = per_epoch * o->epochs;
  TRY(grow(net->X, (size_t)B * net->I * 4));
  TRY(grow(net->T, (size_t)B * net->P * 4));
  TRY(net_ws(net, B, true));
  TRY(grow(net->scal, 64 * 8));
  uint64_t ka, ks, kn;
  train_keys(o->seed, &ka, &ks, &kn);
  EventPair ev;
  HIP_TRY(hipEventCreate(&ev.a));
  HIP_TRY(hipEventCreate(&ev.b));
  HIP_TRY(hipEventRecord(ev.a, s));
  const int window = (int)std::min<int64_t>(16, total);
  // per-step losses of the first and last `window` steps land in scal[0..32)
  for (int64_t step = 0; step < total; ++step) {
    const int64_t off = (step % per_epoch) * B;
    launch_noisy_batch(D->dhat.as<float>(), D->Kp, D->L, D->is_complex ? 0 : 1, D->d,
                       D->params.as<float>(), D->nparam, dmean(net), dstdv(net), dlogm(net), ka, ks, kn,
                       off, B, o->snr_lo, o->snr_hi, net->X.as<float>(), D->K, net->T.as<float>(),
                       nullptr, s);
    int nb = 0;
    TRY(net_loss_grad(net, net->X.as<float>(), net->T.as<float>(), B, &nb, s));
    if (step < window) launch_reduce_sum(net->red.as<double>(), nb, net->scal.as<double>() + step, s);
    else if (step >= total - window)
      launch_reduce_sum(net->red.as<double>(), nb, net->scal.as<double>() + 16 + (step - (total - window)), s);
    const double frac = (double)step / (double)std::max<int64_t>(1, total - 1);
    const float lr = (float)(o->lr_min + 0.5 * (o->lr - o->lr_min) * (1.0 + std::cos(M_PI * frac)));
    net->t += 1;
    ++net->wver;
    launch_adam(net->w.as<float>(), net->g.as<float>(), net->m.as<float>(), net->v.as<float>(),
                net->nw, lr, 0.9f, 0.999f, 1e-8f, net->t, s);
    LAUNCH_CHECK("train step");
  }
  HIP_TRY(hipEventRecord(ev.b, s));
  std::vector<double> l(32, 0.0);
  HIP_TRY(hipMemcpyAsync(l.data(), net->scal.p, 32 * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (st) {
    st->steps = (int32_t)total;
    double a = 0, b = 0;
    for (int i = 0; i < window; ++i) {
      a += l[(size_t)i];
      b += l[(size_t)(16 + i)];
    }
    st->first_loss = a / window / ((double)B * net->P);
    st->last_loss = b / window / ((double)B * net->P);
    HIP_TRY(hipEventElapsedTime(&st->ms, ev.a, ev.b));
  }
  return MRF_OK;
}

// ---------------------------------------------------------------------------
// learned / local matched filter
// ---------------------------------------------------------------------------
namespace mrf {

void launch_mark(const int32_t *list, int64_t cnt, int32_t *flags, hipStream_t s,
                 const unsigned int *dcnt = nullptr);

mrf_status check_learned(const mrf_dict_s *D, const mrf_match_opts *o, bool need_net) {
  if (D->grid_dims.empty()) return fail(MRF_E_UNSUPPORTED, "local search needs a product-grid dictionary (grid_dims)");
  if (D->nparam > 4) return fail(MRF_E_UNSUPPORTED, "local search supports at most 4 parameters");
  if (o->box_radius < 0 || o->box_radius > 64) return fail(MRF_E_INVAL, "box_radius %d not in 0..64", o->box_radius);
  if (o->recentre < 0 || o->recentre > 16) return fail(MRF_E_INVAL, "recentre %d not in 0..16", o->recentre);
  if (!std::isfinite(o->fallback_corr)) return fail(MRF_E_INVAL, "non-finite fallback_corr");
  if (D->has_tree && (std::isnan(o->eps) || (std::isinf(o->eps) && o->eps > 0.f)))
    return fail(MRF_E_INVAL, "eps of the cover-tree fallback must be finite (negative: exhaustive fallback)");
  if (D->has_tree && o->tree_capacity < 0) return fail(MRF_E_INVAL, "tree_capacity < 0");
  if (need_net) {
    if (!o->net) return fail(MRF_E_INVAL, "MRF_LEARNED needs a network");
    if (o->net->I != D->K || o->net->P != D->nparam)
      return fail(MRF_E_INVAL, "network sizes (%d in, %d out) do not fit the dictionary (K %d, %d params)",
                  o->net->I, o->net->P, D->K, D->nparam);
    if (!o->net->has_std) return fail(MRF_E_INVAL, "network has no target standardisation (train it first)");
  }
  return MRF_OK;
}

// The device counter of fallback voxels (all calls), created zeroed.
mrf_status fallback_total_buf(mrf_dict_s *D, hipStream_t s) {
  if (D->fbtot.p) return MRF_OK;
  TRY(grow(D->fbtot, 64));
  launch_zero(D->fbtot.p, 8, s);
  LAUNCH_CHECK("fallback counter");
  return MRF_OK;
}

mrf_status read_fallback_total(mrf_dict_s *D, hipStream_t s, int64_t *out) {
  *out = 0;
  if (!D->fbtot.p) return MRF_OK;
  unsigned long long v = 0;
  HIP_TRY(hipMemcpyAsync(&v, D->fbtot.p, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *out = (int64_t)v;
  return MRF_OK;
}

mrf_status ensure_x3(mrf_dict_s *D, hipStream_t s) {
  if (D->dx3.p) return MRF_OK;
  TRY(grow(D->dx3, (size_t)D->d_pad * 2 * D->Kx * 2));
  launch_split_x3(D->dhat.as<float>(), D->Kp, D->d_pad, D->Kx, D->dx3.as<uint16_t>(), s);
  LAUNCH_CHECK("split atoms");
  D->bytes += (int64_t)D->d_pad * 2 * D->Kx * 2;
  return MRF_OK;
}

mrf_status match_learned(mrf_dict_s *D, const mrf_match_opts *o, int64_t n, const int32_t *warm,
                         int32_t *idx, float *pd, float *corr, float *params_out, int32_t *cells_in,
                         int32_t *fallback_out, mrf_match_stats *st, hipStream_t s) {
  const int P = D->nparam;
  const int r = o->box_radius > 0 ? o->box_radius : 3;
  const float thr = o->fallback_corr == 0.f ? 0.98f : o->fallback_corr;
  // the packing leaves out the FP32 rows only where nothing below reads them
  if (!D->zp_fresh && !learned_split_rows_only(D, o, warm, cells_in != nullptr))
    return fail(MRF_E_UNSUPPORTED, "learned match: the voxels were packed without their FP32 rows");
  GridDims g;
  for (int p = 0; p < 4; ++p) g.dims[p] = p < P ? D->grid_dims[(size_t)p] : 1;
  EventPair ev;
  hipEvent_t e_prop0 = nullptr, e_prop1 = nullptr, e_ls0 = nullptr, e_ls1 = nullptr;
  if (st) {
    HIP_TRY(hipEventCreate(&e_ls0));
    HIP_TRY(hipEventCreate(&e_ls1));
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    HIP_TRY(hipEventCreate(&ev.c));
    HIP_TRY(hipEventCreate(&ev.d));
    HIP_TRY(hipEventCreate(&e_prop0));
    HIP_TRY(hipEventCreate(&e_prop1));
  }
  struct EvGuard {
    hipEvent_t a, b, c, d;
    ~EvGuard() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      if (c) (void)hipEventDestroy(c);
      if (d) (void)hipEventDestroy(d);
    }
  } eg{e_prop0, e_prop1, e_ls0, e_ls1};
  TRY(grow(D->gamma, (size_t)n * 4));
  TRY(grow(D->best_s, (size_t)n * 4));
  TRY(grow(D->best_j, (size_t)n * 4));
  TRY(grow(D->list_a, (size_t)n * 4));
  TRY(grow(D->list_b, (size_t)n * 4));
  TRY(grow(D->list_c, (size_t)n * 4));
  TRY(grow(D->keys, (size_t)n * 4));
  TRY(grow(D->cnt, 128));  // [0] fallback count, [1..16] re-centring rounds
  TRY(grow(D->counters, 64));
#ifndef MRF_LS_SHIFT
#define MRF_LS_SHIFT 2
#endif
#ifndef MRF_LS_RC_SHIFT
#define MRF_LS_RC_SHIFT 1
#endif
  const int shift = MRF_LS_SHIFT;  // coarse cells of 2^shift grid steps per parameter (a tuning constant)
  const int nkeys = coarse_key_count(g, P, shift);
  // re-centring rounds take few, scattered voxels: finer cells keep each
  // tile's bounding box close to its voxels' own boxes (also a tuning constant)
  const int shift_rc = MRF_LS_RC_SHIFT;
  const int nkeys_rc = coarse_key_count(g, P, shift_rc);
  TRY(grow(D->hist, (size_t)(4 * std::max(nkeys, nkeys_rc) + 8) * 4));
  auto group_bufs = [&](int nk) {
    GroupBufs b;
    b.hist = D->hist.as<unsigned int>();
    b.off = b.hist + nk;
    b.cursor = b.off + nk;
    b.toff = b.cursor + nk;
    return b;
  };
  const GroupBufs gb = group_bufs(nkeys), gb_rc = group_bufs(nkeys_rc);
  // per-call counters, 32-bit words of D->cnt: [0] fallback count, [1..16]
  // re-centring list lengths, [18..21] two 64-bit work counters (scored rows,
  // first-launch box atoms); all cleared by the preparation kernel with the
  // identity list and the per-voxel best keys
  unsigned int *cntw = D->cnt.as<unsigned int>();
  unsigned int *rcount = cntw + 1;
  unsigned long long *work = reinterpret_cast<unsigned long long *>(cntw + 18);
  TRY(grow(D->bestkey, (size_t)n * 8));
  unsigned long long *bkey = D->bestkey.as<unsigned long long>();
  // first pass: every voxel, grouped by coarse proposal cell
  int32_t *la = D->list_a.as<int32_t>(), *lb = D->list_b.as<int32_t>(), *lc = D->list_c.as<int32_t>();
  // start of the call (identity list, best keys, counters, histogram),
  // folded into the cells launch where the network runs
  const LearnedPrep prep{la, bkey, cntw, 22, gb.hist, nkeys};
  bool prepped = false;
  int32_t *cells = cells_in;
  if (!cells) {
    TRY(grow(D->cells, (size_t)n * P * 4));
    cells = D->cells.as<int32_t>();
    mrf_net_s *net = o->net;
    TRY(grow(D->inv, (size_t)n * 4));
    TRY(grow(D->h1, (size_t)n * net->H * 4));
    TRY(grow(D->h2, (size_t)n * net->H * 4));
    TRY(grow(D->yout, (size_t)n * P * 4));
    if (st) HIP_TRY(hipEventRecord(e_prop0, s));
    if (!D->inv_fresh) launch_inv_norm(D->znorm.as<float>(), n, D->inv.as<float>(), s);
    if (o->precision == MRF_BF16X3 && D->zx3_fresh && net_split_ok(net, D))
      TRY(net_forward_bf16_split(net, D, D->zx3.as<uint16_t>(), n, D->inv.as<float>(), D->yout.as<float>(),
                                 D->h1.as<uint16_t>(), s));
    else if (net_bf16_ok(net, D->Kp, D->Kp))
      TRY(net_forward_bf16(net, D->zp.as<float>(), D->Kp, D->Kp, n, D->inv.as<float>(), D->yout.as<float>(),
                           D->h1.as<uint16_t>(), s));
    else
      TRY(net_forward_rows(net, D->zp.as<float>(), D->Kp, n, D->inv.as<float>(), D->yout.as<float>(),
                           D->h1.as<float>(), D->h2.as<float>(), s));
    launch_cells(D->yout.as<float>(), n, P, dmean(net), dstdv(net), dlogm(net), D->axes.as<float>(),
                 D->aoff.as<int>(), D->dims.as<int>(), cells, s, &prep);
    prepped = true;
    LAUNCH_CHECK("cells");
    if (st) HIP_TRY(hipEventRecord(e_prop1, s));
  }
  if (!prepped) launch_learned_prep(prep, n, s);
  const bool x3 = o->precision == MRF_BF16X3;
  if (x3) TRY(ensure_x3(D, s));
  if (st) HIP_TRY(hipEventRecord(ev.a, s));
  if (x3 && !D->zx3_fresh) {
    TRY(grow(D->zx3, (size_t)n * 2 * D->Kx * 2));
    launch_split_x3(D->zp.as<float>(), D->Kp, n, D->Kx, D->zx3.as<uint16_t>(), s);
    LAUNCH_CHECK("split voxels");
  }
  const void *Dop = x3 ? D->dx3.p : D->dhat.p;
  const void *Zop = x3 ? D->zx3.p : D->zp.p;
  const int pitch = x3 ? D->Kx : D->Kp;
  launch_group(la, n, cells, P, shift, g, D->keys.as<int32_t>(), gb, lb, s, nullptr, true);
  if (st) HIP_TRY(hipEventRecord(e_ls0, s));
  launch_local_score(Dop, Zop, pitch, x3, lb, n, gb, nkeys, cells, P, g, r, shift, bkey, work, work + 1, s);
  // the best keys stay packed until every round is done: the face test reads
  // them, and one pass unpacks them all at the end
  if (st) HIP_TRY(hipEventRecord(e_ls1, s));
  LAUNCH_CHECK("local search");
  // re-centring rounds over the voxels whose best atom sits on an interior
  // face of their box: the face test writes the list into lc (and moves the
  // cells), the grouping sorts it into whichever of la / lb was not scored last.
  // The list lengths stay on the device (round rd's in rcount[rd]); every
  // grid is sized for all n voxels and its surplus exits at once, so the host
  // enqueues the rounds without waiting for the first launch to finish.
  int32_t *prev = lb;
  const unsigned int *prev_cnt = nullptr;  // device length of prev (null: all n)
  for (int rd = 0; rd < o->recentre; ++rd) {
    unsigned int *count = rcount + rd;
    // the face test also resets the listed voxels' best keys and clears the
    // histogram of the grouping that follows
    launch_face(prev, n, nullptr, cells, P, g, r, lc, count, s, prev_cnt, bkey, gb_rc.hist, nkeys_rc);
    int32_t *sorted = (prev == lb) ? la : lb;
    launch_group(lc, n, cells, P, shift_rc, g, D->keys.as<int32_t>(), gb_rc, sorted, s, count, true);
    launch_local_score(Dop, Zop, pitch, x3, sorted, n, gb_rc, nkeys_rc, cells, P, g, r, shift_rc, bkey, work,
                       nullptr, s);
    LAUNCH_CHECK("local search (re-centre)");
    prev = sorted;
    prev_cnt = count;
  }
  // unpacked here, or by the fallback selection below in the same pass
  const bool unpack_with_select = !warm && thr >= 0.f;
  // without a warm start or the certificate, the selection finishes the
  // voxels that do not fall back and the fallback's scatter the others, in
  // place of the closing merge pass
  const bool cert = o->certify_local != 0;
  const bool finish_early = unpack_with_select && !cert;
  const FinishArgs fin{D->d, D->znorm.as<float>(), warm, D->inv_norm.as<float>(), D->params.as<float>(),
                       D->nparam, idx, pd, corr, params_out, D->gamma.as<float>()};
  const FinishArgs *fe = finish_early ? &fin : nullptr;
  if (!unpack_with_select) launch_best_keys(nullptr, n, bkey, D->best_s.as<float>(), D->best_j.as<int32_t>(), 1, s);
  // the previous atom competes (non-expansive safeguard of the inexact projection)
  launch_warm_best(warm, n, D->d, D->zp.as<float>(), D->dhat.as<float>(), D->Kp, D->znorm.as<float>(),
                   D->best_s.as<float>(), D->best_j.as<int32_t>(), s);
  LAUNCH_CHECK("warm start");
  if (st) HIP_TRY(hipEventRecord(ev.b, s));
  // exhaustive fallback below the correlation threshold
  int64_t nfb = 0;
  bool tree_ran = false;
  if (fallback_out) launch_zero(fallback_out, n * 4, s);
  int32_t *fbflag = nullptr;  // certified: the exhaustive fallbacks, for the rescan
  if (cert) {
    TRY(grow(D->lc_fb, (size_t)n * 4));
    fbflag = D->lc_fb.as<int32_t>();
    launch_zero(fbflag, n * 4, s);
  }
  if (st) HIP_TRY(hipEventRecord(ev.c, s));
  bool nfb_on_device = false;  // the fallback count stayed on the device (read back only for stats)
  unsigned int *count = cntw;  // cleared by the preparation kernel
  if (thr >= 0.f) {
    if (unpack_with_select)
      launch_best_select(n, bkey, D->best_s.as<float>(), D->best_j.as<int32_t>(), D->znorm.as<float>(), thr, la,
                         count, s, fe);
    else
      launch_select_fallback(n, D->best_s.as<float>(), D->best_j.as<int32_t>(), D->znorm.as<float>(), thr,
                             la, count, s);
    TRY(fallback_total_buf(D, s));
    const bool tree_fb = D->has_tree && o->eps >= 0.f;
    if (x3 && !tree_fb) {
      // split-BF16 exhaustive fallback sized on the device (gather, filter and
      // merge read the count there): the host does not wait for the count
      const int64_t n_pad = round_up(n, kRowPad);
      TRY(grow(D->rows, (size_t)n_pad * D->Kx * 4));
      TRY(grow(D->part_s, (size_t)64 * n * 4));
      TRY(grow(D->part_j, (size_t)64 * n * 4));
      launch_gather_rows_dev(reinterpret_cast<const float *>(D->zx3.p), D->Kx, la, n, count, D->rows.as<float>(),
                             s, D->fbtot.as<unsigned long long>());
      launch_score_x3_dev(D->dx3.as<uint16_t>(), D->rows.as<uint16_t>(), D->d, D->d_pad, n, count, D->Kx,
                          D->part_s.as<float>(), D->part_j.as<int>(), s);
      launch_scatter_best(la, n, D->part_s.as<float>(), D->part_j.as<int>(), 1, D->best_s.as<float>(),
                          D->best_j.as<int32_t>(), s, count, (int)(D->d_pad / 256), fe);
      if (fallback_out) launch_mark(la, n, fallback_out, s, count);
      if (fbflag) launch_mark(la, n, fbflag, s, count);
      LAUNCH_CHECK("fallback (sized on the device)");
      nfb_on_device = true;
    }
  }
  if (thr >= 0.f && !nfb_on_device) {
    launch_add_count(D->fbtot.as<unsigned long long>(), count, s);
    unsigned int hc = 0;
    HIP_TRY(hipMemcpyAsync(&hc, count, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    nfb = hc;
    if (nfb > 0 && D->has_tree && o->eps >= 0.f) {
      // the cover tree (Algorithm 1, inaccuracy eps; eps = 0 is exact)
      // warm-started at each voxel's local best, on the FP32 rows
      const int64_t cnt_pad = round_up(nfb, kRowPad);
      TRY(grow(D->fb_rows, (size_t)cnt_pad * D->Kp * 4));
      TRY(grow(D->fb_norm, (size_t)nfb * 4));
      TRY(grow(D->fb_warm, (size_t)nfb * 4));
      TRY(grow(D->fb_s, (size_t)nfb * 4));
      TRY(grow(D->fb_j, (size_t)nfb * 4));
      launch_gather_rows(D->zp.as<float>(), D->Kp, la, nfb, cnt_pad, D->fb_rows.as<float>(), s);
      launch_gather_queries(la, nfb, D->znorm.as<float>(), D->best_j.as<int32_t>(), D->d, D->fb_norm.as<float>(),
                            D->fb_warm.as<int32_t>(), s);
      LAUNCH_CHECK("fallback queries");
      const int cap = o->tree_capacity > 0 ? o->tree_capacity : 1024;
      TRY(grow(D->ts_evals, 64));
      if (st) launch_zero(D->ts_evals.p, 8, s);
      tree_ran = true;
      TRY(tree_search(D, D->fb_rows.as<float>(), D->fb_norm.as<float>(), D->fb_warm.as<int32_t>(), nfb, o->eps, cap,
                      D->fb_s.as<float>(), D->fb_j.as<int32_t>(), D->list_c, D->rows, D->part_s, D->part_j, nullptr,
                      s));
      launch_scatter_best(la, nfb, D->fb_s.as<float>(), D->fb_j.as<int>(), 1, D->best_s.as<float>(),
                          D->best_j.as<int32_t>(), s, nullptr, 0, fe);
      if (fallback_out) launch_mark(la, nfb, fallback_out, s);
      if (fbflag) launch_mark(la, nfb, fbflag, s);
      LAUNCH_CHECK("fallback (cover tree)");
    } else if (nfb > 0) {
      const int64_t cnt_pad = round_up(nfb, kRowPad);
      TRY(grow(D->rows, (size_t)cnt_pad * std::max(D->Kp, D->Kx) * 4));
      int splits = 0;
      if (x3) {
        // split rows are 2 Kx BF16 = Kx words: gathered as rows of Kx floats
        launch_gather_rows(reinterpret_cast<const float *>(D->zx3.p), D->Kx, la, nfb, cnt_pad,
                           D->rows.as<float>(), s);
        splits = auto_splits_x3(D, nfb);
        TRY(grow(D->part_s, (size_t)splits * nfb * 4));
        TRY(grow(D->part_j, (size_t)splits * nfb * 4));
        launch_score_x3(D->dx3.as<uint16_t>(), D->rows.as<uint16_t>(), D->d, D->d_pad, nfb, cnt_pad, D->Kx,
                        splits, D->part_s.as<float>(), D->part_j.as<int>(), s);
      } else {
        launch_gather_rows(D->zp.as<float>(), D->Kp, la, nfb, cnt_pad, D->rows.as<float>(), s);
        const int64_t nvt = (nfb + 127) / 128;
        const int64_t nvt8 = (nvt + 7) / 8 * 8;
        int64_t sp = (1024 + nvt8 - 1) / nvt8;
        sp = std::max<int64_t>(1, std::min<int64_t>(sp, std::min<int64_t>(64, D->d_pad / 128)));
        splits = (int)sp;
        TRY(grow(D->part_s, (size_t)splits * nfb * 4));
        TRY(grow(D->part_j, (size_t)splits * nfb * 4));
        launch_score_f32(D->dhat.as<float>(), D->rows.as<float>(), D->d, D->d_pad, nfb, cnt_pad, D->Kp,
                         splits, D->part_s.as<float>(), D->part_j.as<int>(), s);
      }
      launch_scatter_best(la, nfb, D->part_s.as<float>(), D->part_j.as<int>(), splits,
                          D->best_s.as<float>(), D->best_j.as<int32_t>(), s, nullptr, 0, fe);
      if (fallback_out) launch_mark(la, nfb, fallback_out, s);
      if (fbflag) launch_mark(la, nfb, fbflag, s);
      LAUNCH_CHECK("fallback");
    }
  }
  if (st) HIP_TRY(hipEventRecord(ev.d, s));
  if (cert) {
    // Certified local search: the answer's exact score b, every box atom
    // whose local-pass score reaches b minus the pass's error bound (a second
    // pass over every voxel's final box, grouped afresh as the re-centring
    // moved the cells), all of them and the warm atom rescored exactly;
    // overflowing voxels and the exhaustive fallbacks go to the rescan of the
    // exhaustive certificate (FP32 collect, exact rescore, full exact scan).
    TRY(grow(D->cert, 64));
    TRY(grow(D->cert_list, (size_t)n * 4));
    TRY(grow(D->cert_thr, (size_t)n * 4));
    TRY(grow(D->cert_ccount, (size_t)n * 4));
    TRY(grow(D->cert_scan, (size_t)n * 4));
    TRY(grow(D->cert_cand, (size_t)n * kCertCap * 4));
    TRY(grow(D->lc_thr, (size_t)n * 4));
    TRY(grow(D->lc_count, (size_t)n * 4));
    TRY(grow(D->lc_cand, (size_t)n * kCertCap * 4));
    TRY(grow(D->lc_bex, (size_t)n * 8));
    TRY(grow(D->lc_bjx, (size_t)n * 4));
    launch_zero(D->cert.p, 64, s);
    unsigned int *cq = D->cert.as<unsigned int>();
    const CertQueue q{cq, D->cert_list.as<int32_t>(), D->cert_thr.as<float>(), D->cert_ccount.as<unsigned int>(),
                      cq + 1, D->cert_scan.as<int32_t>(), reinterpret_cast<unsigned long long *>(cq + 2)};
    const CertOut out{D->znorm.as<float>(), warm, D->inv_norm.as<float>(), D->params.as<float>(), D->nparam, idx,
                      pd, corr, params_out, D->gamma.as<float>()};
    const float cE = cert_coeff(o->precision, D->K), cE32 = cert_coeff(MRF_FP32, D->K);
    launch_local_line(D->best_s.as<float>(), D->best_j.as<int32_t>(), fbflag, n, D->d, D->zp.as<float>(),
                      D->dhat.as<float>(), D->Kp, D->K, cE, cE32, kCertAbs, out, D->lc_thr.as<float>(),
                      D->lc_count.as<unsigned int>(), D->lc_bex.as<double>(), D->lc_bjx.as<int32_t>(), q, s);
    LAUNCH_CHECK("local certificate line");
    launch_iota(lc, n, s);
    launch_group(lc, n, cells, P, shift, g, D->keys.as<int32_t>(), gb, lb, s, nullptr, false);
    const LocalCollect lcol{D->lc_thr.as<float>(), D->lc_count.as<unsigned int>(), D->lc_cand.as<int32_t>(),
                            kCertCap};
    launch_local_score(Dop, Zop, pitch, x3, lb, n, gb, nkeys, cells, P, g, r, shift, nullptr, nullptr, nullptr, s,
                       &lcol);
    LAUNCH_CHECK("local certificate collect");
    launch_rescore_local(D->zp.as<float>(), D->dhat.as<float>(), D->Kp, D->K, D->d, n,
                         D->lc_count.as<unsigned int>(), D->lc_cand.as<int32_t>(), kCertCap, D->lc_bex.as<double>(),
                         D->lc_bjx.as<int32_t>(), warm, fbflag, cE32, kCertAbs, out, q, s);
    launch_collect_f32_dev(D->dhat.as<float>(), D->zp.as<float>(), q.list, D->d, D->d_pad, n, q.count, D->Kp, q.thr,
                           q.ccount, D->cert_cand.as<int32_t>(), kCertCap, s);
    launch_rescore_collected(D->zp.as<float>(), D->dhat.as<float>(), D->Kp, D->K, D->d, n, q,
                             D->cert_cand.as<int32_t>(), kCertCap, out, s);
    launch_scan_exact(D->zp.as<float>(), D->dhat.as<float>(), D->Kp, D->K, D->d, n, q, out, s);
    LAUNCH_CHECK("local certificate rescore");
  } else if (!finish_early) {
    launch_merge_argmax(D->best_s.as<float>(), D->best_j.as<int>(), 1, n, D->d, D->znorm.as<float>(), warm,
                        D->inv_norm.as<float>(), D->params.as<float>(), D->nparam, idx, pd, corr, params_out,
                        D->gamma.as<float>(), s);
    LAUNCH_CHECK("merge");
  }
  if (st) {
    unsigned long long wk[2] = {0, 0}, ev_count = 0;
    unsigned int rc[16] = {0}, dev_nfb = 0, cc[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(wk, work, 16, hipMemcpyDeviceToHost, s));
    if (cert) HIP_TRY(hipMemcpyAsync(cc, D->cert.p, 16, hipMemcpyDeviceToHost, s));
    if (nfb_on_device) HIP_TRY(hipMemcpyAsync(&dev_nfb, count, 4, hipMemcpyDeviceToHost, s));
    if (o->recentre > 0) HIP_TRY(hipMemcpyAsync(rc, rcount, 4 * o->recentre, hipMemcpyDeviceToHost, s));
    if (tree_ran) HIP_TRY(hipMemcpyAsync(&ev_count, D->ts_evals.p, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    st->fallbacks = nfb_on_device ? (int64_t)dev_nfb : nfb;
    int64_t recentred = 0;
    for (int rd = 0; rd < o->recentre; ++rd) recentred += rc[rd];
    st->recentred = recentred;
    st->local_atoms = (int64_t)wk[0];
    st->first_box_atoms = (int64_t)wk[1];
    st->distance_evals = (int64_t)ev_count;
    if (cert) {
      st->cert_rescanned = cc[0];
      st->cert_scanned = cc[1];
      st->cert_rescored = (int64_t)(cc[2] | ((unsigned long long)cc[3] << 32));
    }
    HIP_TRY(hipEventElapsedTime(&st->search_ms, ev.a, ev.b));
    HIP_TRY(hipEventElapsedTime(&st->score_ms, e_ls0, e_ls1));
    HIP_TRY(hipEventElapsedTime(&st->fallback_ms, ev.c, ev.d));
    if (!cells_in) HIP_TRY(hipEventElapsedTime(&st->proposal_ms, e_prop0, e_prop1));
  }
  return MRF_OK;
}

}  // namespace mrf

extern "C" mrf_status mrf_match_local(mrf_dict D, const mrf_match_opts *opts, int64_t n, const void *Z,
                                      int32_t z_layout, int64_t slice_voxels, int32_t *cells,
                                      const int32_t *warm_idx, int32_t *idx, float *pd, float *corr,
                                      int32_t *fallback, void *X_out, float *params_out,
                                      mrf_match_stats *stats, mrf_stream stream) {
  last_error().clear();
  if (!D || !opts) return fail(MRF_E_INVAL, "mrf_match_local: null dictionary or options");
  TRY(check_learned(D, opts, false));
  if (opts->precision != MRF_FP32 && opts->precision != MRF_BF16X3)
    return fail(MRF_E_INVAL, "mrf_match_local: precision must be MRF_FP32 or MRF_BF16X3");
  if (n < 0) return fail(MRF_E_INVAL, "mrf_match_local: n < 0");
  if (n > 0 && (!Z || !idx || !cells)) return fail(MRF_E_INVAL, "mrf_match_local: null Z, cells or idx");
  if (z_layout != MRF_VOXEL_MAJOR && z_layout != MRF_FRAME_MAJOR)
    return fail(MRF_E_INVAL, "mrf_match_local: bad z_layout %d", z_layout);
  if (z_layout == MRF_FRAME_MAJOR && (slice_voxels < 1 || n % slice_voxels != 0))
    return fail(MRF_E_INVAL, "mrf_match_local: slice_voxels must divide n");
  if (n > ((int64_t)1 << 31) - 1024) return fail(MRF_E_INVAL, "mrf_match_local: n too large");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (n == 0) return MRF_OK;
  EventPair ev;
  if (stats) {
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    HIP_TRY(hipEventRecord(ev.a, s));
  }
  TRY(pack_voxels(D, Z, z_layout, slice_voxels, n, s, opts && opts->precision == MRF_BF16X3,
                  !learned_split_rows_only(D, opts, warm_idx, true), stats != nullptr));
  TRY(match_learned(D, opts, n, warm_idx, idx, pd, corr, params_out, cells, fallback, stats, s));
  if (X_out) {
    launch_write_x(idx, D->gamma.as<float>(), D->dhat.as<float>(), D->Kp, D->is_complex ? 0 : 1, n, D->L,
                   z_layout == MRF_FRAME_MAJOR, slice_voxels, static_cast<float2 *>(X_out), nullptr,
                   nullptr, nullptr, nullptr, s, D->align ? D->vphase.as<float2>() : nullptr);
    LAUNCH_CHECK("write_x");
  }
  if (stats) {
    HIP_TRY(hipEventRecord(ev.b, s));
    unsigned long long cnt[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(cnt, D->counters.p, sizeof cnt, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipEventElapsedTime(&stats->ms, ev.a, ev.b));
    stats->n = n;
    stats->zero_voxels = (int64_t)cnt[0];
    stats->nonfinite = (int64_t)cnt[1];
    if (cnt[1] > 0) return fail(MRF_E_NUMERIC, "mrf_match_local: %llu voxel(s) with non-finite entries", cnt[1]);
  }
  return MRF_OK;
}
