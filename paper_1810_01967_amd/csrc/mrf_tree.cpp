// Host side of the cover-tree comparator: tree upload and export, and the
// level-synchronous batched search used by MRF_COVERTREE (Algorithm 1 per
// voxel on Z_v/||Z_v||, warm-started as in Algorithm 2), with the exhaustive
// filter for queries whose candidate set outgrows its capacity.
#include "host_common.h"

using namespace mrf;

namespace mrf {

mrf_status upload_tree(mrf_dict_s *D, const double *Xnorm) {
  HostTree &T = D->tree;
  build_cover_tree(Xnorm, D->d, D->K, T);
  FlatTree F;
  flatten_cover_tree(T, F);
  const int64_t E = (int64_t)F.node.size();
  if (E >= ((int64_t)1 << 31)) return fail(MRF_E_UNSUPPORTED, "cover tree too large");
  std::vector<int32_t> cb((size_t)E), ce((size_t)E);
  for (int64_t e = 0; e < E; ++e) {
    cb[(size_t)e] = (int32_t)F.child_begin[(size_t)e];
    ce[(size_t)e] = (int32_t)F.child_end[(size_t)e];
  }
  const size_t u = T.rep.size();
  TRY(grow(D->t_node, (size_t)E * 4));
  TRY(grow(D->t_cb, (size_t)E * 4));
  TRY(grow(D->t_ce, (size_t)E * 4));
  TRY(grow(D->t_md, (size_t)E * 4));
  TRY(grow(D->t_self, (size_t)E));
  TRY(grow(D->t_rep, u * 4));
  TRY(grow(D->t_uniq, (size_t)D->d * 4));
  HIP_TRY(hipMemcpy(D->t_node.p, F.node.data(), (size_t)E * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(D->t_cb.p, cb.data(), (size_t)E * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(D->t_ce.p, ce.data(), (size_t)E * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(D->t_md.p, F.maxdist.data(), (size_t)E * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(D->t_self.p, F.is_self.data(), (size_t)E, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(D->t_rep.p, T.rep.data(), u * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(D->t_uniq.p, T.uniq_of.data(), (size_t)D->d * 4, hipMemcpyHostToDevice));
  D->tree_entries = E;
  D->has_tree = true;
  D->bytes += (int64_t)(D->t_node.cap + D->t_cb.cap + D->t_ce.cap + D->t_md.cap + D->t_self.cap +
                        D->t_rep.cap + D->t_uniq.cap);
  return MRF_OK;
}

mrf_status tree_search(mrf_dict_s *D, const float *Q, const float *qnorm, const int32_t *warm, int64_t n,
                       float eps, int cap, float *out_s, int32_t *out_j, DevBuf &ovf, DevBuf &rows, DevBuf &ps,
                       DevBuf &pj, int64_t *n_overflow, hipStream_t s) {
  TRY(grow(D->ts_active, (size_t)n * 4));
  TRY(grow(D->ts_qc, (size_t)n * 4));
  TRY(grow(D->ts_cnt, (size_t)n * 4));
  TRY(grow(D->ts_flags, (size_t)n * 4));
  TRY(grow(D->ts_dmin, (size_t)n * 4));
  TRY(grow(D->ts_Qe0, (size_t)n * cap * 4));
  TRY(grow(D->ts_Qe1, (size_t)n * cap * 4));
  TRY(grow(D->ts_Qd0, (size_t)n * cap * 4));
  TRY(grow(D->ts_Qd1, (size_t)n * cap * 4));
  TRY(grow(D->ts_evals, 64));
  TRY(grow(ovf, (size_t)n * 4));
  TRY(grow(D->cnt, 64));
  TreeDev t;
  t.dhat = D->dhat.as<float>();
  t.node = D->t_node.as<int32_t>();
  t.rep = D->t_rep.as<int32_t>();
  t.uniq_of = D->t_uniq.as<int32_t>();
  t.child_begin = D->t_cb.as<int32_t>();
  t.child_end = D->t_ce.as<int32_t>();
  t.maxdist = D->t_md.as<float>();
  t.is_self = D->t_self.as<uint8_t>();
  t.d = D->d;
  t.sigma = (float)D->tree.sigma;
  t.imax = D->tree.imax;
  TreeState ts;
  ts.active = D->ts_active.as<int32_t>();
  ts.qc = D->ts_qc.as<int32_t>();
  ts.cnt = D->ts_cnt.as<int32_t>();
  ts.flags = D->ts_flags.as<int32_t>();
  ts.dmin = D->ts_dmin.as<float>();
  ts.Qe = D->ts_Qe0.as<int32_t>();
  ts.Qd = D->ts_Qd0.as<float>();
  ts.cap = cap;
  ts.evals = D->ts_evals.as<unsigned long long>();
  launch_tree_init(t, Q, D->Kp, qnorm, warm, n, ts, s);
  LAUNCH_CHECK("tree init");
  const float inv_eps = eps > 0.f ? 1.f / eps : INFINITY;
  int32_t *qe_next = D->ts_Qe1.as<int32_t>();
  float *qd_next = D->ts_Qd1.as<float>();
  for (int level = 0; level < t.imax; ++level) {
    launch_tree_level(t, Q, D->Kp, qnorm, n, level, inv_eps, ts, qe_next, qd_next, s);
    LAUNCH_CHECK("tree level");
    std::swap(ts.Qe, qe_next);
    std::swap(ts.Qd, qd_next);
  }
  launch_tree_finish(t, Q, D->Kp, D->K, qnorm, n, ts, out_s, out_j, s);
  LAUNCH_CHECK("tree finish");
  // queries whose candidate set overflowed: exhaustive filter
  unsigned int *count = D->cnt.as<unsigned int>();
  launch_zero(count, 4, s);
  launch_tree_select(ts, n, ovf.as<int32_t>(), count, s);
  unsigned int hc = 0;
  HIP_TRY(hipMemcpyAsync(&hc, count, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t nfb = hc;
  if (nfb > 0) {
    const int64_t cnt_pad = round_up(nfb, kRowPad);
    TRY(grow(rows, (size_t)cnt_pad * D->Kp * 4));
    launch_gather_rows(Q, D->Kp, ovf.as<int32_t>(), nfb, cnt_pad, rows.as<float>(), s);
    const int64_t nvt = (nfb + 127) / 128, nvt8 = (nvt + 7) / 8 * 8;
    int64_t sp = (1024 + nvt8 - 1) / nvt8;
    sp = std::max<int64_t>(1, std::min<int64_t>(sp, std::min<int64_t>(64, D->d_pad / 128)));
    TRY(grow(ps, (size_t)sp * nfb * 4));
    TRY(grow(pj, (size_t)sp * nfb * 4));
    launch_score_f32(D->dhat.as<float>(), rows.as<float>(), D->d, D->d_pad, nfb, cnt_pad, D->Kp, (int)sp,
                     ps.as<float>(), pj.as<int>(), s);
    launch_scatter_best(ovf.as<int32_t>(), nfb, ps.as<float>(), pj.as<int>(), (int)sp, out_s, out_j, s);
    LAUNCH_CHECK("tree fallback");
  }
  if (n_overflow) *n_overflow = nfb;
  return MRF_OK;
}

mrf_status match_tree(mrf_dict_s *D, const mrf_match_opts *o, int64_t n, const int32_t *warm,
                      int32_t *idx, float *pd, float *corr, float *params_out, mrf_match_stats *st,
                      hipStream_t s) {
  const int cap = o->tree_capacity > 0 ? o->tree_capacity : 1024;
  TRY(grow(D->gamma, (size_t)n * 4));
  TRY(grow(D->best_s, (size_t)n * 4));
  TRY(grow(D->best_j, (size_t)n * 4));
  TRY(grow(D->ts_evals, 64));
  EventPair ev;
  if (st) {
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    HIP_TRY(hipEventRecord(ev.a, s));
  }
  // the counter accumulates over searches: reset here for a direct call with
  // stats, by the projected-gradient entry points otherwise
  if (st) launch_zero(D->ts_evals.p, 8, s);
  int64_t nfb = 0;
  TRY(tree_search(D, D->zp.as<float>(), D->znorm.as<float>(), warm, n, o->eps, cap, D->best_s.as<float>(),
                  D->best_j.as<int32_t>(), D->list_a, D->rows, D->part_s, D->part_j, &nfb, s));
  launch_merge_argmax(D->best_s.as<float>(), D->best_j.as<int>(), 1, n, D->d, D->znorm.as<float>(), warm,
                      D->inv_norm.as<float>(), D->params.as<float>(), D->nparam, idx, pd, corr, params_out,
                      D->gamma.as<float>(), s);
  LAUNCH_CHECK("merge");
  if (st) {
    HIP_TRY(hipEventRecord(ev.b, s));
    unsigned long long ev_count = 0;
    HIP_TRY(hipMemcpyAsync(&ev_count, D->ts_evals.p, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipEventElapsedTime(&st->search_ms, ev.a, ev.b));
    st->distance_evals = (int64_t)ev_count;
    st->fallbacks = nfb;
    st->tree_levels = D->tree.imax;
  }
  return MRF_OK;
}

}  // namespace mrf

extern "C" mrf_status mrf_dict_tree_info(mrf_dict D, mrf_tree_info *info) {
  last_error().clear();
  if (!D || !info) return fail(MRF_E_INVAL, "mrf_dict_tree_info: null argument");
  if (!D->has_tree) return fail(MRF_E_UNSUPPORTED, "dictionary built without MRF_BUILD_COVERTREE");
  info->unique_atoms = (int32_t)D->tree.rep.size();
  info->imax = D->tree.imax;
  info->entries = D->tree_entries;
  info->sigma = D->tree.sigma;
  return MRF_OK;
}

extern "C" mrf_status mrf_dict_tree_export(mrf_dict D, int32_t *rep, int32_t *ins_level, int32_t *parent,
                                           float *maxdist) {
  last_error().clear();
  if (!D || !rep || !ins_level || !parent) return fail(MRF_E_INVAL, "mrf_dict_tree_export: null argument");
  if (!D->has_tree) return fail(MRF_E_UNSUPPORTED, "dictionary built without MRF_BUILD_COVERTREE");
  const HostTree &T = D->tree;
  for (size_t i = 0; i < T.rep.size(); ++i) {
    rep[i] = T.rep[i];
    ins_level[i] = T.ins_level[i];
    parent[i] = T.parent[i];
  }
  if (maxdist) {
    size_t k = 0;
    for (size_t i = 0; i < T.levels.size(); ++i)
      for (size_t j = 0; j < T.levels[i].size(); ++j) maxdist[k++] = T.maxdist[i][j];
  }
  return MRF_OK;
}
