// Host-side driver of the C ABI for the sanitizer build: argument
// validation of every entry point, and the host work that runs before the
// first device call (dictionary normalisation over the caller's arrays,
// network construction, the non-uniform plan's checks of offsets and
// coordinates) followed by the error path a machine without a GPU takes.
// Exits non-zero on the first unexpected status; any sanitizer report
// aborts the run.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "mrf.h"

static int failures = 0;

static void expect(const char *what, mrf_status got, bool ok) {
  const char *msg = mrf_last_error();
  if (!ok) {
    std::printf("FAIL %s: status %d (%s)\n", what, (int)got, msg ? msg : "");
    ++failures;
  } else {
    std::printf("ok   %s: status %d (%s)\n", what, (int)got, msg ? msg : "");
  }
}

static void expect_inval(const char *what, mrf_status got) {
  expect(what, got, got == MRF_E_INVAL && std::strlen(mrf_last_error()) > 0);
}

int main() {
  if (std::strncmp(mrf_version(), "mrf-mi355x", 10) != 0) return 2;

  // dictionaries
  mrf_dict D = nullptr;
  expect_inval("dict_build null desc", mrf_dict_build(nullptr, nullptr, &D));
  std::vector<double> atoms(4 * 3, 1.0), params(4, 0.0);
  mrf_dict_desc desc{};
  desc.d = 0; desc.L = 3; desc.nparam = 1; desc.is_complex = 0;
  desc.atoms = atoms.data(); desc.atoms_dtype = MRF_F64; desc.params = params.data();
  expect_inval("dict_build d = 0", mrf_dict_build(&desc, nullptr, &D));
  desc.d = 4; desc.flags = 0x100;
  expect_inval("dict_build unknown flag", mrf_dict_build(&desc, nullptr, &D));
  desc.flags = 0;
  int32_t gd = 3;  // product 3 != d = 4
  desc.grid_dims = &gd;
  expect_inval("dict_build grid mismatch", mrf_dict_build(&desc, nullptr, &D));
  desc.grid_dims = nullptr;
  atoms[5] = NAN;
  expect_inval("dict_build non-finite atom", mrf_dict_build(&desc, nullptr, &D));
  atoms[5] = 1.0;
  for (int t = 0; t < 3; ++t) atoms[2 * 3 + t] = 0.0;  // atom 2 has zero norm
  expect_inval("dict_build zero-norm atom", mrf_dict_build(&desc, nullptr, &D));
  for (int t = 0; t < 3; ++t) atoms[2 * 3 + t] = 1.0 + t;
  // a valid descriptor: host normalisation, then the first device call
  std::vector<float> atoms32(6 * 5 * 2);
  for (size_t i = 0; i < atoms32.size(); ++i) atoms32[i] = std::sin(0.37f * (float)(i + 1));
  std::vector<double> p2(6 * 2, 1.0);
  int32_t gd2[2] = {2, 3};
  mrf_dict_desc ok{};
  ok.d = 6; ok.L = 5; ok.nparam = 2; ok.is_complex = 1; ok.atoms = atoms32.data();
  ok.atoms_dtype = MRF_F32; ok.params = p2.data(); ok.grid_dims = gd2; ok.flags = MRF_STORE_BF16;
  mrf_status st = mrf_dict_build(&ok, nullptr, &D);
  expect("dict_build valid (device step fails or succeeds)", st, st == MRF_OK || st == MRF_E_HIP || st == MRF_E_NOMEM);
  if (st == MRF_OK) mrf_dict_destroy(D);
  D = nullptr;
  expect("dict_destroy null", mrf_dict_destroy(nullptr), true);
  mrf_dict_info info;
  expect_inval("dict_query null", mrf_dict_query(nullptr, &info));
  expect_inval("dict_copy_atoms null", mrf_dict_copy_atoms(nullptr, MRF_FP32, nullptr, nullptr, nullptr));
  mrf_dict C = nullptr;
  expect_inval("dict_compress null", mrf_dict_compress(nullptr, 4, 0, nullptr, &C));
  expect_inval("dict_align null", mrf_dict_align(nullptr, 0, nullptr, &C));
  expect_inval("dict_subspace null", mrf_dict_subspace(nullptr, nullptr, nullptr));
  mrf_tree_info ti;
  expect_inval("dict_tree_info null", mrf_dict_tree_info(nullptr, &ti));

  // matched filter and local search
  mrf_match_opts mo{};
  mo.method = MRF_EXHAUSTIVE; mo.precision = MRF_FP32; mo.topk = 8;
  expect_inval("match null dict", mrf_match(nullptr, &mo, 1, nullptr, MRF_VOXEL_MAJOR, 0, nullptr, nullptr,
                                            nullptr, nullptr, nullptr, nullptr, nullptr, nullptr));
  expect_inval("match_local null dict",
               mrf_match_local(nullptr, &mo, 1, nullptr, MRF_VOXEL_MAJOR, 0, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr));

  // forward model and solver
  mrf_op bad{};
  bad.nx = 48; bad.ny = 64; bad.L = 10; bad.nslices = 1;  // 48 is not a power of two
  expect_inval("op_forward bad nx", mrf_op_forward(&bad, nullptr, nullptr, nullptr, nullptr, nullptr));
  expect_inval("op_adjoint null op", mrf_op_adjoint(nullptr, nullptr, 1, nullptr, nullptr));
  expect_inval("ipg_step null dict", mrf_ipg_step(nullptr, &bad, nullptr, nullptr, nullptr, nullptr, nullptr,
                                                  nullptr, 1.f, &mo, nullptr, nullptr));
  mrf_solve_opts so{};
  expect_inval("ipg_solve null dict", mrf_ipg_solve(nullptr, &bad, nullptr, &so, nullptr, nullptr, nullptr,
                                                    nullptr, nullptr, nullptr));

  // encoders
  expect_inval("quantize_rows null", mrf_quantize_rows(nullptr, 1, 4, 4, MRF_BF16, nullptr, 4, nullptr, nullptr));

  // networks: bad sizes, then a valid network whose device allocation may fail
  mrf_net net = nullptr;
  expect_inval("net_create null out", mrf_net_create(8, 16, 2, 1, nullptr));
  expect_inval("net_create bad sizes", mrf_net_create(0, 16, 2, 1, &net));
  expect_inval("net_create nout 9", mrf_net_create(8, 16, 9, 1, &net));
  st = mrf_net_create(8, 16, 2, 1, &net);
  expect("net_create valid (device step fails or succeeds)", st, st == MRF_OK || st == MRF_E_HIP || st == MRF_E_NOMEM);
  if (st == MRF_OK) mrf_net_destroy(net);
  expect("net_destroy null", mrf_net_destroy(nullptr), true);
  int64_t cnt = 0;
  expect_inval("net_size null", mrf_net_size(nullptr, &cnt));
  mrf_train_opts to{};
  expect_inval("net_train null", mrf_net_train(nullptr, nullptr, &to, nullptr, nullptr));

  // non-uniform plans: offsets and coordinates are checked on the host
  std::vector<int64_t> off = {0, 3, 5};
  std::vector<float> co = {0.1f, 0.2f, -0.3f, 0.4f, 0.0f, 0.5f, 0.25f, -0.25f, 0.125f, 0.0625f};
  mrf_nufft plan = nullptr;
  expect_inval("nufft_create null out", mrf_nufft_create(16, 16, 2, 1, 5, off.data(), co.data(), 7, nullptr));
  off[1] = 6;  // not monotone
  expect_inval("nufft_create bad offsets", mrf_nufft_create(16, 16, 2, 1, 5, off.data(), co.data(), 7, &plan));
  off[1] = 3;
  co[3] = NAN;
  expect_inval("nufft_create non-finite coordinate", mrf_nufft_create(16, 16, 2, 1, 5, off.data(), co.data(), 7, &plan));
  co[3] = 2048.f;
  expect_inval("nufft_create coordinate beyond 1024", mrf_nufft_create(16, 16, 2, 1, 5, off.data(), co.data(), 7, &plan));
  co[3] = 0.4f;
  expect_inval("nufft_create bad width", mrf_nufft_create(16, 16, 2, 1, 5, off.data(), co.data(), 3, &plan));
  st = mrf_nufft_create(16, 16, 2, 1, 5, off.data(), co.data(), 7, &plan);
  expect("nufft_create valid (device step fails or succeeds)", st, st == MRF_OK || st == MRF_E_HIP || st == MRF_E_NOMEM);
  if (st == MRF_OK) mrf_nufft_destroy(plan);
  expect("nufft_destroy null", mrf_nufft_destroy(nullptr), true);

  std::printf("%d failure(s)\n", failures);
  return failures ? 1 : 0;
}
