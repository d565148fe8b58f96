// Test driver: reads normalised FP64 rows (d, K, then d*K doubles) from a
// file, builds the library's cover tree with its host builder, and writes
// sigma, imax, then per unique atom (rep, ins_level, parent).
#include <cstdio>
#include <vector>

#include "../paper_1810_01967_amd/csrc/covertree.h"

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  FILE *f = std::fopen(argv[1], "rb");
  if (!f) return 3;
  long long d = 0, K = 0;
  if (std::fread(&d, 8, 1, f) != 1 || std::fread(&K, 8, 1, f) != 1) return 4;
  std::vector<double> X((size_t)(d * K));
  if (std::fread(X.data(), 8, X.size(), f) != X.size()) return 5;
  std::fclose(f);
  mrf::HostTree T;
  mrf::build_cover_tree(X.data(), d, K, T);
  mrf::FlatTree F;
  mrf::flatten_cover_tree(T, F);
  FILE *o = std::fopen(argv[2], "w");
  std::fprintf(o, "%.17g %d %zu %zu\n", T.sigma, T.imax, T.rep.size(), F.node.size());
  for (size_t i = 0; i < T.rep.size(); ++i) std::fprintf(o, "%d %d %d\n", T.rep[i], T.ins_level[i], T.parent[i]);
  for (size_t i = 0; i < T.levels.size(); ++i)
    for (size_t j = 0; j < T.levels[i].size(); ++j) std::fprintf(o, "%.9g\n", T.maxdist[i][j]);
  // flattened form: per entry node, child range, self flag
  for (size_t e = 0; e < F.node.size(); ++e)
    std::fprintf(o, "%d %lld %lld %d\n", F.node[e], (long long)F.child_begin[e], (long long)F.child_end[e],
                 (int)F.is_self[e]);
  for (size_t i = 0; i < F.level_begin.size(); ++i) std::fprintf(o, "%lld\n", (long long)F.level_begin[i]);
  std::fclose(o);
  return 0;
}
