// Cover tree over the normalised, de-duplicated atoms: host build and its
// flattened (per level, per node) form for the device traversal.
#pragma once

#include <cstdint>
#include <vector>

namespace mrf {

struct HostTree {
  double sigma = 0.0;
  int imax = 0;                              // deepest level (all unique atoms are nodes)
  std::vector<int32_t> rep;                  // unique atom -> lowest dictionary index
  std::vector<int32_t> uniq_of;              // dictionary index -> unique atom
  std::vector<std::vector<int32_t>> levels;  // S_0 .. S_imax (unique indices, ascending)
  std::vector<int32_t> parent;               // parent (in S_{l-1}) of a node first added at level l
  std::vector<int32_t> ins_level;            // level at which each unique atom became a node
  std::vector<std::vector<float>> maxdist;   // per level, aligned with levels[i]
  static double dist(const double *X, int64_t K, int32_t a, int32_t b);
};

struct FlatTree {
  std::vector<int64_t> level_begin;  // entries of level i: [level_begin[i], level_begin[i+1])
  std::vector<int32_t> node;         // unique atom of the entry
  std::vector<int64_t> child_begin, child_end;  // children: entries of the next level
  std::vector<float> maxdist;
  std::vector<uint8_t> is_self;      // the entry is its parent's self-child
};

// Xall: normalised FP64 rows [d][K] (the real contraction form of the atoms).
void build_cover_tree(const double *Xall, int64_t d, int64_t K, HostTree &T);
void flatten_cover_tree(const HostTree &T, FlatTree &F);

}  // namespace mrf
