// Host construction of the cover tree (Section "Cover trees") over the
// normalised, de-duplicated atoms, FP64.
//
// The tree is the greedy nested-net tree: root S_0 = {atom 0}, sigma =
// max_j ||D_0 - D_j||; level i+1 (radius r = sigma 2^-(i+1)) starts from S_i
// and scans the remaining atoms in increasing index, adding an atom when its
// distance to every node already in S_{i+1} exceeds r; a new node's parent is
// its nearest node of S_i (ties: lower index).
//
// Exact pruned evaluation: every atom a keeps the list L(a) of nodes of S_i
// within 3 sigma 2^-i.  Any node of S_{i+1} within r of a, and a's nearest node
// of S_i, have their parent in L(a) (triangle inequality with the covering
// radius), and the nodes of S_{i+1} within 3r of a are children of L(a).  The
// coverage test against old nodes and the refresh of L run in parallel over
// atoms; only the scan against nodes added at the current level is
// sequential.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>
#include <unordered_map>
#include <vector>

#include "covertree.h"

namespace mrf {

namespace {

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn) {
  unsigned nt = std::max(1u, std::thread::hardware_concurrency());
  if (nt > 32) nt = 32;
  if (n < 256 || nt == 1) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  std::atomic<int64_t> next(0);
  const int64_t chunk = std::max<int64_t>(64, n / (nt * 8));
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (;;) {
        const int64_t b = next.fetch_add(chunk);
        if (b >= n) break;
        fn(b, std::min(n, b + chunk));
      }
    });
  for (auto &t : th) t.join();
}

struct Near {
  int32_t node;
  double dist;
};

}  // namespace

double HostTree::dist(const double *X, int64_t K, int32_t a, int32_t b) {
  const double *x = X + (int64_t)a * K, *y = X + (int64_t)b * K;
  double s = 0.0;
  for (int64_t k = 0; k < K; ++k) {
    const double t = x[k] - y[k];
    s += t * t;
  }
  return std::sqrt(s);
}

void build_cover_tree(const double *Xall, int64_t d, int64_t K, HostTree &T) {
  // de-duplicate exactly equal rows (keep the lowest index)
  std::vector<uint64_t> hash((size_t)d);
  parallel_for(d, [&](int64_t b, int64_t e) {
    for (int64_t j = b; j < e; ++j) {
      uint64_t h = 1469598103934665603ull;
      const unsigned char *p = reinterpret_cast<const unsigned char *>(Xall + j * K);
      for (int64_t k = 0; k < K * 8; ++k) {
        h ^= p[k];
        h *= 1099511628211ull;
      }
      hash[(size_t)j] = h;
    }
  });
  std::unordered_map<uint64_t, std::vector<int64_t>> buckets;
  T.uniq_of.assign((size_t)d, -1);
  T.rep.clear();
  for (int64_t j = 0; j < d; ++j) {
    auto &b = buckets[hash[(size_t)j]];
    int64_t found = -1;
    for (int64_t k : b)
      if (std::memcmp(Xall + k * K, Xall + j * K, (size_t)K * 8) == 0) {
        found = k;
        break;
      }
    if (found >= 0) {
      T.uniq_of[(size_t)j] = T.uniq_of[(size_t)found];
    } else {
      b.push_back(j);
      T.uniq_of[(size_t)j] = (int32_t)T.rep.size();
      T.rep.push_back((int32_t)j);
    }
  }
  const int64_t u = (int64_t)T.rep.size();
  std::vector<double> X((size_t)(u * K));
  for (int64_t i = 0; i < u; ++i)
    std::memcpy(&X[(size_t)(i * K)], Xall + (int64_t)T.rep[(size_t)i] * K, (size_t)K * 8);
  // sigma and the initial near lists
  std::vector<std::vector<Near>> L((size_t)u);
  std::vector<double> d0((size_t)u);
  parallel_for(u, [&](int64_t b, int64_t e) {
    for (int64_t a = b; a < e; ++a) d0[(size_t)a] = HostTree::dist(X.data(), K, (int32_t)a, 0);
  });
  double sigma = 0.0;
  for (int64_t a = 0; a < u; ++a) sigma = std::max(sigma, d0[(size_t)a]);
  T.sigma = sigma;
  std::vector<char> inS((size_t)u, 0);
  std::vector<int32_t> ins_level((size_t)u, 0);
  std::vector<int32_t> parent((size_t)u, -1);
  inS[0] = 1;
  for (int64_t a = 1; a < u; ++a) L[(size_t)a].push_back({0, d0[(size_t)a]});
  T.levels.clear();
  T.levels.push_back({0});
  int64_t remaining = u - 1;
  int level = 0;
  while (remaining > 0 && sigma > 0.0) {
    const double r = sigma * std::ldexp(1.0, -(level + 1));
    // (1) coverage by nodes already present (parallel)
    std::vector<char> covered((size_t)u, 0);
    parallel_for(u, [&](int64_t b, int64_t e) {
      for (int64_t a = b; a < e; ++a) {
        if (inS[(size_t)a]) continue;
        for (const Near &nr : L[(size_t)a])
          if (nr.dist <= r) {
            covered[(size_t)a] = 1;
            break;
          }
      }
    });
    // (2) sequential greedy scan against nodes added at this level
    std::unordered_map<int32_t, std::vector<int32_t>> newkids;
    std::vector<int32_t> added;
    for (int64_t a = 0; a < u; ++a) {
      if (inS[(size_t)a] || covered[(size_t)a]) continue;
      bool cov = false;
      for (const Near &nr : L[(size_t)a]) {
        auto it = newkids.find(nr.node);
        if (it == newkids.end()) continue;
        for (int32_t nn : it->second)
          if (HostTree::dist(X.data(), K, (int32_t)a, nn) <= r) {
            cov = true;
            break;
          }
        if (cov) break;
      }
      if (cov) continue;
      // nearest node of S_i (L is in increasing node order: ties to the lower index)
      int32_t best = -1;
      double bd = INFINITY;
      for (const Near &nr : L[(size_t)a])
        if (nr.dist < bd) {
          bd = nr.dist;
          best = nr.node;
        }
      parent[(size_t)a] = best;
      newkids[best].push_back((int32_t)a);
      added.push_back((int32_t)a);
    }
    for (int32_t a : added) {
      inS[(size_t)a] = 1;
      ins_level[(size_t)a] = level + 1;
    }
    remaining -= (int64_t)added.size();
    std::vector<int32_t> lev = T.levels.back();
    lev.insert(lev.end(), added.begin(), added.end());
    std::sort(lev.begin(), lev.end());
    T.levels.push_back(lev);
    // (3) refresh the near lists: children of L(a) within 3r (parallel)
    parallel_for(u, [&](int64_t b, int64_t e) {
      std::vector<Near> nl;
      for (int64_t a = b; a < e; ++a) {
        if (inS[(size_t)a]) {
          std::vector<Near>().swap(L[(size_t)a]);
          continue;
        }
        nl.clear();
        for (const Near &nr : L[(size_t)a]) {
          if (nr.dist <= 3.0 * r) nl.push_back(nr);  // self-child keeps its distance
          auto it = newkids.find(nr.node);
          if (it == newkids.end()) continue;
          for (int32_t nn : it->second) {
            const double dd = HostTree::dist(X.data(), K, (int32_t)a, nn);
            if (dd <= 3.0 * r) nl.push_back({nn, dd});
          }
        }
        std::sort(nl.begin(), nl.end(), [](const Near &x, const Near &y) { return x.node < y.node; });
        L[(size_t)a] = nl;
      }
    });
    ++level;
  }
  if (sigma == 0.0) {
    // every unique atom is the root (u == 1)
  }
  T.imax = (int)T.levels.size() - 1;
  T.parent = parent;
  T.ins_level = ins_level;
  // maxdist per (level, node): max distance to the atoms whose ancestor at that level is the node
  const int nl = T.imax + 1;
  T.maxdist.assign((size_t)nl, std::vector<float>());
  std::vector<std::unordered_map<int32_t, double>> md((size_t)nl);
  std::vector<double> anc_d((size_t)(u * nl), 0.0);
  std::vector<int32_t> anc((size_t)(u * nl), -1);
  parallel_for(u, [&](int64_t b, int64_t e) {
    for (int64_t a = b; a < e; ++a) {
      int32_t q = (int32_t)a;
      for (int i = nl - 1; i >= 0; --i) {
        // ancestor of a at level i: a itself while i >= its insertion level
        if (i < ins_level[(size_t)q]) q = parent[(size_t)q];
        anc[(size_t)(a * nl + i)] = q;
        anc_d[(size_t)(a * nl + i)] = (q == (int32_t)a) ? 0.0 : HostTree::dist(X.data(), K, (int32_t)a, q);
      }
    }
  });
  for (int64_t a = 0; a < u; ++a)
    for (int i = 0; i < nl; ++i) {
      double &m = md[(size_t)i][anc[(size_t)(a * nl + i)]];
      m = std::max(m, anc_d[(size_t)(a * nl + i)]);
    }
  for (int i = 0; i < nl; ++i) {
    T.maxdist[(size_t)i].resize(T.levels[(size_t)i].size());
    for (size_t k = 0; k < T.levels[(size_t)i].size(); ++k)
      T.maxdist[(size_t)i][k] = (float)md[(size_t)i][T.levels[(size_t)i][k]];
  }
}

// Flatten into per-(level, node) entries, level-major; inside level i+1 the
// entries are sorted by (parent, node) so the children of an entry of level i
// are one contiguous range (its own self-child included).
void flatten_cover_tree(const HostTree &T, FlatTree &F) {
  const int nl = T.imax + 1;
  F.level_begin.assign((size_t)nl + 1, 0);
  F.node.clear();
  F.child_begin.clear();
  F.child_end.clear();
  F.maxdist.clear();
  F.is_self.clear();
  std::vector<std::vector<int32_t>> order((size_t)nl);
  order[0] = T.levels[0];
  for (int i = 1; i < nl; ++i) {
    std::vector<int32_t> v = T.levels[(size_t)i];
    auto par = [&](int32_t q) { return (i - 1 >= T.ins_level[(size_t)q]) ? q : T.parent[(size_t)q]; };
    std::stable_sort(v.begin(), v.end(), [&](int32_t a, int32_t b) {
      const int32_t pa = par(a), pb = par(b);
      return pa != pb ? pa < pb : a < b;
    });
    order[(size_t)i] = v;
  }
  int64_t total = 0;
  for (int i = 0; i < nl; ++i) {
    F.level_begin[(size_t)i] = total;
    total += (int64_t)order[(size_t)i].size();
  }
  F.level_begin[(size_t)nl] = total;
  F.node.resize((size_t)total);
  F.child_begin.assign((size_t)total, 0);
  F.child_end.assign((size_t)total, 0);
  F.maxdist.resize((size_t)total);
  F.is_self.assign((size_t)total, 0);
  for (int i = 0; i < nl; ++i) {
    // maxdist lookup by node for this level
    std::unordered_map<int32_t, float> mdl;
    for (size_t k = 0; k < T.levels[(size_t)i].size(); ++k) mdl[T.levels[(size_t)i][k]] = T.maxdist[(size_t)i][k];
    for (size_t k = 0; k < order[(size_t)i].size(); ++k) {
      const int64_t e = F.level_begin[(size_t)i] + (int64_t)k;
      const int32_t q = order[(size_t)i][k];
      F.node[(size_t)e] = q;
      F.maxdist[(size_t)e] = mdl[q];
      if (i > 0) F.is_self[(size_t)e] = (i - 1 >= T.ins_level[(size_t)q]) ? 1 : 0;
    }
  }
  for (int i = 0; i + 1 < nl; ++i) {
    std::unordered_map<int32_t, int64_t> entry_of;  // node -> entry at level i
    for (int64_t e = F.level_begin[(size_t)i]; e < F.level_begin[(size_t)i + 1]; ++e) entry_of[F.node[(size_t)e]] = e;
    for (int64_t e = F.level_begin[(size_t)i + 1]; e < F.level_begin[(size_t)i + 2]; ++e) {
      const int32_t q = F.node[(size_t)e];
      const int32_t p = (i >= T.ins_level[(size_t)q]) ? q : T.parent[(size_t)q];
      const int64_t pe = entry_of[p];
      if (F.child_end[(size_t)pe] == 0) F.child_begin[(size_t)pe] = e;
      F.child_end[(size_t)pe] = e + 1;
    }
  }
}

}  // namespace mrf
