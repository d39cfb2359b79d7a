// remesh.cpp -- host side of mesh adaptation: where every cell of a new
// tree takes its state from in the old tree (Sec. 8).
#include "remesh.h"

#include <algorithm>

#include "grid_builder.h"

namespace lbm {

namespace {

// coordinates of one level packed into a sortable key (21 bits per axis)
inline uint64_t pack(int64_t x, int64_t y, int64_t z) {
  return (uint64_t)x | ((uint64_t)y << 21) | ((uint64_t)z << 42);
}

struct FlowIndex {
  std::vector<std::vector<std::pair<uint64_t, int32_t>>> lev;  // sorted per level
  int32_t find(int l, int64_t x, int64_t y, int64_t z) const {
    if (l < 0 || l >= (int)lev.size()) return -1;
    const auto &v = lev[l];
    const uint64_t k = pack(x, y, z);
    auto it = std::lower_bound(v.begin(), v.end(), std::make_pair(k, (int32_t)-1));
    return (it != v.end() && it->first == k) ? it->second : -1;
  }
};

// volume shares of the old flow cells inside cell (l, x, y, z), depth first,
// children in x-major order
void inside(const FlowIndex &fi, int D, int deepest, int l, int64_t x, int64_t y, int64_t z, double share,
            std::vector<std::pair<int32_t, double>> *acc) {
  if (l >= deepest) return;
  const double w = share / (double)(1 << D);
  for (int ox = 0; ox < 2; ++ox)
    for (int oy = 0; oy < (D > 1 ? 2 : 1); ++oy)
      for (int oz = 0; oz < (D > 2 ? 2 : 1); ++oz) {
        const int64_t cx = 2 * x + ox, cy = 2 * y + oy, cz = D > 2 ? 2 * z + oz : 0;
        const int32_t c = fi.find(l + 1, cx, cy, cz);
        if (c >= 0) acc->push_back({c, w});
        else inside(fi, D, deepest, l + 1, cx, cy, cz, w, acc);
      }
}

bool sources_of(const FlowIndex &fi, int D, int deepest, int l, int64_t x, int64_t y, int64_t z,
                std::vector<std::pair<int32_t, double>> *acc) {
  acc->clear();
  for (int up = l; up >= 0; --up) {
    const int s = l - up;
    const int32_t c = fi.find(up, x >> s, y >> s, z >> s);
    if (c >= 0) {
      acc->push_back({c, 1.0});
      return true;
    }
  }
  inside(fi, D, deepest, l, x, y, z, 1.0, acc);
  double tot = 0.0;
  for (auto &p : *acc) tot += p.second;
  if (acc->empty() || !(tot > 0.0)) return false;
  for (auto &p : *acc) p.second /= tot;
  return true;
}

}  // namespace

int remesh_sources(const HostGrid &old, const HostGrid &nw, std::vector<int64_t> *off, std::vector<int32_t> *src,
                   std::vector<double> *wt, std::string *err) {
  FlowIndex fi;
  fi.lev.resize(old.L);
  int deepest = 0;
  for (int64_t c = 0; c < old.n; ++c) {
    if (old.flag[c] & F_FINE_GHOST) continue;
    const int l = old.lev[c];
    fi.lev[l].push_back({pack(old.xyz[3 * c], old.xyz[3 * c + 1], old.xyz[3 * c + 2]), (int32_t)c});
    deepest = std::max(deepest, l);
  }
#pragma omp parallel for schedule(static)
  for (int l = 0; l < old.L; ++l) std::sort(fi.lev[l].begin(), fi.lev[l].end());
  const int64_t n = nw.n;
  const int D = nw.D;
  off->assign(n + 1, 0);
  int bad = 0;
  int64_t bad_cell = -1;
#pragma omp parallel
  {
    std::vector<std::pair<int32_t, double>> acc;
#pragma omp for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
      if (!sources_of(fi, D, deepest, nw.lev[j], nw.xyz[3 * j], nw.xyz[3 * j + 1], nw.xyz[3 * j + 2], &acc)) {
#pragma omp critical
        {
          bad = 1;
          bad_cell = j;
        }
        continue;
      }
      (*off)[j + 1] = (int64_t)acc.size();
    }
  }
  if (bad) {
    *err = "remesh: new cell " + std::to_string(bad_cell) + " covers no flow cell of the old grid";
    return -1;
  }
  for (int64_t j = 0; j < n; ++j) (*off)[j + 1] += (*off)[j];
  src->resize((*off)[n]);
  wt->resize((*off)[n]);
#pragma omp parallel
  {
    std::vector<std::pair<int32_t, double>> acc;
#pragma omp for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
      sources_of(fi, D, deepest, nw.lev[j], nw.xyz[3 * j], nw.xyz[3 * j + 1], nw.xyz[3 * j + 2], &acc);
      int64_t k = (*off)[j];
      for (auto &p : acc) {
        (*src)[k] = p.first;
        (*wt)[k] = p.second;
        ++k;
      }
    }
  }
  return 0;
}

}  // namespace lbm
