// Cluster tree, lockstep block partition and greedy colouring (host side).
#include "h2_structure.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace h2 {

namespace {

struct Box {
  double lo[3], hi[3];
  bool empty = true;
};

double diam(const Box& b) {
  double s = 0.0;
  for (int d = 0; d < 3; ++d) s += (b.hi[d] - b.lo[d]) * (b.hi[d] - b.lo[d]);
  return std::sqrt(s);
}

double dist(const Box& a, const Box& b) {
  double s = 0.0;
  for (int d = 0; d < 3; ++d) {
    double g = std::max(0.0, std::max(b.lo[d] - a.hi[d], a.lo[d] - b.hi[d]));
    s += g * g;
  }
  return std::sqrt(s);
}

}  // namespace

bool build_structure(const double* pts, int64_t n, double h, int leaf, double eta, Structure& S,
                     std::vector<char>& msg) {
  S = Structure();
  S.N = n;
  // levels of index lists (caller numbering)
  std::vector<std::vector<std::vector<int64_t>>> lev(1);
  lev[0].emplace_back(n);
  for (int64_t i = 0; i < n; ++i) lev[0][0][i] = i;
  for (;;) {
    bool need = false;
    for (auto& c : lev.back())
      if ((int64_t)c.size() > leaf) need = true;
    if (!need) break;
    std::vector<std::vector<int64_t>> next;
    next.reserve(lev.back().size() * 2);
    for (auto& c : lev.back()) {
      std::vector<int64_t> left, right;
      if (!c.empty()) {
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) lo[d] = hi[d] = pts[3 * c[0] + d];
        for (int64_t i : c)
          for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], pts[3 * i + d]);
            hi[d] = std::max(hi[d], pts[3 * i + d]);
          }
        int axis = 0;
        double best = hi[0] - lo[0];
        for (int d = 1; d < 3; ++d)
          if (hi[d] - lo[d] > best) {
            best = hi[d] - lo[d];
            axis = d;
          }
        double mid = 0.5 * (lo[axis] + hi[axis]);
        for (int64_t i : c) (pts[3 * i + axis] < mid ? left : right).push_back(i);
        if ((int64_t)c.size() > leaf && left.empty()) {
          const char* m = "points cannot be bisected (duplicate points)";
          msg.assign(m, m + std::strlen(m) + 1);
          return false;
        }
      }
      next.push_back(std::move(left));
      next.push_back(std::move(right));
    }
    lev.push_back(std::move(next));
    if (lev.size() > 62) {
      const char* m = "cluster tree deeper than 62 levels";
      msg.assign(m, m + std::strlen(m) + 1);
      return false;
    }
  }
  S.L = (int)lev.size() - 1;
  const int L = S.L;
  S.perm.clear();
  S.perm.reserve(n);
  for (auto& c : lev[L]) S.perm.insert(S.perm.end(), c.begin(), c.end());
  S.start.resize(L + 1);
  S.size.resize(L + 1);
  for (int l = 0; l <= L; ++l) {
    size_t nc = lev[l].size();
    S.start[l].resize(nc);
    S.size[l].resize(nc);
    int64_t o = 0;
    for (size_t t = 0; t < nc; ++t) {
      S.start[l][t] = o;
      S.size[l][t] = (int64_t)lev[l][t].size();
      o += S.size[l][t];
    }
  }
  // cell-support boxes
  std::vector<std::vector<Box>> box(L + 1);
  for (int l = 0; l <= L; ++l) {
    box[l].resize(lev[l].size());
    for (size_t t = 0; t < lev[l].size(); ++t) {
      auto& c = lev[l][t];
      if (c.empty()) continue;
      Box& b = box[l][t];
      b.empty = false;
      for (int d = 0; d < 3; ++d) b.lo[d] = b.hi[d] = pts[3 * c[0] + d];
      for (int64_t i : c)
        for (int d = 0; d < 3; ++d) {
          b.lo[d] = std::min(b.lo[d], pts[3 * i + d]);
          b.hi[d] = std::max(b.hi[d], pts[3 * i + d]);
        }
      for (int d = 0; d < 3; ++d) {
        b.lo[d] = b.lo[d] - 0.5 * h;
        b.hi[d] = b.hi[d] + 0.5 * h;
      }
    }
  }
  S.near.assign(L + 1, {});
  S.adm.assign(L + 1, {});
  S.near[0].push_back({0, 0});
  for (int l = 1; l <= L; ++l) {
    for (const Pair& p : S.near[l - 1]) {
      for (int tc = 2 * p.first; tc <= 2 * p.first + 1; ++tc) {
        if (box[l][tc].empty) continue;
        for (int sc = 2 * p.second; sc <= 2 * p.second + 1; ++sc) {
          if (box[l][sc].empty) continue;
          const Box &bt = box[l][tc], &bs = box[l][sc];
          double dm = std::max(diam(bt), diam(bs));
          if (dm <= eta * dist(bt, bs) * (1.0 + 1e-10))
            S.adm[l].push_back({tc, sc});
          else
            S.near[l].push_back({tc, sc});
        }
      }
    }
    std::sort(S.near[l].begin(), S.near[l].end());
    std::sort(S.adm[l].begin(), S.adm[l].end());
  }
  S.l0 = -1;
  for (int l = 0; l <= L; ++l)
    if (!S.adm[l].empty()) {
      S.l0 = l;
      break;
    }
  // greedy colouring per level
  S.colour.resize(L + 1);
  S.ncolours.assign(L + 1, 0);
  for (int l = 0; l <= L; ++l) {
    int nc = (int)lev[l].size();
    std::vector<std::vector<int32_t>> nb(nc);
    for (const Pair& p : S.near[l])
      if (p.first != p.second) nb[p.first].push_back(p.second);
    std::vector<int32_t>& col = S.colour[l];
    col.assign(nc, -1);
    std::vector<char> used;
    for (int t = 0; t < nc; ++t) {
      if (lev[l][t].empty()) continue;
      used.assign(nb[t].size() + 2, 0);
      for (int32_t s : nb[t])
        if (col[s] >= 0 && col[s] < (int32_t)used.size()) used[col[s]] = 1;
      int c = 0;
      while (used[c]) ++c;
      col[t] = c;
      S.ncolours[l] = std::max(S.ncolours[l], c + 1);
    }
  }
  return true;
}

}  // namespace h2
