// Cluster tree, block partition and per-level colouring (host side).
//
// Tree (Sec. II): every cluster is bisected at the midpoint of the longest
// side of its points' bounding box (first axis on ties, "coord < mid" goes
// left, input order kept) until all clusters of the deepest level hold at
// most `leaf` points; the depth is uniform.  Admissibility is eq. 1 on
// cell-support boxes (centres +- h/2): max(diam_t, diam_s) <= eta * dist(t, s)
// with a relative tie tolerance of 1e-10, tested level by level on the
// children of inadmissible pairs (a lockstep traversal from (root, root)).
// Clusters of a level are coloured greedily on the graph of inadmissible
// pairs so that one colour holds mutually admissible clusters only.
#pragma once

#include <cstdint>
#include <utility>
#include <vector>

namespace h2 {

using Pair = std::pair<int32_t, int32_t>;

struct Structure {
  int64_t N = 0;
  int L = 0;
  int l0 = -1;                                   // coarsest level with an admissible pair
  std::vector<int64_t> perm;                     // tree order -> caller's index
  std::vector<std::vector<int64_t>> start;       // [level][cluster] offset in tree order
  std::vector<std::vector<int64_t>> size;        // [level][cluster] point count
  std::vector<std::vector<Pair>> near;           // [level] inadmissible pairs, sorted, incl. (t,t)
  std::vector<std::vector<Pair>> adm;            // [level] admissible pairs, sorted
  std::vector<std::vector<int32_t>> colour;      // [level][cluster], -1 for empty clusters
  std::vector<int> ncolours;                     // [level]
  int nclusters(int l) const { return (int)start[l].size(); }
};

// Returns false (with msg) when the points cannot be split (duplicates).
bool build_structure(const double* pts, int64_t n, double h, int leaf, double eta, Structure& S,
                     std::vector<char>& msg);

}  // namespace h2
