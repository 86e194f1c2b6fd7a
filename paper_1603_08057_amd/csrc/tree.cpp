// Quadtree over the observation sites (Section 2.1 of the paper; adaptive as
// in the remark on the tree).  Host code: the tree is pure geometry, built once
// per point set and shared by every factorization and sweep on it.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "rsf.h"

namespace rsf {

// Checks one instance's sites: finite, unique (the nugget is a delta on
// observation indices).  Returns its bounding box.
static void check_sites(const double* xy, int64_t n, int inst, double bb[4]) {
  const std::string who = inst >= 0 ? " of instance " + std::to_string(inst) : std::string();
  double xmin = xy[0], xmax = xy[0], ymin = xy[1], ymax = xy[1];
  for (int64_t i = 0; i < n; ++i) {
    const double x = xy[2 * i], y = xy[2 * i + 1];
    RSF_CHECK(std::isfinite(x) && std::isfinite(y), RSF_E_NONFINITE,
              "non-finite coordinate at point " + std::to_string(i) + who);
    xmin = std::min(xmin, x);
    xmax = std::max(xmax, x);
    ymin = std::min(ymin, y);
    ymax = std::max(ymax, y);
  }
  std::vector<int64_t> o(n);
  std::iota(o.begin(), o.end(), 0);
  std::sort(o.begin(), o.end(), [&](int64_t a, int64_t b) {
    return xy[2 * a] < xy[2 * b] || (xy[2 * a] == xy[2 * b] && xy[2 * a + 1] < xy[2 * b + 1]);
  });
  for (int64_t i = 1; i < n; ++i)
    RSF_CHECK(!(xy[2 * o[i]] == xy[2 * o[i - 1]] && xy[2 * o[i] + 1] == xy[2 * o[i - 1] + 1]), RSF_E_DUPLICATE,
              "duplicate observation site (points " + std::to_string(o[i - 1]) + " and " + std::to_string(o[i]) +
                  ")" + who);
  bb[0] = xmin;
  bb[1] = xmax;
  bb[2] = ymin;
  bb[3] = ymax;
}

Tree build_tree(const double* xy, int64_t n, int leaf) {
  return build_forest(std::vector<const double*>{xy}, std::vector<int64_t>{n}, leaf);
}

// Independent instances share one breadth-first numbering: the depth-0 boxes
// are the instances' root squares, and every depth holds the boxes of all
// instances (instance by instance), so each level is processed by one set of
// launches.  Instance i occupies the tree-order range [ioff[i], ioff[i + 1])
// and its caller indices are ioff[i] + local index.
Tree build_forest(const std::vector<const double*>& xys, const std::vector<int64_t>& ns, int leaf) {
  const int ni = (int)xys.size();
  RSF_CHECK(ni >= 1 && ns.size() == xys.size(), RSF_E_INVALID, "no instances");
  RSF_CHECK(leaf >= 1, RSF_E_INVALID, "leaf must be >= 1");
  Tree t;
  t.ninst = ni;
  t.ioff.assign(ni + 1, 0);
  for (int i = 0; i < ni; ++i) {
    RSF_CHECK(ns[i] >= 1, RSF_E_INVALID, "n must be >= 1" + (ni > 1 ? " (instance " + std::to_string(i) + ")" : std::string()));
    t.ioff[i + 1] = t.ioff[i] + ns[i];
  }
  const int64_t n = t.ioff[ni];
  RSF_CHECK(n < (int64_t(1) << 31), RSF_E_INVALID, "n must fit in 31 bits");
  t.n = n;
  t.perm.assign(n, 0);
  std::vector<std::pair<int, std::vector<int>>> frontier;
  for (int i = 0; i < ni; ++i) {
    double bb[4];
    check_sites(xys[i], ns[i], ni > 1 ? i : -1, bb);
    double h = std::max(bb[1] - bb[0], bb[3] - bb[2]) / 2.0;
    if (!(h > 0.0)) h = 0.5;
    t.cx.push_back((bb[0] + bb[1]) / 2.0);
    t.cy.push_back((bb[2] + bb[3]) / 2.0);
    t.half.push_back(h);
    t.depth.push_back(0);
    t.parent.push_back(-1);
    t.quad.push_back(-1);
    t.begin.push_back((int)t.ioff[i]);
    t.count.push_back((int)ns[i]);
    t.child.push_back({-1, -1, -1, -1});
    t.inst.push_back(i);
    std::vector<int> all(ns[i]);
    std::iota(all.begin(), all.end(), 0);
    frontier.emplace_back(i, std::move(all));
  }
  const int max_depth = 40;
  while (!frontier.empty()) {
    std::vector<std::pair<int, std::vector<int>>> next;
    for (auto& fb : frontier) {
      const int b = fb.first, in = t.inst[b];
      const double* xy = xys[in];
      std::vector<int>& idx = fb.second;
      if ((int)idx.size() > leaf && t.depth[b] < max_depth) {
        std::vector<int> q[4];
        const double cx = t.cx[b], cy = t.cy[b];
        for (int i : idx) {
          const bool east = xy[2 * (int64_t)i] >= cx, north = xy[2 * (int64_t)i + 1] >= cy;
          q[north ? (east ? 1 : 0) : (east ? 3 : 2)].push_back(i);
        }
        int off = t.begin[b];
        const double hh = t.half[b] / 2.0;
        for (int c = 0; c < 4; ++c) {
          if (q[c].empty()) continue;
          const int id = (int)t.cx.size();
          t.cx.push_back((c == 1 || c == 3) ? cx + hh : cx - hh);
          t.cy.push_back((c == 0 || c == 1) ? cy + hh : cy - hh);
          t.half.push_back(hh);
          t.depth.push_back(t.depth[b] + 1);
          t.parent.push_back(b);
          t.quad.push_back(c);
          t.begin.push_back(off);
          t.count.push_back((int)q[c].size());
          t.child.push_back({-1, -1, -1, -1});
          t.inst.push_back(in);
          t.child[b][c] = id;
          off += (int)q[c].size();
          next.emplace_back(id, std::move(q[c]));
        }
      } else {
        for (size_t u = 0; u < idx.size(); ++u) t.perm[t.begin[b] + u] = (int)(t.ioff[in] + idx[u]);
      }
    }
    frontier.swap(next);
  }
  const int nb = t.nbox();
  t.leaf.assign(nb, 0);
  for (int b = 0; b < nb; ++b)
    t.leaf[b] = (t.child[b][0] < 0 && t.child[b][1] < 0 && t.child[b][2] < 0 && t.child[b][3] < 0);
  t.maxdepth = *std::max_element(t.depth.begin(), t.depth.end());
  t.lev.assign(t.maxdepth + 2, 0);
  for (int b = 0; b < nb; ++b) t.lev[t.depth[b] + 1] = b + 1;  // ids are sorted by depth
  for (int d = 1; d <= t.maxdepth + 1; ++d) t.lev[d] = std::max(t.lev[d], t.lev[d - 1]);
  return t;
}

}  // namespace rsf
