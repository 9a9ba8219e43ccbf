// kd-tree domain decomposition (Sec. 3.1: cell-split rule, InitialTree,
// MakeTree).  Each cell is split on the coordinate axis along which its own
// points have the largest variance, at the median of that coordinate.  The
// median split is taken by rank: points ordered by (coordinate, input
// index), the first ceil(m/2) form the left cell, the threshold is the
// largest left coordinate.  A cell with at most leaf_max points is a leaf;
// its points are listed by input index.  Nodes are numbered in preorder.
#include <algorithm>
#include <cmath>
#include <future>
#include <memory>

#include "internal.h"

namespace mlb {
namespace {

struct Cell {
  int64_t b, e;
  int32_t axis = -1;
  double thr = 0.0;
  std::unique_ptr<Cell> l, r;
};

struct Splitter {
  const double* P;
  int32_t d;
  int32_t leaf_max;
  int64_t* idx;

  int32_t max_var_axis(int64_t b, int64_t e) const {
    const double m = double(e - b);
    int32_t best = 0;
    double best_var = -1.0;
    for (int32_t k = 0; k < d; ++k) {
      double s = 0.0;
      for (int64_t i = b; i < e; ++i) s += P[idx[i] * d + k];
      const double mean = s / m;
      double v = 0.0;
      for (int64_t i = b; i < e; ++i) {
        const double t = P[idx[i] * d + k] - mean;
        v += t * t;
      }
      v /= m;
      if (v > best_var) {  // strict: the lowest axis wins ties
        best_var = v;
        best = k;
      }
    }
    return best;
  }

  std::unique_ptr<Cell> make(int64_t b, int64_t e, int depth) {
    auto c = std::make_unique<Cell>();
    c->b = b;
    c->e = e;
    if (e - b <= leaf_max) {
      std::sort(idx + b, idx + e);
      return c;
    }
    const int32_t ax = max_var_axis(b, e);
    const int64_t nl = (e - b + 1) / 2;
    const double* P_ = P;
    const int32_t d_ = d;
    auto less = [P_, d_, ax](int64_t u, int64_t v) {
      const double cu = P_[u * d_ + ax], cv = P_[v * d_ + ax];
      return cu < cv || (cu == cv && u < v);
    };
    std::nth_element(idx + b, idx + b + nl - 1, idx + e, less);
    // nth_element leaves [b, b+nl-1) <= element b+nl-1 <= [b+nl, e)
    c->axis = ax;
    c->thr = P[idx[b + nl - 1] * d + ax];
    for (int64_t i = b; i < b + nl; ++i) c->thr = std::max(c->thr, P[idx[i] * d + ax]);
    if (depth < 4 && (e - b) > 8192) {
      auto fl = std::async(std::launch::async, [this, b, nl, depth] { return make(b, b + nl, depth + 1); });
      c->r = make(b + nl, e, depth + 1);
      c->l = fl.get();
    } else {
      c->l = make(b, b + nl, depth + 1);
      c->r = make(b + nl, e, depth + 1);
    }
    return c;
  }
};

int32_t flatten(const Cell* c, int32_t depth, int32_t parent, Tree& t) {
  const int32_t v = (int32_t)t.begin.size();
  t.begin.push_back(c->b);
  t.end.push_back(c->e);
  t.depth.push_back(depth);
  t.axis.push_back(c->axis);
  t.threshold.push_back(c->l ? c->thr : 0.0);
  t.left.push_back(-1);
  t.right.push_back(-1);
  t.parent.push_back(parent);
  t.max_depth = std::max(t.max_depth, depth);
  if (c->l) {
    const int32_t l = flatten(c->l.get(), depth + 1, v, t);
    const int32_t r = flatten(c->r.get(), depth + 1, v, t);
    t.left[v] = l;
    t.right[v] = r;
  }
  return v;
}

}  // namespace

int build_tree(const double* pts, int64_t n, int32_t d, int32_t leaf_max, Tree& t) {
  if (!pts || n < 1 || d < 1 || d > 64 || leaf_max < 1)
    return fail(MLBLUP_EINVAL, "build_tree: need pts != NULL, n >= 1, 1 <= d <= 64, leaf_max >= 1");
  for (int64_t i = 0; i < n * d; ++i)
    if (!std::isfinite(pts[i])) return fail(MLBLUP_EINVAL, "build_tree: non-finite coordinate");
  t = Tree();
  t.n = n;
  t.d = d;
  t.leaf_max = leaf_max;
  t.pts.assign(pts, pts + n * d);
  t.perm.resize(n);
  for (int64_t i = 0; i < n; ++i) t.perm[i] = i;
  Splitter s{t.pts.data(), d, leaf_max, t.perm.data()};
  std::unique_ptr<Cell> root = s.make(0, n, 0);
  flatten(root.get(), 0, -1, t);
  return MLBLUP_OK;
}

}  // namespace mlb
