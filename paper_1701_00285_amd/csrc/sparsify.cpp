// Sparsity pattern of the multilevel covariance matrix (Sec. 4.1: the tree
// search SearchTree / LocalSearchTree with the left and right rules, and
// the construction of the sparse blocks C~^{i,j}_W).
//
// For a cell B_a at level i and a target depth j >= i, the search walks the
// kd-tree from the root: a node at depth j is reported, a leaf above depth j
// ends the walk, and a split (axis k, threshold s) is entered on its left
// side when min_{x in B_a} x_k - tau <= s and on its right side when
// max_{x in B_a} x_k + tau > s, i.e. when B_a's bounding box widened by tau
// reaches that side.  The block of wavelets of B_a against those of a
// reported cell B_b is kept.  Blocks with i <= j come from the search at
// the coarser cell and are mirrored; for two cells of one level the block
// is kept when either search reaches the other.  Every other block of
// C~^n_W is zero.  tau = inf keeps every block (the exact C^n_W).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "internal.h"

namespace mlb {

static int32_t wavelets(const Basis& B, int32_t v) { return B.desc[v].m - B.desc[v].a; }

int32_t pattern_cells(const Basis& B, int32_t level) {
  int32_t nc = 0;
  for (int32_t v = 0; v < (int32_t)B.desc.size(); ++v)
    if (B.depth[v] >= level && wavelets(B, v) > 0) ++nc;
  return nc;
}

void build_pattern(const Basis& B, int32_t level, double tau, Pattern& P) {
  const int32_t nn = (int32_t)B.desc.size();
  const int d = B.d;
  // cells in the row order of C^n_W: their wavelet rows start at w_off
  std::vector<int32_t> cell_of(nn, -1), cells;
  for (int32_t v = 0; v < nn; ++v)
    if (B.depth[v] >= level && wavelets(B, v) > 0) cells.push_back(v);
  std::sort(cells.begin(), cells.end(), [&](int32_t x, int32_t y) { return B.desc[x].w_off < B.desc[y].w_off; });
  const int32_t nc = (int32_t)cells.size();
  for (int32_t c = 0; c < nc; ++c) cell_of[cells[c]] = c;
  int64_t nt = 0;
  for (int32_t c = 0; c < nc; ++c) nt += wavelets(B, cells[c]);
  P.nc = nc;
  P.rowcell.assign((size_t)nt, 0);
  for (int32_t c = 0; c < nc; ++c) {
    const int64_t o = B.desc[cells[c]].w_off;
    std::fill(P.rowcell.begin() + o, P.rowcell.begin() + o + wavelets(B, cells[c]), c);
  }
  P.keep.assign((size_t)nc * nc, 0);
  if (std::isinf(tau)) {
    std::fill(P.keep.begin(), P.keep.end(), 1);
    P.nnz = nt * nt;
    return;
  }
  // bounding boxes, children before parents (preorder numbers parents first)
  std::vector<double> lo((size_t)nn * d), hi((size_t)nn * d);
  for (int32_t v = nn - 1; v >= 0; --v) {
    double* l = &lo[(size_t)v * d];
    double* h = &hi[(size_t)v * d];
    if (B.left[v] < 0) {
      std::fill(l, l + d, INFINITY);
      std::fill(h, h + d, -INFINITY);
      for (int64_t i = B.begin[v]; i < B.end[v]; ++i)
        for (int k = 0; k < d; ++k) {
          const double x = B.pts_tree[(size_t)i * d + k];
          l[k] = std::min(l[k], x);
          h[k] = std::max(h[k], x);
        }
    } else {
      const double* la = &lo[(size_t)B.left[v] * d];
      const double* lb = &lo[(size_t)B.right[v] * d];
      const double* ha = &hi[(size_t)B.left[v] * d];
      const double* hb = &hi[(size_t)B.right[v] * d];
      for (int k = 0; k < d; ++k) {
        l[k] = std::min(la[k], lb[k]);
        h[k] = std::max(ha[k], hb[k]);
      }
    }
  }
  std::vector<int32_t> stack;
  for (int32_t c = 0; c < nc; ++c) {
    const int32_t a = cells[c];
    const double* l = &lo[(size_t)a * d];
    const double* h = &hi[(size_t)a * d];
    for (int32_t j = B.depth[a]; j < B.levels; ++j) {
      stack.assign(1, 0);
      while (!stack.empty()) {
        const int32_t v = stack.back();
        stack.pop_back();
        if (B.depth[v] == j) {
          const int32_t cb = cell_of[v];
          if (cb >= 0) P.keep[(size_t)c * nc + cb] = P.keep[(size_t)cb * nc + c] = 1;
          continue;
        }
        if (B.left[v] < 0) continue;
        const int k = B.axis[v];
        const double s = B.threshold[v];
        if (h[k] + tau > s) stack.push_back(B.right[v]);
        if (l[k] - tau <= s) stack.push_back(B.left[v]);
      }
    }
  }
  int64_t nnz = 0;
  for (int32_t x = 0; x < nc; ++x)
    for (int32_t y = 0; y < nc; ++y)
      if (P.keep[(size_t)x * nc + y]) nnz += (int64_t)wavelets(B, cells[x]) * wavelets(B, cells[y]);
  P.nnz = nnz;
}

}  // namespace mlb
