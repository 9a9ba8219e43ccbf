// Host analysis for the sparse factorization of the sparsified multilevel
// covariance matrix C~^n_W (Sec. 4.1, the blocks the tree search keeps;
// Sec. 6.1, the Cholesky factor that gives the log-determinant and the
// quadratic form of the reduced likelihood).
//
// The matrix is block-sparse with one block row and column per cell that
// owns wavelets at levels >= n (Pattern).  The factorization works on those
// blocks:
//  1. Fill-reducing order: minimum degree on the cell graph (cells joined
//     when their block is kept), the degree of a cell being the number of
//     rows of its not yet eliminated neighbours; eliminating a cell joins its
//     neighbours pairwise, and those neighbours are the block pattern of its
//     factor column.
//  2. Block structure of the factor L: column k holds its diagonal block and
//     one block per later neighbour; the row structure (for each column j,
//     the earlier columns k whose pattern contains j) drives the
//     left-looking updates, L_ij = A_ij - sum_k L_ik L_jk^T over the k in
//     both row structures.
//  3. Dense tail: the last columns of the order (the separators the
//     minimum-degree order leaves to the end) are nearly full; from the
//     position where that pays (by the estimated time of the block kernels
//     against the dense blocked Cholesky) they form one dense matrix, which
//     the block columns before it update and the dense factorization then
//     finishes.
//  4. Schedule of the block columns before the tail: the elimination tree
//     (parent = first column of the pattern) by height; the columns of one
//     height depend on lower heights only.
//  5. The wavelet vectors of every cell on the points of its subtree,
//     bottom-up from the basis' orthogonal blocks (a leaf's candidates are
//     its points' unit vectors, an internal cell's the scaling vectors of
//     its two children, left first), so that a kept block is
//     Psi_a^T C(S_a, S_b) Psi_b.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "internal.h"

namespace mlb {

namespace {

int32_t wavelets_of(const Basis& B, int32_t v) { return B.desc[v].m - B.desc[v].a; }

}  // namespace

int sparse_analyse(const Basis& B, int32_t level, double tau, SparseSymbolic& S, int32_t dense_tail,
                   int64_t max_tail) {
  S = SparseSymbolic();
  S.level = level;
  S.tau = tau;
  Pattern P;
  build_pattern(B, level, tau, P);
  S.kept_entries = P.nnz;
  const int32_t nc = P.nc;
  S.nc = nc;
  // cells in row order (the pattern's numbering), their node ids and sizes
  std::vector<int32_t> cells;
  for (int32_t v = 0; v < (int32_t)B.desc.size(); ++v)
    if (B.depth[v] >= level && wavelets_of(B, v) > 0) cells.push_back(v);
  std::sort(cells.begin(), cells.end(), [&](int32_t x, int32_t y) { return B.desc[x].w_off < B.desc[y].w_off; });
  if ((int32_t)cells.size() != nc) return fail(MLBLUP_EINVAL, "sparse loglik: cell count does not match the pattern");
  std::vector<int32_t> wc(nc);
  S.rows = 0;
  for (int32_t c = 0; c < nc; ++c) {
    wc[c] = wavelets_of(B, cells[c]);
    if (wc[c] > kSparseMaxBlock)
      return fail(MLBLUP_EINVAL, "sparse loglik: a cell has " + std::to_string(wc[c]) + " wavelets (at most " +
                                     std::to_string(kSparseMaxBlock) + ": leaf size and trend dimension up to 64)");
    S.rows += wc[c];
  }
  if (nc == 0) {
    S.tail = 0;
    return MLBLUP_OK;
  }

  // 1. minimum degree on the cell graph, with the fill
  const int words = (nc + 63) / 64;
  std::vector<uint64_t> adj((size_t)nc * words, 0);
  for (int32_t x = 0; x < nc; ++x)
    for (int32_t y = 0; y < nc; ++y)
      if (x != y && P.keep[(size_t)x * nc + y]) adj[(size_t)x * words + y / 64] |= 1ull << (y % 64);
  std::vector<int64_t> deg(nc, 0);
  auto degree = [&](int32_t u) {
    int64_t s = 0;
    const uint64_t* a = &adj[(size_t)u * words];
    for (int q = 0; q < words; ++q)
      for (uint64_t m = a[q]; m; m &= m - 1) s += wc[q * 64 + __builtin_ctzll(m)];
    return s;
  };
  for (int32_t u = 0; u < nc; ++u) deg[u] = degree(u);
  std::vector<uint8_t> done(nc, 0);
  std::vector<int32_t> order(nc), pos(nc);
  std::vector<std::vector<int32_t>> patc(nc);   // per elimination step: neighbours (cells)
  std::vector<uint64_t> nb(words);
  for (int32_t step = 0; step < nc; ++step) {
    int32_t k = -1;
    for (int32_t u = 0; u < nc; ++u)
      if (!done[u] && (k < 0 || deg[u] < deg[k])) k = u;
    order[step] = k;
    pos[k] = step;
    done[k] = 1;
    std::copy(&adj[(size_t)k * words], &adj[(size_t)k * words] + words, nb.begin());
    std::vector<int32_t>& pk = patc[step];
    for (int q = 0; q < words; ++q)
      for (uint64_t m = nb[q]; m; m &= m - 1) pk.push_back(q * 64 + __builtin_ctzll(m));
    for (int32_t u : pk) {
      uint64_t* a = &adj[(size_t)u * words];
      for (int q = 0; q < words; ++q) a[q] |= nb[q];
      a[u / 64] &= ~(1ull << (u % 64));
      a[k / 64] &= ~(1ull << (k % 64));
    }
    for (int32_t u : pk) deg[u] = degree(u);
  }

  // 2. block structure in elimination positions
  S.order = order;
  S.w.resize(nc);
  S.row0.resize(nc);
  S.ypos.resize(nc);
  for (int32_t k = 0; k < nc; ++k) {
    S.w[k] = wc[order[k]];
    S.row0[k] = B.desc[cells[order[k]]].w_off;
    S.node.push_back(cells[order[k]]);
  }
  int64_t yp = 0;
  for (int32_t k = 0; k < nc; ++k) {
    S.ypos[k] = yp;
    yp += S.w[k];
  }
  S.col_ptr.assign(nc + 1, 0);
  for (int32_t k = 0; k < nc; ++k) S.col_ptr[k + 1] = S.col_ptr[k] + 1 + (int64_t)patc[k].size();
  const int64_t nblk = S.col_ptr[nc];
  S.blk_row.resize(nblk);
  S.blk_col.resize(nblk);
  S.blk_off.resize(nblk + 1);
  S.blk_kept.resize(nblk);
  int64_t off = 0;
  for (int32_t k = 0; k < nc; ++k) {
    std::vector<int32_t> rows;
    rows.reserve(patc[k].size());
    for (int32_t u : patc[k]) rows.push_back(pos[u]);
    std::sort(rows.begin(), rows.end());
    int64_t b = S.col_ptr[k];
    S.blk_row[b] = k;
    S.blk_col[b] = k;
    S.blk_off[b] = off;
    S.blk_kept[b] = 1;
    off += (int64_t)S.w[k] * S.w[k];
    for (int32_t i : rows) {
      ++b;
      S.blk_row[b] = i;
      S.blk_col[b] = k;
      S.blk_off[b] = off;
      S.blk_kept[b] = P.keep[(size_t)order[i] * nc + order[k]];
      off += (int64_t)S.w[i] * S.w[k];
    }
  }
  S.blk_off[nblk] = off;
  S.factor_entries = off;
  // row structure: for column j, the earlier columns k with j in pattern(k), ascending k, with blk(j, k)
  std::vector<int64_t> cnt(nc + 1, 0);
  for (int64_t b = 0; b < nblk; ++b)
    if (S.blk_row[b] != S.blk_col[b]) ++cnt[S.blk_row[b] + 1];
  S.row_ptr.assign(nc + 1, 0);
  for (int32_t j = 0; j < nc; ++j) S.row_ptr[j + 1] = S.row_ptr[j] + cnt[j + 1];
  S.row_col.resize(S.row_ptr[nc]);
  S.row_blk.resize(S.row_ptr[nc]);
  std::vector<int64_t> fillp(S.row_ptr.begin(), S.row_ptr.end() - 1);
  for (int32_t k = 0; k < nc; ++k)   // columns ascending: each row list comes out sorted by k
    for (int64_t b = S.col_ptr[k] + 1; b < S.col_ptr[k + 1]; ++b) {
      const int32_t j = S.blk_row[b];
      S.row_col[fillp[j]] = k;
      S.row_blk[fillp[j]] = b;
      ++fillp[j];
    }

  // factor flops per column: a w^3/3 factor, w_i w_k^2 per block below it, and per pair of its
  // blocks (i >= j) 2 w_i w_j w_k for the update of block (i, j)
  std::vector<double> colfl(nc, 0.0);
  for (int32_t k = 0; k < nc; ++k) {
    const double wk = S.w[k];
    double fl = wk * wk * wk / 3.0;
    double sw = 0.0, sw2 = 0.0;
    for (int64_t b = S.col_ptr[k] + 1; b < S.col_ptr[k + 1]; ++b) {
      const double wi = S.w[S.blk_row[b]];
      fl += wi * wk * wk;
      sw += wi;
      sw2 += wi * wi;
    }
    fl += wk * (sw * sw + sw2);   // sum over i >= j of 2 w_i w_j w_k = w_k ((sum w)^2 + sum w^2)
    colfl[k] = fl;
  }
  // elimination tree heights (the parent of a column is the first block row below its diagonal)
  std::vector<int32_t> height(nc, 0);
  for (int32_t k = 0; k < nc; ++k) {
    if (S.col_ptr[k + 1] - S.col_ptr[k] > 1) {
      const int32_t parent = S.blk_row[S.col_ptr[k] + 1];
      height[parent] = std::max(height[parent], height[k] + 1);
    }
  }
  // 3. dense tail: the start q minimising the estimated time (flops of the block columns before q) /
  // kSparseBlockRate + (their heights) kSparseHeightTime + rows(q)^3 / 3 / kSparseDenseRate, with at
  // most max_tail rows in the tail; a child precedes its parent in the order, so the heights of the
  // columns before q are those of the whole tree
  {
    int32_t best = nc;
    double pre = 0.0, best_t = 0.0;
    int32_t hall = -1;
    for (int32_t k = 0; k < nc; ++k) {
      best_t += colfl[k];
      hall = std::max(hall, height[k]);
    }
    best_t = best_t / kSparseBlockRate + (hall + 1) * kSparseHeightTime;
    if (dense_tail < 0) {
      int32_t hpre = -1;
      for (int32_t q = 0; q < nc; ++q) {
        const double rows = (double)(S.rows - S.ypos[q]);
        if (rows <= (double)std::min<int64_t>(max_tail, kSparseMaxTail)) {
          const double est =
              pre / kSparseBlockRate + (hpre + 1) * kSparseHeightTime + rows * rows * rows / 3.0 / kSparseDenseRate;
          if (est < best_t) {
            best_t = est;
            best = q;
          }
        }
        pre += colfl[q];
        hpre = std::max(hpre, height[q]);
      }
    } else {
      best = std::min<int32_t>(dense_tail, nc);
      if (S.rows - (best < nc ? S.ypos[best] : S.rows) > kSparseMaxTail)
        return fail(MLBLUP_EINVAL, "sparse loglik: forced dense tail above the row limit");
    }
    S.tail = best;
    S.tail_rows = best < nc ? S.rows - S.ypos[best] : 0;
    const double tr = (double)S.tail_rows;
    S.flops_tail = tr * tr * tr / 3.0;
    S.flops = 0.0;
    for (int32_t k = 0; k < best; ++k) S.flops += colfl[k];
    for (int32_t k = best; k < nc; ++k) {
      S.tail_cols.push_back(k);
      for (int64_t b = S.col_ptr[k]; b < S.col_ptr[k + 1]; ++b) S.tail_blks.push_back(b);
    }
  }

  // 4. the heights of the columns before the tail, one launch group each
  const int32_t ntail0 = S.tail;
  int32_t hmax = -1;
  for (int32_t k = 0; k < ntail0; ++k) hmax = std::max(hmax, height[k]);
  S.lvl_ptr.assign(hmax + 2, 0);
  for (int32_t k = 0; k < ntail0; ++k) ++S.lvl_ptr[height[k] + 1];
  for (int32_t h = 0; h <= hmax; ++h) S.lvl_ptr[h + 1] += S.lvl_ptr[h];
  S.lvl_cols.resize(ntail0);
  std::vector<int64_t> lp(S.lvl_ptr.begin(), S.lvl_ptr.end() - 1);
  for (int32_t k = 0; k < ntail0; ++k) S.lvl_cols[lp[height[k]]++] = k;
  // per height: the blocks of its columns (diagonal first within a column), for the launches
  S.lvl_blk_ptr.assign(hmax + 2, 0);
  for (int32_t h = 0; h <= hmax; ++h) {
    int64_t c = 0;
    for (int64_t q = S.lvl_ptr[h]; q < S.lvl_ptr[h + 1]; ++q) {
      const int32_t k = S.lvl_cols[q];
      c += S.col_ptr[k + 1] - S.col_ptr[k];
    }
    S.lvl_blk_ptr[h + 1] = S.lvl_blk_ptr[h] + c;
  }
  S.lvl_blks.resize(S.lvl_blk_ptr[hmax + 1]);
  {
    int64_t q2 = 0;
    for (int32_t h = 0; h <= hmax; ++h)
      for (int64_t q = S.lvl_ptr[h]; q < S.lvl_ptr[h + 1]; ++q) {
        const int32_t k = S.lvl_cols[q];
        for (int64_t b = S.col_ptr[k]; b < S.col_ptr[k + 1]; ++b) S.lvl_blks[q2++] = b;
      }
  }

  // 5. wavelet vectors of every cell on its points (and the scaling vectors they are built from)
  const int32_t nn = (int32_t)B.desc.size();
  std::vector<std::vector<double>> phi(nn);
  S.psi_off.assign(nc + 1, 0);
  for (int32_t k = 0; k < nc; ++k) {
    const int32_t v = S.node[k];
    S.psi_off[k + 1] = S.psi_off[k] + (B.end[v] - B.begin[v]) * (int64_t)S.w[k];
  }
  S.psi.assign((size_t)S.psi_off[nc], 0.0);
  // nodes at depth >= level, deepest first (preorder numbers parents before children)
  std::vector<int32_t> cell_pos(nn, -1);
  for (int32_t k = 0; k < nc; ++k) cell_pos[S.node[k]] = k;
  for (int32_t v = nn - 1; v >= 0; --v) {
    if (B.depth[v] < level) continue;
    const NodeDesc& nd = B.desc[v];
    const int32_t m = nd.m, a = nd.a, wv = m - a;
    const int64_t sv = B.end[v] - B.begin[v];
    const double* V = &B.V[(size_t)nd.v_off];
    // candidates of v as rows over its points: cand (sv x m)
    std::vector<double> cand;
    if (B.left[v] < 0) {
      cand.assign((size_t)sv * m, 0.0);
      for (int64_t r = 0; r < sv && r < m; ++r) cand[(size_t)r * m + r] = 1.0;
    } else {
      const int32_t L = B.left[v], R = B.right[v];
      const int32_t aL = B.desc[L].a, aR = B.desc[R].a;
      const int64_t sL = B.end[L] - B.begin[L], sR = B.end[R] - B.begin[R];
      cand.assign((size_t)sv * m, 0.0);
      for (int64_t r = 0; r < sL; ++r)
        for (int32_t i = 0; i < aL; ++i) cand[(size_t)r * m + i] = phi[L][(size_t)r * aL + i];
      for (int64_t r = 0; r < sR; ++r)
        for (int32_t i = 0; i < aR; ++i) cand[(size_t)(sL + r) * m + aL + i] = phi[R][(size_t)r * aR + i];
      phi[L].clear();
      phi[L].shrink_to_fit();
      phi[R].clear();
      phi[R].shrink_to_fit();
    }
    // scaling vectors (first a columns of V) and wavelets (the rest)
    phi[v].assign((size_t)sv * a, 0.0);
    double* psi = cell_pos[v] >= 0 ? &S.psi[(size_t)S.psi_off[cell_pos[v]]] : nullptr;
    for (int64_t r = 0; r < sv; ++r) {
      const double* cr = &cand[(size_t)r * m];
      for (int32_t c = 0; c < m; ++c) {
        double s = 0.0;
        for (int32_t i = 0; i < m; ++i) s += cr[i] * V[(size_t)i * m + c];
        if (c < a)
          phi[v][(size_t)r * a + c] = s;
        else if (psi)
          psi[(size_t)r * wv + (c - a)] = s;
      }
    }
  }
  return MLBLUP_OK;
}

}  // namespace mlb
