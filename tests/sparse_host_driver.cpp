// Host check of the analysis behind the sparse block Cholesky of C~^n_W
// (sparse_chol.cpp): for trees and bases over several point sets, levels
// and distances tau it verifies
//  * the wavelet vectors of every cell: orthonormal, with vanishing moments
//    against the monomials of the trend degree on the cell's points;
//  * the block structure: every kept cell pair is a block of the factor, the
//    pattern of each column is closed under elimination (for i > j in the
//    pattern of k, block (i, j) exists), the row structure lists exactly
//    the blocks below the diagonals, and every column and block sits in one
//    elimination-tree height, after all the columns it depends on;
//  * the numbers: the block algorithm the device kernels run (assembly from
//    the wavelet vectors, left-looking updates over the merged row
//    structures, diagonal factor and inverse, products with the inverse,
//    the data vector as a border row), written here in plain loops with the
//    same indexing, against a dense Cholesky of the same sparsified matrix:
//    log det and quadratic form to 1e-9 relative.
// Built with the address/undefined sanitizers by tests/test_host_sanitizers.py.
// Exit status 0 and the line "sparse driver: ok" mean no finding.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "internal.h"

namespace mlb {
int fail(int status, const std::string& msg) {
  std::fprintf(stderr, "  (status %d: %s)\n", status, msg.c_str());
  return status;
}
void clear_error() {}
}  // namespace mlb

static int g_fail = 0;
#define CHECK(cond, ...)                  \
  do {                                    \
    if (!(cond)) {                        \
      std::printf("FAIL: " __VA_ARGS__);  \
      std::printf("\n");                  \
      ++g_fail;                           \
      return;                             \
    }                                     \
  } while (0)

static double cov(const double* a, const double* b, int d, double rho) {
  double s = 0.0;
  for (int k = 0; k < d; ++k) s += (a[k] - b[k]) * (a[k] - b[k]);
  return std::exp(-std::sqrt(s) / rho);
}

// mode: 0 the tail start chosen by the analysis, 1 no dense tail, 2 all dense, 3 dense from the middle
static void check_case(const char* name, const mlb::Basis& B, int level, double tau, double rho, int mode) {
  mlb::SparseSymbolic S;
  int st = mlb::sparse_analyse(B, level, tau, S);
  CHECK(st == MLBLUP_OK, "%s: sparse_analyse status %d", name, st);
  if (mode > 0) {
    const int forced = mode == 1 ? S.nc : (mode == 2 ? 0 : S.nc / 2);
    st = mlb::sparse_analyse(B, level, tau, S, forced);
    CHECK(st == MLBLUP_OK && S.tail == forced, "%s: forced tail %d status %d", name, forced, st);
  }
  const int nc = S.nc;
  const int d = B.d;
  if (nc == 0) return;
  // wavelet vectors: orthonormal, vanishing moments
  for (int k = 0; k < nc; ++k) {
    const int v = S.node[k], w = S.w[k];
    const int64_t s = B.end[v] - B.begin[v];
    const double* P = &S.psi[S.psi_off[k]];
    CHECK(S.psi_off[k + 1] - S.psi_off[k] == s * w, "%s: psi size of position %d", name, k);
    for (int a = 0; a < w; ++a)
      for (int b = 0; b < w; ++b) {
        double g = 0.0;
        for (int64_t r = 0; r < s; ++r) g += P[r * w + a] * P[r * w + b];
        CHECK(std::fabs(g - (a == b ? 1.0 : 0.0)) < 1e-10, "%s: psi not orthonormal (cell %d: %d,%d = %g)", name, k,
              a, b, g);
      }
    // moments in the cell's frame (centre and half width of its box)
    std::vector<double> lo(d, 1e300), hi(d, -1e300);
    for (int64_t r = 0; r < s; ++r)
      for (int q = 0; q < d; ++q) {
        const double x = B.pts_tree[(B.begin[v] + r) * d + q];
        lo[q] = std::min(lo[q], x);
        hi[q] = std::max(hi[q], x);
      }
    double h = 0.0;
    for (int q = 0; q < d; ++q) h = std::max(h, 0.5 * (hi[q] - lo[q]));
    if (h == 0.0) h = 1.0;
    for (const auto& e : B.exps)
      for (int a = 0; a < w; ++a) {
        double m = 0.0, mabs = 0.0;
        for (int64_t r = 0; r < s; ++r) {
          double mono = 1.0;
          for (int q = 0; q < d; ++q) {
            const double u = (B.pts_tree[(B.begin[v] + r) * d + q] - 0.5 * (lo[q] + hi[q])) / h;
            for (int t = 0; t < e[q]; ++t) mono *= u;
          }
          m += P[r * w + a] * mono;
          mabs += std::fabs(P[r * w + a] * mono);
        }
        CHECK(std::fabs(m) <= 1e-9 * std::max(1.0, mabs), "%s: moment of cell %d wavelet %d = %g", name, k, a, m);
      }
  }
  // block structure
  const int64_t nblk = S.col_ptr[nc];
  auto find_blk = [&](int i, int j) -> int64_t {  // block (i, j), i >= j, or -1
    for (int64_t b = S.col_ptr[j]; b < S.col_ptr[j + 1]; ++b)
      if (S.blk_row[b] == i) return b;
    return -1;
  };
  mlb::Pattern Pat;
  mlb::build_pattern(B, level, tau, Pat);
  std::vector<int> pos(nc);
  for (int k = 0; k < nc; ++k) pos[S.order[k]] = k;
  for (int x = 0; x < nc; ++x)
    for (int y = 0; y < nc; ++y)
      if (Pat.keep[(size_t)x * nc + y]) {
        const int i = std::max(pos[x], pos[y]), j = std::min(pos[x], pos[y]);
        const int64_t b = find_blk(i, j);
        CHECK(b >= 0 && S.blk_kept[b], "%s: kept pair (%d,%d) has no kept block", name, x, y);
      }
  for (int64_t b = 0; b < nblk; ++b) {
    const int i = S.blk_row[b], j = S.blk_col[b];
    CHECK(i >= j && S.blk_off[b + 1] - S.blk_off[b] == (int64_t)S.w[i] * S.w[j], "%s: block %lld shape", name,
          (long long)b);
    CHECK(S.blk_kept[b] == Pat.keep[(size_t)S.order[i] * nc + S.order[j]] || i == j, "%s: kept flag of block %lld",
          name, (long long)b);
  }
  for (int k = 0; k < nc; ++k) {
    CHECK(S.blk_row[S.col_ptr[k]] == k, "%s: column %d does not start at its diagonal", name, k);
    for (int64_t a = S.col_ptr[k] + 1; a < S.col_ptr[k + 1]; ++a) {
      CHECK(a == S.col_ptr[k] + 1 || S.blk_row[a] > S.blk_row[a - 1], "%s: column %d rows not ascending", name, k);
      for (int64_t b = S.col_ptr[k] + 1; b < a; ++b)
        CHECK(find_blk(S.blk_row[a], S.blk_row[b]) >= 0, "%s: fill block (%d,%d) missing", name, S.blk_row[a],
              S.blk_row[b]);
    }
  }
  int64_t rows_listed = 0;
  for (int j = 0; j < nc; ++j)
    for (int64_t p = S.row_ptr[j]; p < S.row_ptr[j + 1]; ++p) {
      const int64_t b = S.row_blk[p];
      CHECK(S.blk_row[b] == j && S.blk_col[b] == S.row_col[p] && S.row_col[p] < j, "%s: row structure of %d", name,
            j);
      CHECK(p == S.row_ptr[j] || S.row_col[p] > S.row_col[p - 1], "%s: row structure of %d not ascending", name, j);
      ++rows_listed;
    }
  CHECK(rows_listed == nblk - nc, "%s: row structure lists %lld of %lld blocks", name, (long long)rows_listed,
        (long long)(nblk - nc));
  const int P = S.tail;
  CHECK(P >= 0 && P <= nc && (int)S.tail_cols.size() == nc - P, "%s: tail %d", name, P);
  CHECK(S.tail_rows == (P < nc ? S.rows - S.ypos[P] : 0), "%s: tail rows", name);
  for (int q = 0; q < nc - P; ++q) CHECK(S.tail_cols[q] == P + q, "%s: tail columns", name);
  std::vector<int> hof(nc, -1);
  const int heights = (int)S.lvl_ptr.size() - 1;
  for (int h = 0; h < heights; ++h)
    for (int64_t q = S.lvl_ptr[h]; q < S.lvl_ptr[h + 1]; ++q) {
      CHECK(S.lvl_cols[q] < P && hof[S.lvl_cols[q]] < 0, "%s: column in two heights or in the tail", name);
      hof[S.lvl_cols[q]] = h;
    }
  for (int k = 0; k < P; ++k) {
    CHECK(hof[k] >= 0, "%s: column %d in no height", name, k);
    for (int64_t b = S.col_ptr[k] + 1; b < S.col_ptr[k + 1]; ++b)
      CHECK(S.blk_row[b] >= P || hof[S.blk_row[b]] > hof[k], "%s: column %d not below %d in the tree", name, k,
            S.blk_row[b]);
  }
  {
    std::vector<int> seen(nblk, 0);
    for (int h = 0; h < heights; ++h)
      for (int64_t q = S.lvl_blk_ptr[h]; q < S.lvl_blk_ptr[h + 1]; ++q) {
        const int64_t b = S.lvl_blks[q];
        CHECK(hof[S.blk_col[b]] == h && !seen[b], "%s: block %lld listed at the wrong height", name, (long long)b);
        seen[b] = 1;
      }
    for (int64_t b : S.tail_blks) {
      CHECK(S.blk_col[b] >= P && !seen[b], "%s: tail block %lld", name, (long long)b);
      seen[b] = 1;
    }
    for (int64_t b = 0; b < nblk; ++b) CHECK(seen[b], "%s: block %lld in no height", name, (long long)b);
  }

  // the device algorithm in plain loops
  const int64_t nt = S.rows;
  std::vector<double> L(S.factor_entries, 0.0), Linv, z(nt), y(nt, 0.0), zt(nt, 0.0), logd(nt, 0.0);
  std::vector<int64_t> inv_off(nc);
  int64_t io = 0;
  for (int k = 0; k < nc; ++k) {
    inv_off[k] = io;
    io += (int64_t)S.w[k] * S.w[k];
  }
  Linv.assign(io, 0.0);
  std::mt19937_64 g(7);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (auto& v : z) v = nd(g);
  for (int64_t b = 0; b < nblk; ++b) {
    if (!S.blk_kept[b]) continue;
    const int i = S.blk_row[b], k = S.blk_col[b];
    const int wi = S.w[i], wk = S.w[k];
    const int vi = S.node[i], vk = S.node[k];
    const int64_t si = B.end[vi] - B.begin[vi], sk = B.end[vk] - B.begin[vk];
    const double* Pi = &S.psi[S.psi_off[i]];
    const double* Pk = &S.psi[S.psi_off[k]];
    std::vector<double> T(si * wk, 0.0);
    for (int64_t a = 0; a < si; ++a)
      for (int64_t c = 0; c < sk; ++c) {
        const double kv = cov(&B.pts_tree[(B.begin[vi] + a) * d], &B.pts_tree[(B.begin[vk] + c) * d], d, rho);
        for (int q = 0; q < wk; ++q) T[a * wk + q] += kv * Pk[c * wk + q];
      }
    for (int r = 0; r < wi; ++r)
      for (int q = 0; q < wk; ++q) {
        double s = 0.0;
        for (int64_t a = 0; a < si; ++a) s += Pi[a * wi + r] * T[a * wk + q];
        L[S.blk_off[b] + r * wk + q] = s;
      }
  }
  // dense copy of the assembled matrix (symmetric) for the reference
  std::vector<double> A((size_t)nt * nt, 0.0);
  for (int64_t b = 0; b < nblk; ++b) {
    const int i = S.blk_row[b], k = S.blk_col[b];
    for (int r = 0; r < S.w[i]; ++r)
      for (int q = 0; q < S.w[k]; ++q) {
        const double v = L[S.blk_off[b] + r * S.w[k] + q];
        A[(size_t)(S.ypos[i] + r) * nt + S.ypos[k] + q] = v;
        A[(size_t)(S.ypos[k] + q) * nt + S.ypos[i] + r] = v;
      }
  }
  bool broke = false;
  for (int h = 0; h < heights; ++h) {
    // update
    for (int64_t q = S.lvl_blk_ptr[h]; q < S.lvl_blk_ptr[h + 1]; ++q) {
      const int64_t b = S.lvl_blks[q];
      const int i = S.blk_row[b], j = S.blk_col[b];
      const int wi = S.w[i], wj = S.w[j];
      int64_t p = S.row_ptr[i], r = S.row_ptr[j];
      while (p < S.row_ptr[i + 1] && r < S.row_ptr[j + 1]) {
        if (S.row_col[p] == S.row_col[r]) {
          const int k = S.row_col[p], wk = S.w[k];
          const double* la = &L[S.blk_off[S.row_blk[p]]];
          const double* lb = &L[S.blk_off[S.row_blk[r]]];
          for (int x = 0; x < wi; ++x)
            for (int c = 0; c < wj; ++c) {
              double s = 0.0;
              for (int t = 0; t < wk; ++t) s += la[x * wk + t] * lb[c * wk + t];
              L[S.blk_off[b] + x * wj + c] -= s;
            }
          ++p;
          ++r;
        } else if (S.row_col[p] < S.row_col[r]) {
          ++p;
        } else {
          ++r;
        }
      }
    }
    for (int64_t q = S.lvl_ptr[h]; q < S.lvl_ptr[h + 1]; ++q) {
      const int j = S.lvl_cols[q], wj = S.w[j];
      for (int c = 0; c < wj; ++c) {
        double v = z[S.ypos[j] + c];
        for (int64_t p = S.row_ptr[j]; p < S.row_ptr[j + 1]; ++p) {
          const int k = S.row_col[p], wk = S.w[k];
          for (int t = 0; t < wk; ++t) v -= L[S.blk_off[S.row_blk[p]] + c * wk + t] * y[S.ypos[k] + t];
        }
        zt[S.ypos[j] + c] = v;
      }
    }
    // factor
    for (int64_t q = S.lvl_ptr[h]; q < S.lvl_ptr[h + 1]; ++q) {
      const int j = S.lvl_cols[q], w = S.w[j];
      double* M = &L[S.blk_off[S.col_ptr[j]]];
      for (int c = 0; c < w; ++c) {
        double piv = M[c * w + c];
        if (!(piv > 0.0)) {
          broke = true;
          piv = 1.0;
        }
        M[c * w + c] = std::sqrt(piv);
        for (int r = c + 1; r < w; ++r) M[r * w + c] /= M[c * w + c];
        for (int r = c + 1; r < w; ++r)
          for (int t = c + 1; t <= r; ++t) M[r * w + t] -= M[r * w + c] * M[t * w + c];
      }
      for (int r = 0; r < w; ++r)
        for (int c = r + 1; c < w; ++c) M[r * w + c] = 0.0;
      double* X = &Linv[inv_off[j]];
      for (int c = 0; c < w; ++c)
        for (int r = c; r < w; ++r) {
          double s = (r == c) ? 1.0 : 0.0;
          for (int t = c; t < r; ++t) s -= M[r * w + t] * X[t * w + c];
          X[r * w + c] = s / M[r * w + r];
        }
      for (int r = 0; r < w; ++r) {
        double s = 0.0;
        for (int t = 0; t <= r; ++t) s += X[r * w + t] * zt[S.ypos[j] + t];
        y[S.ypos[j] + r] = s;
        logd[S.ypos[j] + r] = std::log(M[r * w + r]);
      }
    }
    // products with the inverse
    for (int64_t q = S.lvl_blk_ptr[h]; q < S.lvl_blk_ptr[h + 1]; ++q) {
      const int64_t b = S.lvl_blks[q];
      const int i = S.blk_row[b], j = S.blk_col[b];
      if (i == j) continue;
      const int wi = S.w[i], wj = S.w[j];
      const double* X = &Linv[inv_off[j]];
      std::vector<double> tmp((size_t)wi * wj);
      for (int r = 0; r < wi; ++r)
        for (int c = 0; c < wj; ++c) {
          double s = 0.0;
          for (int t = 0; t < wj; ++t) s += L[S.blk_off[b] + r * wj + t] * X[c * wj + t];
          tmp[(size_t)r * wj + c] = s;
        }
      std::copy(tmp.begin(), tmp.end(), L.begin() + S.blk_off[b]);
    }
  }
  double ld = 0.0, qf = 0.0;
  const int64_t nsp = P < nc ? S.ypos[P] : nt;
  for (int64_t r = 0; r < nsp; ++r) {
    ld += 2.0 * logd[r];
    qf += y[r] * y[r];
  }
  if (P < nc) {
    // the tail's blocks updated by the columns before it, its data rows, then a dense Cholesky
    for (int64_t b : S.tail_blks) {
      const int i = S.blk_row[b], j = S.blk_col[b];
      const int wi = S.w[i], wj = S.w[j];
      int64_t p = S.row_ptr[i], r = S.row_ptr[j];
      while (p < S.row_ptr[i + 1] && r < S.row_ptr[j + 1] && S.row_col[p] < P && S.row_col[r] < P) {
        if (S.row_col[p] == S.row_col[r]) {
          const int k = S.row_col[p], wk = S.w[k];
          for (int x = 0; x < wi; ++x)
            for (int c = 0; c < wj; ++c) {
              double s = 0.0;
              for (int t2 = 0; t2 < wk; ++t2)
                s += L[S.blk_off[S.row_blk[p]] + x * wk + t2] * L[S.blk_off[S.row_blk[r]] + c * wk + t2];
              L[S.blk_off[b] + x * wj + c] -= s;
            }
          ++p;
          ++r;
        } else if (S.row_col[p] < S.row_col[r]) {
          ++p;
        } else {
          ++r;
        }
      }
    }
    for (int j = P; j < nc; ++j)
      for (int c = 0; c < S.w[j]; ++c) {
        double v = z[S.ypos[j] + c];
        for (int64_t p = S.row_ptr[j]; p < S.row_ptr[j + 1] && S.row_col[p] < P; ++p) {
          const int k = S.row_col[p], wk = S.w[k];
          for (int t2 = 0; t2 < wk; ++t2) v -= L[S.blk_off[S.row_blk[p]] + c * wk + t2] * y[S.ypos[k] + t2];
        }
        zt[S.ypos[j] + c] = v;
      }
    const int64_t T = S.tail_rows, y0 = S.ypos[P];
    std::vector<double> D((size_t)T * T, 0.0);
    for (int64_t b : S.tail_blks) {
      const int i = S.blk_row[b], j = S.blk_col[b];
      for (int r = 0; r < S.w[i]; ++r)
        for (int c = 0; c < S.w[j]; ++c) {
          if (i == j && c > r) continue;   // the lower triangle of a diagonal block, as the device does
          const double v = L[S.blk_off[b] + r * S.w[j] + c];
          D[(size_t)(S.ypos[i] - y0 + r) * T + S.ypos[j] - y0 + c] = v;
          D[(size_t)(S.ypos[j] - y0 + c) * T + S.ypos[i] - y0 + r] = v;
        }
    }
    std::vector<double> yt(T);
    for (int64_t c = 0; c < T && !broke; ++c) {
      double piv = D[c * T + c];
      for (int64_t t2 = 0; t2 < c; ++t2) piv -= D[c * T + t2] * D[c * T + t2];
      if (!(piv > 0.0)) {
        broke = true;
        break;
      }
      D[c * T + c] = std::sqrt(piv);
      for (int64_t r = c + 1; r < T; ++r) {
        double s = D[r * T + c];
        for (int64_t t2 = 0; t2 < c; ++t2) s -= D[r * T + t2] * D[c * T + t2];
        D[r * T + c] = s / D[c * T + c];
      }
    }
    if (!broke)
      for (int64_t r = 0; r < T; ++r) {
        double s = zt[y0 + r];
        for (int64_t t2 = 0; t2 < r; ++t2) s -= D[r * T + t2] * yt[t2];
        yt[r] = s / D[r * T + r];
        ld += 2.0 * std::log(D[r * T + r]);
        qf += yt[r] * yt[r];
      }
  }
  // dense Cholesky of the same matrix, data vector in the same order
  bool dbroke = false;
  for (int64_t c = 0; c < nt; ++c) {
    double piv = A[c * nt + c];
    for (int64_t t = 0; t < c; ++t) piv -= A[c * nt + t] * A[c * nt + t];
    if (!(piv > 0.0)) {
      dbroke = true;
      break;
    }
    A[c * nt + c] = std::sqrt(piv);
    for (int64_t r = c + 1; r < nt; ++r) {
      double s = A[r * nt + c];
      for (int64_t t = 0; t < c; ++t) s -= A[r * nt + t] * A[c * nt + t];
      A[r * nt + c] = s / A[c * nt + c];
    }
  }
  CHECK(broke == dbroke, "%s: breakdown differs (block %d, dense %d)", name, (int)broke, (int)dbroke);
  if (dbroke) {
    std::printf("%s level %d tau %g: indefinite, both stop\n", name, level, tau);
    return;
  }
  double dld = 0.0, dqf = 0.0;
  std::vector<double> yy(nt);
  for (int64_t r = 0; r < nt; ++r) {
    double s = z[r];
    for (int64_t t = 0; t < r; ++t) s -= A[r * nt + t] * yy[t];
    yy[r] = s / A[r * nt + r];
    dld += 2.0 * std::log(A[r * nt + r]);
    dqf += yy[r] * yy[r];
  }
  std::printf("%s level %d tau %g tail %d/%d: N~ %lld, blocks %lld, heights %d, logdet %.12g / %.12g, quad %.12g / %.12g\n",
              name, level, tau, P, nc, (long long)nt, (long long)nblk, heights, ld, dld, qf, dqf);
  CHECK(std::fabs(ld - dld) <= 1e-9 * std::max(1.0, std::fabs(dld)), "%s: log det %g vs %g", name, ld, dld);
  CHECK(std::fabs(qf - dqf) <= 1e-9 * std::max(1.0, std::fabs(dqf)), "%s: quadratic form %g vs %g", name, qf, dqf);
}

static void run(const char* name, int64_t n, int d, int leaf, int w, double rho, unsigned seed) {
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  std::vector<double> pts((size_t)n * d);
  for (auto& v : pts) v = u(g);
  mlb::Tree t;
  if (mlb::build_tree(pts.data(), n, d, leaf, t) != MLBLUP_OK) {
    std::printf("FAIL: %s build_tree\n", name);
    ++g_fail;
    return;
  }
  mlb::Basis b;
  if (mlb::build_basis(t, w, 1e-10, b) != MLBLUP_OK) {
    std::printf("FAIL: %s build_basis\n", name);
    ++g_fail;
    return;
  }
  const int top = b.levels - 1;
  for (int level : {top, top - 1, top - 2, 0})
    for (double tau : {0.0, 0.05, 0.15, 1e9}) {
      if (level < 0) continue;
      for (int mode = 0; mode < 4; ++mode) check_case(name, b, level, tau, rho, mode);
    }
}

int main() {
  run("uniform2d", 600, 2, 32, 2, 0.1, 1);
  run("uniform3d", 700, 3, 64, 1, 0.2, 2);
  run("uniform5d", 400, 5, 40, 1, 0.3, 3);
  if (g_fail) {
    std::printf("sparse driver: %d failures\n", g_fail);
    return 1;
  }
  std::printf("sparse driver: ok\n");
  return 0;
}
