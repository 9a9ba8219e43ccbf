// Multilevel basis construction (Sec. 3.1: construction of W and L from the
// kd-tree; operators W, L, P).
//
// For every cell, bottom-up, the candidate vectors (a leaf: the unit vectors
// of its points; an internal cell: the scaling vectors of its two children,
// left first) are combined by an orthogonal m x m matrix V whose first a
// columns span the range of M^T, M = X^T [candidates] (p x m moments against
// the degree-w monomials), and whose remaining m - a columns span null(M):
// those are the cell's wavelets, orthogonal to every monomial (vanishing
// moments); the first a are the scaling vectors passed to the parent.
//
// The paper takes V from an SVD of M; any orthogonal V with the same two
// subspaces gives the same W up to a rotation inside each cell, and every
// result of the solve is invariant under such rotations.  This code uses
// Householder QR with column pivoting of M^T (rank revealing, exact
// orthogonality, cheaper).  Moments are taken in cell-local coordinates
// u = (x - c)/h (c = box centre, h = half of the widest box side), which
// spans the same polynomial space; a child's scaling moments are carried to
// the parent's frame by the exact binomial change of variables.
#include <algorithm>
#include <cmath>
#include <functional>
#include <thread>

#include "internal.h"

namespace mlb {

std::vector<std::vector<int32_t>> td_exponents(int32_t d, int32_t w) {
  std::vector<std::vector<int32_t>> out;
  std::vector<int32_t> cur(d, 0);
  // exponents of total degree `deg`, decreasing lexicographic order
  std::function<void(int32_t, int32_t)> rec = [&](int32_t pos, int32_t rem) {
    if (pos == d - 1) {
      cur[pos] = rem;
      out.push_back(cur);
      return;
    }
    for (int32_t e = rem; e >= 0; --e) {
      cur[pos] = e;
      rec(pos + 1, rem - e);
    }
  };
  for (int32_t deg = 0; deg <= w; ++deg) rec(0, deg);
  return out;
}

namespace {

struct Frame {
  std::vector<double> c;
  double h = 1.0;
};

// Householder QR with column pivoting of A (m x p, column-major, lda = m).
// On return A holds R in its upper triangle and the reflectors below it,
// piv the column permutation, tau the reflector scales.
void qr_pivot(int m, int p, std::vector<double>& A, std::vector<int>& piv, std::vector<double>& tau) {
  const int K = std::min(m, p);
  piv.resize(p);
  for (int j = 0; j < p; ++j) piv[j] = j;
  tau.assign(K, 0.0);
  for (int k = 0; k < K; ++k) {
    // pivot: largest remaining column norm (recomputed, no downdating)
    int jbest = k;
    double nbest = -1.0;
    for (int j = k; j < p; ++j) {
      double s = 0.0;
      for (int i = k; i < m; ++i) s += A[(size_t)j * m + i] * A[(size_t)j * m + i];
      if (s > nbest) {
        nbest = s;
        jbest = j;
      }
    }
    if (jbest != k) {
      for (int i = 0; i < m; ++i) std::swap(A[(size_t)k * m + i], A[(size_t)jbest * m + i]);
      std::swap(piv[k], piv[jbest]);
    }
    double* x = &A[(size_t)k * m];
    const double xnorm = std::sqrt(std::max(nbest, 0.0));
    if (xnorm == 0.0) {
      tau[k] = 0.0;
      continue;
    }
    const double alpha = x[k] >= 0 ? -xnorm : xnorm;
    const double v0 = x[k] - alpha;
    // v = [1, x[k+1:]/v0], tau = (alpha - x_k) / alpha... computed as -v0/alpha
    for (int i = k + 1; i < m; ++i) x[i] /= v0;
    tau[k] = -v0 / alpha;
    x[k] = alpha;
    for (int j = k + 1; j < p; ++j) {
      double* y = &A[(size_t)j * m];
      double s = y[k];
      for (int i = k + 1; i < m; ++i) s += x[i] * y[i];
      s *= tau[k];
      y[k] -= s;
      for (int i = k + 1; i < m; ++i) y[i] -= s * x[i];
    }
  }
}

// Q = H_0 H_1 ... H_{K-1} (m x m), written row-major into Q.
void form_q(int m, int p, const std::vector<double>& A, const std::vector<double>& tau, double* Q) {
  const int K = std::min(m, p);
  std::vector<double> Qc((size_t)m * m, 0.0);  // column-major work
  for (int i = 0; i < m; ++i) Qc[(size_t)i * m + i] = 1.0;
  for (int k = K - 1; k >= 0; --k) {
    if (tau[k] == 0.0) continue;
    const double* v = &A[(size_t)k * m];
    for (int j = k; j < m; ++j) {
      double* y = &Qc[(size_t)j * m];
      double s = y[k];
      for (int i = k + 1; i < m; ++i) s += v[i] * y[i];
      s *= tau[k];
      y[k] -= s;
      for (int i = k + 1; i < m; ++i) y[i] -= s * v[i];
    }
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) Q[(size_t)i * m + j] = Qc[(size_t)j * m + i];
}

double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// T[beta][alpha]: moments in the child frame -> moments in the parent frame.
// With u = (x - c_child)/h_child and y = (x - c_parent)/h_parent,
// y_k = s u_k + b_k (s = h_child/h_parent, b_k = (c_child,k - c_parent,k)/h_parent),
// so y^beta = sum_{alpha <= beta} prod_k C(beta_k, alpha_k) s^alpha_k b_k^(beta_k - alpha_k) u^alpha.
void frame_transform(const std::vector<std::vector<int32_t>>& E, int32_t w, const Frame& ch, const Frame& pa,
                     std::vector<double>& T) {
  const int p = (int)E.size(), d = (int)ch.c.size();
  const double s = ch.h / pa.h;
  std::vector<double> spow(w + 1), bpow((size_t)d * (w + 1));
  spow[0] = 1.0;
  for (int e = 1; e <= w; ++e) spow[e] = spow[e - 1] * s;
  for (int k = 0; k < d; ++k) {
    const double b = (ch.c[k] - pa.c[k]) / pa.h;
    bpow[(size_t)k * (w + 1)] = 1.0;
    for (int e = 1; e <= w; ++e) bpow[(size_t)k * (w + 1) + e] = bpow[(size_t)k * (w + 1) + e - 1] * b;
  }
  T.assign((size_t)p * p, 0.0);
  for (int be = 0; be < p; ++be)
    for (int al = 0; al < p; ++al) {
      double t = 1.0;
      int deg = 0;
      for (int k = 0; k < d; ++k) {
        const int B = E[be][k], A = E[al][k];
        if (A > B) {
          t = 0.0;
          break;
        }
        if (B) t *= binom(B, A) * bpow[(size_t)k * (w + 1) + (B - A)];
        deg += A;
      }
      T[(size_t)be * p + al] = t * spow[deg];
    }
}

}  // namespace

int build_basis(const Tree& t, int32_t w, double rank_rtol, Basis& B) {
  if (w < 0 || w > 16) return fail(MLBLUP_EINVAL, "build_multilevel_basis: degree_w must be in [0, 16]");
  if (rank_rtol <= 0) rank_rtol = 1e-10;
  const int32_t d = t.d;
  const int64_t n = t.n;
  B = Basis();
  B.n = n;
  B.d = d;
  B.w = w;
  B.exps = td_exponents(d, w);
  const int p = (int)B.exps.size();
  B.p = p;
  if (n <= p) return fail(MLBLUP_EINVAL, "build_multilevel_basis: need N > p = binomial(d+w, w)");
  B.levels = t.max_depth + 1;
  const int32_t nn = t.n_nodes();
  B.begin = t.begin;
  B.end = t.end;
  B.left = t.left;
  B.right = t.right;
  B.depth = t.depth;
  B.axis = t.axis;
  B.threshold = t.threshold;

  B.pts_tree.resize((size_t)n * d);
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < d; ++k) B.pts_tree[(size_t)i * d + k] = t.pts[(size_t)t.perm[i] * d + k];

  // frames
  std::vector<Frame> fr(nn);
  for (int32_t v = 0; v < nn; ++v) {
    std::vector<double> lo(d, INFINITY), hi(d, -INFINITY);
    for (int64_t i = t.begin[v]; i < t.end[v]; ++i)
      for (int k = 0; k < d; ++k) {
        const double x = B.pts_tree[(size_t)i * d + k];
        lo[k] = std::min(lo[k], x);
        hi[k] = std::max(hi[k], x);
      }
    fr[v].c.resize(d);
    double h = 0.0;
    for (int k = 0; k < d; ++k) {
      fr[v].c[k] = 0.5 * (lo[k] + hi[k]);
      h = std::max(h, 0.5 * (hi[k] - lo[k]));
    }
    fr[v].h = h > 0 ? h : 1.0;
  }

  // candidate counts and V offsets are known only bottom-up; process by level
  std::vector<int32_t> m_of(nn, 0), a_of(nn, 0);
  std::vector<std::vector<double>> Vblk(nn);
  std::vector<std::vector<double>> Hblk(nn);
  std::vector<std::vector<double>> Ms(nn);   // p x a, row-major
  std::vector<std::vector<int32_t>> by_level(B.levels);
  for (int32_t v = 0; v < nn; ++v) by_level[t.depth[v]].push_back(v);

  const unsigned hw = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  for (int q = B.levels - 1; q >= 0; --q) {
    const auto& nodes = by_level[q];
    auto work = [&](size_t lo, size_t hi_) {
      std::vector<double> A, tau, T;
      std::vector<int> piv;
      for (size_t s = lo; s < hi_; ++s) {
        const int32_t v = nodes[s];
        int m;
        if (t.leaf(v)) {
          m = (int)(t.end[v] - t.begin[v]);
          A.assign((size_t)m * p, 0.0);
          for (int i = 0; i < m; ++i) {
            const double* x = &B.pts_tree[(size_t)(t.begin[v] + i) * d];
            for (int be = 0; be < p; ++be) {
              double val = 1.0;
              for (int k = 0; k < d; ++k) {
                const double u = (x[k] - fr[v].c[k]) / fr[v].h;
                for (int e = 0; e < B.exps[be][k]; ++e) val *= u;
              }
              A[(size_t)be * m + i] = val;
            }
          }
        } else {
          const int32_t L = t.left[v], R = t.right[v];
          m = a_of[L] + a_of[R];
          A.assign((size_t)m * p, 0.0);
          int row = 0;
          for (int32_t c : {L, R}) {
            frame_transform(B.exps, w, fr[c], fr[v], T);
            const int ac = a_of[c];
            for (int j = 0; j < ac; ++j, ++row)
              for (int be = 0; be < p; ++be) {
                double s2 = 0.0;
                for (int al = 0; al < p; ++al) s2 += T[(size_t)be * p + al] * Ms[c][(size_t)al * ac + j];
                A[(size_t)be * m + row] = s2;
              }
          }
        }
        m_of[v] = m;
        if (m == 0) {
          a_of[v] = 0;
          continue;
        }
        qr_pivot(m, p, A, piv, tau);
        const int K = std::min(m, p);
        const double r00 = std::fabs(A[0]);
        int a = 0;
        while (a < K && r00 > 0 && std::fabs(A[(size_t)a * m + a]) > rank_rtol * r00) ++a;
        a_of[v] = a;
        Vblk[v].resize((size_t)m * m);
        form_q(m, p, A, tau, Vblk[v].data());
        // the same V as a compact WY product (R. Schreiber and C. Van Loan, "A storage-efficient WY
        // representation for products of Householder transformations", SIAM J. Sci. Stat. Comput.
        // 10, 1989): V = H_0 ... H_{K-1} = I - Y T Y^T, Y = [h_0 ... h_{K-1}] (h_k = [0 (k entries),
        // 1, A[k+1..m-1] of column k]), T upper triangular with T_kk = tau_k and column k above the
        // diagonal -tau_k T_{0..k-1,0..k-1} Y_{0..k-1}^T h_k.  Stored as Y (K rows of m), then T (K x K).
        Hblk[v].assign((size_t)K * m + (size_t)K * K, 0.0);
        double* Y = Hblk[v].data();
        double* Tm = Y + (size_t)K * m;
        std::vector<double> yh(K);
        for (int k = 0; k < K; ++k) {
          double* h = Y + (size_t)k * m;
          h[k] = 1.0;
          for (int i = k + 1; i < m; ++i) h[i] = A[(size_t)k * m + i];
          for (int j = 0; j < k; ++j) {
            double s = 0.0;
            for (int i = k; i < m; ++i) s += Y[(size_t)j * m + i] * h[i];
            yh[j] = s;
          }
          for (int r = 0; r < k; ++r) {
            double s = 0.0;
            for (int j = r; j < k; ++j) s += Tm[(size_t)r * K + j] * yh[j];
            Tm[(size_t)r * K + k] = -tau[k] * s;
          }
          Tm[(size_t)k * K + k] = tau[k];
        }
        Ms[v].assign((size_t)p * a, 0.0);
        for (int j = 0; j < a; ++j)
          for (int k = j; k < p; ++k) Ms[v][(size_t)piv[k] * a + j] = A[(size_t)k * m + j];
      }
    };
    const size_t cnt = nodes.size();
    const unsigned nt = (unsigned)std::min<size_t>(hw, std::max<size_t>(1, cnt / 4));
    if (nt <= 1) {
      work(0, cnt);
    } else {
      std::vector<std::thread> th;
      for (unsigned i = 0; i < nt; ++i) th.emplace_back(work, cnt * i / nt, cnt * (i + 1) / nt);
      for (auto& x : th) x.join();
    }
    // children's moments are no longer needed
    for (int32_t v : nodes)
      if (!t.leaf(v)) {
        std::vector<double>().swap(Ms[t.left[v]]);
        std::vector<double>().swap(Ms[t.right[v]]);
      }
  }
  if (a_of[0] != p)
    return fail(MLBLUP_ERANK, "build_multilevel_basis: rank of the design matrix on the points is " +
                                  std::to_string(a_of[0]) + " < p = " + std::to_string(p) +
                                  " (collinear or duplicate points for this degree?)");
  B.root_c = fr[0].c;
  B.root_h = fr[0].h;
  B.root_moments = Ms[0];  // p x p

  // schedule: wavelet offsets level-major (finest first), preorder inside a level
  B.desc.resize(nn);
  B.level_counts.assign(B.levels, 0);
  int64_t woff = 0;
  for (int q = B.levels - 1; q >= 0; --q)
    for (int32_t v : by_level[q]) {  // by_level lists nodes in increasing (preorder) id
      B.desc[v].w_off = woff;
      woff += m_of[v] - a_of[v];
      B.level_counts[q] += m_of[v] - a_of[v];
    }
  // scaling slots: children of each internal node are contiguous
  int64_t soff = 0;
  for (int32_t v = 0; v < nn; ++v) B.desc[v].scal_off = -1;
  for (int32_t v = 0; v < nn; ++v)
    if (!t.leaf(v)) {
      B.desc[t.left[v]].scal_off = soff;
      soff += a_of[t.left[v]];
      B.desc[t.right[v]].scal_off = soff;
      soff += a_of[t.right[v]];
    }
  B.scal_total = soff;
  int64_t voff = 0, hoff = 0;
  for (int32_t v = 0; v < nn; ++v) {
    NodeDesc& D = B.desc[v];
    D.m = m_of[v];
    D.a = a_of[v];
    D.leaf = t.leaf(v) ? 1 : 0;
    D.nref = std::min(m_of[v], p);
    D.in_off = t.leaf(v) ? t.begin[v] : B.desc[t.left[v]].scal_off;
    D.v_off = voff;
    voff += (int64_t)m_of[v] * m_of[v];
    D.h_off = hoff;
    hoff += (int64_t)Hblk[v].size();
  }
  B.V.resize((size_t)voff);
  B.H.resize((size_t)hoff);
  for (int32_t v = 0; v < nn; ++v) {
    std::copy(Vblk[v].begin(), Vblk[v].end(), B.V.begin() + B.desc[v].v_off);
    std::copy(Hblk[v].begin(), Hblk[v].end(), B.H.begin() + B.desc[v].h_off);
  }
  B.lvl_begin.assign(B.levels + 1, 0);
  B.level_nodes.clear();
  for (int q = 0; q < B.levels; ++q) {
    B.lvl_begin[q] = (int32_t)B.level_nodes.size();
    for (int32_t v : by_level[q]) B.level_nodes.push_back(v);
  }
  B.lvl_begin[B.levels] = (int32_t)B.level_nodes.size();
  if (woff != n - p) return fail(MLBLUP_ERANK, "build_multilevel_basis: wavelet count != N - p");
  return MLBLUP_OK;
}

}  // namespace mlb
