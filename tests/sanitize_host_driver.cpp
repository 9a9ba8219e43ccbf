// Driver of the address/undefined-behaviour sanitizer build of the host C++
// (kd-tree, multilevel basis, sparsity pattern, general-nu tables): builds
// trees and bases over ordinary, tied, collinear, tiny and high-dimensional
// point sets and walks every output array, so that an out-of-bounds index
// or an undefined operation anywhere in those sources stops the run.
// Compiled and run by tests/test_host_sanitizers.py.  Exit status 0 and the
// line "sanitize driver: ok" mean no finding.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "genu.h"
#include "internal.h"

namespace mlb {
int fail(int status, const std::string& msg) {
  std::fprintf(stderr, "  (status %d: %s)\n", status, msg.c_str());
  return status;
}
void clear_error() {}
}  // namespace mlb

static double g_sink = 0.0;

static int run_case(const char* name, std::vector<double> pts, int64_t n, int d, int leaf, int w, bool expect_ok) {
  mlb::Tree t;
  int st = mlb::build_tree(pts.data(), n, d, leaf, t);
  if (st != MLBLUP_OK) {
    std::printf("%s: build_tree status %d\n", name, st);
    return expect_ok ? 1 : 0;
  }
  for (int32_t v = 0; v < t.n_nodes(); ++v) g_sink += (double)(t.end[v] - t.begin[v]) + t.threshold[v];
  for (int64_t i = 0; i < n; ++i) g_sink += (double)t.perm[i];
  mlb::Basis b;
  st = mlb::build_basis(t, w, 1e-10, b);
  if (st != MLBLUP_OK) {
    std::printf("%s: build_basis status %d\n", name, st);
    return expect_ok ? 1 : 0;
  }
  for (double v : b.V) g_sink += v;
  for (const auto& D : b.desc) g_sink += (double)(D.in_off + D.w_off + D.v_off + D.m + D.a);
  // the compact WY form of every block: I - Y T Y^T equals V, and T's diagonal holds the reflectors'
  // scales (H_k h_k = -h_k, i.e. tau_k h_k.h_k = 2 for every reflector that is not the identity)
  double worst = 0.0;
  for (const auto& D : b.desc) {
    const int m = D.m, K = D.nref;
    if (m == 0) continue;
    if (K != std::min(m, b.p)) {
      std::printf("%s: node with m=%d has %d reflectors\n", name, m, K);
      return 1;
    }
    const double* Y = &b.H[(size_t)D.h_off];
    const double* T = Y + (size_t)K * m;
    for (int k = 0; k < K; ++k) {
      double hh = 0.0;
      for (int i = 0; i < m; ++i) hh += Y[(size_t)k * m + i] * Y[(size_t)k * m + i];
      const double tk = T[(size_t)k * K + k];
      if (tk != 0.0) worst = std::max(worst, std::fabs(tk * hh - 2.0));
      for (int r = k + 1; r < K; ++r) worst = std::max(worst, std::fabs(T[(size_t)r * K + k]));   // upper
    }
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        double s = i == j ? 1.0 : 0.0;
        for (int k = 0; k < K; ++k) {
          double tyj = 0.0;
          for (int l = 0; l < K; ++l) tyj += T[(size_t)k * K + l] * Y[(size_t)l * m + j];
          s -= Y[(size_t)k * m + i] * tyj;
        }
        worst = std::max(worst, std::fabs(s - b.V[(size_t)D.v_off + (size_t)i * m + j]));
      }
  }
  // the transform kernels' three steps (w = Y^T x, u = T^T w or T w, x - Y u, with their index
  // ranges) against V^T x and V x from the dense block
  for (const auto& D : b.desc) {
    const int m = D.m, K = D.nref;
    if (m == 0 || m > 256) continue;
    const double* Y = &b.H[(size_t)D.h_off];
    const double* T = Y + (size_t)K * m;
    std::vector<double> x(m), w(K), u(K);
    for (int i = 0; i < m; ++i) x[i] = std::sin(0.7 * i + 0.1 * D.v_off);
    for (int analysis = 0; analysis < 2; ++analysis) {
      const int G = K <= 64 ? 64 / K : 1;   // lanes sharing a row of Y in the kernel
      for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int g = 0; g < G; ++g) {
          double part = 0.0;
          for (int i = k + g; i < m; i += G) part += Y[(size_t)k * m + i] * x[i];
          s += part;
        }
        w[k] = s;
      }
      for (int k = 0; k < K; ++k) {
        double s = 0.0;
        if (analysis)
          for (int j = 0; j <= k; ++j) s += T[(size_t)j * K + k] * w[j];
        else
          for (int j = k; j < K; ++j) s += T[(size_t)k * K + j] * w[j];
        u[k] = s;
      }
      for (int i = 0; i < m; ++i) {
        double s = x[i];
        const int kmax = i < K ? i + 1 : K;
        for (int k = 0; k < kmax; ++k) s -= Y[(size_t)k * m + i] * u[k];
        double ref = 0.0;
        for (int j = 0; j < m; ++j)
          ref += (analysis ? b.V[(size_t)D.v_off + (size_t)j * m + i] : b.V[(size_t)D.v_off + (size_t)i * m + j]) * x[j];
        worst = std::max(worst, std::fabs(s - ref));
      }
    }
  }
  if (worst > 1e-12) {
    std::printf("%s: compact WY form differs from V by %g\n", name, worst);
    return 1;
  }
  for (int32_t level = 0; level < b.levels; ++level) {
    for (double tau : {0.0, 0.05, 0.2, 1e9}) {
      mlb::Pattern P;
      mlb::build_pattern(b, level, tau, P);
      g_sink += (double)P.nnz + (double)mlb::pattern_cells(b, level);
      for (uint8_t k : P.keep) g_sink += k;
    }
  }
  std::printf("%s: n=%lld d=%d p=%d levels=%d ok\n", name, (long long)n, d, b.p, b.levels);
  return expect_ok ? 0 : 1;
}

int main() {
  std::mt19937_64 g(1701);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  auto cloud = [&](int64_t n, int d) {
    std::vector<double> p((size_t)(n * d));
    for (auto& v : p) v = u(g);
    return p;
  };
  int bad = 0;
  bad += run_case("uniform d=2", cloud(1000, 2), 1000, 2, 32, 1, true);
  bad += run_case("uniform d=3 quadratic", cloud(4099, 3), 4099, 3, 64, 2, true);
  bad += run_case("uniform d=10 linear", cloud(777, 10), 777, 10, 64, 1, true);
  bad += run_case("uniform d=20 linear", cloud(1300, 20), 1300, 20, 64, 1, true);
  bad += run_case("unit square degree 8", cloud(200, 2), 200, 2, 64, 8, true);
  {
    // ties: coordinates on a coarse grid
    std::vector<double> p = cloud(600, 3);
    for (auto& v : p) v = std::floor(v * 4.0) / 4.0 + 0.001 * (&v - p.data()) / (double)p.size();
    bad += run_case("ties d=3", p, 600, 3, 16, 1, true);
  }
  {
    // one point per leaf
    bad += run_case("leaf 1", cloud(40, 2), 40, 2, 1, 0, true);
  }
  {
    // n equal to the leaf size: a single leaf
    bad += run_case("single leaf", cloud(64, 3), 64, 3, 64, 1, true);
  }
  {
    // collinear points: the linear trend in d = 2 has rank 2 < p = 3
    std::vector<double> p(2 * 300);
    for (int i = 0; i < 300; ++i) {
      const double s = u(g);
      p[2 * i] = s;
      p[2 * i + 1] = 2.0 * s;
    }
    bad += run_case("collinear (rank error expected)", p, 300, 2, 32, 1, false);
  }
  // general-nu tables and their evaluation over the whole range of s
  for (double nu : {0.3, 0.75, 1.0, 1.25, 2.0, 3.7, 7.5, 8.0}) {
    std::vector<double> tab;
    if (!mlb::genu_build(nu, tab)) {
      std::printf("genu_build(%g) failed\n", nu);
      ++bad;
      continue;
    }
    for (double s = 1e-300; s < 1e5; s = s * 1.7 + 1e-3) g_sink += mlb::genu_f(s, tab.data());
  }
  {
    std::vector<double> tab;
    if (mlb::genu_build(9.0, tab) || mlb::genu_build(0.0, tab)) {
      std::printf("genu_build accepted a nu out of range\n");
      ++bad;
    }
  }
  for (int d = 1; d <= 25; d += 3)
    for (int w = 0; w <= 3; ++w) g_sink += (double)mlb::td_exponents(d, w).size();
  if (!std::isfinite(g_sink)) std::printf("non-finite checksum\n");
  std::printf("sanitize driver: %s\n", bad ? "FAILED" : "ok");
  return bad ? 1 : 0;
}
