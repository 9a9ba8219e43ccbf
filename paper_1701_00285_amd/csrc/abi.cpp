// C ABI entry points and the host drivers of the solve (Sec. 6.2 predictor
// iteration; Sec. 5.2 eqs. Spatial:eqn2-3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "device.h"
#include "genu.h"
#include "internal.h"
#include "precond.h"


namespace mlb {

namespace {
thread_local std::string g_err;
}

int fail(int status, const std::string& msg) {
  g_err = msg;
  return status;
}
void clear_error() { g_err.clear(); }

namespace {

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

int nu2_of_nu(double nu) {
  if (std::isinf(nu) && nu > 0) return 0;
  const double n2 = 2.0 * nu;
  for (int c : {1, 3, 5})
    if (std::fabs(n2 - c) < 1e-12) return c;
  if (nu > 0.0 && nu <= 8.0) return kNuGeneral;
  return -1;
}

// Device view of the multilevel transform of an uploaded basis.
TransformDev transform_dev(const Basis& B) {
  const char* img = (const char*)B.dev_base;
  TransformDev T;
  T.desc = (const NodeDesc*)(img + B.off_desc);
  T.level_nodes = (const int32_t*)(img + B.off_levels);
  T.lvl_begin_host = B.lvl_begin.data();
  T.levels = B.levels;
  T.V = (const double*)(img + B.off_V);
  T.H = (const double*)(img + B.off_H);
  T.children = (const int32_t*)(img + B.off_children);
  T.n_nodes = (int32_t)B.desc.size();
  return T;
}

namespace {

// progress log of long solves: MLBLUP_LOG_EVERY=k prints the residual every k iterations to stderr
int log_every() {
  static const int k = [] {
    const char* e = std::getenv("MLBLUP_LOG_EVERY");
    return e ? std::atoi(e) : 0;
  }();
  return k;
}

int nu2_of(const mlblup_matern* k) { return k ? nu2_of_nu(k->nu) : -1; }

int check_kernel(const mlblup_matern* k) {
  if (!k) return fail(MLBLUP_EINVAL, "NULL covariance parameters");
  if (nu2_of(k) == -1) return fail(MLBLUP_EINVAL, "nu must be in (0, 8] or +inf (Gaussian)");
  if (!(k->rho > 0) || !std::isfinite(k->rho)) return fail(MLBLUP_EINVAL, "rho must be finite and > 0");
  if (!(k->sigma2 > 0) || !std::isfinite(k->sigma2)) return fail(MLBLUP_EINVAL, "sigma2 must be finite and > 0");
  return MLBLUP_OK;
}

// Coefficients of x^g in prod_k (s x_k + b_k)^(a_k):  S[a][g] = prod_k C(a_k, g_k) s^g_k b_k^(a_k - g_k)
std::vector<double> shift_matrix(const std::vector<std::vector<int32_t>>& E, double s, const std::vector<double>& b) {
  const int p = (int)E.size(), d = (int)b.size();
  auto binom = [](int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
  };
  std::vector<double> S((size_t)p * p, 0.0);
  for (int a = 0; a < p; ++a)
    for (int g = 0; g < p; ++g) {
      double t = 1.0;
      for (int k = 0; k < d; ++k) {
        const int A = E[a][k], G = E[g][k];
        if (G > A) {
          t = 0.0;
          break;
        }
        t *= binom(A, G) * std::pow(s, G) * std::pow(b[k], A - G);
      }
      S[(size_t)a * p + g] = t;
    }
  return S;
}

// Solve A x = y (p x p row-major) by Gaussian elimination with partial pivoting.
bool dense_solve(std::vector<double> A, std::vector<double>& y, int p) {
  for (int k = 0; k < p; ++k) {
    int piv = k;
    for (int i = k + 1; i < p; ++i)
      if (std::fabs(A[(size_t)i * p + k]) > std::fabs(A[(size_t)piv * p + k])) piv = i;
    if (A[(size_t)piv * p + k] == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < p; ++j) std::swap(A[(size_t)k * p + j], A[(size_t)piv * p + j]);
      std::swap(y[k], y[piv]);
    }
    for (int i = k + 1; i < p; ++i) {
      const double f = A[(size_t)i * p + k] / A[(size_t)k * p + k];
      for (int j = k; j < p; ++j) A[(size_t)i * p + j] -= f * A[(size_t)k * p + j];
      y[i] -= f * y[k];
    }
  }
  for (int k = p - 1; k >= 0; --k) {
    double s = y[k];
    for (int j = k + 1; j < p; ++j) s -= A[(size_t)k * p + j] * y[j];
    y[k] = s / A[(size_t)k * p + k];
  }
  return true;
}

// Layout of the device image written by mlblup_basis_upload.
void image_layout(Basis& B) {
  const int64_t nn = (int64_t)B.desc.size();
  const int64_t nv = (int64_t)B.V.size();
  int64_t off = 0;
  B.off_desc = off;
  off = align_up(off + nn * (int64_t)sizeof(NodeDesc));
  B.off_levels = off;
  off = align_up(off + nn * (int64_t)sizeof(int32_t));
  B.off_exps = off;
  off = align_up(off + (int64_t)B.p * B.d * (int64_t)sizeof(int32_t));
  B.off_rootc = off;
  off = align_up(off + B.d * (int64_t)sizeof(double));
  B.off_V = off;
  off = align_up(off + nv * (int64_t)sizeof(double));
  B.off_H = off;
  off = align_up(off + (int64_t)B.H.size() * (int64_t)sizeof(double));
  B.off_pts = off;
  off = align_up(off + B.n * B.d * (int64_t)sizeof(double));
  B.off_children = off;
  off = align_up(off + 2 * nn * (int64_t)sizeof(int32_t));
  B.dev_bytes = off;
}


// Workspace of the solve/predict/grad drivers.
struct Ws {
  int64_t r, p, q, z, dx, r2, p2, q2, z2, sc2, a, b, scal, part, sc, cov, zw, v, vw, lv, beta, gam, gamw, total;
  int64_t cov_bytes;
};

Ws ws_layout(const Basis& B, int64_t mt) {
  Ws w{};
  const int64_t N = B.n, nw = B.n - B.p, D = sizeof(double);
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  w.r = take(nw * D);
  w.p = take(nw * D);
  w.q = take(nw * D);
  w.z = take(nw * D);
  w.dx = take(nw * D);
  w.r2 = take(nw * D);
  w.p2 = take(nw * D);
  w.q2 = take(nw * D);
  w.z2 = take(nw * D);
  w.sc2 = take(S_COUNT * D);
  w.a = take(N * D);
  w.b = take(N * D);
  w.scal = take(std::max<int64_t>(B.scal_total, 1) * D);
  w.part = take(2 * kRedBlocks * D);
  w.sc = take(S_COUNT * D);
  int64_t cb = 0;
  for (int prec = MLBLUP_FP64; prec <= MLBLUP_MFMA_BF16X3; ++prec) {
    cb = std::max(cb, pair_workspace_bytes(N, N, B.d, prec, 3));
    if (mt > 0) cb = std::max(cb, pair_workspace_bytes(mt, N, B.d, prec, 3));
  }
  w.cov_bytes = std::max<int64_t>(cb, kAlign);
  w.cov = take(w.cov_bytes);
  w.zw = take(nw * D);
  w.v = take(N * D);
  w.vw = take(nw * D);
  w.lv = take(B.p * D);
  w.beta = take(B.p * D);
  w.gam = take(N * D);
  w.gamw = take(nw * D);
  w.total = off;
  return w;
}

struct Ctx {
  const Basis& B;
  hipStream_t s;
  char* base;
  Ws w;
  TransformDev T;
  const double* pts;
  mlblup_matern k;
  int nu2;
  double sc_host[S_COUNT];

  double* at(int64_t off) const { return (double*)(base + off); }

  Ctx(const Basis& b, const mlblup_matern& km, void* work, const Ws& ws, hipStream_t st)
      : B(b), s(st), base((char*)work), w(ws), k(km) {
    const char* img = (const char*)B.dev_base;
    T = transform_dev(B);
    pts = (const double*)(img + B.off_pts);
    nu2 = nu2_of(&km);
  }

  int pair(const double* rows, int64_t m, const double* x, double* y, double* dy, int prec, int outputs) {
    PairArgs a{rows, m, pts, B.n, B.d, nu2, k.rho, k.sigma2, prec, outputs, x, y, dy, k.nu, nullptr};
    return pair_launch(a, at(w.cov), w.cov_bytes, s);
  }

  // out = W C W^T in  (N - p vectors)
  int matvec_cw(const double* in, double* out, int prec) {
    int st = transform_synthesis(T, in, nullptr, at(w.a), at(w.scal), s);
    if (st) return st;
    st = pair(pts, B.n, at(w.a), at(w.b), nullptr, prec, MLBLUP_VALUE);
    if (st) return st;
    return transform_analysis(T, at(w.b), out, nullptr, at(w.scal), s);
  }

  int read_scalars(const double* sc) {
    MLB_HIP(hipMemcpyAsync(sc_host, sc, sizeof(sc_host), hipMemcpyDeviceToHost, s));
    MLB_HIP(hipStreamSynchronize(s));
    return MLBLUP_OK;
  }

  // |a|_2 read back to the host
  int norm(const double* a, int64_t n, double* out) {
    int st = vec_dot(a, a, n, at(w.part), at(w.sc) + S_DOT, s);
    if (st) return st;
    st = read_scalars(at(w.sc));
    if (st) return st;
    *out = std::sqrt(sc_host[S_DOT]);
    return MLBLUP_OK;
  }

  int dot(const double* a, const double* b, int64_t n, double* out) {
    int st = vec_dot(a, b, n, at(w.part), at(w.sc) + S_DOT, s);
    if (st) return st;
    st = read_scalars(at(w.sc));
    if (st) return st;
    *out = sc_host[S_DOT];
    return MLBLUP_OK;
  }

  // PCG on C_W d = rhs from d = 0 with the pair kernel in precision `prec`.
  // Vectors r, p, q, z and scalars sc are this loop's own; stops when the
  // recurrence residual drops to tol_abs or the iteration budget is spent.
  // history: record |r_k| / bnorm per iteration (plain FP64 solve only).
  int inner_pcg(const double* rhs, double* d, double tol_abs, int prec, const Precond* pc, int& iters_left,
                const mlblup_pcg_opts& o, mlblup_pcg_info& info, double bnorm, bool history, bool resume = false) {
    const int64_t nw = B.n - B.p;
    double* r = at(w.r);
    double* p = at(w.p);
    double* q = at(w.q);
    double* z = at(w.z);
    double* sc = at(w.sc);
    int st;
    // Krylov state of the FP64 recurrence kept for a later call: r, p and r.z
    double* state = (prec == MLBLUP_FP64) ? o.state_dev : nullptr;
    auto save_state = [&]() -> int {
      if (!state) return MLBLUP_OK;
      int e;
      if ((e = vec_copy(r, state, nw, s))) return e;
      if ((e = vec_copy(p, state + nw, nw, s))) return e;
      return hip_check(hipMemcpyAsync(state + 2 * nw, sc + S_RZ, sizeof(double), hipMemcpyDeviceToDevice, s),
                       "state copy");
    };
    if ((st = vec_zero(d, nw, s))) return st;
    const double* zz = r;
    if (pc) zz = z;
    if (state && resume) {
      if ((st = vec_copy(state, r, nw, s))) return st;
      if ((st = vec_copy(state + nw, p, nw, s))) return st;
      MLB_HIP(hipMemcpyAsync(sc + S_RZ, state + 2 * nw, sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
      if ((st = vec_copy(rhs, r, nw, s))) return st;
      if (pc && (st = precond_apply(*pc, r, z, s))) return st;
      if ((st = vec_copy(zz, p, nw, s))) return st;
      if ((st = pcg_start(r, zz, nw, at(w.part), sc, s))) return st;
    }
    while (iters_left > 0) {
      if ((st = matvec_cw(p, q, prec))) return st;
      if (prec == MLBLUP_FP64) info.fp64_matvecs++;
      else info.lowp_matvecs++;
      if ((st = pcg_alpha(p, q, nw, at(w.part), sc, s))) return st;
      if ((st = pcg_update_xr(d, r, p, q, nw, at(w.part), sc, s))) return st;
      if (pc) {
        if ((st = precond_apply(*pc, r, z, s))) return st;
        if ((st = pcg_rz_partial(r, z, nw, at(w.part), s))) return st;
      }
      if ((st = pcg_finish_beta(at(w.part), pc != nullptr, sc, s))) return st;
      if ((st = read_scalars(sc))) return st;
      --iters_left;
      if (history && o.history_host && info.inner_iters < o.history_cap)
        o.history_host[info.inner_iters] = std::sqrt(sc_host[S_RR]) / bnorm;
      info.inner_iters++;
      if (log_every() > 0 && info.inner_iters % log_every() == 0) {
        std::fprintf(stderr, "mlblup: iteration %d (precision %d) relres %.3e\n", info.inner_iters, prec,
                     std::sqrt(sc_host[S_RR]) / bnorm);
        std::fflush(stderr);
      }
      if (sc_host[S_FLAG] != 0.0) return fail(MLBLUP_EBREAKDOWN, "pcg_solve: breakdown (p.q <= 0 or non-finite scalar)");
      if (std::sqrt(sc_host[S_RR]) <= tol_abs) break;
      if ((st = pcg_update_p(p, zz, nw, sc, s))) return st;
    }
    return save_state();
  }

  // Reduced precision, reliable updates (G. L. G. Sleijpen and H. A. van der
  // Vorst, "Reliable updated residuals in hybrid Bi-CG methods", Computing
  // 56, 1996): one PCG recurrence whose products use the reduced-precision
  // pair kernel, with x, r, p and every dot in FP64.  When the recurred
  // residual has fallen by the factor delta since the last true residual,
  // or below the target, zw - C_W x is formed with the FP64 product and
  // replaces it; the search direction is kept and beta is taken from the
  // replaced residual, so the recurrence is never restarted.  On entry r2
  // holds the true residual of x, of norm rnorm.
  int reliable_pcg(const double* zw, double* x, double rnorm, double bnorm, const Precond* pc, int iters_left,
                   const mlblup_pcg_opts& o, mlblup_pcg_info& info) {
    const int64_t nw = B.n - B.p;
    const int prec = o.precision;
    const double delta = o.inner_rtol > 0 ? o.inner_rtol : 1e-2;
    const double tol = o.rtol * bnorm;
    double* r = at(w.r2);
    double* p = at(w.p);
    double* q = at(w.q);
    double* z = at(w.z);
    double* sc = at(w.sc);
    double* part = at(w.part);
    int st;
    const double* zz = r;
    if (pc) {
      if ((st = precond_apply(*pc, r, z, s))) return st;
      zz = z;
    }
    if ((st = vec_copy(zz, p, nw, s))) return st;
    if ((st = pcg_start(r, zz, nw, part, sc, s))) return st;
    if ((st = read_scalars(sc))) return st;
    double rz_prev = sc_host[S_RZ];
    double rcheck = rnorm;  // norm of the last true residual
    info.relres_fp64 = rnorm / bnorm;
    for (;;) {
      if (iters_left <= 0) return fail(MLBLUP_ENOCONV, "pcg_solve: tolerance not reached (relres " +
                                                           std::to_string(info.relres_fp64) + ")");
      if ((st = matvec_cw(p, q, prec))) return st;
      info.lowp_matvecs++;
      if ((st = pcg_alpha(p, q, nw, part, sc, s))) return st;
      if ((st = pcg_update_xr(x, r, p, q, nw, part, sc, s))) return st;
      if (pc) {
        if ((st = precond_apply(*pc, r, z, s))) return st;
        if ((st = pcg_rz_partial(r, z, nw, part, s))) return st;
      }
      if ((st = pcg_finish_beta(part, pc != nullptr, sc, s))) return st;
      if ((st = read_scalars(sc))) return st;
      --iters_left;
      const double rr = std::sqrt(sc_host[S_RR]);
      if (o.history_host && info.inner_iters < o.history_cap) o.history_host[info.inner_iters] = rr / bnorm;
      info.inner_iters++;
      if (log_every() > 0 && info.inner_iters % log_every() == 0) {
        std::fprintf(stderr, "mlblup: iteration %d (precision %d, reliable) relres %.3e\n", info.inner_iters, prec,
                     rr / bnorm);
        std::fflush(stderr);
      }
      if (sc_host[S_FLAG] != 0.0) return fail(MLBLUP_EBREAKDOWN, "pcg_solve: breakdown (p.q <= 0 or non-finite scalar)");
      if (rr <= tol || rr <= delta * rcheck) {
        // replace the recurred residual by the true one
        if ((st = true_residual(zw, x, r, &rnorm, info))) return st;
        info.outer_iters++;
        info.relres_fp64 = rnorm / bnorm;
        if (!std::isfinite(rnorm)) return fail(MLBLUP_EBREAKDOWN, "pcg_solve: non-finite residual");
        if (rnorm <= tol) return MLBLUP_OK;
        if (info.outer_iters >= o.refine_max)
          return fail(MLBLUP_ENOCONV, "pcg_solve: tolerance not reached after " + std::to_string(o.refine_max) +
                                          " residual replacements (relres " + std::to_string(info.relres_fp64) + ")");
        rcheck = rnorm;
        if ((st = pcg_rr_partial(r, nw, part, s))) return st;
        if (pc) {
          if ((st = precond_apply(*pc, r, z, s))) return st;
          if ((st = pcg_rz_partial(r, z, nw, part, s))) return st;
        }
        if ((st = pcg_finish_beta_from(part, pc != nullptr, rz_prev, sc, s))) return st;
        if ((st = read_scalars(sc))) return st;
      }
      rz_prev = sc_host[S_RZ];
      if ((st = pcg_update_p(p, zz, nw, sc, s))) return st;
    }
  }

  // true residual r_out = zw - C_W x (FP64 product); returns |r_out|
  int true_residual(const double* zw, const double* x, double* r_out, double* rnorm, mlblup_pcg_info& info) {
    const int64_t nw = B.n - B.p;
    int st;
    if ((st = matvec_cw(x, r_out, MLBLUP_FP64))) return st;
    info.fp64_matvecs++;
    if ((st = vec_sub_from(zw, r_out, nw, s))) return st;
    return norm(r_out, nw, rnorm);
  }

  // Solve C_W x = zw to |zw - C_W x| <= rtol |zw| (FP64 product, unpreconditioned
  // residual).  FP64: PCG, then the true residual; if rounding drift left it
  // above rtol, PCG restarts from x on the true residual.  Reduced
  // precision: flexible CG in FP64 (FP64 products, vectors and dots) whose
  // preconditioner is an inner PCG solve with the reduced-precision pair
  // kernel to relative tolerance inner_rtol -- a Krylov-accelerated
  // iterative refinement; the FP64 recurrence residual is confirmed by a
  // true residual at the end.
  // floor_abs: a right-hand side with |zw| <= floor_abs is treated as zero
  // (data in the trend space up to rounding: gamma_W = 0).
  int solve(const double* zw, double* x, bool use_x0, const mlblup_pcg_opts& o, mlblup_pcg_info& info,
            double floor_abs = 0.0) {
    const int64_t nw = B.n - B.p;
    info = mlblup_pcg_info{};
    double bnorm = 0.0;
    int st = norm(zw, nw, &bnorm);
    if (st) return st;
    if (!std::isfinite(bnorm)) return fail(MLBLUP_EINVAL, "pcg_solve: non-finite right-hand side");
    info.zw_norm = bnorm;
    if (bnorm <= floor_abs) {
      info.relres_fp64 = 0.0;
      return vec_zero(x, nw, s);
    }
    if (!use_x0 && (st = vec_zero(x, nw, s))) return st;
    const int prec = o.precision;
    const Precond* pc = o.precond ? &o.precond->p : nullptr;
    if (pc && (!pc->uploaded || pc->nw != nw))
      return fail(MLBLUP_ESTATE, "pcg_solve: preconditioner not uploaded or of another basis");
    int iters_left = o.max_iter;
    double* r2 = at(w.r2);
    double* p2 = at(w.p2);
    double* q2 = at(w.q2);
    double* z2 = at(w.z2);
    double* sc2 = at(w.sc2);
    double rnorm = bnorm;
    if (use_x0) {
      if ((st = true_residual(zw, x, r2, &rnorm, info))) return st;
    } else if ((st = vec_copy(zw, r2, nw, s))) {
      return st;
    }
    auto noconv = [&](double rel) {
      return fail(MLBLUP_ENOCONV, "pcg_solve: tolerance not reached (relres " + std::to_string(rel) + ")");
    };
    if (prec == MLBLUP_FP64) {
      for (int outer = 0;; ++outer) {
        const double relres = rnorm / bnorm;
        info.relres_fp64 = relres;
        if (!std::isfinite(relres)) return fail(MLBLUP_EBREAKDOWN, "pcg_solve: non-finite residual");
        if (relres <= o.rtol) return MLBLUP_OK;
        if (outer >= std::max(o.refine_max, 1) || iters_left <= 0) return noconv(relres);
        info.outer_iters++;
        // the first inner solve continues a stored recurrence when asked to
        st = inner_pcg(r2, z2, 0.7 * o.rtol * bnorm, MLBLUP_FP64, pc, iters_left, o, info, bnorm, true,
                       o.resume != 0 && outer == 0);
        const int st2 = vec_axpy(1.0, z2, x, nw, s);  // keep the progress even on breakdown
        if (st) return st;
        if (st2) return st2;
        if ((st = true_residual(zw, x, r2, &rnorm, info))) return st;
      }
    }
    if (o.mixed_scheme == MLBLUP_MIXED_RELIABLE) {
      info.relres_fp64 = rnorm / bnorm;
      if (rnorm <= o.rtol * bnorm) return MLBLUP_OK;
      return reliable_pcg(zw, x, rnorm, bnorm, pc, iters_left, o, info);
    }
    // flexible CG outer loop (FP64), reduced-precision inner solves
    const double inner = o.inner_rtol > 0 ? o.inner_rtol : 1e-2;
    const int max_outer = std::max(o.refine_max, 1);
    for (int k = 0;; ++k) {
      double relres = rnorm / bnorm;
      info.relres_fp64 = relres;
      if (!std::isfinite(relres)) return fail(MLBLUP_EBREAKDOWN, "pcg_solve: non-finite residual");
      if (relres <= o.rtol) {
        // confirm with the true FP64 residual; on drift restart the directions
        if ((st = true_residual(zw, x, r2, &rnorm, info))) return st;
        relres = rnorm / bnorm;
        info.relres_fp64 = relres;
        if (relres <= o.rtol) return MLBLUP_OK;
        k = 0;
      }
      if (info.outer_iters >= max_outer || iters_left <= 0) return noconv(relres);
      info.outer_iters++;
      if ((st = inner_pcg(r2, z2, inner * rnorm, prec, pc, iters_left, o, info, bnorm, false))) return st;
      if (o.history_host && info.outer_iters - 1 < o.history_cap) o.history_host[info.outer_iters - 1] = relres;
      if (k == 0) {
        if ((st = vec_copy(z2, p2, nw, s))) return st;
      } else {
        if ((st = vec_dot(z2, q2, nw, at(w.part), sc2 + S_DOT, s))) return st;  // q2 = C_W p_prev
        if ((st = fcg_update_p(p2, z2, nw, sc2, s))) return st;
      }
      if ((st = matvec_cw(p2, q2, MLBLUP_FP64))) return st;
      info.fp64_matvecs++;
      if ((st = pcg_start(r2, p2, nw, at(w.part), sc2, s))) return st;  // sc2[RZ] = r . p
      if ((st = pcg_alpha(p2, q2, nw, at(w.part), sc2, s))) return st;
      if ((st = pcg_update_xr(x, r2, p2, q2, nw, at(w.part), sc2, s))) return st;
      if ((st = pcg_finish_beta(at(w.part), false, sc2, s))) return st;
      if ((st = read_scalars(sc2))) return st;
      if (sc_host[S_FLAG] != 0.0) return fail(MLBLUP_EBREAKDOWN, "pcg_solve: breakdown in the outer iteration");
      rnorm = std::sqrt(sc_host[S_RR]);
    }
  }
};

int check_basis_dev(const mlblup_basis b) {
  if (!b) return fail(MLBLUP_EINVAL, "NULL basis");
  if (!b->b.uploaded) return fail(MLBLUP_ESTATE, "basis not uploaded (call mlblup_basis_upload first)");
  return MLBLUP_OK;
}

int check_ws(const mlblup_basis b, int64_t mt, void* work, int64_t bytes, Ws* out) {
  *out = ws_layout(b->b, mt);
  if (!work || bytes < out->total)
    return fail(MLBLUP_EINVAL, "workspace too small (need " + std::to_string(out->total) + " bytes)");
  if (((uintptr_t)work) % kAlign) return fail(MLBLUP_EINVAL, "workspace must be 256-byte aligned");
  return MLBLUP_OK;
}

mlblup_pcg_opts default_opts() {
  mlblup_pcg_opts o{};
  o.rtol = 1e-8;
  o.max_iter = 1000;
  o.precision = MLBLUP_FP64;
  o.refine_max = 200;
  o.inner_rtol = 1e-2;
  o.precond = nullptr;
  o.history_cap = 0;
  o.history_host = nullptr;
  o.mixed_scheme = MLBLUP_MIXED_FLEXIBLE;
  o.state_dev = nullptr;
  o.resume = 0;
  return o;
}

}  // namespace
}  // namespace mlb

using namespace mlb;

extern "C" {

const char* mlblup_last_error(void) { return g_err.c_str(); }
int32_t mlblup_version(void) { return 100; }

int mlblup_build_tree(const double* pts_host, int64_t n, int32_t d, int32_t leaf_max, mlblup_tree* out) {
  clear_error();
  if (!out) return fail(MLBLUP_EINVAL, "build_tree: out is NULL");
  *out = nullptr;
  std::unique_ptr<mlblup_tree_s> t(new (std::nothrow) mlblup_tree_s);
  if (!t) return fail(MLBLUP_EINVAL, "build_tree: out of host memory");
  const int st = build_tree(pts_host, n, d, leaf_max, t->t);
  if (st) return st;
  *out = t.release();
  return MLBLUP_OK;
}

int mlblup_tree_info(mlblup_tree t, int64_t* n, int32_t* d, int32_t* n_nodes, int32_t* max_depth) {
  clear_error();
  if (!t) return fail(MLBLUP_EINVAL, "NULL tree");
  if (n) *n = t->t.n;
  if (d) *d = t->t.d;
  if (n_nodes) *n_nodes = t->t.n_nodes();
  if (max_depth) *max_depth = t->t.max_depth;
  return MLBLUP_OK;
}

int mlblup_tree_perm(mlblup_tree t, int64_t* perm_host) {
  clear_error();
  if (!t || !perm_host) return fail(MLBLUP_EINVAL, "NULL argument");
  std::memcpy(perm_host, t->t.perm.data(), t->t.perm.size() * sizeof(int64_t));
  return MLBLUP_OK;
}

int mlblup_tree_nodes(mlblup_tree t, int64_t* begin, int64_t* end, int32_t* depth, int32_t* axis, int32_t* left,
                      int32_t* right, double* threshold) {
  clear_error();
  if (!t) return fail(MLBLUP_EINVAL, "NULL tree");
  const Tree& T = t->t;
  const size_t nn = T.begin.size();
  if (begin) std::memcpy(begin, T.begin.data(), nn * sizeof(int64_t));
  if (end) std::memcpy(end, T.end.data(), nn * sizeof(int64_t));
  if (depth) std::memcpy(depth, T.depth.data(), nn * sizeof(int32_t));
  if (axis) std::memcpy(axis, T.axis.data(), nn * sizeof(int32_t));
  if (left) std::memcpy(left, T.left.data(), nn * sizeof(int32_t));
  if (right) std::memcpy(right, T.right.data(), nn * sizeof(int32_t));
  if (threshold) std::memcpy(threshold, T.threshold.data(), nn * sizeof(double));
  return MLBLUP_OK;
}

void mlblup_tree_free(mlblup_tree t) { delete t; }

int mlblup_build_multilevel_basis(mlblup_tree t, int32_t degree_w, double rank_rtol, mlblup_basis* out) {
  clear_error();
  if (!t || !out) return fail(MLBLUP_EINVAL, "NULL argument");
  *out = nullptr;
  std::unique_ptr<mlblup_basis_s> b(new (std::nothrow) mlblup_basis_s);
  if (!b) return fail(MLBLUP_EINVAL, "out of host memory");
  const int st = build_basis(t->t, degree_w, rank_rtol, b->b);
  if (st) return st;
  image_layout(b->b);
  *out = b.release();
  return MLBLUP_OK;
}

int mlblup_basis_info(mlblup_basis b, int32_t* p, int32_t* levels, int64_t* n_minus_p, int64_t* device_bytes) {
  clear_error();
  if (!b) return fail(MLBLUP_EINVAL, "NULL basis");
  if (p) *p = b->b.p;
  if (levels) *levels = b->b.levels;
  if (n_minus_p) *n_minus_p = b->b.n - b->b.p;
  if (device_bytes) *device_bytes = b->b.dev_bytes;
  return MLBLUP_OK;
}

int mlblup_basis_transform_bytes(mlblup_basis b, int64_t* bytes) {
  clear_error();
  if (!b || !bytes) return fail(MLBLUP_EINVAL, "NULL argument");
  int64_t s = 0;
  for (const auto& nd : b->b.desc) s += transform_node_doubles(nd);
  *bytes = 8 * s + 16 * b->b.n;
  return MLBLUP_OK;
}

int mlblup_basis_level_counts(mlblup_basis b, int64_t* counts_host) {
  clear_error();
  if (!b || !counts_host) return fail(MLBLUP_EINVAL, "NULL argument");
  std::memcpy(counts_host, b->b.level_counts.data(), b->b.level_counts.size() * sizeof(int64_t));
  return MLBLUP_OK;
}

int mlblup_basis_dense(mlblup_basis bb, double* W_host, double* L_host) {
  clear_error();
  if (!bb) return fail(MLBLUP_EINVAL, "NULL basis");
  const Basis& B = bb->b;
  const int64_t N = B.n;
  if (W_host) std::fill(W_host, W_host + (size_t)(N - B.p) * N, 0.0);
  // Expand every cell's vectors bottom-up as dense columns over the cell's
  // point range [begin, end): candidates times the cell's orthogonal block.
  const int32_t nn = (int32_t)B.desc.size();
  std::vector<std::vector<double>> scal(nn);  // (end-begin) x a, row-major
  for (int q = B.levels - 1; q >= 0; --q)
    for (int32_t s = B.lvl_begin[q]; s < B.lvl_begin[q + 1]; ++s) {
      const int32_t v = B.level_nodes[s];
      const NodeDesc& D = B.desc[v];
      const int64_t lo = B.begin[v], len = B.end[v] - B.begin[v];
      std::vector<double> cand((size_t)len * D.m, 0.0);
      if (D.leaf) {
        for (int i = 0; i < D.m; ++i) cand[(size_t)i * D.m + i] = 1.0;
      } else {
        int col = 0;
        for (int32_t c : {B.left[v], B.right[v]}) {
          const int ac = B.desc[c].a;
          for (int64_t i = 0; i < B.end[c] - B.begin[c]; ++i)
            for (int j = 0; j < ac; ++j)
              cand[(size_t)(B.begin[c] - lo + i) * D.m + col + j] = scal[c][(size_t)i * ac + j];
          col += ac;
          std::vector<double>().swap(scal[c]);
        }
      }
      const double* Vb = &B.V[D.v_off];
      std::vector<double> out((size_t)len * D.m, 0.0);
      for (int64_t i = 0; i < len; ++i)
        for (int kk = 0; kk < D.m; ++kk) {
          const double c = cand[(size_t)i * D.m + kk];
          if (c == 0.0) continue;
          for (int j = 0; j < D.m; ++j) out[(size_t)i * D.m + j] += c * Vb[(size_t)kk * D.m + j];
        }
      scal[v].assign((size_t)len * D.a, 0.0);
      for (int64_t i = 0; i < len; ++i)
        for (int j = 0; j < D.m; ++j) {
          const double val = out[(size_t)i * D.m + j];
          if (j < D.a) scal[v][(size_t)i * D.a + j] = val;
          else if (W_host) W_host[(size_t)(D.w_off + j - D.a) * N + lo + i] = val;
        }
    }
  if (L_host)
    for (int j = 0; j < B.p; ++j)
      for (int64_t i = 0; i < N; ++i) L_host[(size_t)j * N + i] = scal[0][(size_t)i * B.p + j];
  return MLBLUP_OK;
}

int mlblup_basis_upload(mlblup_basis bb, void* dev_buf, int64_t bytes, void* stream) {
  clear_error();
  if (!bb || !dev_buf) return fail(MLBLUP_EINVAL, "NULL argument");
  Basis& B = bb->b;
  if (bytes < B.dev_bytes)
    return fail(MLBLUP_EINVAL, "basis_upload: buffer too small (need " + std::to_string(B.dev_bytes) + ")");
  if (((uintptr_t)dev_buf) % kAlign) return fail(MLBLUP_EINVAL, "basis_upload: buffer must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)dev_buf;
  const int32_t nn = (int32_t)B.desc.size();
  MLB_HIP(hipMemcpyAsync(base + B.off_desc, B.desc.data(), nn * sizeof(NodeDesc), hipMemcpyHostToDevice, s));
  MLB_HIP(hipMemcpyAsync(base + B.off_levels, B.level_nodes.data(), nn * sizeof(int32_t), hipMemcpyHostToDevice, s));
  std::vector<int32_t> ex((size_t)B.p * B.d);
  for (int b = 0; b < B.p; ++b)
    for (int k = 0; k < B.d; ++k) ex[(size_t)b * B.d + k] = B.exps[b][k];
  MLB_HIP(hipMemcpyAsync(base + B.off_exps, ex.data(), ex.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  MLB_HIP(hipMemcpyAsync(base + B.off_rootc, B.root_c.data(), B.d * sizeof(double), hipMemcpyHostToDevice, s));
  MLB_HIP(hipMemcpyAsync(base + B.off_V, B.V.data(), B.V.size() * sizeof(double), hipMemcpyHostToDevice, s));
  MLB_HIP(hipMemcpyAsync(base + B.off_H, B.H.data(), B.H.size() * sizeof(double), hipMemcpyHostToDevice, s));
  MLB_HIP(hipMemcpyAsync(base + B.off_pts, B.pts_tree.data(), B.pts_tree.size() * sizeof(double),
                         hipMemcpyHostToDevice, s));
  MLB_HIP(hipMemcpyAsync(base + B.off_children, B.left.data(), nn * sizeof(int32_t), hipMemcpyHostToDevice, s));
  MLB_HIP(hipMemcpyAsync(base + B.off_children + nn * sizeof(int32_t), B.right.data(), nn * sizeof(int32_t),
                         hipMemcpyHostToDevice, s));
  MLB_HIP(hipStreamSynchronize(s));  // host staging buffers die here
  B.dev_base = dev_buf;
  B.uploaded = true;
  return MLBLUP_OK;
}

int mlblup_basis_points_dev(mlblup_basis b, const double** pts_dev) {
  clear_error();
  const int st = check_basis_dev(b);
  if (st) return st;
  if (!pts_dev) return fail(MLBLUP_EINVAL, "NULL argument");
  *pts_dev = (const double*)((const char*)b->b.dev_base + b->b.off_pts);
  return MLBLUP_OK;
}

void mlblup_basis_free(mlblup_basis b) { delete b; }

int mlblup_cov_workspace_bytes(int64_t m, int64_t n, int32_t d, int32_t precision, int32_t outputs, int64_t* bytes) {
  clear_error();
  if (!bytes || m < 0 || n < 0 || d < 1 || d > 64 || outputs < 1 || outputs > 3)
    return fail(MLBLUP_EINVAL, "cov_workspace_bytes: bad argument");
  *bytes = pair_workspace_bytes(m, n, d, precision, outputs);
  return MLBLUP_OK;
}

int mlblup_matern_host(const mlblup_matern* k, const double* r_host, int64_t n, double* phi_host) {
  clear_error();
  int st = check_kernel(k);
  if (st) return st;
  if (n < 0 || (n > 0 && (!r_host || !phi_host))) return fail(MLBLUP_EINVAL, "matern_host: bad arguments");
  const int nu2 = nu2_of(k);
  const double* tab = nu2 == kNuGeneral ? genu_table_cached(k->nu) : nullptr;
  if (nu2 == kNuGeneral && !tab) return fail(MLBLUP_EINVAL, "matern_host: nu out of range");
  const double zs = kernel_scale(nu2, k->nu, k->rho);
  for (int64_t i = 0; i < n; ++i) {
    const double z = r_host[i] * zs;
    double f;
    if (nu2 == kNuGeneral) f = genu_f(z * z + 1e-300, tab);
    else if (nu2 == 0) f = std::exp(-0.5 * z * z);
    else if (nu2 == 1) f = std::exp(-z);
    else if (nu2 == 3) f = (1.0 + z) * std::exp(-z);
    else f = (1.0 + z + z * z / 3.0) * std::exp(-z);
    phi_host[i] = k->sigma2 * f;
  }
  return MLBLUP_OK;
}

int mlblup_cov_matvec(const mlblup_matern* k, const double* rows_dev, int64_t m, const double* cols_dev, int64_t n,
                      int32_t d, int32_t precision, int32_t outputs, const double* x_dev, double* y_dev,
                      double* dy_dev, void* work_dev, int64_t work_bytes, void* stream) {
  clear_error();
  int st = check_kernel(k);
  if (st) return st;
  PairArgs a{rows_dev, m, cols_dev, n, d, nu2_of(k), k->rho, k->sigma2, precision, outputs, x_dev, y_dev, dy_dev,
             k->nu, nullptr};
  return pair_launch(a, work_dev, work_bytes, (hipStream_t)stream);
}

int mlblup_cov_matvec_noalloc(const mlblup_matern* k, const double* rows_dev, int64_t m, const double* cols_dev,
                              int64_t n, int32_t d, int32_t precision, int32_t outputs, const double* x_dev,
                              double* y_dev, double* dy_dev, void* stream) {
  clear_error();
  int st = check_kernel(k);
  if (st) return st;
  PairArgs a{rows_dev, m, cols_dev, n, d, nu2_of(k), k->rho, k->sigma2, precision, outputs, x_dev, y_dev, dy_dev,
             k->nu, nullptr};
  return pair_launch_noalloc(a, (hipStream_t)stream);
}

int mlblup_transform_workspace_bytes(mlblup_basis b, int64_t* bytes) {
  clear_error();
  if (!b || !bytes) return fail(MLBLUP_EINVAL, "NULL argument");
  *bytes = align_up(std::max<int64_t>(b->b.scal_total, 1) * (int64_t)sizeof(double));
  return MLBLUP_OK;
}

static int transform_common(mlblup_basis b, void* work, int64_t work_bytes, TransformDev* T) {
  int st = check_basis_dev(b);
  if (st) return st;
  const Basis& B = b->b;
  if (!work || work_bytes < std::max<int64_t>(B.scal_total, 1) * (int64_t)sizeof(double))
    return fail(MLBLUP_EINVAL, "transform workspace too small");
  *T = transform_dev(B);
  return MLBLUP_OK;
}

int mlblup_apply_W(mlblup_basis b, const double* v_dev, double* vw_dev, double* vl_dev, void* work_dev,
                   int64_t work_bytes, void* stream) {
  clear_error();
  TransformDev T;
  int st = transform_common(b, work_dev, work_bytes, &T);
  if (st) return st;
  if (!v_dev || !vw_dev) return fail(MLBLUP_EINVAL, "apply_W: NULL vector");
  return transform_analysis(T, v_dev, vw_dev, vl_dev, (double*)work_dev, (hipStream_t)stream);
}

int mlblup_apply_Wt(mlblup_basis b, const double* vw_dev, const double* vl_dev, double* v_dev, void* work_dev,
                    int64_t work_bytes, void* stream) {
  clear_error();
  TransformDev T;
  int st = transform_common(b, work_dev, work_bytes, &T);
  if (st) return st;
  if (!v_dev || !vw_dev) return fail(MLBLUP_EINVAL, "apply_Wt: NULL vector");
  return transform_synthesis(T, vw_dev, vl_dev, v_dev, (double*)work_dev, (hipStream_t)stream);
}

int mlblup_solve_workspace_bytes(mlblup_basis b, const mlblup_pcg_opts* opts, int64_t m_targets, int64_t* bytes) {
  clear_error();
  (void)opts;
  if (!b || !bytes || m_targets < 0) return fail(MLBLUP_EINVAL, "bad argument");
  *bytes = ws_layout(b->b, m_targets).total;
  return MLBLUP_OK;
}

static int check_opts(const mlblup_pcg_opts* opts, mlblup_pcg_opts* o) {
  *o = opts ? *opts : default_opts();
  if (o->history_cap < 0 || (o->history_cap > 0 && !o->history_host)) return fail(MLBLUP_EINVAL, "pcg options: bad history");
  if (!(o->rtol > 0) || o->max_iter < 0 || o->precision < MLBLUP_FP64 || o->precision > MLBLUP_MFMA_BF16X3)
    return fail(MLBLUP_EINVAL, "pcg options: need rtol > 0, max_iter >= 0, known precision");
  if (o->mixed_scheme != MLBLUP_MIXED_FLEXIBLE && o->mixed_scheme != MLBLUP_MIXED_RELIABLE)
    return fail(MLBLUP_EINVAL, "pcg options: unknown mixed_scheme");
  if (o->refine_max <= 0) o->refine_max = 200;
  return MLBLUP_OK;
}

int mlblup_cw_matvec(mlblup_basis b, const mlblup_matern* k, const double* in_dev, double* out_dev,
                     int32_t precision, void* work_dev, int64_t work_bytes, void* stream) {
  clear_error();
  int st = check_basis_dev(b);
  if (st) return st;
  if ((st = check_kernel(k))) return st;
  if (!in_dev || !out_dev || in_dev == out_dev) return fail(MLBLUP_EINVAL, "cw_matvec: NULL or aliased vectors");
  if (precision < MLBLUP_FP64 || precision > MLBLUP_MFMA_BF16X3) return fail(MLBLUP_EINVAL, "unknown precision");
  Ws w;
  if ((st = check_ws(b, 0, work_dev, work_bytes, &w))) return st;
  Ctx c(b->b, *k, work_dev, w, (hipStream_t)stream);
  return c.matvec_cw(in_dev, out_dev, precision);
}

int mlblup_pcg_solve(mlblup_basis b, const mlblup_matern* k, const double* zw_dev, double* gw_dev, int32_t use_x0,
                     const mlblup_pcg_opts* opts, void* work_dev, int64_t work_bytes, mlblup_pcg_info* info,
                     void* stream) {
  clear_error();
  int st = check_basis_dev(b);
  if (st) return st;
  if ((st = check_kernel(k))) return st;
  mlblup_pcg_opts o;
  if ((st = check_opts(opts, &o))) return st;
  if (!zw_dev || !gw_dev) return fail(MLBLUP_EINVAL, "pcg_solve: NULL vector");
  if (o.resume && (!o.state_dev || !use_x0 || o.precision != MLBLUP_FP64))
    return fail(MLBLUP_EINVAL, "pcg_solve: resume needs state_dev, use_x0 = 1 and MLBLUP_FP64");
  Ws w;
  if ((st = check_ws(b, 0, work_dev, work_bytes, &w))) return st;
  Ctx c(b->b, *k, work_dev, w, (hipStream_t)stream);
  mlblup_pcg_info inf{};
  st = c.solve(zw_dev, gw_dev, use_x0 != 0, o, inf);
  if (info) *info = inf;
  return st;
}

int mlblup_blup_predict(mlblup_basis b, const mlblup_matern* k, const double* z_dev, const double* tgt_dev,
                        int64_t m_t, const mlblup_pcg_opts* opts, int32_t predict_precision, int32_t warm_start,
                        double* zhat_dev, double* beta_host, double* gamma_dev, double* gamma_w_dev,
                        double* interp_res_host, void* work_dev, int64_t work_bytes, mlblup_pcg_info* info,
                        void* stream) {
  clear_error();
  int st = check_basis_dev(b);
  if (st) return st;
  if ((st = check_kernel(k))) return st;
  mlblup_pcg_opts o;
  if ((st = check_opts(opts, &o))) return st;
  if (!z_dev || m_t < 0 || (m_t > 0 && (!tgt_dev || !zhat_dev)))
    return fail(MLBLUP_EINVAL, "blup_predict: bad z / target arguments");
  if (predict_precision < MLBLUP_FP64 || predict_precision > MLBLUP_MFMA_BF16X3)
    return fail(MLBLUP_EINVAL, "blup_predict: unknown predict precision");
  Ws w;
  if ((st = check_ws(b, m_t, work_dev, work_bytes, &w))) return st;
  const Basis& B = b->b;
  hipStream_t s = (hipStream_t)stream;
  Ctx c(B, *k, work_dev, w, s);
  const int64_t N = B.n, nw = B.n - B.p;
  double* zw = c.at(w.zw);
  double* gw = gamma_w_dev ? gamma_w_dev : c.at(w.gamw);
  double* gam = gamma_dev ? gamma_dev : c.at(w.gam);
  // Z_W = W z
  if ((st = transform_analysis(c.T, z_dev, zw, nullptr, c.at(w.scal), s))) return st;
  // |Z_W| at rounding level of |z| means z lies in the trend space: gamma_W = 0
  double znorm = 0.0;
  if ((st = c.norm(z_dev, N, &znorm))) return st;
  if (!std::isfinite(znorm)) return fail(MLBLUP_EINVAL, "blup_predict: non-finite observations");
  mlblup_pcg_info inf{};
  if (warm_start && !gamma_w_dev) return fail(MLBLUP_EINVAL, "blup_predict: warm start needs gamma_w_dev");
  const int solve_st = c.solve(zw, gw, warm_start != 0, o, inf, 1e-13 * znorm);
  if (info) *info = inf;
  if (solve_st != MLBLUP_OK && solve_st != MLBLUP_ENOCONV) return solve_st;
  const std::string solve_msg = solve_st ? std::string(mlblup_last_error()) : std::string();
  // gamma = W^T gamma_W ; v = z - C gamma ; (r_W, L v) = (W v, L v)
  if ((st = transform_synthesis(c.T, gw, nullptr, gam, c.at(w.scal), s))) return st;
  double* v = c.at(w.v);
  if ((st = c.pair(c.pts, N, gam, v, nullptr, MLBLUP_FP64, MLBLUP_VALUE))) return st;
  if ((st = vec_sub_from(z_dev, v, N, s))) return st;
  double* vw = c.at(w.vw);
  double* lv = c.at(w.lv);
  if ((st = transform_analysis(c.T, v, vw, lv, c.at(w.scal), s))) return st;
  double rw = 0.0;
  if ((st = c.norm(vw, nw, &rw))) return st;
  if (interp_res_host) *interp_res_host = rw;
  // beta in the root frame: (L X_loc) beta_loc = L v with L X_loc = Ms^T
  std::vector<double> lvh(B.p);
  MLB_HIP(hipMemcpyAsync(lvh.data(), lv, B.p * sizeof(double), hipMemcpyDeviceToHost, s));
  MLB_HIP(hipStreamSynchronize(s));
  std::vector<double> A((size_t)B.p * B.p);
  for (int i = 0; i < B.p; ++i)
    for (int j = 0; j < B.p; ++j) A[(size_t)i * B.p + j] = B.root_moments[(size_t)j * B.p + i];
  std::vector<double> bl = lvh;
  if (!dense_solve(A, bl, B.p)) return fail(MLBLUP_ERANK, "blup_predict: singular root moment matrix");
  if (beta_host) {
    // raw-coordinate coefficients: u = (x - c)/h = s x + b, s = 1/h, b = -c/h
    std::vector<double> bvec(B.d);
    for (int kk = 0; kk < B.d; ++kk) bvec[kk] = -B.root_c[kk] / B.root_h;
    const std::vector<double> S = shift_matrix(B.exps, 1.0 / B.root_h, bvec);
    for (int g = 0; g < B.p; ++g) {
      double acc = 0.0;
      for (int a = 0; a < B.p; ++a) acc += bl[a] * S[(size_t)a * B.p + g];
      beta_host[g] = acc;
    }
  }
  if (m_t > 0) {
    double* betad = c.at(w.beta);
    MLB_HIP(hipMemcpyAsync(betad, bl.data(), B.p * sizeof(double), hipMemcpyHostToDevice, s));
    if ((st = c.pair(tgt_dev, m_t, gam, zhat_dev, nullptr, predict_precision, MLBLUP_VALUE))) return st;
    const char* img = (const char*)B.dev_base;
    const int32_t* ex = (const int32_t*)(img + B.off_exps);
    const double* rc = (const double*)(img + B.off_rootc);
    if ((st = trend_add(tgt_dev, m_t, B.d, ex, B.p, rc, B.root_h, betad, zhat_dev, s))) return st;
    MLB_HIP(hipStreamSynchronize(s));  // bl (host) must outlive the copy
  }
  if (solve_st) return fail(solve_st, solve_msg);
  return MLBLUP_OK;
}

int mlblup_dd_workspace_bytes(mlblup_basis b, int64_t m_t, int64_t* bytes) {
  clear_error();
  if (!b || !bytes || m_t < 0) return fail(MLBLUP_EINVAL, "dd_workspace_bytes: bad argument");
  *bytes = dd_workspace_bytes(b->b.n, m_t);
  return MLBLUP_OK;
}

int mlblup_blup_predict_dd(mlblup_basis b, const mlblup_matern* k, const double* z_dev, const double* tgt_dev,
                           int64_t m_t, double rtol, int32_t max_iter, double* zhat_dev, double* beta_host,
                           double* cw_dev, double* info_host, void* work_dev, int64_t work_bytes, void* stream) {
  clear_error();
  int st = check_basis_dev(b);
  if (st) return st;
  if ((st = check_kernel(k))) return st;
  const Basis& B = b->b;
  const int nu2 = nu2_of(k);
  if (nu2 == kNuGeneral) return fail(MLBLUP_EINVAL, "blup_predict_dd: nu must be 1/2, 3/2, 5/2 or +inf");
  if (B.n > kDdMaxN || m_t < 0 || m_t > kDdMaxN)
    return fail(MLBLUP_EINVAL, "blup_predict_dd: N and the target count must be at most " + std::to_string(kDdMaxN));
  if (!z_dev || !info_host || (m_t > 0 && (!tgt_dev || !zhat_dev)) || !(rtol >= 0) || max_iter < 0)
    return fail(MLBLUP_EINVAL, "blup_predict_dd: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = B.n, m = n - B.p;
  std::vector<double> P((size_t)n * n), W((size_t)m * n), Lm((size_t)B.p * n);
  if ((st = mlblup_basis_dense(b, W.data(), Lm.data()))) return st;
  std::copy(W.begin(), W.end(), P.begin());
  std::copy(Lm.begin(), Lm.end(), P.begin() + (size_t)m * n);
  std::vector<double> tgt((size_t)std::max<int64_t>(m_t, 1) * B.d);
  if (m_t > 0) {
    MLB_HIP(hipMemcpyAsync(tgt.data(), tgt_dev, (size_t)m_t * B.d * 8, hipMemcpyDeviceToHost, s));
    MLB_HIP(hipStreamSynchronize(s));
  }
  return dd_blup_predict(B, P, nu2, k->nu, k->rho, k->sigma2, z_dev, tgt_dev, tgt.data(), m_t, rtol, max_iter,
                         zhat_dev, beta_host, cw_dev, info_host, work_dev, work_bytes, s);
}

int mlblup_blup_grad(mlblup_basis b, const mlblup_matern* k, const double* z_dev, const double* gamma_dev,
                     const double* lambda_dev, int32_t precision, double* Q_host, double* dQ_dlogrho_host,
                     void* work_dev, int64_t work_bytes, void* stream) {
  clear_error();
  int st = check_basis_dev(b);
  if (st) return st;
  if ((st = check_kernel(k))) return st;
  if (!gamma_dev) return fail(MLBLUP_EINVAL, "blup_grad: NULL gamma");
  if (precision < MLBLUP_FP64 || precision > MLBLUP_MFMA_BF16X3) return fail(MLBLUP_EINVAL, "unknown precision");
  Ws w;
  if ((st = check_ws(b, 0, work_dev, work_bytes, &w))) return st;
  const Basis& B = b->b;
  Ctx c(B, *k, work_dev, w, (hipStream_t)stream);
  if (Q_host) {
    if (!z_dev) return fail(MLBLUP_EINVAL, "blup_grad: Q needs z");
    if ((st = c.dot(z_dev, gamma_dev, B.n, Q_host))) return st;
  }
  if (dQ_dlogrho_host) {
    double* g = c.at(w.b);
    if ((st = c.pair(c.pts, B.n, gamma_dev, nullptr, g, precision, MLBLUP_DLOGRHO))) return st;
    double dd = 0.0;
    if ((st = c.dot(lambda_dev ? lambda_dev : gamma_dev, g, B.n, &dd))) return st;
    *dQ_dlogrho_host = -dd;
  }
  return MLBLUP_OK;
}

int mlblup_loglik_workspace_bytes(mlblup_basis b, int32_t level, int64_t* bytes, int64_t* rows) {
  clear_error();
  if (!b || !bytes) return fail(MLBLUP_EINVAL, "NULL argument");
  if (level < 0 || level >= b->b.levels)
    return fail(MLBLUP_EINVAL, "loglik: level must be in [0, " + std::to_string(b->b.levels - 1) + "]");
  const LoglikLayout L = loglik_layout(b->b, level);
  *bytes = L.total;
  if (rows) *rows = L.rows;
  return MLBLUP_OK;
}

static int loglik_common(mlblup_basis b, const mlblup_matern* k, const double* z_dev, int32_t level, double tau,
                         void* work_dev, int64_t work_bytes, TransformDev* T, LoglikLayout* L, PairArgs* a,
                         int64_t* nnz, hipStream_t stream) {
  int st = check_basis_dev(b);
  if (st) return st;
  if ((st = check_kernel(k))) return st;
  const Basis& B = b->b;
  if (level < 0 || level >= B.levels)
    return fail(MLBLUP_EINVAL, "loglik: level must be in [0, " + std::to_string(B.levels - 1) + "]");
  if (!(tau >= 0)) return fail(MLBLUP_EINVAL, "loglik: tau must be >= 0 (inf = no sparsification)");
  if (!z_dev) return fail(MLBLUP_EINVAL, "loglik: NULL data vector");
  *L = loglik_layout(B, level);
  if (!work_dev || work_bytes < L->total)
    return fail(MLBLUP_EINVAL, "loglik: workspace too small (need " + std::to_string(L->total) + " bytes)");
  *T = transform_dev(B);
  *a = PairArgs{nullptr, 0, nullptr, B.n, B.d, nu2_of(k), k->rho, k->sigma2, MLBLUP_FP64, MLBLUP_VALUE,
                nullptr, nullptr, nullptr, k->nu, nullptr};
  *nnz = L->rows * L->rows;
  if (std::isfinite(tau)) {
    Pattern P;
    build_pattern(B, level, tau, P);
    *nnz = P.nnz;
    if ((st = loglik_upload_pattern(P, work_dev, *L, stream))) return st;
  }
  return MLBLUP_OK;
}

int mlblup_sparsity_pattern(mlblup_basis b, int32_t level, double tau, int64_t* nnz, uint8_t* mask_host) {
  clear_error();
  if (!b || !nnz) return fail(MLBLUP_EINVAL, "NULL argument");
  const Basis& B = b->b;
  if (level < 0 || level >= B.levels)
    return fail(MLBLUP_EINVAL, "sparsity_pattern: level must be in [0, " + std::to_string(B.levels - 1) + "]");
  if (!(tau >= 0)) return fail(MLBLUP_EINVAL, "sparsity_pattern: tau must be >= 0 (inf = no sparsification)");
  Pattern P;
  build_pattern(B, level, tau, P);
  *nnz = P.nnz;
  if (mask_host) {
    const int64_t nt = (int64_t)P.rowcell.size();
    for (int64_t r = 0; r < nt; ++r) {
      const uint8_t* kr = &P.keep[(size_t)P.rowcell[r] * P.nc];
      for (int64_t c = 0; c < nt; ++c) mask_host[r * nt + c] = kr[P.rowcell[c]];
    }
  }
  return MLBLUP_OK;
}

int mlblup_loglik(mlblup_basis b, const mlblup_matern* k, const double* z_dev, int32_t level, double tau,
                  double* out4_host, void* work_dev, int64_t work_bytes, void* stream) {
  clear_error();
  if (!out4_host) return fail(MLBLUP_EINVAL, "loglik: NULL output");
  TransformDev T;
  LoglikLayout L;
  PairArgs a;
  int64_t nnz = 0;
  int st = loglik_common(b, k, z_dev, level, tau, work_dev, work_bytes, &T, &L, &a, &nnz, (hipStream_t)stream);
  if (st) return st;
  if ((st = loglik_device(b->b, T, a, level, z_dev, work_dev, L, std::isfinite(tau), out4_host, (hipStream_t)stream)))
    return st;
  out4_host[3] = (double)nnz;
  return MLBLUP_OK;
}

// the sparse analysis of (level, tau), from the basis' cache or built now
// MLBLUP_SPARSE_TAIL=none | all overrides the choice of the dense tail (-1 = chosen by the analysis)
static int sparse_tail_request() {
  const char* e = std::getenv("MLBLUP_SPARSE_TAIL");
  if (!e) return -1;
  if (!std::strcmp(e, "none")) return -2;
  if (!std::strcmp(e, "all")) return 0;
  return -1;
}

// MLBLUP_SPARSE_TAIL_MAX=<rows> lowers the row limit of a chosen dense tail (at most kSparseMaxTail)
static int64_t sparse_tail_cap() {
  const char* e = std::getenv("MLBLUP_SPARSE_TAIL_MAX");
  if (!e) return kSparseMaxTail;
  char* end = nullptr;
  const long long v = std::strtoll(e, &end, 10);
  if (end == e || *end || v < 0) return kSparseMaxTail;
  return std::min<int64_t>(v, kSparseMaxTail);
}

static int sparse_symbolic(mlblup_basis b, int32_t level, double tau, std::shared_ptr<const SparseSymbolic>* out) {
  std::lock_guard<std::mutex> g(b->sparse_mu);
  const int req = sparse_tail_request();
  const int64_t cap = sparse_tail_cap();
  const bool same_tau = (std::isinf(tau) && b->sparse && std::isinf(b->sparse->tau)) || (b->sparse && b->sparse->tau == tau);
  if (b->sparse && b->sparse->level == level && same_tau && b->sparse_req == req && b->sparse_cap == cap) {
    *out = b->sparse;
    return MLBLUP_OK;
  }
  auto S = std::make_shared<SparseSymbolic>();
  const int st = sparse_analyse(b->b, level, tau, *S, req == -2 ? std::numeric_limits<int32_t>::max() : req, cap);
  b->sparse_req = req;
  b->sparse_cap = cap;
  if (st) return st;
  b->sparse = S;
  *out = S;
  return MLBLUP_OK;
}

int mlblup_loglik_sparse_workspace_bytes(mlblup_basis b, int32_t level, double tau, int64_t* bytes,
                                         double* info8_host) {
  clear_error();
  if (!b || !bytes) return fail(MLBLUP_EINVAL, "NULL argument");
  if (level < 0 || level >= b->b.levels)
    return fail(MLBLUP_EINVAL, "sparse loglik: level must be in [0, " + std::to_string(b->b.levels - 1) + "]");
  if (!(tau >= 0)) return fail(MLBLUP_EINVAL, "sparse loglik: tau must be >= 0 (inf = no sparsification)");
  std::shared_ptr<const SparseSymbolic> S;
  int st = sparse_symbolic(b, level, tau, &S);
  if (st) return st;
  *bytes = sparse_layout(b->b, *S).total;
  if (info8_host) {
    info8_host[0] = (double)S->rows;
    info8_host[1] = (double)S->kept_entries;
    info8_host[2] = (double)S->factor_entries;
    info8_host[3] = (double)S->tail;
    info8_host[4] = S->lvl_ptr.empty() ? 0.0 : (double)(S->lvl_ptr.size() - 1);
    info8_host[5] = S->flops;
    info8_host[6] = (double)S->tail_rows;
    info8_host[7] = S->flops_tail;
  }
  return MLBLUP_OK;
}

int mlblup_loglik_sparse(mlblup_basis b, const mlblup_matern* k, const double* z_dev, int32_t level, double tau,
                         double* out4_host, void* work_dev, int64_t work_bytes, void* stream) {
  clear_error();
  if (!out4_host) return fail(MLBLUP_EINVAL, "sparse loglik: NULL output");
  int st = check_basis_dev(b);
  if (st) return st;
  if ((st = check_kernel(k))) return st;
  const Basis& B = b->b;
  if (level < 0 || level >= B.levels)
    return fail(MLBLUP_EINVAL, "sparse loglik: level must be in [0, " + std::to_string(B.levels - 1) + "]");
  if (!(tau >= 0)) return fail(MLBLUP_EINVAL, "sparse loglik: tau must be >= 0 (inf = no sparsification)");
  if (!z_dev) return fail(MLBLUP_EINVAL, "sparse loglik: NULL data vector");
  std::shared_ptr<const SparseSymbolic> S;
  if ((st = sparse_symbolic(b, level, tau, &S))) return st;
  const SparseLayout Ly = sparse_layout(B, *S);
  if (!work_dev || work_bytes < Ly.total)
    return fail(MLBLUP_EINVAL, "sparse loglik: workspace too small (need " + std::to_string(Ly.total) + " bytes)");
  const TransformDev T = transform_dev(B);
  const PairArgs a{nullptr, 0, nullptr, B.n, B.d, nu2_of(k), k->rho, k->sigma2, MLBLUP_FP64, MLBLUP_VALUE,
                   nullptr, nullptr, nullptr, k->nu, nullptr};
  if ((st = loglik_sparse_device(B, T, a, *S, z_dev, work_dev, Ly, out4_host, (hipStream_t)stream))) return st;
  out4_host[3] = (double)S->kept_entries;
  return MLBLUP_OK;
}

// golden-section search for the maximum of f(log rho) on [log rho_lo, log rho_hi]
static int golden_log_rho(const std::function<int(double, double*)>& f, double rho_lo, double rho_hi,
                          double log_rho_tol, double* out4_host) {
  const double g = 0.6180339887498949;
  int evals = 0;
  auto ev = [&](double x, double* v) {
    ++evals;
    return f(x, v);
  };
  double lo = std::log(rho_lo), hi = std::log(rho_hi);
  double x1 = hi - g * (hi - lo), x2 = lo + g * (hi - lo), f1, f2;
  int st;
  if ((st = ev(x1, &f1)) || (st = ev(x2, &f2))) return st;
  while (hi - lo > log_rho_tol) {
    if (f1 >= f2) {
      hi = x2;
      x2 = x1;
      f2 = f1;
      x1 = hi - g * (hi - lo);
      if ((st = ev(x1, &f1))) return st;
    } else {
      lo = x1;
      x1 = x2;
      f1 = f2;
      x2 = lo + g * (hi - lo);
      if ((st = ev(x2, &f2))) return st;
    }
  }
  const double lr = 0.5 * (lo + hi);
  double fm;
  if ((st = ev(lr, &fm))) return st;
  out4_host[0] = std::exp(lr);
  out4_host[1] = fm;
  out4_host[2] = (double)evals;
  out4_host[3] = hi - lo;
  return MLBLUP_OK;
}

static int check_mle_rho_args(const double* out4_host, double rho_lo, double rho_hi, double log_rho_tol) {
  if (!out4_host) return fail(MLBLUP_EINVAL, "mle_rho: NULL output");
  if (!(rho_lo > 0) || !(rho_hi > rho_lo) || !std::isfinite(rho_hi))
    return fail(MLBLUP_EINVAL, "mle_rho: need 0 < rho_lo < rho_hi < inf");
  if (!(log_rho_tol > 0)) return fail(MLBLUP_EINVAL, "mle_rho: log_rho_tol must be > 0");
  return MLBLUP_OK;
}

int mlblup_mle_rho(mlblup_basis b, const mlblup_matern* k0, const double* z_dev, int32_t level, double tau,
                   double rho_lo, double rho_hi, double log_rho_tol, double* out4_host, void* work_dev,
                   int64_t work_bytes, void* stream) {
  clear_error();
  int st = check_mle_rho_args(out4_host, rho_lo, rho_hi, log_rho_tol);
  if (st) return st;
  TransformDev T;
  LoglikLayout L;
  PairArgs a;
  int64_t nnz = 0;
  if ((st = loglik_common(b, k0, z_dev, level, tau, work_dev, work_bytes, &T, &L, &a, &nnz, (hipStream_t)stream)))
    return st;
  const bool masked = std::isfinite(tau);
  return golden_log_rho(
      [&](double lr, double* v) {
        PairArgs q = a;
        q.rho = std::exp(lr);
        double out[3];
        const int s2 = loglik_device(b->b, T, q, level, z_dev, work_dev, L, masked, out, (hipStream_t)stream);
        *v = out[0];
        return s2;
      },
      rho_lo, rho_hi, log_rho_tol, out4_host);
}

int mlblup_mle_rho_sparse(mlblup_basis b, const mlblup_matern* k0, const double* z_dev, int32_t level, double tau,
                          double rho_lo, double rho_hi, double log_rho_tol, double* out4_host, void* work_dev,
                          int64_t work_bytes, void* stream) {
  clear_error();
  int st = check_mle_rho_args(out4_host, rho_lo, rho_hi, log_rho_tol);
  if (st) return st;
  if (!k0) return fail(MLBLUP_EINVAL, "mle_rho: NULL kernel");
  // every evaluation validates its arguments; the analysis of (level, tau) is built once
  const mlblup_matern k = *k0;
  return golden_log_rho(
      [&](double lr, double* v) {
        mlblup_matern q = k;
        q.rho = std::exp(lr);
        double out[4];
        const int s2 = mlblup_loglik_sparse(b, &q, z_dev, level, tau, out, work_dev, work_bytes, stream);
        *v = out[0];
        return s2;
      },
      rho_lo, rho_hi, log_rho_tol, out4_host);
}

// profile likelihood over nu: golden section, each point the rho maximum of `mle`
static int golden_nu(const std::function<int(const mlblup_matern*, double*)>& mle, double sigma2, double nu_lo,
                     double nu_hi, double nu_tol, double* out5_host) {
  if (!out5_host) return fail(MLBLUP_EINVAL, "mle_nu_rho: NULL output");
  if (!(nu_lo > 0) || !(nu_hi > nu_lo) || nu_hi > 8.0) return fail(MLBLUP_EINVAL, "mle_nu_rho: need 0 < nu_lo < nu_hi <= 8");
  if (!(nu_tol > 0)) return fail(MLBLUP_EINVAL, "mle_nu_rho: nu_tol must be > 0");
  int evals = 0;
  auto profile = [&](double nu, double* val, double* rho) {
    const mlblup_matern k{nu, 1.0, sigma2};
    double o[4];
    const int s2 = mle(&k, o);
    if (s2) return s2;
    evals += (int)o[2];
    *rho = o[0];
    *val = o[1];
    return MLBLUP_OK;
  };
  const double g = 0.6180339887498949;
  double lo = nu_lo, hi = nu_hi;
  double x1 = hi - g * (hi - lo), x2 = lo + g * (hi - lo), f1, f2, r1, r2;
  int st;
  if ((st = profile(x1, &f1, &r1)) || (st = profile(x2, &f2, &r2))) return st;
  while (hi - lo > nu_tol) {
    if (f1 >= f2) {
      hi = x2;
      x2 = x1;
      f2 = f1;
      r2 = r1;
      x1 = hi - g * (hi - lo);
      if ((st = profile(x1, &f1, &r1))) return st;
    } else {
      lo = x1;
      x1 = x2;
      f1 = f2;
      r1 = r2;
      x2 = lo + g * (hi - lo);
      if ((st = profile(x2, &f2, &r2))) return st;
    }
  }
  const double nu = 0.5 * (lo + hi);
  double fm, rm;
  if ((st = profile(nu, &fm, &rm))) return st;
  out5_host[0] = nu;
  out5_host[1] = rm;
  out5_host[2] = fm;
  out5_host[3] = (double)evals;
  out5_host[4] = hi - lo;
  return MLBLUP_OK;
}

int mlblup_mle_nu_rho(mlblup_basis b, double sigma2, const double* z_dev, int32_t level, double tau, double nu_lo,
                      double nu_hi, double nu_tol, double rho_lo, double rho_hi, double log_rho_tol,
                      double* out5_host, void* work_dev, int64_t work_bytes, void* stream) {
  clear_error();
  return golden_nu(
      [&](const mlblup_matern* k, double* o) {
        return mlblup_mle_rho(b, k, z_dev, level, tau, rho_lo, rho_hi, log_rho_tol, o, work_dev, work_bytes, stream);
      },
      sigma2, nu_lo, nu_hi, nu_tol, out5_host);
}

int mlblup_mle_nu_rho_sparse(mlblup_basis b, double sigma2, const double* z_dev, int32_t level, double tau,
                             double nu_lo, double nu_hi, double nu_tol, double rho_lo, double rho_hi,
                             double log_rho_tol, double* out5_host, void* work_dev, int64_t work_bytes, void* stream) {
  clear_error();
  return golden_nu(
      [&](const mlblup_matern* k, double* o) {
        return mlblup_mle_rho_sparse(b, k, z_dev, level, tau, rho_lo, rho_hi, log_rho_tol, o, work_dev, work_bytes,
                                     stream);
      },
      sigma2, nu_lo, nu_hi, nu_tol, out5_host);
}

}  // extern "C"
