// The multilevel predictor with the covariance blocks formed in double-double
// arithmetic, for the accuracy experiment of Sec. 8 ("prediction numerical
// accuracy under ill-conditioning": Gaussian kernel, a few hundred sites).
//
// W annihilates the polynomials of degree <= w (Sec. 3.1), so W C W^T keeps
// only the part of the kernel's Taylor expansion above that degree.  For the
// flat Gaussians of the experiment that part is some 25 orders of magnitude
// below the entries of C, far under the rounding of FP64 products of C; here
// every entry of P C P^T (P = [W; L], the dense multilevel basis) and of
// K(targets, S) P^T is formed in double-double (about 32 digits) from the
// FP64 coordinates and basis, so the cancellation happens without noise.
// C_W gamma_W = W Z is then solved by CG in FP64 on the rounded C_W
// (stopping at the relative residual, the iteration limit, or a breakdown
// p.q <= 0, whose last iterate is kept), and the GLS coefficients and the
// predictions come from gamma_W in double-double:
//   L v = L Z - (L C W^T) gamma_W,  (L X) beta = L v  (the Sec. 5.2 least
//   squares, since col(X) = row(L)),  Zhat = X(targets) beta + (K W^T) gamma_W.
// Kernels are plain (one thread per output entry): the sizes are small.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "dd.h"
#include "device.h"
#include "internal.h"

namespace mlb {
namespace {

constexpr int kT = 256;
constexpr int kCgT = 1024;

struct DdKernel {
  int nu2;       // 0 Gaussian, 1/3/5 half-integer Matern
  dd scale;      // Gaussian: 1 / (2 rho^2); Matern: sqrt(2 nu) / rho
  double sigma2;
};

__device__ dd dd_phi(const double* __restrict__ a, const double* __restrict__ b, int d, const DdKernel& K) {
  dd s = dd_make(0.0);
  for (int k = 0; k < d; ++k) {
    const dd u = two_sum(a[k], -b[k]);  // the exact difference
    s = dd_add(s, dd_mul(u, u));
  }
  dd f;
  if (K.nu2 == 0) {
    f = dd_exp(dd_neg(dd_mul(s, K.scale)));
  } else {
    const dd z = dd_mul(dd_sqrt(s), K.scale);
    const dd e = dd_exp(dd_neg(z));
    dd poly = dd_make(1.0);
    if (K.nu2 == 3) poly = dd_add_d(z, 1.0);
    if (K.nu2 == 5) poly = dd_add_d(dd_add(z, dd_div_d(dd_mul(z, z), 3.0)), 1.0);
    f = dd_mul(poly, e);
  }
  return dd_mul_d(f, K.sigma2);
}

// C[i][j] = sigma2 phi(|a_i - b_j|) in double-double (hi, lo arrays, ld nb)
__global__ __launch_bounds__(kT) void k_dd_cov(const double* __restrict__ A, int64_t na, const double* __restrict__ B,
                                               int64_t nb, int d, DdKernel K, double* __restrict__ chi,
                                               double* __restrict__ clo) {
  const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= nb || i >= na) return;
  const dd f = dd_phi(A + i * d, B + j * d, d, K);
  chi[i * nb + j] = f.hi;
  clo[i * nb + j] = f.lo;
}

// U[i][r] = sum_j C[i][j] P[r][j]  (C: nr x n double-double, P: np x n FP64; U: nr x np)
__global__ __launch_bounds__(kT) void k_dd_times_pt(const double* __restrict__ chi, const double* __restrict__ clo,
                                                    int64_t nr, int64_t n, const double* __restrict__ P, int64_t np,
                                                    double* __restrict__ uhi, double* __restrict__ ulo) {
  const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (r >= np || i >= nr) return;
  dd acc = dd_make(0.0);
  for (int64_t j = 0; j < n; ++j) {
    const double pr = P[r * n + j];
    if (pr == 0.0) continue;
    acc = dd_add(acc, dd_mul_d(dd{chi[i * n + j], clo[i * n + j]}, pr));
  }
  uhi[i * np + r] = acc.hi;
  ulo[i * np + r] = acc.lo;
}

// G[r][s] = sum_i P[r][i] U[i][s]  (P: np x n FP64, U: n x np double-double)
__global__ __launch_bounds__(kT) void k_p_times_dd(const double* __restrict__ P, int64_t np, int64_t n,
                                                   const double* __restrict__ uhi, const double* __restrict__ ulo,
                                                   double* __restrict__ ghi, double* __restrict__ glo) {
  const int64_t s = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (s >= np || r >= np) return;
  dd acc = dd_make(0.0);
  for (int64_t i = 0; i < n; ++i) {
    const double pr = P[r * n + i];
    if (pr == 0.0) continue;
    acc = dd_add(acc, dd_mul_d(dd{uhi[i * np + s], ulo[i * np + s]}, pr));
  }
  ghi[r * np + s] = acc.hi;
  glo[r * np + s] = acc.lo;
}

// y[r] = sum_j P[r][j] z[j] in double-double
__global__ __launch_bounds__(kT) void k_p_times_z(const double* __restrict__ P, int64_t np, int64_t n,
                                                  const double* __restrict__ z, double* __restrict__ yhi,
                                                  double* __restrict__ ylo) {
  const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (r >= np) return;
  dd acc = dd_make(0.0);
  for (int64_t j = 0; j < n; ++j) acc = dd_add(acc, two_prod(P[r * n + j], z[j]));
  yhi[r] = acc.hi;
  ylo[r] = acc.lo;
}

__device__ double block_sum(double v, double* red) {
  // fixed-order sum over the workgroup (deterministic)
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
  return t;
}

// CG on the dense m x m matrix A (row stride lda), FP64, one workgroup.
// info: [iterations, breakdown flag, recurrence relres, true relres]
__global__ __launch_bounds__(kCgT) void k_dense_cg(const double* __restrict__ A, int64_t m, int64_t lda,
                                                   const double* __restrict__ b, double rtol, int max_iter,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ p, double* __restrict__ q,
                                                   double* __restrict__ info) {
  __shared__ double red[kCgT / 64];
  const int tid = threadIdx.x;
  double part = 0.0;
  for (int64_t i = tid; i < m; i += kCgT) {
    x[i] = 0.0;
    r[i] = b[i];
    p[i] = b[i];
    part = fma(b[i], b[i], part);
  }
  const double bb = block_sum(part, red);
  const double bn = sqrt(bb);
  double rr = bb;
  int it = 0, flag = 0;
  if (bn > 0.0) {
    while (it < max_iter) {
      __syncthreads();
      part = 0.0;
      for (int64_t i = tid; i < m; i += kCgT) {
        double s = 0.0;
        for (int64_t j = 0; j < m; ++j) s = fma(A[i * lda + j], p[j], s);
        q[i] = s;
        part = fma(p[i], s, part);
      }
      const double pq = block_sum(part, red);
      if (!(pq > 0.0) || !isfinite(pq)) {
        flag = 1;
        break;
      }
      const double alpha = rr / pq;
      part = 0.0;
      for (int64_t i = tid; i < m; i += kCgT) {
        x[i] = fma(alpha, p[i], x[i]);
        r[i] = fma(-alpha, q[i], r[i]);
        part = fma(r[i], r[i], part);
      }
      const double rn = block_sum(part, red);
      ++it;
      if (sqrt(rn) <= rtol * bn) {
        rr = rn;
        break;
      }
      const double beta = rn / rr;
      rr = rn;
      __syncthreads();
      for (int64_t i = tid; i < m; i += kCgT) p[i] = fma(beta, p[i], r[i]);
    }
  }
  // true residual |b - A x| / |b|
  __syncthreads();
  part = 0.0;
  for (int64_t i = tid; i < m; i += kCgT) {
    double s = b[i];
    for (int64_t j = 0; j < m; ++j) s = fma(-A[i * lda + j], x[j], s);
    part = fma(s, s, part);
  }
  const double tr = block_sum(part, red);
  if (tid == 0) {
    info[0] = it;
    info[1] = flag;
    info[2] = bn > 0.0 ? sqrt(rr) / bn : 0.0;
    info[3] = bn > 0.0 ? sqrt(tr) / bn : 0.0;
  }
}

// out[k] = y0[k] - sum_s M[k][s] g[s] (M: rows x m double-double with row stride ldm), in double-double
__global__ __launch_bounds__(kT) void k_dd_residual(const double* __restrict__ mhi, const double* __restrict__ mlo,
                                                    int64_t rows, int64_t m, int64_t ldm,
                                                    const double* __restrict__ y0hi, const double* __restrict__ y0lo,
                                                    const double* __restrict__ g, double sign,
                                                    double* __restrict__ ohi, double* __restrict__ olo) {
  const int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (k >= rows) return;
  dd acc = y0hi ? dd{y0hi[k], y0lo[k]} : dd_make(0.0);
  for (int64_t s = 0; s < m; ++s) acc = dd_add(acc, dd_mul_d(dd{mhi[k * ldm + s], mlo[k * ldm + s]}, sign * g[s]));
  ohi[k] = acc.hi;
  olo[k] = acc.lo;
}

struct DdLayout {
  int64_t P, chi, clo, uhi, ulo, ghi, glo, khi, klo, kphi, kplo, pzhi, pzlo, x, r, p, q, info, lvhi, lvlo, zkhi, zklo,
      total;
};

DdLayout dd_layout(int64_t n, int64_t mt) {
  DdLayout L{};
  int64_t o = 0;
  auto take = [&](int64_t doubles) {
    const int64_t at = o;
    o += (std::max<int64_t>(doubles, 1) * 8 + 255) / 256 * 256;
    return at;
  };
  L.P = take(n * n);
  L.chi = take(n * n);
  L.clo = take(n * n);
  L.uhi = take(n * n);
  L.ulo = take(n * n);
  L.ghi = take(n * n);
  L.glo = take(n * n);
  L.khi = take(mt * n);
  L.klo = take(mt * n);
  L.kphi = take(mt * n);
  L.kplo = take(mt * n);
  L.pzhi = take(n);
  L.pzlo = take(n);
  L.x = take(n);
  L.r = take(n);
  L.p = take(n);
  L.q = take(n);
  L.info = take(8);
  L.lvhi = take(n);
  L.lvlo = take(n);
  L.zkhi = take(std::max<int64_t>(mt, 1));
  L.zklo = take(std::max<int64_t>(mt, 1));
  L.total = o;
  return L;
}

dd dd_monomial(const double* x, const std::vector<int32_t>& e) {
  dd v = dd_make(1.0);
  for (size_t k = 0; k < e.size(); ++k)
    for (int t = 0; t < e[k]; ++t) v = dd_mul_d(v, x[k]);
  return v;
}

// (A | y) by Gaussian elimination with partial pivoting in double-double
bool dd_solve(std::vector<dd> A, std::vector<dd>& y, int p) {
  for (int k = 0; k < p; ++k) {
    int piv = k;
    for (int i = k + 1; i < p; ++i)
      if (std::fabs(A[(size_t)i * p + k].hi) > std::fabs(A[(size_t)piv * p + k].hi)) piv = i;
    if (A[(size_t)piv * p + k].hi == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < p; ++j) std::swap(A[(size_t)k * p + j], A[(size_t)piv * p + j]);
      std::swap(y[k], y[piv]);
    }
    for (int i = k + 1; i < p; ++i) {
      const dd f = dd_div(A[(size_t)i * p + k], A[(size_t)k * p + k]);
      for (int j = k; j < p; ++j) A[(size_t)i * p + j] = dd_sub(A[(size_t)i * p + j], dd_mul(f, A[(size_t)k * p + j]));
      y[i] = dd_sub(y[i], dd_mul(f, y[k]));
    }
  }
  for (int k = p - 1; k >= 0; --k) {
    dd s = y[k];
    for (int j = k + 1; j < p; ++j) s = dd_sub(s, dd_mul(A[(size_t)k * p + j], y[j]));
    y[k] = dd_div(s, A[(size_t)k * p + k]);
  }
  return true;
}

}  // namespace

int64_t dd_workspace_bytes(int64_t n, int64_t mt) { return dd_layout(n, mt).total; }

int dd_blup_predict(const Basis& B, const std::vector<double>& P_host, int nu2, double nu, double rho, double sigma2,
                    const double* z_dev, const double* tgt_dev, const double* tgt_host, int64_t mt, double rtol,
                    int32_t max_iter, double* zhat_dev, double* beta_host, double* cw_dev, double* info_host,
                    void* work, int64_t work_bytes, hipStream_t s) {
  const int64_t n = B.n, p = B.p, m = n - p;
  const DdLayout L = dd_layout(n, mt);
  if (!work || work_bytes < L.total)
    return fail(MLBLUP_EINVAL, "blup_predict_dd: workspace too small (need " + std::to_string(L.total) + ")");
  char* w = (char*)work;
  auto at = [&](int64_t off) { return (double*)(w + off); };
  const double* pts = (const double*)((const char*)B.dev_base + B.off_pts);
  DdKernel K{};
  K.nu2 = nu2;
  K.sigma2 = sigma2;
  if (nu2 == 0) {
    K.scale = dd_div(dd_make(1.0), dd_mul_d(two_prod(rho, rho), 2.0));
  } else {
    K.scale = dd_div(dd_sqrt(dd_make(2.0 * nu)), dd_make(rho));
  }
  MLB_HIP(hipMemcpyAsync(at(L.P), P_host.data(), (size_t)n * n * 8, hipMemcpyHostToDevice, s));
  // P C P^T
  hipLaunchKernelGGL(k_dd_cov, dim3((unsigned)((n + kT - 1) / kT), (unsigned)n), dim3(kT), 0, s, pts, n, pts, n, B.d,
                     K, at(L.chi), at(L.clo));
  hipLaunchKernelGGL(k_dd_times_pt, dim3((unsigned)((n + kT - 1) / kT), (unsigned)n), dim3(kT), 0, s, at(L.chi),
                     at(L.clo), n, n, at(L.P), n, at(L.uhi), at(L.ulo));
  hipLaunchKernelGGL(k_p_times_dd, dim3((unsigned)((n + kT - 1) / kT), (unsigned)n), dim3(kT), 0, s, at(L.P), n, n,
                     at(L.uhi), at(L.ulo), at(L.ghi), at(L.glo));
  // P z
  hipLaunchKernelGGL(k_p_times_z, dim3((unsigned)((n + kT - 1) / kT)), dim3(kT), 0, s, at(L.P), n, n, z_dev,
                     at(L.pzhi), at(L.pzlo));
  // K(targets, S) P^T
  if (mt > 0) {
    hipLaunchKernelGGL(k_dd_cov, dim3((unsigned)((n + kT - 1) / kT), (unsigned)mt), dim3(kT), 0, s, tgt_dev, mt, pts, n,
                       B.d, K, at(L.khi), at(L.klo));
    hipLaunchKernelGGL(k_dd_times_pt, dim3((unsigned)((n + kT - 1) / kT), (unsigned)mt), dim3(kT), 0, s, at(L.khi),
                       at(L.klo), mt, n, at(L.P), n, at(L.kphi), at(L.kplo));
  }
  MLB_HIP(hipGetLastError());
  // CG on the rounded C_W = G[0:m, 0:m] (row stride n)
  hipLaunchKernelGGL(k_dense_cg, dim3(1), dim3(kCgT), 0, s, at(L.ghi), m, n, at(L.pzhi), rtol, max_iter, at(L.x),
                     at(L.r), at(L.p), at(L.q), at(L.info));
  MLB_HIP(hipGetLastError());
  if (cw_dev) MLB_HIP(hipMemcpy2DAsync(cw_dev, m * 8, at(L.ghi), n * 8, m * 8, m, hipMemcpyDeviceToDevice, s));
  // L v = L z - (L C W^T) gamma_W ;  (K W^T) gamma_W
  hipLaunchKernelGGL(k_dd_residual, dim3((unsigned)((p + kT - 1) / kT)), dim3(kT), 0, s, at(L.ghi) + m * n,
                     at(L.glo) + m * n, p, m, n, at(L.pzhi) + m, at(L.pzlo) + m, at(L.x), -1.0, at(L.lvhi), at(L.lvlo));
  if (mt > 0)
    hipLaunchKernelGGL(k_dd_residual, dim3((unsigned)((mt + kT - 1) / kT)), dim3(kT), 0, s, at(L.kphi), at(L.kplo), mt,
                       m, n, nullptr, nullptr, at(L.x), 1.0, at(L.zkhi), at(L.zklo));
  MLB_HIP(hipGetLastError());
  std::vector<double> info(4), lv(2 * p), zk(2 * std::max<int64_t>(mt, 1));
  MLB_HIP(hipMemcpyAsync(info.data(), at(L.info), 4 * 8, hipMemcpyDeviceToHost, s));
  MLB_HIP(hipMemcpyAsync(lv.data(), at(L.lvhi), p * 8, hipMemcpyDeviceToHost, s));
  MLB_HIP(hipMemcpyAsync(lv.data() + p, at(L.lvlo), p * 8, hipMemcpyDeviceToHost, s));
  if (mt > 0) {
    MLB_HIP(hipMemcpyAsync(zk.data(), at(L.zkhi), mt * 8, hipMemcpyDeviceToHost, s));
    MLB_HIP(hipMemcpyAsync(zk.data() + mt, at(L.zklo), mt * 8, hipMemcpyDeviceToHost, s));
  }
  MLB_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < 4; ++k) info_host[k] = info[k];
  // (L X) beta = L v in double-double: X the raw-coordinate monomials at the sites (tree order)
  const int pp = (int)p;
  std::vector<dd> R((size_t)pp * pp, dd_make(0.0)), beta(pp);
  for (int a = 0; a < pp; ++a) {
    const double* Lrow = &P_host[(size_t)(m + a) * n];
    for (int g = 0; g < pp; ++g) {
      dd acc = dd_make(0.0);
      for (int64_t i = 0; i < n; ++i)
        if (Lrow[i] != 0.0) acc = dd_add(acc, dd_mul_d(dd_monomial(&B.pts_tree[(size_t)i * B.d], B.exps[g]), Lrow[i]));
      R[(size_t)a * pp + g] = acc;
    }
    beta[a] = dd{lv[a], lv[p + a]};
  }
  if (!dd_solve(R, beta, pp)) return fail(MLBLUP_ERANK, "blup_predict_dd: singular L X");
  if (beta_host)
    for (int g = 0; g < pp; ++g) beta_host[g] = beta[g].hi + beta[g].lo;
  if (mt > 0) {
    std::vector<double> zh(mt);
    for (int64_t t = 0; t < mt; ++t) {
      dd acc = dd{zk[t], zk[mt + t]};
      for (int g = 0; g < pp; ++g) acc = dd_add(acc, dd_mul(dd_monomial(&tgt_host[(size_t)t * B.d], B.exps[g]), beta[g]));
      zh[t] = acc.hi + acc.lo;
    }
    MLB_HIP(hipMemcpyAsync(zhat_dev, zh.data(), mt * 8, hipMemcpyHostToDevice, s));
    MLB_HIP(hipStreamSynchronize(s));
  }
  return MLBLUP_OK;
}

}  // namespace mlb
