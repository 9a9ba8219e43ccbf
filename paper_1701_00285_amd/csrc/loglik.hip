// Multilevel log-likelihood of the partial transform (Sec. 5.1, the reduced
// likelihoods and the Proposition on nested condition numbers):
//
//   l_n(theta) = -N~/2 log(2 pi) - 1/2 log det C^n_W - 1/2 (Z^n_W)^T (C^n_W)^-1 Z^n_W,
//
// with Z^n_W = [W_t; ...; W_n] Z (the first N~ rows of W, finest level
// first) and C^n_W the leading N~ x N~ block of C_W = W C W^T.  The
// determinant and the quadratic form come from one Cholesky factor G of
// C^n_W (Sec. 6.1, estimator computation): log det = 2 sum log G_ii, and the
// quadratic form is |y|^2 with G y = Z^n_W.
//
// Device steps (all FP64):
//  1. Phi = sigma^2 phi(|x_i - x_j|), N x N, row-major (dense_cov);
//  2. A = (W Phi) restricted to the first N~ rows: the multilevel analysis
//     applied to column blocks of Phi, level by level from the finest to n
//     (batched_analysis: one workgroup per cell and 256 columns);
//  3. A^T (tiled transpose), then C^n_W = (W A^T) restricted to N~ rows;
//  4. blocked right-looking Cholesky: panels of 256 columns, each factored
//     in blocks of 64 (the diagonal factor and its inverse in one wave, the
//     panel below as a product with that inverse, the update of the panel's
//     remaining columns), then the rank-256 update of the trailing lower
//     triangle in 128 x 128 tiles on the FP64 matrix cores: the next panel's
//     columns first, the rest on a second stream while the next panel is
//     factored;
//  5. G y = Z^n_W inside the factorization: Z^n_W is appended as row N~ of
//     the matrix, which the panel products and updates turn into y;
//     2 sum log G_ii and |y|^2 by fixed-order reductions.
// With a finite distance tau, the blocks of cell pairs that the tree search
// of Sec. 4.1 does not connect are zeroed after step 3 (apply_pattern), which
// gives the sparsified C~^n_W and l~_n.  The paper factorizes C~^n_W with a
// sparse Cholesky and nested dissection; here the factorization is dense
// (288 GB of HBM hold C^n_W for N~ up to about 10^5), so the zeros do not
// shorten it, and tau = inf gives the exact C^n_W.
//
// The same dense formation and bordered Cholesky give the coarse block of
// C_W used by the coarse preconditioner (coarse_inverse_factor, at the end).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "device.h"
#include "internal.h"
#include "pairmath.h"

namespace mlb {
namespace {

constexpr int kT = 256;
constexpr int kNb = 64;       // Cholesky block
constexpr int kTr = 32;       // transpose tile
constexpr int kColBatch = 4096;

// ---- 1. dense covariance -------------------------------------------------------
// columns [j0, j0 + ncols) of Phi into phi (row i at phi + i ld)
template <int NU2>
__global__ __launch_bounds__(kT) void dense_cov(const double* __restrict__ pts, int64_t n, int d, double zs,
                                                double sigma2, const double* __restrict__ gtab,
                                                double* __restrict__ phi, int64_t j0, int64_t ncols, int64_t ld) {
  __shared__ double tab[kExpTab];
  exp_table_fill(tab);
  const double* gt = gtab;
  if constexpr (NU2 == kNuGeneralT) {
    __shared__ double gsh[kGenuDoubles];
    const int nd = kGenuOffPoly + (int)gtab[5] * (kGenuDeg + 1);
    for (int i = threadIdx.x; i < nd; i += blockDim.x) gsh[i] = gtab[i];
    gt = gsh;
  }
  __syncthreads();
  const int64_t jl = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (jl >= ncols) return;
  const int64_t j = j0 + jl;
  for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
    double s = 1e-300;  // keeps the self pair away from sqrt(0) in the series branch
    for (int k = 0; k < d; ++k) {
      const double t = (pts[i * d + k] - pts[j * d + k]) * zs;
      s = fma(t, t, s);
    }
    double f = 0.0, g = 0.0;
    pair_value<NU2, 1, false>(s, tab, f, g, gt);
    phi[i * ld + jl] = sigma2 * f;
  }
}

__global__ void clear_flag(int* __restrict__ flag) {
  if (threadIdx.x == 0) flag[0] = 0;
}

// ---- 2./3. batched analysis: Y[row - row_lo] = (W X)[row] for the rows
// row_lo <= row < row_lo + ny of W produced by the cells of one level -------
__global__ __launch_bounds__(kT) void batched_analysis(const NodeDesc* __restrict__ desc,
                                                       const int32_t* __restrict__ lnodes,
                                                       const double* __restrict__ V, const double* __restrict__ X,
                                                       int64_t ldx, double* __restrict__ scal, int64_t lds,
                                                       double* __restrict__ Y, int64_t ldy, int64_t row_lo,
                                                       int64_t ny, int64_t ncols) {
  const NodeDesc D = desc[lnodes[blockIdx.y]];
  const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (j >= ncols) return;
  const double* cin = D.leaf ? X + D.in_off * ldx : scal + D.in_off * lds;
  const int64_t ldc = D.leaf ? ldx : lds;
  const double* B = V + D.v_off;
  const int m = D.m;
  for (int k0 = 0; k0 < m; k0 += 16) {
    double acc[16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) acc[kk] = 0.0;
    for (int i = 0; i < m; ++i) {
      const double c = cin[(int64_t)i * ldc + j];
#pragma unroll
      for (int kk = 0; kk < 16; ++kk)
        if (k0 + kk < m) acc[kk] = fma(B[(int64_t)i * m + k0 + kk], c, acc[kk]);
    }
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int k = k0 + kk;
      if (k >= m) break;
      if (k < D.a) {
        if (D.scal_off >= 0) scal[(D.scal_off + k) * lds + j] = acc[kk];
      } else {
        const int64_t row = D.w_off + (k - D.a) - row_lo;
        if (row >= 0 && row < ny) Y[row * ldy + j] = acc[kk];
      }
    }
  }
}

// out (cols x rows) = in^T (in: rows x cols)
__global__ __launch_bounds__(kTr * 8) void transpose(const double* __restrict__ in, int64_t rows, int64_t cols,
                                                     int64_t ldi, double* __restrict__ out, int64_t ldo) {
  __shared__ double t[kTr][kTr + 1];
  const int64_t r0 = (int64_t)blockIdx.y * kTr, c0 = (int64_t)blockIdx.x * kTr;
  const int tx = threadIdx.x % kTr, ty = threadIdx.x / kTr;
  for (int r = ty; r < kTr; r += 8) {
    const int64_t gr = r0 + r, gc = c0 + tx;
    if (gr < rows && gc < cols) t[r][tx] = in[gr * ldi + gc];
  }
  __syncthreads();
  for (int c = ty; c < kTr; c += 8) {
    const int64_t gc = c0 + c, gr = r0 + tx;
    if (gc < cols && gr < rows) out[gc * ldo + gr] = t[tx][c];
  }
}

// ---- 3b. sparsity pattern: zero the blocks of unconnected cell pairs --------
// One thread per column, rows strided over grid.y; rowcell maps a row or a
// column of C^n_W to its cell, keep is the nc x nc cell-pair matrix.
__global__ __launch_bounds__(kT) void apply_pattern(double* __restrict__ C, int64_t nt,
                                                    const int32_t* __restrict__ rowcell,
                                                    const uint8_t* __restrict__ keep, int32_t nc) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c >= nt) return;
  const int64_t cc = rowcell[c];
  for (int64_t r = blockIdx.y; r < nt; r += gridDim.y)
    if (!keep[(int64_t)rowcell[r] * nc + cc]) C[r * nt + c] = 0.0;
}

// rows [0, nc) of an nc x nc row-major block set to the identity
__global__ __launch_bounds__(kT) void identity_rows(double* __restrict__ Y, int64_t nc) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c >= nc) return;
  for (int64_t r = blockIdx.y; r < nc; r += gridDim.y) Y[r * nc + c] = r == c ? 1.0 : 0.0;
}

// ---- 4. blocked Cholesky (lower), A is n x n with leading dimension ld --------
// Factor of the diagonal block at k0 (size nb <= kNb) and the inverse of that
// factor (into linv, kNb x kNb row-major), which turns the panel solve and
// the forward substitution into products.  One wave: lane i keeps row i of
// the block in registers.  Step j takes the pivot from lane j, scales each
// lane's column-j entry, passes the scaled column through LDS and updates
// every lane's row with it (right-looking, no workgroup-wide barrier beyond
// the wave's own).  A pivot that is not positive and finite sets flag[0]
// (the factor then continues with 1).  The inverse: lane c forms column c of
// G^-1 by forward substitution, reading the factor's rows from LDS (the same
// address on every lane).
__global__ __launch_bounds__(kNb) void potrf_diag(double* __restrict__ A, int64_t ld, int64_t k0, int nb,
                                                  double* __restrict__ linv, int* __restrict__ flag) {
  __shared__ double s[kNb][kNb + 1];
  __shared__ double col[kNb];
  const int i = threadIdx.x;
  for (int e = i; e < kNb * kNb; e += kNb) {
    const int r = e / kNb, c = e % kNb;
    s[r][c] = (r < nb && c <= r) ? A[(k0 + r) * ld + k0 + c] : 0.0;
  }
  __syncthreads();
  double a[kNb];
#pragma unroll
  for (int c = 0; c < kNb; ++c) a[c] = s[i][c];
  bool bad = false;
#pragma unroll
  for (int j = 0; j < kNb; ++j) {
    if (j < nb) {
      col[i] = a[j];
      __syncthreads();
      double p = col[j];
      if (!(p > 0.0 && __builtin_isfinite(p))) {
        bad = true;
        p = 1.0;
      }
      const double d = sqrt(p), rd = 1.0 / d;
      const double lij = i > j ? a[j] * rd : (i == j ? d : 0.0);
      a[j] = lij;
      __syncthreads();
      col[i] = lij;
      __syncthreads();
#pragma unroll
      for (int c = j + 1; c < kNb; ++c) a[c] = fma(-lij, col[c], a[c]);
      __syncthreads();
    }
  }
  if (bad && i == 0) flag[0] = 1;
#pragma unroll
  for (int c = 0; c < kNb; ++c) s[i][c] = c <= i ? a[c] : 0.0;
  __syncthreads();
  for (int e = i; e < kNb * kNb; e += kNb) {
    const int r = e / kNb, c = e % kNb;
    if (r < nb && c <= r) A[(k0 + r) * ld + k0 + c] = s[r][c];
  }
  // column i of the inverse: x_r = (delta_ri - sum_{k<r} G_rk x_k) / G_rr
  double x[kNb];
#pragma unroll
  for (int r = 0; r < kNb; ++r) {
    double t = r == i ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < r; ++k) t = fma(-s[r][k], x[k], t);
    x[r] = r < nb ? t / s[r][r] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < kNb; ++r) linv[r * kNb + i] = x[r];
}

// panel below the diagonal block: rows [k0 + nb, n), columns [k0, k0 + nb):
// X = B G_kk^-T, one 64-row tile per workgroup, 4 x 4 outputs per thread
__global__ __launch_bounds__(kT) void trsm_panel(double* __restrict__ A, int64_t ld, int64_t n, int64_t k0, int nb,
                                                 const double* __restrict__ linv) {
  __shared__ double Bt[kNb][kNb + 1];  // [k][row]
  __shared__ double Li[kNb][kNb + 1];  // [k][col]: Li[k][c] = G^-1[c][k]
  const int tid = threadIdx.x;
  const int64_t r0 = k0 + nb + (int64_t)blockIdx.x * kNb;
  for (int e = tid; e < kNb * kNb; e += kT) {
    const int r = e / kNb, k = e % kNb;
    Bt[k][r] = (k < nb && r0 + r < n) ? A[(r0 + r) * ld + k0 + k] : 0.0;
    Li[k][r] = linv[r * kNb + k];
  }
  __syncthreads();
  const int tx = tid % 16, ty = tid / 16;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int k = 0; k < nb; ++k) {
    double x[4], y[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) x[a] = Bt[k][ty * 4 + a];
#pragma unroll
    for (int b = 0; b < 4; ++b) y[b] = Li[k][tx * 4 + b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = fma(x[a], y[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t r = r0 + ty * 4 + a;
    if (r >= n) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int c = tx * 4 + b;
      if (c < nb) A[r * ld + k0 + c] = acc[a][b];
    }
  }
}

// Rank-K update of the lower triangle: A[r][c] -= sum_{k < K} A[r][kc + k] A[c][kc + k]
// for rows r in [rb, n) and columns c in [cb, ce) with c <= r.  Tiles of
// kUp x kUp on the FP64 matrix cores: each of the four waves owns a 64 x 64
// quarter as 4 x 4 blocks of v_mfma_f64_16x16x4 (operands from LDS, one
// double per lane for each of A and B; the product of block (R, C) lands in
// lane l's four registers as rows l/16 + 4j, column l%16).  The matrix
// cores have the FP64 peak of the vector units, but read their operands
// from registers: a k-step of 4 reads 8 doubles per lane from LDS for 16
// products of 1,024 FMAs, where FMAs from LDS need a read per 4 FMAs.
// tri: the tiles I >= J of the square [rb, n)^2 (the trailing matrix after a
// panel of K = 256 columns); otherwise a rectangular grid of row tiles x nct
// column tiles (updates of one panel's columns).  The panel rows go through
// LDS in chunks of kUpK columns, stored k-major; each thread fetches its
// share of the next chunk into registers while the current one is used.
constexpr int kUp = 128;
constexpr int kUpK = 16;
constexpr int kOuter = 256;        // panel width of the trailing update
typedef double d4 __attribute__((ext_vector_type(4)));
// two workgroups per CU: the registers stay within 256 per lane
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(2, 2))) void update_tiles(
    double* __restrict__ A, int64_t ld, int64_t n, int64_t kc, int K, int64_t rb, int64_t cb, int64_t ce,
    int64_t nct, int tri) {
  __shared__ double Pi[kUpK][kUp + 2];  // [k][row]
  __shared__ double Pj[kUpK][kUp + 2];
  const int64_t t = blockIdx.x;
  int64_t I, J;
  if (tri) {
    I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    J = t - I * (I + 1) / 2;
  } else {
    I = t / nct;
    J = t % nct;
  }
  const int64_t ri = rb + I * kUp, rj = cb + J * kUp;
  const int tid = threadIdx.x;
  const int l = tid % 64, w = tid / 64;
  const int wr = (w / 2) * 64, wc = (w % 2) * 64;   // the wave's quarter
  const int li = l % 16, lk = l / 16;
  d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  constexpr int kPf = kUp * kUpK / kT;
  double fi[kPf], fj[kPf];
  // element q of a thread: tile row pr + q kT / kUpK, chunk column pk
  const int pr = tid / kUpK, pk = tid % kUpK;
  const int64_t oi = (ri + pr) * ld + kc + pk, oj = (rj + pr) * ld + kc + pk;
  const int64_t step = (int64_t)(kT / kUpK) * ld;
  auto fetch = [&](int kh) {
    const bool ok = kh + pk < K;
#pragma unroll
    for (int q = 0; q < kPf; ++q) {
      const int64_t r = pr + q * (kT / kUpK);
      fi[q] = (ok && ri + r < n) ? A[oi + q * step + kh] : 0.0;
      fj[q] = (ok && rj + r < ce) ? A[oj + q * step + kh] : 0.0;
    }
  };
  fetch(0);
  for (int kh = 0; kh < K; kh += kUpK) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPf; ++q) {
      Pi[pk][pr + q * (kT / kUpK)] = fi[q];
      Pj[pk][pr + q * (kT / kUpK)] = fj[q];
    }
    __syncthreads();
    if (kh + kUpK < K) fetch(kh + kUpK);
#pragma unroll 2
    for (int k4 = 0; k4 < kUpK; k4 += 4) {
      double x[4], y[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) x[a] = Pi[k4 + lk][wr + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 4; ++b) y[b] = Pj[k4 + lk][wc + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[a], y[b], acc[a][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t r = ri + wr + a * 16 + lk + 4 * j;
      if (r >= n) continue;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t c = rj + wc + b * 16 + li;
        if (c < ce && c <= r) A[r * ld + c] -= acc[a][b][j];
      }
    }
}

// ---- 5. the two reductions ------------------------------------------------------
// 2 sum log G_ii and |y|^2 in one fixed-order pass (y = G^-1 Z^n_W, the
// border row of the factor)
__global__ __launch_bounds__(kT) void logdet_quad(const double* __restrict__ A, int64_t ld, int64_t n,
                                                  const double* __restrict__ y, double* __restrict__ out) {
  __shared__ double s0[kT], s1[kT];
  const int tid = threadIdx.x;
  double a = 0.0, q = 0.0;
  for (int64_t i = tid; i < n; i += kT) {
    a += log(A[i * ld + i]);
    q = fma(y[i], y[i], q);
  }
  s0[tid] = a;
  s1[tid] = q;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if (tid < w) {
      s0[tid] += s0[tid + w];
      s1[tid] += s1[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = 2.0 * s0[0];
    out[1] = s1[0];
  }
}

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

// A second stream per device (default priority, created once) for the
// trailing updates, which then run beside the factorization of the next
// panel; events order the two.
int side_stream(hipStream_t* out) {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  MLB_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(MLBLUP_EHIP, "loglik: device index out of range");
  std::lock_guard<std::mutex> g(mu);
  if (!streams[dev]) MLB_HIP(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
  *out = streams[dev];
  return MLBLUP_OK;
}

struct Events {
  hipEvent_t e[3] = {nullptr, nullptr, nullptr};
  ~Events() {
    for (hipEvent_t x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

}  // namespace

// rows of [W_t; ...; W_n]: wavelets of the cells at depth >= n
int64_t loglik_rows(const Basis& B, int32_t level) {
  int64_t r = 0;
  for (int q = level; q < B.levels; ++q) r += B.level_counts[q];
  return r;
}

LoglikLayout loglik_layout(const Basis& B, int32_t level) {
  LoglikLayout L;
  const int64_t n = B.n, nt = loglik_rows(B, level);
  const int64_t batch = std::min<int64_t>(std::max<int64_t>(n, 1), kColBatch);
  int64_t o = 0;
  L.phi = o;
  o += align256(n * n * 8);
  L.a = o;
  o += align256(std::max<int64_t>(nt * n, 1) * 8);
  L.scal = o;
  o += align256(std::max<int64_t>(B.scal_total, 1) * batch * 8);
  L.zw = o;
  o += align256(std::max<int64_t>(n, 1) * 8);
  L.scalz = o;
  o += align256(std::max<int64_t>(B.scal_total, 1) * 8);
  L.out = o;
  o += 256;
  L.flag = o;
  o += 256;
  L.gtab = o;
  o += align256(kGenuBytes);
  L.linv = o;  // the inverse of every diagonal block of the factor
  o += align256(std::max<int64_t>((nt + kNb - 1) / kNb, 1) * kNb * kNb * 8);
  L.cells = pattern_cells(B, level);
  L.rowcell = o;
  o += align256(std::max<int64_t>(nt, 1) * 4);
  L.keep = o;
  o += align256(std::max<int64_t>((int64_t)L.cells * L.cells, 1));
  L.total = o;
  L.rows = nt;
  L.batch = batch;
  return L;
}

// rows [row_lo, row_lo + ny) of W X for the column range of X (levels B.levels-1 .. level)
static int analysis_batched(const Basis& B, const TransformDev& T, int32_t level, const double* X, int64_t ldx,
                            int64_t ncols, double* scal, int64_t batch, double* Y, int64_t ldy, int64_t row_lo,
                            int64_t ny, hipStream_t s) {
  for (int64_t c0 = 0; c0 < ncols; c0 += batch) {
    const int64_t nc = std::min(batch, ncols - c0);
    for (int q = B.levels - 1; q >= level; --q) {
      const int32_t lb = B.lvl_begin[q], cnt = B.lvl_begin[q + 1] - lb;
      if (cnt <= 0) continue;
      dim3 grid((unsigned)((nc + kT - 1) / kT), (unsigned)cnt);
      hipLaunchKernelGGL(batched_analysis, grid, dim3(kT), 0, s, T.desc, T.level_nodes + lb, T.V, X + c0, ldx, scal,
                         batch, Y + c0, ldy, row_lo, ny, nc);
    }
  }
  return hip_check(hipGetLastError(), "batched analysis launch");
}

// Phi = sigma^2 phi(|x_i - x_j|), N x N row-major; gtab: device room for the
// general-nu table
static int dense_phi(const Basis& B, const PairArgs& k, double* phi, double* gtab, hipStream_t s, int64_t j0 = 0,
                     int64_t ncols = -1, int64_t ld = -1) {
  const int64_t n = B.n;
  if (ncols < 0) ncols = n;
  if (ld < 0) ld = n;
  const double* pts = (const double*)((const char*)B.dev_base + B.off_pts);
  const double zs = kernel_scale(k.nu2, k.nu, k.rho);
  const double* gt = nullptr;
  if (k.nu2 == kNuGeneral) {
    const double* host = genu_table_cached(k.nu);
    if (!host) return fail(MLBLUP_EINVAL, "dense covariance: nu out of range for the general-nu table");
    MLB_HIP(hipMemcpyAsync(gtab, host, kGenuBytes, hipMemcpyHostToDevice, s));
    gt = gtab;
  }
  dim3 grid((unsigned)((ncols + kT - 1) / kT), (unsigned)std::min<int64_t>(n, 65535));
  switch (k.nu2) {
    case 0: hipLaunchKernelGGL(dense_cov<0>, grid, dim3(kT), 0, s, pts, n, B.d, zs, k.sigma2, gt, phi, j0, ncols, ld); break;
    case 1: hipLaunchKernelGGL(dense_cov<1>, grid, dim3(kT), 0, s, pts, n, B.d, zs, k.sigma2, gt, phi, j0, ncols, ld); break;
    case 3: hipLaunchKernelGGL(dense_cov<3>, grid, dim3(kT), 0, s, pts, n, B.d, zs, k.sigma2, gt, phi, j0, ncols, ld); break;
    case 5: hipLaunchKernelGGL(dense_cov<5>, grid, dim3(kT), 0, s, pts, n, B.d, zs, k.sigma2, gt, phi, j0, ncols, ld); break;
    default:
      hipLaunchKernelGGL(dense_cov<kNuGeneralT>, grid, dim3(kT), 0, s, pts, n, B.d, zs, k.sigma2, gt, phi, j0, ncols,
                         ld);
  }
  return hip_check(hipGetLastError(), "dense covariance launch");
}

// (W Phi W^T) restricted to the rows and columns [row_lo, row_lo + ny) of W,
// levels >= level: A = (W Phi)[rows, :] (ny x N), A^T into Phi's storage,
// then W A^T restricted to the same rows, into A's storage with ld ny
static int dense_cw_block(const Basis& B, const TransformDev& T, int32_t level, double* phi, double* A,
                          double* scal, int64_t batch, int64_t row_lo, int64_t ny, hipStream_t s) {
  const int64_t n = B.n;
  int st;
  if ((st = analysis_batched(B, T, level, phi, n, n, scal, batch, A, n, row_lo, ny, s))) return st;
  dim3 grid((unsigned)((n + kTr - 1) / kTr), (unsigned)((ny + kTr - 1) / kTr));
  hipLaunchKernelGGL(transpose, grid, dim3(kTr * 8), 0, s, A, ny, n, n, phi, ny);
  if ((st = hip_check(hipGetLastError(), "transpose launch"))) return st;
  return analysis_batched(B, T, level, phi, ny, ny, scal, batch, A, ny, row_lo, ny, s);
}

// Blocked right-looking Cholesky of the nt x nt lower triangle of C (ld nt),
// with the rows [nt, nr) below it as border rows: panels of kOuter columns,
// each factored in blocks of kNb (diagonal factor and inverse into linv,
// panel product, update of the panel's remaining columns), then the rank-
// kOuter update of the trailing matrix.  The border rows B end as B G^-T:
// a vector z as one border row gives y = G^-1 z (forward substitution), the
// identity gives G^-T.  Lookahead: after panel [ob, oe) is factored, the
// main stream updates only the next panel's columns [oe, oe2) and goes on to
// factor it, while the side stream updates the columns >= oe2; the next
// lookahead writes columns that this trailing update writes too, so it
// waits for it.  A pivot that is not positive sets flag[0].
static int cholesky_bordered(double* C, int64_t nt, int64_t nr, double* linv, int* flag, hipStream_t s) {
  int st;
  hipStream_t side;
  if ((st = side_stream(&side))) return st;
  Events ev;
  for (hipEvent_t& e : ev.e) MLB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hipEvent_t ev_fork = ev.e[0], ev_panel = ev.e[1], ev_trail = ev.e[2];
  MLB_HIP(hipEventRecord(ev_fork, s));
  MLB_HIP(hipStreamWaitEvent(side, ev_fork, 0));
  bool trail_pending = false;
  for (int64_t ob = 0; ob < nt; ob += kOuter) {
    const int64_t oe = std::min<int64_t>(nt, ob + kOuter);
    for (int64_t k0 = ob; k0 < oe; k0 += kNb) {
      const int nb = (int)std::min<int64_t>(kNb, nt - k0);
      double* li = linv + (k0 / kNb) * kNb * kNb;
      hipLaunchKernelGGL(potrf_diag, dim3(1), dim3(kNb), 0, s, C, nt, k0, nb, li, flag);
      const int64_t below = nr - k0 - nb;
      if (below > 0)
        hipLaunchKernelGGL(trsm_panel, dim3((unsigned)((below + kNb - 1) / kNb)), dim3(kT), 0, s, C, nt, nr, k0, nb,
                           li);
      const int64_t cb = k0 + nb;
      if (cb < oe) {
        const int64_t nct = (oe - cb + kUp - 1) / kUp, nrt = (nr - cb + kUp - 1) / kUp;
        hipLaunchKernelGGL(update_tiles, dim3((unsigned)(nrt * nct)), dim3(kT), 0, s, C, nt, nr, k0, nb, cb, cb, oe,
                           nct, 0);
      }
    }
    if (oe >= nt) break;
    const int64_t oe2 = std::min<int64_t>(nt, oe + kOuter), K = oe - ob;
    if (oe2 < nt) {
      MLB_HIP(hipEventRecord(ev_panel, s));
    }
    if (trail_pending) MLB_HIP(hipStreamWaitEvent(s, ev_trail, 0));
    {
      const int64_t nct = (oe2 - oe + kUp - 1) / kUp, nrt = (nr - oe + kUp - 1) / kUp;
      hipLaunchKernelGGL(update_tiles, dim3((unsigned)(nrt * nct)), dim3(kT), 0, s, C, nt, nr, ob, (int)K, oe, oe,
                         oe2, nct, 0);
    }
    if (oe2 < nt) {
      MLB_HIP(hipStreamWaitEvent(side, ev_panel, 0));
      const int64_t ut = (nr - oe2 + kUp - 1) / kUp;
      hipLaunchKernelGGL(update_tiles, dim3((unsigned)(ut * (ut + 1) / 2)), dim3(kT), 0, side, C, nt, nr, ob, (int)K,
                         oe2, oe2, nt, (int64_t)1, 1);
      MLB_HIP(hipEventRecord(ev_trail, side));
      trail_pending = true;
    }
  }
  if (trail_pending) MLB_HIP(hipStreamWaitEvent(s, ev_trail, 0));
  return hip_check(hipGetLastError(), "Cholesky launch");
}

int dense_cholesky_logdet(double* C, int64_t nt, double* linv, int* flag, double* dout, hipStream_t s) {
  int st = cholesky_bordered(C, nt, nt + 1, linv, flag, s);
  if (st) return st;
  hipLaunchKernelGGL(logdet_quad, dim3(1), dim3(kT), 0, s, C, nt, nt, C + nt * nt, dout);
  return hip_check(hipGetLastError(), "reduction launch");
}

int64_t dense_cholesky_linv_doubles(int64_t nt) { return std::max<int64_t>((nt + kNb - 1) / kNb, 1) * kNb * kNb; }

int loglik_upload_pattern(const Pattern& P, void* work, const LoglikLayout& L, hipStream_t s) {
  if (P.nc != L.cells || (int64_t)P.rowcell.size() != L.rows)
    return fail(MLBLUP_EINVAL, "loglik: sparsity pattern does not match the level");
  char* w = (char*)work;
  if (L.rows > 0) {
    MLB_HIP(hipMemcpyAsync(w + L.rowcell, P.rowcell.data(), P.rowcell.size() * 4, hipMemcpyHostToDevice, s));
    MLB_HIP(hipMemcpyAsync(w + L.keep, P.keep.data(), P.keep.size(), hipMemcpyHostToDevice, s));
  }
  MLB_HIP(hipStreamSynchronize(s));
  return MLBLUP_OK;
}

int loglik_device(const Basis& B, const TransformDev& T, const PairArgs& k, int32_t level, const double* z,
                  void* work, const LoglikLayout& L, bool masked, double out[3], hipStream_t s) {
  char* w = (char*)work;
  double* phi = (double*)(w + L.phi);
  double* A = (double*)(w + L.a);
  double* scal = (double*)(w + L.scal);
  double* zw = (double*)(w + L.zw);
  double* scalz = (double*)(w + L.scalz);
  double* dout = (double*)(w + L.out);
  int* flag = (int*)(w + L.flag);
  double* linv = (double*)(w + L.linv);
  const int64_t nt = L.rows;
  hipLaunchKernelGGL(clear_flag, dim3(1), dim3(64), 0, s, flag);
  // 1. Phi
  int st = dense_phi(B, k, phi, (double*)(w + L.gtab), s);
  if (st) return st;
  // Z^n_W: the first N~ entries of W z
  if ((st = transform_analysis(T, z, zw, nullptr, scalz, s))) return st;
  if (nt == 0) {
    out[0] = out[1] = 0.0;
    out[2] = 0.0;
    return MLBLUP_OK;
  }
  // 2./3. C^n_W = (W Phi W^T)[0:N~, 0:N~] into A's storage (ld N~)
  if ((st = dense_cw_block(B, T, level, phi, A, scal, L.batch, 0, nt, s))) return st;
  double* C = A;
  if (masked) {
    dim3 grid((unsigned)((nt + kT - 1) / kT), (unsigned)std::min<int64_t>(nt, 65535));
    hipLaunchKernelGGL(apply_pattern, grid, dim3(kT), 0, s, C, nt, (const int32_t*)(w + L.rowcell),
                       (const uint8_t*)(w + L.keep), L.cells);
    if ((st = hip_check(hipGetLastError(), "sparsity pattern launch"))) return st;
  }
  // 4./5. Cholesky with Z^n_W as the border row nt: row nt ends as y = G^-1 Z^n_W
  double* y = C + nt * nt;   // A's storage holds nt x n >= (nt + 1) x nt doubles
  MLB_HIP(hipMemcpyAsync(y, zw, nt * sizeof(double), hipMemcpyDeviceToDevice, s));
  if ((st = cholesky_bordered(C, nt, nt + 1, linv, flag, s))) return st;
  // 2 sum log G_ii and |y|^2
  hipLaunchKernelGGL(logdet_quad, dim3(1), dim3(kT), 0, s, C, nt, nt, y, dout);
  if ((st = hip_check(hipGetLastError(), "reduction launch"))) return st;
  double host[2];
  int hflag = 0;
  MLB_HIP(hipMemcpyAsync(host, dout, sizeof(host), hipMemcpyDeviceToHost, s));
  MLB_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  MLB_HIP(hipStreamSynchronize(s));
  if (hflag) return fail(MLBLUP_EBREAKDOWN, "loglik: C^n_W is not numerically positive definite");
  const double kLog2Pi = 1.8378770664093453;
  out[1] = host[0];
  out[2] = host[1];
  out[0] = -0.5 * ((double)nt * kLog2Pi + host[0] + host[1]);
  return MLBLUP_OK;
}

// ---- coarse block of C_W for the preconditioner ------------------------------
// The rows [c0, c0 + nc) of W (the coarse levels: they come last) give
// C_c = (W C W^T)[c0:, c0:].  Formed without any N x N array: Phi is made in
// panels of `batch` columns, and the batched analysis of each panel keeps
// the rows [c0, c0 + nc) of W Phi, giving A = (W Phi)[c0:, :] (nc x N);
// A^T (N x nc) then goes through the analysis once more, which gives C_c
// in A's storage (2 nc <= N since c0 >= nc).  C_c is factored G G^T = C_c
// with the identity as nc border rows, which end as Y = G^-T; then
// C_c^-1 = G^-T G^-1 = Y Y^T.  Y (nc x nc, row-major) is copied to the host.
// Workspace: N batch + 2 N nc doubles (13 GB at 65,536 points and nc = 10,230).
CoarseLayout coarse_layout(const Basis& B, int64_t nc) {
  CoarseLayout L;
  const int64_t n = B.n;
  const int64_t batch = std::min<int64_t>(std::max<int64_t>(n, 1), kColBatch);
  int64_t o = 0;
  L.phi = o;   // the Phi panel (N x batch), later A^T (N x nc)
  o += align256(std::max<int64_t>(n * std::max(batch, nc), 1) * 8);
  L.a = o;     // A (nc x N), later C_c and its border rows (2 nc x nc)
  o += align256(std::max<int64_t>(std::max(nc * n, 2 * nc * nc), 1) * 8);
  L.scal = o;
  o += align256(std::max<int64_t>(B.scal_total, 1) * batch * 8);
  L.flag = o;
  o += 256;
  L.gtab = o;
  o += align256(kGenuBytes);
  L.linv = o;
  o += align256(std::max<int64_t>((nc + kNb - 1) / kNb, 1) * kNb * kNb * 8);
  L.total = o;
  L.batch = batch;
  return L;
}

int coarse_inverse_factor(const Basis& B, const PairArgs& k, int64_t c0, int64_t nc, void* work, int64_t work_bytes,
                          std::vector<double>& Y, hipStream_t s) {
  const CoarseLayout L = coarse_layout(B, nc);
  if (!work || work_bytes < L.total)
    return fail(MLBLUP_EINVAL, "coarse preconditioner: workspace too small (need " + std::to_string(L.total) + ")");
  if (nc <= 0 || c0 < nc || c0 + nc > B.n - B.p)
    return fail(MLBLUP_EINVAL, "coarse preconditioner: bad row range (need nc <= c0, c0 + nc <= N - p)");
  char* w = (char*)work;
  double* panel = (double*)(w + L.phi);
  double* A = (double*)(w + L.a);
  double* scal = (double*)(w + L.scal);
  int* flag = (int*)(w + L.flag);
  const int64_t n = B.n;
  const TransformDev T = transform_dev(B);
  hipLaunchKernelGGL(clear_flag, dim3(1), dim3(64), 0, s, flag);
  int st;
  for (int64_t j0 = 0; j0 < n; j0 += L.batch) {
    const int64_t nb = std::min(L.batch, n - j0);
    if ((st = dense_phi(B, k, panel, (double*)(w + L.gtab), s, j0, nb, nb))) return st;
    if ((st = analysis_batched(B, T, 0, panel, nb, nb, scal, L.batch, A + j0, n, c0, nc, s))) return st;
  }
  double* at = panel;  // A^T, N x nc
  {
    dim3 grid((unsigned)((n + kTr - 1) / kTr), (unsigned)((nc + kTr - 1) / kTr));
    hipLaunchKernelGGL(transpose, grid, dim3(kTr * 8), 0, s, A, nc, n, n, at, nc);
    if ((st = hip_check(hipGetLastError(), "transpose launch"))) return st;
  }
  double* C = A;
  if ((st = analysis_batched(B, T, 0, at, nc, nc, scal, L.batch, C, nc, c0, nc, s))) return st;
  double* border = C + nc * nc;
  {
    dim3 grid((unsigned)((nc + kT - 1) / kT), (unsigned)std::min<int64_t>(nc, 65535));
    hipLaunchKernelGGL(identity_rows, grid, dim3(kT), 0, s, border, nc);
    if ((st = hip_check(hipGetLastError(), "identity launch"))) return st;
  }
  if ((st = cholesky_bordered(C, nc, 2 * nc, (double*)(w + L.linv), flag, s))) return st;
  Y.resize((size_t)nc * nc);
  int hflag = 0;
  MLB_HIP(hipMemcpyAsync(Y.data(), border, (size_t)nc * nc * sizeof(double), hipMemcpyDeviceToHost, s));
  MLB_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  MLB_HIP(hipStreamSynchronize(s));
  if (hflag) return fail(MLBLUP_EBREAKDOWN, "coarse preconditioner: the coarse block of C_W is not positive definite");
  return MLBLUP_OK;
}

}  // namespace mlb
