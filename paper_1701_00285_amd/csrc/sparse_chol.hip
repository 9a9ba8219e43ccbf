// Sparse block Cholesky of the sparsified multilevel covariance matrix
// C~^n_W (Sec. 4.1 kept blocks; Sec. 6.1: log det C~^n_W = 2 sum log L_ii
// and the quadratic form |L^-1 Z^n_W|^2 from one factor), on the device in
// FP64.  The block structure, elimination order and schedule come from the
// host analysis (sparse_analyse); every block is at most 64 x 64.
//
//  1. Assembly: every kept block of two cells a, b is
//     Psi_a^T C(S_a, S_b) Psi_b, Psi the cells' wavelet vectors on their
//     points; one workgroup per block walks S_a and S_b in chunks of 64
//     points: the 64 x 64 kernel tile in LDS, T = K Psi_b accumulated over
//     the S_b chunks in LDS, then the block += Psi_a^T T.  Fill blocks start
//     at zero.
//  2. Left-looking factorization by elimination-tree height; per height
//     three launches:
//     update: every block (i, j) of the height's columns becomes
//       A_ij - sum_k L_ik L_jk^T over the earlier columns k whose pattern
//       holds both i and j (a merge of the two row structures), one
//       workgroup per block; and per column the data block
//       z_j - sum_k L_jk y_k (the forward substitution, as a border row);
//     factor: per column, the Cholesky of the diagonal block in LDS (a
//       pivot that is not positive raises the flag), its triangular
//       inverse, y_j = L_jj^-1 (z_j - ...) and log L_jj[r][r];
//     solve: every block below a diagonal, L_ij = A_ij L_jj^-T (a product
//       with the inverse).
//     The columns of the dense tail (the last ones of the order, nearly
//     full) are not scheduled by height: one update launch applies the
//     block columns before the tail to all of its blocks and its data rows,
//     the blocks are scattered into a dense matrix with the data rows as a
//     border row, and the dense blocked Cholesky of the estimator finishes it.
//  3. Fixed-order reductions: sum log L_rr and |y|^2 over the block
//     columns, plus the dense tail's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "device.h"
#include "internal.h"
#include "pairmath.h"

namespace mlb {
namespace {

constexpr int kT = 256;
constexpr int kB = kSparseMaxBlock;   // 64
constexpr int kLd = kB + 1;           // LDS row stride (doubles)

inline int64_t al256(int64_t b) { return (b + 255) / 256 * 256; }

typedef double d4 __attribute__((ext_vector_type(4)));

// ---- 1. assembly of the kept blocks ---------------------------------------------
template <int NU2>
__global__ __launch_bounds__(kT) void sp_assemble(const double* __restrict__ pts, int d, double zs, double sigma2,
                                                  const double* __restrict__ gtab, const double* __restrict__ psi,
                                                  const int64_t* __restrict__ psi_off,
                                                  const int64_t* __restrict__ sup_beg,
                                                  const int64_t* __restrict__ sup_cnt, const int32_t* __restrict__ w,
                                                  const int32_t* __restrict__ blk_row,
                                                  const int32_t* __restrict__ blk_col,
                                                  const int64_t* __restrict__ blk_off,
                                                  const int64_t* __restrict__ list, double* __restrict__ L) {
  __shared__ double tab[kExpTab];
  __shared__ double Kt[kB * kLd];
  __shared__ double Ts[kB * kLd];
  exp_table_fill(tab);
  const double* gt = gtab;
  if constexpr (NU2 == kNuGeneralT) {
    __shared__ double gsh[kGenuDoubles];
    const int nd = kGenuOffPoly + (int)gtab[5] * (kGenuDeg + 1);
    for (int i = threadIdx.x; i < nd; i += blockDim.x) gsh[i] = gtab[i];
    gt = gsh;
  }
  const int64_t b = list[blockIdx.x];
  const int bi = blk_row[b], bk = blk_col[b];
  const int wi = w[bi], wk = w[bk];
  const int64_t si = sup_cnt[bi], sk = sup_cnt[bk];
  const double* xi = pts + sup_beg[bi] * d;
  const double* xk = pts + sup_beg[bk] * d;
  const double* Pi = psi + psi_off[bi];
  const double* Pk = psi + psi_off[bk];
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
  for (int64_t a0 = 0; a0 < si; a0 += kB) {
    const int na = (int)min<int64_t>(kB, si - a0);
    double tac[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) tac[r][c] = 0.0;
    for (int64_t b0 = 0; b0 < sk; b0 += kB) {
      const int nb = (int)min<int64_t>(kB, sk - b0);
      __syncthreads();
      for (int e = t; e < kB * kB; e += kT) {
        const int a = e >> 6, c = e & 63;
        double v = 0.0;
        if (a < na && c < nb) {
          double s = 1e-300;  // keeps the self pair away from sqrt(0) in the series branch
          for (int q = 0; q < d; ++q) {
            const double u = (xi[(a0 + a) * d + q] - xk[(b0 + c) * d + q]) * zs;
            s = fma(u, u, s);
          }
          double f = 0.0, g = 0.0;
          pair_value<NU2, 1, false>(s, tab, f, g, gt);
          v = sigma2 * f;
        }
        Kt[a * kLd + c] = v;
      }
      __syncthreads();
      // T[a][c] += sum_b K[a][b] Psi_k[b][c]  (rows 4 tr .. 4 tr + 3, columns 4 tc .. 4 tc + 3)
      for (int bb = 0; bb < nb; ++bb) {
        const double* prow = Pk + (b0 + bb) * wk;
        double pc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) pc[c] = (4 * tc + c < wk) ? prow[4 * tc + c] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double kv = Kt[(4 * tr + r) * kLd + bb];
#pragma unroll
          for (int c = 0; c < 4; ++c) tac[r][c] = fma(kv, pc[c], tac[r][c]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) Ts[(4 * tr + r) * kLd + 4 * tc + c] = tac[r][c];
    __syncthreads();
    // block[r][c] += sum_a Psi_i[a][r] T[a][c]
    for (int a = 0; a < na; ++a) {
      const double* prow = Pi + (a0 + a) * wi;
      double pr[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) pr[r] = (4 * tr + r < wi) ? prow[4 * tr + r] : 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double tv = Ts[a * kLd + 4 * tc + c];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r][c] = fma(pr[r], tv, acc[r][c]);
      }
    }
  }
  double* out = L + blk_off[b];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (4 * tr + r < wi && 4 * tc + c < wk) out[(4 * tr + r) * wk + 4 * tc + c] = acc[r][c];
}

// ---- 2. left-looking factorization, one elimination-tree height at a time ----------
// the matched columns of one chunk: at most kMatch (the merge of one batch of 64 entries of row j's
// structure adds at most 64, and a batch starts only while 64 places are left)
constexpr int kMatch = 128;
// row i's structure is searched in LDS when it holds at most this many entries (else in memory)
constexpr int kListCap = 2048;

// blocks [0, nblk): update block lvl[x]; then one data block per column cols[x - nblk]; only the
// columns k < kmax contribute (all earlier ones inside the block part; those before the dense tail
// for the tail's blocks)
__global__ __launch_bounds__(kT) void sp_update(double* __restrict__ L, const int32_t* __restrict__ w,
                                                const int32_t* __restrict__ blk_row,
                                                const int32_t* __restrict__ blk_col,
                                                const int64_t* __restrict__ blk_off,
                                                const int64_t* __restrict__ row_ptr,
                                                const int32_t* __restrict__ row_col,
                                                const int64_t* __restrict__ row_blk, const int64_t* __restrict__ lvl,
                                                int64_t nblk, const int32_t* __restrict__ cols,
                                                const double* __restrict__ zw, const int64_t* __restrict__ row0,
                                                const int64_t* __restrict__ ypos, const double* __restrict__ y,
                                                double* __restrict__ zt, int kmax) {
  __shared__ double La[kB * kLd];   // L_ik transposed: La[q][r]
  __shared__ double Lb[kB * kLd];   // L_jk transposed: Lb[q][c]
  __shared__ int64_t pa[kMatch], pb[kMatch];
  __shared__ int32_t pk[kMatch], pw[kMatch];   // matched column and its width
  __shared__ int np, fin;
  __shared__ int64_t cur[2];
  __shared__ int32_t icols[kListCap];   // row i's structure (columns), when it fits
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  if ((int64_t)blockIdx.x >= nblk) {
    // data block of column j: z_j - sum_k L_jk y_k; wave v takes the entries v, v + 4, ... of row j's
    // structure, lane r the row r, and the four partial sums are added in a fixed order
    const int j = cols[blockIdx.x - nblk];
    const int wj = w[j];
    double v = 0.0;
    if (lane < wj) {
      for (int64_t p = row_ptr[j] + wave; p < row_ptr[j + 1]; p += 4) {
        const int k = row_col[p];
        if (k >= kmax) break;
        const int wk = w[k];
        const double* lb = L + blk_off[row_blk[p]] + (int64_t)lane * wk;
        const double* yk = y + ypos[k];
        for (int q = 0; q < wk; ++q) v = fma(lb[q], yk[q], v);
      }
    }
    La[wave * kB + lane] = v;
    __syncthreads();
    if (t < wj) zt[ypos[j] + t] = zw[row0[j] + t] - ((La[t] + La[kB + t]) + (La[2 * kB + t] + La[3 * kB + t]));
    return;
  }
  const int64_t b = lvl[blockIdx.x];
  const int i = blk_row[b], j = blk_col[b];
  const int wi = w[i], wj = w[j];
  const bool full = wi > 48 && wj > 48;   // every 16 x 16 tile holds rows of the block
  double* A = L + blk_off[b];
  // the sum of the products on the FP64 matrix cores: each wave a 32 x 32 quadrant of the 64 x 64
  // block as 2 x 2 tiles of v_mfma_f64_16x16x4f64 (lane l supplies row l % 16, k l / 16 of the left
  // operand and k l / 16, column l % 16 of the right one; a tile's result lands in lane l as rows
  // l / 16 + 4 j, column l % 16, unlike the FP32 form), the k dimension in steps of 4 with zero rows
  // past w_k
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = d4{0.0, 0.0, 0.0, 0.0};
  if (t == 0) {
    cur[0] = row_ptr[i];
    cur[1] = row_ptr[j];
    fin = 0;
  }
  const int64_t bi = row_ptr[i], ei = row_ptr[i + 1], ej = row_ptr[j + 1];
  const bool ilds = ei - bi <= kListCap;   // block-uniform
  if (ilds)
    for (int64_t e = t; e < ei - bi; e += kT) icols[e] = row_col[bi + e];
  // staging: thread t holds row sr = t / 4 of both blocks at the columns sq + 4 s
  const int sr = t >> 2, sq = t & 3;
  double ra[16], rb[16];
  for (;;) {
    __syncthreads();
    if (wave == 0) {
      // the next matched columns k of the row structures of i and j (ascending lists of distinct
      // columns): each lane takes one entry of j's list and finds it in i's by bisection (in the
      // LDS copy of i's list when it fits); the matches keep the order of j's list
      int64_t p = cur[0], q = cur[1];
      int n = 0, stop = fin;
      while (!stop && n <= kMatch - 64) {
        if (q >= ej) {
          stop = 1;
          break;
        }
        const int64_t qq = q + lane;
        int kq = qq < ej ? row_col[qq] : INT32_MAX;
        if (kq >= kmax) kq = INT32_MAX;
        int64_t lo = p, hi = ei;
        if (ilds) {
          while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (icols[mid - bi] < kq) lo = mid + 1;
            else hi = mid;
          }
        } else {
          while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (row_col[mid] < kq) lo = mid + 1;
            else hi = mid;
          }
        }
        const bool match = kq != INT32_MAX && lo < ei && (ilds ? icols[lo - bi] : row_col[lo]) == kq;
        const uint64_t bal = __ballot(match);
        if (match) {
          const int pos = n + __popcll(bal & ((1ull << lane) - 1ull));
          pa[pos] = row_blk[lo];
          pb[pos] = row_blk[qq];
          pk[pos] = kq;
          pw[pos] = w[kq];
        }
        n += __popcll(bal);
        // a lane past the end of j's list or at kmax ends the merge after this batch; otherwise the
        // next batch starts after lane 63's entry, and its columns lie after lane 63's place in i's list
        if (__ballot(kq == INT32_MAX)) stop = 1;
        q += 64;
        p = __shfl(lo, 63);
      }
      if (lane == 0) {
        cur[0] = p;
        cur[1] = q;
        np = n;
        fin = stop;
      }
    }
    __syncthreads();
    const int n = np;
    if (n == 0) break;
    // software pipeline: the blocks of match m + 1 are loaded into registers while the matrix cores
    // work on match m from LDS
    auto fetch = [&](int m) {
      const int wn = pw[m];
      const double* la = L + blk_off[pa[m]];
      const double* lb = L + blk_off[pb[m]];
#pragma unroll
      for (int s4 = 0; s4 < 16; ++s4) {
        const int q = sq + 4 * s4;
        ra[s4] = (sr < wi && q < wn) ? la[sr * wn + q] : 0.0;
        rb[s4] = (sr < wj && q < wn) ? lb[sr * wn + q] : 0.0;
      }
    };
    fetch(0);
    for (int m = 0; m < n; ++m) {
      const int wk = pw[m], wk4 = (wk + 3) & ~3;
      __syncthreads();
#pragma unroll
      for (int s4 = 0; s4 < 16; ++s4) {
        const int q = sq + 4 * s4;
        if (q < wk4) {   // columns past w_k are zero
          La[q * kLd + sr] = ra[s4];
          Lb[q * kLd + sr] = rb[s4];
        }
      }
      __syncthreads();
      if (m + 1 < n) fetch(m + 1);
      if (full) {
        for (int k4 = 0; k4 < wk4; k4 += 4) {
          double x[2], yv[2];
#pragma unroll
          for (int a = 0; a < 2; ++a) x[a] = La[(k4 + lk) * kLd + wr + a * 16 + li];
#pragma unroll
          for (int c = 0; c < 2; ++c) yv[c] = Lb[(k4 + lk) * kLd + wc + c * 16 + li];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c)
              acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[a], yv[c], acc[a][c], 0, 0, 0);
        }
      } else {
        // a block of at most 48 rows or columns: the tiles wholly past w_i rows or w_j columns
        // are skipped (wave-uniform)
        for (int k4 = 0; k4 < wk4; k4 += 4) {
          double x[2], yv[2];
#pragma unroll
          for (int a = 0; a < 2; ++a) x[a] = La[(k4 + lk) * kLd + wr + a * 16 + li];
#pragma unroll
          for (int c = 0; c < 2; ++c) yv[c] = Lb[(k4 + lk) * kLd + wc + c * 16 + li];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c)
              if (wr + 16 * a < wi && wc + 16 * c < wj)
                acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[a], yv[c], acc[a][c], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int r = wr + a * 16 + lk + 4 * jj;
      if (r >= wi) continue;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int col = wc + c * 16 + li;
        if (col < wj) A[r * wj + col] -= acc[a][c][jj];
      }
    }
}

// Cholesky of the diagonal block of column cols[x], its inverse, y_j and log L_rr
__global__ __launch_bounds__(kT) void sp_factor(double* __restrict__ L, double* __restrict__ Linv,
                                                const int64_t* __restrict__ inv_off, const int32_t* __restrict__ w,
                                                const int64_t* __restrict__ col_ptr,
                                                const int64_t* __restrict__ blk_off, const int32_t* __restrict__ cols,
                                                const int64_t* __restrict__ ypos, const double* __restrict__ zt,
                                                double* __restrict__ y, double* __restrict__ logd,
                                                int* __restrict__ flag) {
  __shared__ double M[kB * kLd];
  __shared__ double X[kB * kLd];
  const int j = cols[blockIdx.x];
  const int wj = w[j];
  double* A = L + blk_off[col_ptr[j]];
  const int t = threadIdx.x;
  for (int e = t; e < wj * wj; e += kT) M[(e / wj) * kLd + e % wj] = A[e];
  for (int c = 0; c < wj; ++c) {
    __syncthreads();
    if (t == 0) {
      double piv = M[c * kLd + c];
      if (!(piv > 0.0)) {
        flag[0] = 1;
        piv = 1.0;
      }
      M[c * kLd + c] = sqrt(piv);
    }
    __syncthreads();
    const double dc = M[c * kLd + c];
    for (int r = c + 1 + t; r < wj; r += kT) M[r * kLd + c] /= dc;
    __syncthreads();
    const int rem = wj - c - 1;
    for (int e = t; e < rem * rem; e += kT) {
      const int r = c + 1 + e / rem, q = c + 1 + e % rem;
      if (q <= r) M[r * kLd + q] = fma(-M[r * kLd + c], M[q * kLd + c], M[r * kLd + q]);
    }
  }
  __syncthreads();
  // inverse of the lower triangle, column c by thread c
  if (t < wj) {
    const int c = t;
    for (int r = 0; r < c; ++r) X[r * kLd + c] = 0.0;
    for (int r = c; r < wj; ++r) {
      double s = (r == c) ? 1.0 : 0.0;
      for (int q = c; q < r; ++q) s = fma(-M[r * kLd + q], X[q * kLd + c], s);
      X[r * kLd + c] = s / M[r * kLd + r];
    }
  }
  __syncthreads();
  double* Xo = Linv + inv_off[j];
  for (int e = t; e < wj * wj; e += kT) {
    const int r = e / wj, c = e % wj;
    A[e] = (c <= r) ? M[r * kLd + c] : 0.0;
    Xo[e] = X[r * kLd + c];
  }
  if (t < wj) {
    const double* z = zt + ypos[j];
    double s = 0.0;
    for (int q = 0; q <= t; ++q) s = fma(X[t * kLd + q], z[q], s);
    y[ypos[j] + t] = s;
    logd[ypos[j] + t] = log(M[t * kLd + t]);
  }
}

// L_ij = A_ij L_jj^-T for the blocks below the diagonals of one height
__global__ __launch_bounds__(kT) void sp_solve(double* __restrict__ L, const double* __restrict__ Linv,
                                               const int64_t* __restrict__ inv_off, const int32_t* __restrict__ w,
                                               const int32_t* __restrict__ blk_row,
                                               const int32_t* __restrict__ blk_col,
                                               const int64_t* __restrict__ blk_off,
                                               const int64_t* __restrict__ lvl) {
  __shared__ double As[kB * kLd];   // A_ij transposed: As[q][r]
  __shared__ double Xs[kB * kLd];   // L_jj^-1 transposed: Xs[q][c] = X[c][q]
  const int64_t b = lvl[blockIdx.x];
  const int i = blk_row[b], j = blk_col[b];
  if (i == j) return;
  const int wi = w[i], wj = w[j];
  double* A = L + blk_off[b];
  const double* X = Linv + inv_off[j];
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
  for (int e = t; e < wi * wj; e += kT) As[(e % wj) * kLd + e / wj] = A[e];
  for (int e = t; e < wj * wj; e += kT) Xs[(e % wj) * kLd + e / wj] = X[e];
  __syncthreads();
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
  for (int q = 0; q < wj; ++q) {
    double av[4], xv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) av[r] = As[q * kLd + 4 * tr + r];
#pragma unroll
    for (int c = 0; c < 4; ++c) xv[c] = Xs[q * kLd + 4 * tc + c];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = fma(av[r], xv[c], acc[r][c]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (4 * tr + r < wi && 4 * tc + c < wj) A[(4 * tr + r) * wj + 4 * tc + c] = acc[r][c];
}

// the tail's blocks into the dense T x T matrix C (rows and columns from the position-ordered
// offsets, minus y0), both triangles from the lower one
__global__ __launch_bounds__(kT) void sp_scatter(const double* __restrict__ L, const int32_t* __restrict__ w,
                                                 const int32_t* __restrict__ blk_row,
                                                 const int32_t* __restrict__ blk_col,
                                                 const int64_t* __restrict__ blk_off,
                                                 const int64_t* __restrict__ ypos, const int64_t* __restrict__ list,
                                                 int64_t y0, int64_t T, double* __restrict__ C) {
  const int64_t b = list[blockIdx.x];
  const int i = blk_row[b], j = blk_col[b];
  const int wi = w[i], wj = w[j];
  const int64_t r0 = ypos[i] - y0, c0 = ypos[j] - y0;
  const double* A = L + blk_off[b];
  for (int e = threadIdx.x; e < wi * wj; e += kT) {
    const int r = e / wj, c = e - r * wj;
    // a diagonal block's two triangles agree only up to rounding: the lower one is kept
    if (i == j && c > r) continue;
    C[(r0 + r) * T + c0 + c] = A[e];
    C[(c0 + c) * T + r0 + r] = A[e];
  }
}

// out = {sum logd, sum y^2} in a fixed order (one workgroup)
__global__ __launch_bounds__(kT) void sp_reduce(const double* __restrict__ logd, const double* __restrict__ y,
                                                int64_t n, double* __restrict__ out) {
  __shared__ double s0[kT], s1[kT];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kT) {
    a += logd[i];
    b = fma(y[i], y[i], b);
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int h = kT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s0[threadIdx.x] += s0[threadIdx.x + h];
      s1[threadIdx.x] += s1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = 2.0 * s0[0];
    out[1] = s1[0];
  }
}

__global__ void sp_clear_flag(int* __restrict__ flag) {
  if (threadIdx.x == 0) flag[0] = 0;
}

template <typename T>
int put(char* w, int64_t off, const std::vector<T>& v, hipStream_t s) {
  if (v.empty()) return MLBLUP_OK;
  MLB_HIP(hipMemcpyAsync(w + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return MLBLUP_OK;
}

}  // namespace

SparseLayout sparse_layout(const Basis& B, const SparseSymbolic& S) {
  SparseLayout Ly;
  const int64_t nc = S.nc, nblk = S.col_ptr.empty() ? 0 : S.col_ptr[nc];
  int64_t inv = 0;
  for (int64_t k = 0; k < nc; ++k) inv += (int64_t)S.w[k] * S.w[k];
  int64_t nkept = 0;
  for (int64_t b = 0; b < nblk; ++b) nkept += S.blk_kept[b];
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    const int64_t r = o;
    o += al256(std::max<int64_t>(bytes, 1));
    return r;
  };
  Ly.L = take(S.factor_entries * 8);
  Ly.linv = take(inv * 8);
  Ly.psi = take((int64_t)S.psi.size() * 8);
  Ly.zw = take(B.n * 8);
  Ly.scal = take(std::max<int64_t>(B.scal_total, 1) * 8);
  Ly.zt = take(S.rows * 8);
  Ly.y = take(S.rows * 8);
  Ly.logd = take(S.rows * 8);
  Ly.out = take(16);
  Ly.flag = take(4);
  Ly.gtab = take(kGenuBytes);
  Ly.w = take(nc * 4);
  Ly.row0 = take(nc * 8);
  Ly.ypos = take(nc * 8);
  Ly.inv_off = take(nc * 8);
  Ly.sup_beg = take(nc * 8);
  Ly.sup_cnt = take(nc * 8);
  Ly.psi_off = take((nc + 1) * 8);
  Ly.col_ptr = take((nc + 1) * 8);
  Ly.blk_row = take(nblk * 4);
  Ly.blk_col = take(nblk * 4);
  Ly.blk_off = take((nblk + 1) * 8);
  Ly.row_ptr = take((nc + 1) * 8);
  Ly.row_col = take((int64_t)S.row_col.size() * 4);
  Ly.row_blk = take((int64_t)S.row_blk.size() * 8);
  Ly.lvl_blks = take(nblk * 8);
  Ly.lvl_cols = take(nc * 4);
  Ly.kept = take(nkept * 8);
  const int64_t T = S.tail_rows;
  Ly.dense = take(T > 0 ? (T + 1) * T * 8 : 8);
  Ly.dense_linv = take(T > 0 ? dense_cholesky_linv_doubles(T) * 8 : 8);
  Ly.dense_out = take(16);
  Ly.tail_blks = take((int64_t)S.tail_blks.size() * 8);
  Ly.tail_cols = take((int64_t)S.tail_cols.size() * 4);
  Ly.total = o;
  Ly.nkept = nkept;
  return Ly;
}

int loglik_sparse_device(const Basis& B, const TransformDev& T, const PairArgs& k, const SparseSymbolic& S,
                         const double* z, void* work, const SparseLayout& Ly, double out[3], hipStream_t s) {
  char* w = (char*)work;
  const int64_t nc = S.nc;
  const int64_t nblk = nc ? S.col_ptr[nc] : 0;
  double* dz = (double*)(w + Ly.zw);
  int st;
  // Z^n_W: the first N~ entries of W z
  if ((st = transform_analysis(T, z, dz, nullptr, (double*)(w + Ly.scal), s))) return st;
  if (S.rows == 0) {
    out[0] = out[1] = out[2] = 0.0;
    return MLBLUP_OK;
  }
  // index arrays
  std::vector<int64_t> inv_off(nc), sup_beg(nc), sup_cnt(nc), kept;
  int64_t io = 0;
  for (int64_t q = 0; q < nc; ++q) {
    inv_off[q] = io;
    io += (int64_t)S.w[q] * S.w[q];
    sup_beg[q] = B.begin[S.node[q]];
    sup_cnt[q] = B.end[S.node[q]] - B.begin[S.node[q]];
  }
  for (int64_t b = 0; b < nblk; ++b)
    if (S.blk_kept[b]) kept.push_back(b);
  if ((st = put(w, Ly.psi, S.psi, s)) || (st = put(w, Ly.w, S.w, s)) || (st = put(w, Ly.row0, S.row0, s)) ||
      (st = put(w, Ly.ypos, S.ypos, s)) || (st = put(w, Ly.inv_off, inv_off, s)) ||
      (st = put(w, Ly.sup_beg, sup_beg, s)) || (st = put(w, Ly.sup_cnt, sup_cnt, s)) ||
      (st = put(w, Ly.psi_off, S.psi_off, s)) || (st = put(w, Ly.col_ptr, S.col_ptr, s)) ||
      (st = put(w, Ly.blk_row, S.blk_row, s)) || (st = put(w, Ly.blk_col, S.blk_col, s)) ||
      (st = put(w, Ly.blk_off, S.blk_off, s)) || (st = put(w, Ly.row_ptr, S.row_ptr, s)) ||
      (st = put(w, Ly.row_col, S.row_col, s)) || (st = put(w, Ly.row_blk, S.row_blk, s)) ||
      (st = put(w, Ly.lvl_blks, S.lvl_blks, s)) || (st = put(w, Ly.lvl_cols, S.lvl_cols, s)) ||
      (st = put(w, Ly.kept, kept, s)) || (st = put(w, Ly.tail_blks, S.tail_blks, s)) ||
      (st = put(w, Ly.tail_cols, S.tail_cols, s)))
    return st;
  double* Ld = (double*)(w + Ly.L);
  double* Linv = (double*)(w + Ly.linv);
  const int32_t* dw = (const int32_t*)(w + Ly.w);
  const int32_t* brow = (const int32_t*)(w + Ly.blk_row);
  const int32_t* bcol = (const int32_t*)(w + Ly.blk_col);
  const int64_t* boff = (const int64_t*)(w + Ly.blk_off);
  int* flag = (int*)(w + Ly.flag);
  hipLaunchKernelGGL(sp_clear_flag, dim3(1), dim3(64), 0, s, flag);
  MLB_HIP(hipMemsetAsync(Ld, 0, S.factor_entries * 8, s));
  // 1. assembly
  const double* pts = (const double*)((const char*)B.dev_base + B.off_pts);
  const double zs = kernel_scale(k.nu2, k.nu, k.rho);
  const double* gt = nullptr;
  if (k.nu2 == kNuGeneral) {
    const double* host = genu_table_cached(k.nu);
    if (!host) return fail(MLBLUP_EINVAL, "sparse loglik: nu out of range for the general-nu table");
    MLB_HIP(hipMemcpyAsync(w + Ly.gtab, host, kGenuBytes, hipMemcpyHostToDevice, s));
    gt = (const double*)(w + Ly.gtab);
  }
  if (!kept.empty()) {
    const dim3 grid((unsigned)kept.size());
    const double* psi = (const double*)(w + Ly.psi);
    const int64_t* po = (const int64_t*)(w + Ly.psi_off);
    const int64_t* sb = (const int64_t*)(w + Ly.sup_beg);
    const int64_t* sc = (const int64_t*)(w + Ly.sup_cnt);
    const int64_t* kl = (const int64_t*)(w + Ly.kept);
#define MLB_SP_ASM(N)                                                                                          \
  hipLaunchKernelGGL(sp_assemble<N>, grid, dim3(kT), 0, s, pts, B.d, zs, k.sigma2, gt, psi, po, sb, sc, dw, brow, \
                     bcol, boff, kl, Ld)
    switch (k.nu2) {
      case 0: MLB_SP_ASM(0); break;
      case 1: MLB_SP_ASM(1); break;
      case 3: MLB_SP_ASM(3); break;
      case 5: MLB_SP_ASM(5); break;
      default: MLB_SP_ASM(kNuGeneralT);
    }
#undef MLB_SP_ASM
    if ((st = hip_check(hipGetLastError(), "sparse assembly launch"))) return st;
  }
  // 2. factorization by elimination-tree height
  const int64_t* rptr = (const int64_t*)(w + Ly.row_ptr);
  const int32_t* rcol = (const int32_t*)(w + Ly.row_col);
  const int64_t* rblk = (const int64_t*)(w + Ly.row_blk);
  const int64_t* lblk = (const int64_t*)(w + Ly.lvl_blks);
  const int32_t* lcol = (const int32_t*)(w + Ly.lvl_cols);
  const int64_t* row0 = (const int64_t*)(w + Ly.row0);
  const int64_t* ypos = (const int64_t*)(w + Ly.ypos);
  const int64_t* ioff = (const int64_t*)(w + Ly.inv_off);
  const int64_t* cptr = (const int64_t*)(w + Ly.col_ptr);
  double* zt = (double*)(w + Ly.zt);
  double* y = (double*)(w + Ly.y);
  double* logd = (double*)(w + Ly.logd);
  const int64_t heights = (int64_t)S.lvl_ptr.size() - 1;
  for (int64_t h = 0; h < heights; ++h) {
    const int64_t c0 = S.lvl_ptr[h], ncol = S.lvl_ptr[h + 1] - c0;
    const int64_t b0 = S.lvl_blk_ptr[h], nb = S.lvl_blk_ptr[h + 1] - b0;
    if (ncol == 0) continue;
    hipLaunchKernelGGL(sp_update, dim3((unsigned)(nb + ncol)), dim3(kT), 0, s, Ld, dw, brow, bcol, boff, rptr, rcol,
                       rblk, lblk + b0, nb, lcol + c0, dz, row0, ypos, y, zt, (int)nc);
    hipLaunchKernelGGL(sp_factor, dim3((unsigned)ncol), dim3(kT), 0, s, Ld, Linv, ioff, dw, cptr, boff, lcol + c0,
                       ypos, zt, y, logd, flag);
    if (nb > ncol)
      hipLaunchKernelGGL(sp_solve, dim3((unsigned)nb), dim3(kT), 0, s, Ld, Linv, ioff, dw, brow, bcol, boff, lblk + b0);
  }
  if ((st = hip_check(hipGetLastError(), "sparse factorization launch"))) return st;
  // dense tail: the updates from the block columns before it, then the dense bordered Cholesky
  double tail_host[2] = {0.0, 0.0};
  double* dtail = (double*)(w + Ly.dense_out);
  const int64_t nT = S.tail_rows;
  if (S.tail < nc && nT > 0) {
    const int64_t ntb = (int64_t)S.tail_blks.size(), ntc = (int64_t)S.tail_cols.size();
    const int64_t* tblk = (const int64_t*)(w + Ly.tail_blks);
    const int32_t* tcol = (const int32_t*)(w + Ly.tail_cols);
    hipLaunchKernelGGL(sp_update, dim3((unsigned)(ntb + ntc)), dim3(kT), 0, s, Ld, dw, brow, bcol, boff, rptr, rcol,
                       rblk, tblk, ntb, tcol, dz, row0, ypos, y, zt, (int)S.tail);
    double* C = (double*)(w + Ly.dense);
    MLB_HIP(hipMemsetAsync(C, 0, nT * nT * 8, s));
    hipLaunchKernelGGL(sp_scatter, dim3((unsigned)ntb), dim3(kT), 0, s, Ld, dw, brow, bcol, boff, ypos, tblk,
                       S.ypos[S.tail], nT, C);
    if ((st = hip_check(hipGetLastError(), "sparse tail launch"))) return st;
    // the data rows of the tail as the border row
    MLB_HIP(hipMemcpyAsync(C + nT * nT, zt + S.ypos[S.tail], nT * 8, hipMemcpyDeviceToDevice, s));
    if ((st = dense_cholesky_logdet(C, nT, (double*)(w + Ly.dense_linv), flag, dtail, s))) return st;
  }
  // 3. reduction over the rows of the block columns
  double* dout = (double*)(w + Ly.out);
  const int64_t nsp = S.tail < nc ? S.ypos[S.tail] : S.rows;
  hipLaunchKernelGGL(sp_reduce, dim3(1), dim3(kT), 0, s, logd, y, nsp, dout);
  if ((st = hip_check(hipGetLastError(), "sparse reduction launch"))) return st;
  double host[2];
  int hflag = 0;
  MLB_HIP(hipMemcpyAsync(host, dout, sizeof(host), hipMemcpyDeviceToHost, s));
  if (S.tail < nc && nT > 0) MLB_HIP(hipMemcpyAsync(tail_host, dtail, sizeof(tail_host), hipMemcpyDeviceToHost, s));
  MLB_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  MLB_HIP(hipStreamSynchronize(s));
  if (hflag) return fail(MLBLUP_EBREAKDOWN, "sparse loglik: C~^n_W is not numerically positive definite");
  host[0] += tail_host[0];
  host[1] += tail_host[1];
  const double kLog2Pi = 1.8378770664093453;
  out[1] = host[0];
  out[2] = host[1];
  out[0] = -0.5 * ((double)S.rows * kLog2Pi + host[0] + host[1]);
  return MLBLUP_OK;
}

}  // namespace mlb
