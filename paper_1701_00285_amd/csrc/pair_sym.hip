// Symmetric square product y = C x (C_ij = C_ji): every unordered pair is
// evaluated once and feeds both row sums.
//
// Blocks of 256 RL points (tree order; RL = 4 rows per lane for d <= 6,
// 3 for d >= 16 in FP64, else 2).  A workgroup (4 waves x 64 lanes x RL
// rows) owns a row block S
// and one column block S'.  Column points stream
// through LDS in chunks of 128; a wave walks each group of 64 columns in 64
// steps in which lane l evaluates column (l + k*delta) mod 64 of the group
// (a lane-varying LDS read) for its RL rows.  Row sums stay in the lane;
// the column sum of the lane's current column travels with it: a register
// is rotated by one lane (DPP wave rotate) after every step, so after 64
// steps lane l holds the wave's whole contribution to column l.  The four
// waves' column sums are added in fixed order through LDS.
//
// Schedule without atomics: diagonal tiles (S, S) are computed as full
// squares (row sums only), each split over 4 column ranges (2 for RL = 3).  Off-diagonal tiles follow a round-robin
// tournament: in round r = 1..T/2, block S pairs with (S + r) mod T (for
// even T the last round keeps S < T/2 only), so in one round every block
// is a row block at most once and a column block at most once; each round
// writes one row-partial and one column-partial vector, and the rounds are
// summed in fixed order.  Results are bitwise reproducible.
//
// Squared distances in FP64: from coordinate differences for d < 8; for
// d >= 8 from |a|^2 + |b|^2 - 2 a.b with both points taken relative to the
// row block's first point (norms of the column points staged with them in
// LDS), which halves the per-pair arithmetic of the distance; the few pairs
// where that form cancels badly are recomputed from the differences.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "pairmath.h"

namespace mlb {
namespace {

constexpr int kT = 256;
constexpr int kChunk = 128; // columns staged per LDS fill
constexpr int kDiagSplit = 4;  // column ranges of a diagonal tile (one partial slot each)

// rows per lane: 4 for small d (amortises the LDS read and the rotation over
// more pairs); from d = 8 on the expanded-form FP64 kernel reads d + 2
// doubles per column step, 3 rows per lane for d >= 16 keep that LDS traffic
// below the LDS bandwidth; a block holds 256 * RL points
constexpr int rows_per_lane(int D) { return D <= 6 ? 4 : (D >= 16 && D <= 20 ? 3 : 2); }
constexpr int rows_per_lane_lp(int D) { return D <= 6 ? 4 : 2; }

// column ranges of a diagonal tile: whole chunks each
constexpr int diag_split(int RL) { return RL == 3 ? 2 : kDiagSplit; }

// (row block, round offset) of an off-diagonal workgroup of a launch of nr
// rounds over T blocks.  Workgroups go to the 8 XCDs in turn (linear id mod
// 8); the ids one XCD receives are renumbered consecutively and walked in
// groups of 8 row blocks x 8 rounds, so the workgroups an XCD runs at one
// time read 8 row blocks and 15 column blocks (S + round) instead of 64 of
// each, and those stay in its L2.  The map is a bijection onto the grid for
// any T and nr (the rows and rounds past whole groups are walked in order),
// and each workgroup still writes its own partial slots, so the results do
// not depend on it.
__device__ __forceinline__ void tile_of(int T, int nr, int& S, int& y) {
  const int total = T * nr;
  const int i = (int)blockIdx.x + T * (int)blockIdx.y;
  const int q = total / 8, rem = total % 8;
  const int x = i % 8, j = i / 8;
  const int v = x < rem ? x * (q + 1) + j : rem * (q + 1) + (x - rem) * q + j;
  const int T8 = T / 8 * 8, n8 = nr / 8 * 8;
  const int full = T8 * n8;
  if (v < full) {
    const int g = v / 64, w = v % 64;
    S = (g % (T8 / 8)) * 8 + w / 8;
    y = (g / (T8 / 8)) * 8 + w % 8;
  } else {
    int u = v - full;
    const int a = (T - T8) * n8;  // row blocks past the groups, rounds inside them
    if (u < a) {
      S = T8 + u % (T - T8);
      y = u / (T - T8);
    } else {
      u -= a;
      S = u % T;
      y = n8 + u / T;
    }
  }
}

template <int D, int NU2, int OUT>
__global__ __launch_bounds__(kT) void sym_kernel(const double* __restrict__ pts, int dd, const double* __restrict__ x,
                                                 int64_t n, int T, int round0, int diag, double zs,
                                                 double* __restrict__ prow, double* __restrict__ pcol,
                                                 double* __restrict__ pdrow, double* __restrict__ pdcol,
                                                 const double* __restrict__ gtab) {
  // D >= 8: squared distances from the expanded form |a|^2 + |b|^2 - 2 a.b
  // (D FMAs instead of 2D), coordinates taken relative to the row block's
  // first point; a pair whose result has lost more than 6 bits to
  // cancellation (s < |a|^2 + |b|^2 times 2^-6, which includes every self
  // pair and near neighbour) is recomputed from the coordinate differences
  constexpr bool kGram = D >= 8;
  constexpr int SD = kGram ? D + 2 : D + 1;  // coordinates, x (and |b|^2)
  constexpr int RL = rows_per_lane(D);
  constexpr int kBlk = 256 * RL;
  constexpr double kGuard = 0.015625;
  static_assert(kBlk % (diag_split(RL) * kChunk) == 0, "a diagonal tile splits into whole chunks");
  // column chunk: each group of 64 columns twice over (slots s and s + 64 hold column s), so that a
  // lane's column index moves by one slot per step without wrapping
  __shared__ double cp[2 * kChunk * SD];
  __shared__ double cred[4][kChunk];
  __shared__ double cdred[4][kChunk];
  __shared__ double tab[kExpTab];
  // diagonal launches: row block blockIdx.x, column range blockIdx.y; others: tile_of
  int S = blockIdx.x, yy = blockIdx.y;
  if (!diag) tile_of(T, (int)gridDim.y, S, yy);
  const int r = round0 + (diag ? 0 : yy);
  int Sp = S;
  if (!diag) {
    Sp = (S + r) % T;
    if ((T % 2 == 0) && (2 * r == T) && S >= T / 2) return;  // whole block exits
  }
  exp_table_fill(tab);
  // general nu: the table in LDS (read by every pair)
  const double* gt = gtab;
  if constexpr (NU2 == kNuGeneralT) {
    __shared__ double gsh[kGenuDoubles];
    const int nd = kGenuOffPoly + (int)gtab[5] * (kGenuDeg + 1);
    for (int i = threadIdx.x; i < nd; i += blockDim.x) gsh[i] = gtab[i];
    gt = gsh;
  }
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // lane rotation direction: after one rotation lane l holds lane (l + delta)'s value
  const int delta = (wave_rotate1_i(lane) - lane) & 63;

  // origin of the expanded form: the row block's first point (o < n)
  const int64_t o = (int64_t)S * kBlk;
  double xr[RL][D], ar[RL], nx[RL];
#pragma unroll
  for (int q = 0; q < RL; ++q) {
    const int64_t i = (int64_t)S * kBlk + wave * (64 * RL) + q * 64 + lane;
    const int64_t ii = i < n ? i : n - 1;
    nx[q] = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double v = k >= dd ? 0.0 : kGram ? (pts[ii * dd + k] - pts[o * dd + k]) * zs : pts[ii * dd + k] * zs;
      nx[q] = fma(v, v, nx[q]);
      xr[q][k] = kGram ? -2.0 * v : v;   // the expanded form keeps -2 a (exact)
    }
    ar[q] = i < n ? x[i] : 0.0;
  }
  double racc[RL], rdacc[RL];
#pragma unroll
  for (int q = 0; q < RL; ++q) racc[q] = rdacc[q] = 0.0;
  const int64_t cbase = (int64_t)Sp * kBlk;
  // a diagonal tile is split over gridDim.y column ranges (one partial slot each)
  const int cfirst = diag ? yy * (kBlk / (int)gridDim.y) : 0;
  const int clast = diag ? cfirst + kBlk / (int)gridDim.y : kBlk;
  for (int c0 = cfirst; c0 < clast; c0 += kChunk) {
    __syncthreads();
    // column j of the chunk goes to slots (j / 64) 128 + j % 64 and that + 64
    for (int e = tid; e < kChunk * D; e += kT) {
      const int j = e / D, k = e - j * D;
      const int64_t gj = cbase + c0 + j;
      const double v = gj < n && k < dd ? (kGram ? (pts[gj * dd + k] - pts[o * dd + k]) * zs : pts[gj * dd + k] * zs)
                                         : 0.0;
      const int sl = (j >> 6) * 128 + (j & 63);
      cp[sl * SD + k] = v;
      cp[(sl + 64) * SD + k] = v;
    }
    for (int j = tid; j < kChunk; j += kT) {
      const int64_t gj = cbase + c0 + j;
      const int sl = (j >> 6) * 128 + (j & 63);
      const double v = gj < n ? x[gj] : 0.0;
      cp[sl * SD + D] = v;
      cp[(sl + 64) * SD + D] = v;
    }
    if constexpr (kGram) {
      __syncthreads();
      for (int j = tid; j < kChunk; j += kT) {
        const int sl = (j >> 6) * 128 + (j & 63);
        double nb = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) nb = fma(cp[sl * SD + k], cp[sl * SD + k], nb);
        cp[sl * SD + D + 1] = nb;
        cp[(sl + 64) * SD + D + 1] = nb;
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int sub = 0; sub < kChunk; sub += 64) {
      double cacc = 0.0, cdacc = 0.0;
      // step k visits column (lane + k delta) mod 64 of the group: slot lane + k (delta = 1) or
      // lane + 64 - k (delta = -1 mod 64); slots are indexed (not stepped by pointer) so that the
      // 128-bit alignment of a slot (SD even) stays visible to the compiler
      const int ds = delta == 1 ? 1 : -1;
      int sl = 2 * sub + lane + (delta == 1 ? 0 : 64);
      {
#pragma unroll 2
        for (int k = 0; k < 64; ++k, sl += ds) {
          const double* cj = &cp[sl * SD];
          double cv[D];
#pragma unroll
          for (int t = 0; t < D; ++t) cv[t] = cj[t];
          const double aj = cj[D];
          double cpart = 0.0, cdpart = 0.0;
#pragma unroll
          for (int q = 0; q < RL; ++q) {
            double s;
            if constexpr (kGram) {
              // |a|^2 + |b|^2 - 2 a.b as one FMA chain from the norms (xr holds -2 a)
              const double tt = nx[q] + cj[D + 1];
              s = tt;
#pragma unroll
              for (int t = 0; t < D; ++t) s = fma(xr[q][t], cv[t], s);
              if (!(s > kGuard * tt)) {
                s = 1e-300;
#pragma unroll
                for (int t = 0; t < D; ++t) {
                  const double u = fma(0.5, xr[q][t], cv[t]);   // b - a, one rounding
                  s = fma(u, u, s);
                }
              }
            } else {
              s = 1e-300;
#pragma unroll
              for (int t = 0; t < D; ++t) {
                const double u = xr[q][t] - cv[t];
                s = fma(u, u, s);
              }
            }
            double f = 0.0, g = 0.0;
            pair_value<NU2, OUT, false>(s, tab, f, g, gt);
            if constexpr (OUT & 1) {
              racc[q] = fma(f, aj, racc[q]);
              cpart = fma(f, ar[q], cpart);
            }
            if constexpr (OUT & 2) {
              rdacc[q] = fma(g, aj, rdacc[q]);
              cdpart = fma(g, ar[q], cdpart);
            }
          }
          if constexpr (OUT & 1) cacc = wave_rotate1(cacc + cpart);
          if constexpr (OUT & 2) cdacc = wave_rotate1(cdacc + cdpart);
        }
      }
      if constexpr (OUT & 1) cred[wave][sub + lane] = cacc;
      if constexpr (OUT & 2) cdred[wave][sub + lane] = cdacc;
    }
    __syncthreads();
    if (!diag && tid < kChunk) {
      const int64_t gj = cbase + c0 + tid;
      if (gj < n) {
        const int64_t slot = (int64_t)yy * n + gj;
        if constexpr (OUT & 1) pcol[slot] = ((cred[0][tid] + cred[1][tid]) + cred[2][tid]) + cred[3][tid];
        if constexpr (OUT & 2) pdcol[slot] = ((cdred[0][tid] + cdred[1][tid]) + cdred[2][tid]) + cdred[3][tid];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RL; ++q) {
    const int64_t i = (int64_t)S * kBlk + wave * (64 * RL) + q * 64 + lane;
    if (i < n) {
      const int64_t slot = (int64_t)yy * n + i;
      if constexpr (OUT & 1) prow[slot] = racc[q];
      if constexpr (OUT & 2) pdrow[slot] = rdacc[q];
    }
  }
}

// FP32 variant.  Coordinates are taken relative to the first point of the
// row block (kd-tree blocks are compact, so row coordinates stay small),
// scaled by the kernel's coordinate scale times lp_scale in FP64 and rounded
// to FP32; the pair value comes from pair_value_lp.  Row sums accumulate in FP32 over 16
// columns and then in FP64; the travelling column sums are FP64.
template <int D, int NU2, int OUT>
__global__ __launch_bounds__(kT) void sym_kernel_lp(const double* __restrict__ pts, int dd, const double* __restrict__ x,
                                                    int64_t n, int T, int round0, int diag, double ws,
                                                    double* __restrict__ prow, double* __restrict__ pcol,
                                                    double* __restrict__ pdrow, double* __restrict__ pdcol) {
  constexpr int SP = (D + 1 + 3) / 4 * 4;  // floats per staged column (coordinates, x), 16-byte rows
  constexpr int RL = rows_per_lane_lp(D);
  constexpr int kBlk = 256 * RL;
  constexpr int kSeg = 16;  // columns per FP32 row-sum segment
  // column chunk: each group of 64 columns twice over (slots s and s + 64 hold column s)
  __shared__ __align__(16) float cp[2 * kChunk * SP];
  // column partials per (wave, column group, segment of kSeg steps, column), FP32 within a segment
  __shared__ float cseg[4][kChunk / 64][64 / kSeg][64];
  __shared__ float cdseg[(OUT & 2) ? 4 : 1][kChunk / 64][64 / kSeg][64];
  // diagonal launches: row block blockIdx.x, column range blockIdx.y; others: tile_of
  int S = blockIdx.x, yy = blockIdx.y;
  if (!diag) tile_of(T, (int)gridDim.y, S, yy);
  const int r = round0 + (diag ? 0 : yy);
  int Sp = S;
  if (!diag) {
    Sp = (S + r) % T;
    if ((T % 2 == 0) && (2 * r == T) && S >= T / 2) return;  // whole block exits
  }
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int delta = (wave_rotate1_i(lane) - lane) & 63;

  const int64_t o = (int64_t)S * kBlk;  // first point of the row block (o < n)
  float xr[RL][D], ar[RL];
#pragma unroll
  for (int q = 0; q < RL; ++q) {
    const int64_t i = o + wave * (64 * RL) + q * 64 + lane;
    const int64_t ii = i < n ? i : n - 1;
#pragma unroll
    for (int k = 0; k < D; ++k) xr[q][k] = k < dd ? (float)((pts[ii * dd + k] - pts[o * dd + k]) * ws) : 0.0f;
    ar[q] = i < n ? (float)x[i] : 0.0f;
  }
  double racc[RL], rdacc[RL];
#pragma unroll
  for (int q = 0; q < RL; ++q) racc[q] = rdacc[q] = 0.0;
  const int64_t cbase = (int64_t)Sp * kBlk;
  const int cfirst = diag ? yy * (kBlk / (int)gridDim.y) : 0;
  const int clast = diag ? cfirst + kBlk / (int)gridDim.y : kBlk;
  for (int c0 = cfirst; c0 < clast; c0 += kChunk) {
    __syncthreads();
    for (int e = tid; e < kChunk * D; e += kT) {
      const int j = e / D, k = e - j * D;
      const int64_t gj = cbase + c0 + j;
      const float v = gj < n && k < dd ? (float)((pts[gj * dd + k] - pts[o * dd + k]) * ws) : 0.0f;
      const int sl = (j >> 6) * 128 + (j & 63);
      cp[sl * SP + k] = v;
      cp[(sl + 64) * SP + k] = v;
    }
    for (int j = tid; j < kChunk; j += kT) {
      const int64_t gj = cbase + c0 + j;
      const float v = gj < n ? (float)x[gj] : 0.0f;
      const int sl = (j >> 6) * 128 + (j & 63);
      cp[sl * SP + D] = v;
      cp[(sl + 64) * SP + D] = v;
    }
    __syncthreads();
#pragma unroll 1
    for (int sub = 0; sub < kChunk; sub += 64) {
      // step k visits column (lane + k delta) mod 64 of the group: slot lane + k (delta = 1) or
      // lane + 64 - k (delta = -1 mod 64)
      const int ds = delta == 1 ? 1 : -1;
      int sl = 2 * sub + lane + (delta == 1 ? 0 : 64);
#pragma unroll 1
      for (int seg = 0; seg < 64; seg += kSeg) {
        float rs[RL], rds[RL];
#pragma unroll
        for (int q = 0; q < RL; ++q) rs[q] = rds[q] = 0.0f;
        // the column sums travel with their columns in FP32 for one segment
        float cacc = 0.0f, cdacc = 0.0f;
#pragma unroll 4
        for (int k = 0; k < kSeg; ++k, sl += ds) {
          const float* cj = &cp[sl * SP];
          float cv[D];
#pragma unroll
          for (int t = 0; t < D; ++t) cv[t] = cj[t];
          const float aj = cj[D];
          float cpart = 0.0f, cdpart = 0.0f;
#pragma unroll
          for (int q = 0; q < RL; ++q) {
            float s = 0.0f;
#pragma unroll
            for (int t = 0; t < D; ++t) {
              const float u = xr[q][t] - cv[t];
              s = fmaf(u, u, s);
            }
            float f = 0.0f, g = 0.0f;
            pair_value_lp<NU2, OUT>(s, f, g);
            if constexpr (OUT & 1) {
              rs[q] = fmaf(f, aj, rs[q]);
              cpart = fmaf(f, ar[q], cpart);
            }
            if constexpr (OUT & 2) {
              rds[q] = fmaf(g, aj, rds[q]);
              cdpart = fmaf(g, ar[q], cdpart);
            }
          }
          if constexpr (OUT & 1) cacc = wave_rotate1_f(cacc + cpart);
          if constexpr (OUT & 2) cdacc = wave_rotate1_f(cdacc + cdpart);
        }
#pragma unroll
        for (int q = 0; q < RL; ++q) {
          if constexpr (OUT & 1) racc[q] += (double)rs[q];
          if constexpr (OUT & 2) rdacc[q] += (double)rds[q];
        }
        // after seg + kSeg steps this lane holds the segment's sum of column lane + (seg + kSeg) delta
        const int col = (lane + (seg + kSeg) * delta) & 63;
        if constexpr (OUT & 1) cseg[wave][sub >> 6][seg / kSeg][col] = cacc;
        if constexpr (OUT & 2) cdseg[wave][sub >> 6][seg / kSeg][col] = cdacc;
      }
    }
    __syncthreads();
    if (!diag && tid < kChunk) {
      const int64_t gj = cbase + c0 + tid;
      if (gj < n) {
        const int64_t slot = (int64_t)yy * n + gj;
        const int g = tid >> 6, cc = tid & 63;
        // per wave the segments in order, then the waves in order (FP64)
        auto colsum = [&](const float* a) {
          double v[4];
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            v[w] = 0.0;
#pragma unroll
            for (int q = 0; q < 64 / kSeg; ++q) v[w] += (double)a[((w * (kChunk / 64) + g) * (64 / kSeg) + q) * 64 + cc];
          }
          return ((v[0] + v[1]) + v[2]) + v[3];
        };
        if constexpr (OUT & 1) pcol[slot] = colsum(&cseg[0][0][0][0]);
        if constexpr (OUT & 2) pdcol[slot] = colsum(&cdseg[0][0][0][0]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RL; ++q) {
    const int64_t i = o + wave * (64 * RL) + q * 64 + lane;
    if (i < n) {
      const int64_t slot = (int64_t)yy * n + i;
      if constexpr (OUT & 1) prow[slot] = racc[q];
      if constexpr (OUT & 2) pdrow[slot] = rdacc[q];
    }
  }
}

// acc += sum over this launch's rounds of row and column partials (fixed
// order); on the last launch y = scale * acc.  acc starts as the diagonal
// partial.
__global__ __launch_bounds__(kT) void sym_reduce(const double* __restrict__ prow, const double* __restrict__ pcol,
                                                 int nr, int rows_summed, int64_t n, int T, int round0, int last,
                                                 double scale, double* __restrict__ acc, double* __restrict__ y,
                                                 int blk_pts) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const int blk = (int)(i / blk_pts);
  double s = acc[i];
  // one row partial for all the launch's rounds, or one per round
  if (rows_summed) s += prow[i];
  for (int q = 0; q < nr; ++q) {
    const int r = round0 + q;
    const bool half = (T % 2 == 0) && (2 * r == T);
    // as a row of block blk: absent in the half round for blk >= T/2
    if (!rows_summed && !(half && blk >= T / 2)) s += prow[(int64_t)q * n + i];
    // as a column: written by block (blk - r) mod T; absent in the half round when that block >= T/2
    const int src = ((blk - r) % T + T) % T;
    if (!(half && src >= T / 2)) s += pcol[(int64_t)q * n + i];
  }
  if (last) y[i] = scale * s;
  else acc[i] = s;
}

template <int D, int NU2, int OUT, bool F>
void launch(const double* pts, int dd, const double* x, int64_t n, int T, int round0, int nr, int diag, double zs,
            double* prow, double* pcol, double* pdrow, double* pdcol, const double* gtab, hipStream_t s) {
  if constexpr (F)
    hipLaunchKernelGGL((sym_kernel_lp<D, NU2, OUT>), dim3(T, nr), dim3(kT), 0, s, pts, dd, x, n, T, round0, diag,
                       zs * lp_scale<NU2>(), prow, pcol, pdrow, pdcol);
  else
    hipLaunchKernelGGL((sym_kernel<D, NU2, OUT>), dim3(T, nr), dim3(kT), 0, s, pts, dd, x, n, T, round0, diag, zs,
                       prow, pcol, pdrow, pdcol, gtab);
}

using LaunchFn = void (*)(const double*, int, const double*, int64_t, int, int, int, int, double, double*, double*,
                          double*, double*, const double*, hipStream_t);

template <int NU2, int OUT, bool F>
LaunchFn pick_d(int d) {
  switch (padded_dim(d)) {
    case 1: return launch<1, NU2, OUT, F>;
    case 2: return launch<2, NU2, OUT, F>;
    case 3: return launch<3, NU2, OUT, F>;
    case 4: return launch<4, NU2, OUT, F>;
    case 5: return launch<5, NU2, OUT, F>;
    case 6: return launch<6, NU2, OUT, F>;
    case 8: return launch<8, NU2, OUT, F>;
    case 10: return launch<10, NU2, OUT, F>;
    case 16: return launch<16, NU2, OUT, F>;
    case 20: return launch<20, NU2, OUT, F>;
    case 24: return launch<24, NU2, OUT, F>;
    case 28: return launch<28, NU2, OUT, F>;
    case 32: return launch<32, NU2, OUT, F>;
    default: return nullptr;
  }
}
template <int NU2, bool F>
LaunchFn pick_out(int out, int d) {
  if (out == 1) return pick_d<NU2, 1, F>(d);
  if (out == 2) return pick_d<NU2, 2, F>(d);
  return pick_d<NU2, 3, F>(d);
}
template <bool F>
LaunchFn pick_nu(int nu2, int out, int d) {
  if constexpr (!F) {
    if (nu2 == kNuGeneral) return out == 1 ? pick_d<kNuGeneralT, 1, false>(d) : nullptr;  // FP64 values only
  }
  if (nu2 == 0) return pick_out<0, F>(out, d);
  if (nu2 == 1) return pick_out<1, F>(out, d);
  if (nu2 == 3) return pick_out<3, F>(out, d);
  return pick_out<5, F>(out, d);
}

constexpr int kRoundsPerLaunch = 16;

__global__ __launch_bounds__(kT) void sum_slots(const double* __restrict__ slots, int k, int64_t n,
                                                double* __restrict__ acc) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int q = 0; q < k; ++q) s += slots[(int64_t)q * n + i];
  acc[i] = s;
}

}  // namespace

bool sym_supported(int d) { return pick_nu<false>(1, 1, d) != nullptr; }

// below this size the tiled row kernel wins (too few blocks to fill the chip)
bool sym_worthwhile(int64_t n) { return n >= 16384; }

int64_t sym_workspace_bytes(int64_t n, int outputs) {
  const int64_t per = (int64_t)(2 * kRoundsPerLaunch + 1 + kDiagSplit) * n * 8;
  const int64_t a = (per + 255) / 256 * 256;
  return a * ((outputs & 1 ? 1 : 0) + (outputs & 2 ? 1 : 0));
}

int sym_schedule(const PairArgs& a, int blk_pts, void* work, hipStream_t s, const SymTileLaunch& fn,
                 bool rows_summed, int diag_splits) {
  const int nsplit = diag_splits > 0 ? std::min(diag_splits, kDiagSplit) : kDiagSplit;
  const int64_t n = a.n;
  const int T = (int)((n + blk_pts - 1) / blk_pts);
  const int64_t per = ((int64_t)(2 * kRoundsPerLaunch + 1 + kDiagSplit) * n * 8 + 255) / 256 * 256;
  double* base_v = (a.outputs & 1) ? (double*)work : nullptr;
  double* base_d = (a.outputs & 2) ? (double*)((char*)work + ((a.outputs & 1) ? per : 0)) : nullptr;
  // per output: [kDiagSplit diagonal slots | accumulator | row partials | column partials]
  auto parts = [&](double* b, double*& pslots, double*& pacc, double*& prow, double*& pcol) {
    pslots = b;
    pacc = b ? b + (int64_t)kDiagSplit * n : nullptr;
    prow = b ? b + (int64_t)(kDiagSplit + 1) * n : nullptr;
    pcol = b ? b + (int64_t)(kDiagSplit + 1 + kRoundsPerLaunch) * n : nullptr;
  };
  double *vs, *vd, *vr, *vc, *ds, *dd, *dr, *dc;
  parts(base_v, vs, vd, vr, vc);
  parts(base_d, ds, dd, dr, dc);
  const unsigned g = (unsigned)((n + kT - 1) / kT);
  // diagonal tiles, each split over nsplit column ranges
  fn(T, 0, nsplit, 1, vs, nullptr, ds, nullptr);
  if (a.outputs & 1) hipLaunchKernelGGL(sum_slots, dim3(g), dim3(kT), 0, s, vs, nsplit, n, vd);
  if (a.outputs & 2) hipLaunchKernelGGL(sum_slots, dim3(g), dim3(kT), 0, s, ds, nsplit, n, dd);
  const int rounds = T / 2;
  int r0 = 1;
  do {
    const int nr = std::max(0, std::min(kRoundsPerLaunch, rounds - r0 + 1));
    if (nr > 0) fn(T, r0, nr, 0, vr, vc, dr, dc);
    const int last = (r0 + nr > rounds) ? 1 : 0;
    if (a.outputs & 1)
      hipLaunchKernelGGL(sym_reduce, dim3(g), dim3(kT), 0, s, vr, vc, nr, (rows_summed && nr > 0) ? 1 : 0, n, T, r0, last,
                         a.sigma2, vd, a.y, blk_pts);
    if (a.outputs & 2)
      hipLaunchKernelGGL(sym_reduce, dim3(g), dim3(kT), 0, s, dr, dc, nr, (rows_summed && nr > 0) ? 1 : 0, n, T, r0, last,
                         a.sigma2, dd, a.dy, blk_pts);
    r0 += kRoundsPerLaunch;
  } while (r0 <= rounds);
  return hip_check(hipGetLastError(), "symmetric pair kernel launch");
}

int sym_launch(const PairArgs& a, double zs, void* work, hipStream_t s) {
  const bool f32 = a.precision != MLBLUP_FP64;
  LaunchFn fn = f32 ? pick_nu<true>(a.nu2, a.outputs, a.d) : pick_nu<false>(a.nu2, a.outputs, a.d);
  if (!fn) return fail(MLBLUP_EINVAL, "symmetric pair kernel: dimension not compiled");
  const int dp = padded_dim(a.d);
  const int rl = f32 ? rows_per_lane_lp(dp) : rows_per_lane(dp);
  return sym_schedule(
      a, 256 * rl, work, s,
      [&](int T, int r0, int nr, int diag, double* prow, double* pcol, double* pdrow, double* pdcol) {
        fn(a.cols, a.d, a.x, a.n, T, r0, nr, diag, zs, prow, pcol, pdrow, pdcol, a.gtab, s);
      },
      false, diag_split(rl));
}

}  // namespace mlb
