// Covariance product with the squared distances from a Gram matrix on the
// matrix cores: r^2 = |a|^2 + |b|^2 - 2 a.b (intended for d >= 8, where the
// d differences per pair dominate the direct form).
//
// A workgroup owns 64 rows (4 waves x one 16-row tile) and one column range.
// All coordinates are scaled by sqrt(2 nu)/rho and centred on one row of the
// block in FP64, then rounded: FP32 for v_mfma_f32_16x16x4_f32, or a BF16
// hi + lo split for v_mfma_f32_16x16x16_bf16 with three products
// (hi.hi + hi.lo + lo.hi).  Centring keeps |a|, |b| small for the near pairs
// that the cancellation in |a|^2 + |b|^2 - 2 a.b would otherwise hurt; the
// 16-column tiles that overlap the workgroup's own rows of a square product
// (self pairs and the nearest neighbours, since points are in tree order)
// take exact FP64 differences instead.  The squared distance is clamped at
// 0, the kernel value uses FP32 sqrt/exp2, sums are FP64.
//
// Fragment layouts of the 16x16 MFMA forms: for 16x16x4 (FP32), lane l
// supplies A[l%16][l/16] and B[l/16][l%16]; for 16x16x16 (BF16) lane l
// supplies A[l%16][4(l/16)+e] and B[4(l/16)+e][l%16], e = 0..3; for
// 16x16x32 (BF16) 8 values of k per lane, the same k for A and B; in all the
// result D[4(l/16)+r][l%16], r = 0..3, sits in the lane's 4 accumulators.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "device.h"
#include "pairmath.h"

namespace mlb {
namespace {

constexpr int kT = 256;
constexpr int kRows = 64;    // rows per workgroup
constexpr int kChunk = 64;   // columns per LDS fill

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// v_mfma_f32_16x16x32_bf16 on BF16 bit patterns: lane l supplies A[l%16][k]
// and B[k][l%16] for the 8 k of its lane group; A and B use the same k
// assignment (k = 8 (l/16) + e here), which is all a dot product needs
__device__ __forceinline__ f4 mfma_bf16_k32(s8 a, s8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

template <int NU2>
__device__ __forceinline__ double value32(double s) {
  s = s > 0.0 ? s : 0.0;
  const float z = __builtin_amdgcn_sqrtf((float)s);
  const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * z);
  return (double)(matern_polyf<NU2>(z) * e);
}

// KP: padded dimension (multiple of 4 for FP32, of 16 for BF16)
template <int KP, int NU2, bool BF>
__global__ __launch_bounds__(kT) void mfma_kernel(const double* __restrict__ rows, int64_t m,
                                                  const double* __restrict__ cols, int64_t n, int d,
                                                  const double* __restrict__ x, double* __restrict__ py, double zs,
                                                  int64_t cps, int self) {
  __shared__ float cf[kChunk * KP];               // FP32 centred coordinates (FP32 mode)
  __shared__ unsigned short chi[kChunk * KP];     // BF16 hi (BF16 mode)
  __shared__ unsigned short clo[kChunk * KP];     // BF16 lo
  __shared__ double cn[kChunk];                   // column squared norms (of the rounded coordinates)
  __shared__ double cx[kChunk];
  __shared__ double ctr[64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t rb = (int64_t)blockIdx.x * kRows;
  // centre: the block's middle row (scaled)
  {
    int64_t ci = rb + 32;
    if (ci >= m) ci = m - 1;
    if (tid < d) ctr[tid] = rows[ci * d + tid] * zs;
  }
  __syncthreads();
  // row fragment: row rb + 16 wave + lr, k indices owned by this lane
  const int64_t irow = rb + 16 * wave + lr;
  const int64_t irc = irow < m ? irow : m - 1;
  float ra[BF ? 1 : KP / 4];
  s4 rhi[BF ? KP / 16 : 1], rlo[BF ? KP / 16 : 1];
  if constexpr (!BF) {
#pragma unroll
    for (int t = 0; t < KP / 4; ++t) {
      const int k = 4 * t + lg;
      ra[t] = k < d ? (float)(rows[irc * d + k] * zs - ctr[k]) : 0.0f;
    }
  } else {
#pragma unroll
    for (int t = 0; t < KP / 16; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 16 * t + 4 * lg + e;
        const float v = k < d ? (float)(rows[irc * d + k] * zs - ctr[k]) : 0.0f;
        const unsigned short h = bf16_rne(v);
        const unsigned short l = bf16_rne(v - bf16_to_f(h));
        rhi[t][e] = (short)h;
        rlo[t][e] = (short)l;
      }
  }
  // squared norms of the 4 rows whose results this lane holds (rows 4 lg + r of the tile)
  double rn[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int64_t i = rb + 16 * wave + 4 * lg + r;
    if (i >= m) i = m - 1;
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
      const float v = (float)(rows[i * d + k] * zs - ctr[k]);
      double vv;
      if constexpr (BF) {
        const unsigned short h = bf16_rne(v);
        vv = (double)bf16_to_f(h) + (double)bf16_to_f(bf16_rne(v - bf16_to_f(h)));
      } else {
        vv = (double)v;
      }
      s = fma(vv, vv, s);
    }
    rn[r] = s;
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t c0 = (int64_t)blockIdx.y * cps;
  const int64_t c1 = (c0 + cps < n) ? c0 + cps : n;
  for (int64_t j0 = c0; j0 < c1; j0 += kChunk) {
    const int cnt = (int)((c1 - j0) < kChunk ? (c1 - j0) : kChunk);
    __syncthreads();
    for (int e = tid; e < kChunk * KP; e += kT) {
      const int j = e / KP, k = e - j * KP;
      const float v = (j < cnt && k < d) ? (float)(cols[(j0 + j) * d + k] * zs - ctr[k]) : 0.0f;
      if constexpr (BF) {
        const unsigned short h = bf16_rne(v);
        chi[e] = h;
        clo[e] = bf16_rne(v - bf16_to_f(h));
      } else {
        cf[e] = v;
      }
    }
    for (int j = tid; j < kChunk; j += kT) cx[j] = j < cnt ? x[j0 + j] : 0.0;
    __syncthreads();
    for (int j = tid; j < kChunk; j += kT) {
      double s = 0.0;
      for (int k = 0; k < d; ++k) {
        double vv;
        if constexpr (BF) vv = (double)bf16_to_f(chi[j * KP + k]) + (double)bf16_to_f(clo[j * KP + k]);
        else vv = (double)cf[j * KP + k];
        s = fma(vv, vv, s);
      }
      cn[j] = s;
    }
    __syncthreads();
#pragma unroll 1
    for (int tile = 0; tile < kChunk / 16; ++tile) {
      const int jc = tile * 16 + lr;          // this lane's column in the chunk
      const int64_t jt = j0 + tile * 16;      // first column of the tile
      const bool near = self && (jt < rb + kRows) && (jt + 16 > rb);
      if (near) {
        // exact FP64 differences
        const int64_t j = j0 + jc;
        const int64_t jj = (jc < cnt) ? j : j0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int64_t i = rb + 16 * wave + 4 * lg + r;
          if (i >= m) i = m - 1;
          double s = 0.0;
          for (int k = 0; k < d; ++k) {
            const double t = (rows[i * d + k] - cols[jj * d + k]) * zs;
            s = fma(t, t, s);
          }
          acc[r] = fma(value32<NU2>(s), cx[jc], acc[r]);
        }
        continue;
      }
      f4 g = {0.0f, 0.0f, 0.0f, 0.0f};
      if constexpr (!BF) {
#pragma unroll
        for (int t = 0; t < KP / 4; ++t) {
          const float b = cf[jc * KP + 4 * t + lg];
          g = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[t], b, g, 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int t = 0; t < KP / 16; ++t) {
          s4 bh, bl;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            bh[e] = (short)chi[jc * KP + 16 * t + 4 * lg + e];
            bl[e] = (short)clo[jc * KP + 16 * t + 4 * lg + e];
          }
          g = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(rhi[t], bh, g, 0, 0, 0);
          g = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(rhi[t], bl, g, 0, 0, 0);
          g = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(rlo[t], bh, g, 0, 0, 0);
        }
      }
      const double nc = cn[jc], xc = cx[jc];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double s = fma(-2.0, (double)g[r], rn[r] + nc);
        acc[r] = fma(value32<NU2>(s), xc, acc[r]);
      }
    }
  }
  // rows 4 lg + r: reduce over the 16 lanes of the group (the 16 columns)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double v = acc[r];
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    acc[r] = v;
  }
  if (lr == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = rb + 16 * wave + 4 * lg + r;
      if (i < m) py[(int64_t)blockIdx.y * m + i] = acc[r];
    }
  }
}

// Symmetric square product on the matrix cores: blocks of 4 waves x kSymRT
// row tiles of 16 points, the tournament schedule of the direct symmetric
// kernel (diagonal tiles split over column ranges, each block a row block
// and a column block at most once per round).  Row sums stay in the lanes
// (FP32 within a chunk, FP64 across chunks; 16 column lanes per row,
// reduced at the end); each lane's column partial over its rows goes to
// LDS, and the 16 partials of a column (4 row groups x 4 waves) are added
// after the chunk.  On diagonal tiles the 16x16 sub-tiles whose rows and
// columns are the same points (self pairs and their nearest neighbours)
// take exact FP64 differences from LDS; every other pair uses the Gram.
constexpr int kSymRT = 4;
constexpr int kSymBlk = 4 * 16 * kSymRT;
constexpr int kMaxDExact = 33;

// exact squared distance of two staged chunk points from their FP64 scaled coordinates
template <int KP>
__device__ __forceinline__ float exact_sq(const double* cexact, int a, int b, int d) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    if (k >= d) break;
    const double t = cexact[a * kMaxDExact + k] - cexact[b * kMaxDExact + k];
    s = fma(t, t, s);
  }
  return (float)s;
}

template <int KP, int NU2, bool BF>
__global__ __launch_bounds__(kT) void mfma_sym_kernel(const double* __restrict__ pts, const double* __restrict__ x,
                                                      int64_t n, int d, int T, int round0, int diag, double zs,
                                                      double* __restrict__ prow, double* __restrict__ pcol) {
  __shared__ float cf[kChunk * KP];
  __shared__ unsigned short chi[kChunk * KP];
  __shared__ unsigned short clo[kChunk * KP];
  __shared__ float cnp[2][kChunk];  // column squared norms, two halves of the coordinates
  __shared__ double cx[kChunk];
  __shared__ double cexact[kChunk * kMaxDExact];
  __shared__ float csum[4][4][kChunk];  // column partials per (wave, row group of 4 lanes x 4 rows)
  __shared__ double ctr[32];
  const int S = blockIdx.x;
  const int rr = round0 + (diag ? 0 : (int)blockIdx.y);
  int Sp = S;
  if (!diag) {
    Sp = (S + rr) % T;
    if ((T % 2 == 0) && (2 * rr == T) && S >= T / 2) return;  // whole block exits
  }
  // wave index in a scalar register: branches on it stay wave-uniform
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t rb = (int64_t)S * kSymBlk, cb = (int64_t)Sp * kSymBlk;
  {
    int64_t ci = rb + kSymBlk / 2;
    if (ci >= n) ci = n - 1;
    if (tid < d) ctr[tid] = pts[ci * d + tid] * zs;
  }
  __syncthreads();
  float af[BF ? 1 : kSymRT][BF ? 1 : KP / 4];
  s4 ahi[BF ? kSymRT : 1][BF ? KP / 16 : 1], alo[BF ? kSymRT : 1][BF ? KP / 16 : 1];
  float rn[kSymRT][4], xr[kSymRT][4];
  double racc[kSymRT][4];
#pragma unroll
  for (int rt = 0; rt < kSymRT; ++rt) {
    const int64_t i0 = rb + wave * (16 * kSymRT) + rt * 16 + lr;  // the row whose A fragment this lane holds
    const int64_t ia = i0 < n ? i0 : n - 1;
    float part = 0.0f;  // this lane's share of |a|^2 for row lr
    if constexpr (!BF) {
#pragma unroll
      for (int t = 0; t < KP / 4; ++t) {
        const int k = 4 * t + lg;
        af[rt][t] = k < d ? (float)(pts[ia * d + k] * zs - ctr[k]) : 0.0f;
        part = fmaf(af[rt][t], af[rt][t], part);
      }
    } else {
#pragma unroll
      for (int t = 0; t < KP / 16; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = 16 * t + 4 * lg + e;
          const float v = k < d ? (float)(pts[ia * d + k] * zs - ctr[k]) : 0.0f;
          const unsigned short h = bf16_rne(v);
          const unsigned short l = bf16_rne(v - bf16_to_f(h));
          ahi[rt][t][e] = (short)h;
          alo[rt][t][e] = (short)l;
          const float vv = bf16_to_f(h) + bf16_to_f(l);
          part = fmaf(vv, vv, part);
        }
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);  // every lane: |a|^2 of row lr
    const float xa = i0 < n ? (float)x[i0] : 0.0f;
    // the result rows of this lane are 4 lg + r: fetch their norm and x from lane 4 lg + r
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      rn[rt][r] = __shfl(part, 4 * lg + r, 64);
      xr[rt][r] = __shfl(xa, 4 * lg + r, 64);
      racc[rt][r] = 0.0;
    }
  }
  const int cfirst = diag ? (int)blockIdx.y * (kSymBlk / (int)gridDim.y) : 0;
  const int clast = diag ? cfirst + kSymBlk / (int)gridDim.y : kSymBlk;
  // column staging: thread t stages column t mod 128 of a chunk, coordinates
  // [h KH, (h+1) KH) with h = t / 128; the next chunk's loads are issued
  // before the current chunk's tiles so that they overlap with them
  constexpr int KH = KP / 2;
  const int sj = tid & (kChunk - 1), sh = tid >> 7;
  double pre[KH];
  double prex = 0.0;
  auto fetch = [&](int cc) {
    const int64_t gj = cb + cc + sj;
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      const int kk = sh * KH + k;
      pre[k] = (gj < n && kk < d) ? pts[gj * d + kk] : 0.0;
    }
    prex = (gj < n && sh == 0) ? x[gj] : 0.0;
  };
  fetch(cfirst);
  for (int c0 = cfirst; c0 < clast; c0 += kChunk) {
    __syncthreads();
    {
      const bool okj = cb + c0 + sj < n;
      float part = 0.0f;
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int kk = sh * KH + k;
        const bool ok = okj && kk < d;
        const double xs = pre[k] * zs;
        const float v = ok ? (float)(xs - ctr[kk]) : 0.0f;
        float vv;
        if constexpr (BF) {
          const unsigned short h = bf16_rne(v);
          const unsigned short l = bf16_rne(v - bf16_to_f(h));
          chi[sj * KP + kk] = h;
          clo[sj * KP + kk] = l;
          vv = bf16_to_f(h) + bf16_to_f(l);
        } else {
          cf[sj * KP + kk] = v;
          vv = v;
        }
        part = fmaf(vv, vv, part);
        if (diag && kk < kMaxDExact) cexact[sj * kMaxDExact + kk] = xs;
      }
      cnp[sh][sj] = part;
      if (sh == 0) cx[sj] = prex;
    }
    __syncthreads();
    if (c0 + kChunk < clast) fetch(c0 + kChunk);
    float rs[kSymRT][4];  // this chunk's row sums (FP32, 8 terms per lane)
#pragma unroll
    for (int rt = 0; rt < kSymRT; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) rs[rt][r] = 0.0f;
    // tiles of this chunk inside the column range (a diagonal split can be narrower than a chunk)
    const int ntile = (clast - c0 < kChunk ? clast - c0 : kChunk) / 16;
    // Gram of the 16 columns of a tile with the wave's kSymRT row tiles
    auto gram = [&](int tile, f4 (&gg)[kSymRT]) {
      const int jc = tile * 16 + lr;
#pragma unroll
      for (int rt = 0; rt < kSymRT; ++rt) gg[rt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      if constexpr (!BF) {
        float bf[KP / 4];
#pragma unroll
        for (int t = 0; t < KP / 4; ++t) bf[t] = cf[jc * KP + 4 * t + lg];
#pragma unroll
        for (int t = 0; t < KP / 4; ++t)
#pragma unroll
          for (int rt = 0; rt < kSymRT; ++rt) gg[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[rt][t], bf[t], gg[rt], 0, 0, 0);
      } else {
        s4 bh[KP / 16], bl[KP / 16];
#pragma unroll
        for (int t = 0; t < KP / 16; ++t)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            bh[t][e] = (short)chi[jc * KP + 16 * t + 4 * lg + e];
            bl[t][e] = (short)clo[jc * KP + 16 * t + 4 * lg + e];
          }
#pragma unroll
        for (int t = 0; t < KP / 16; ++t)
#pragma unroll
          for (int rt = 0; rt < kSymRT; ++rt) {
            gg[rt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi[rt][t], bh[t], gg[rt], 0, 0, 0);
            gg[rt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi[rt][t], bl[t], gg[rt], 0, 0, 0);
            gg[rt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo[rt][t], bh[t], gg[rt], 0, 0, 0);
          }
      }
    };
    // kernel values of a tile from its Gram: row sums in the lanes, the
    // lane's column partial to LDS
    auto values = [&](int tile, const f4 (&gg)[kSymRT]) {
      const int jc = tile * 16 + lr;
      const float xc = (float)cx[jc];
      const float ncol = cnp[0][jc] + cnp[1][jc];
      float cpart = 0.0f;
#pragma unroll
      for (int rt = 0; rt < kSymRT; ++rt) {
        const f4 g = gg[rt];
        const bool same = diag && (wave * (16 * kSymRT) + rt * 16 == c0 + tile * 16);
        float sv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) sv[r] = fmaxf(fmaf(-2.0f, g[r], rn[rt][r] + ncol), 0.0f);
        if (same) {
#pragma unroll
          for (int r = 0; r < 4; ++r) sv[r] = exact_sq<KP>(cexact, tile * 16 + 4 * lg + r, jc, d);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float ph, unused;
          pair_value_w<NU2, 1>(__builtin_amdgcn_sqrtf(sv[r]), ph, unused);
          rs[rt][r] = fmaf(ph, xc, rs[rt][r]);
          cpart = fmaf(ph, xr[rt][r], cpart);
        }
      }
      // column jc: this lane's rows; the row groups and waves are added after the chunk
      if (!diag) csum[wave][lg][jc] = cpart;
    };
#pragma unroll 1
    for (int tile = 0; tile < ntile; ++tile) {
      f4 gg[kSymRT];
      gram(tile, gg);
      values(tile, gg);
    }
#pragma unroll
    for (int rt = 0; rt < kSymRT; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) racc[rt][r] += (double)rs[rt][r];
    __syncthreads();
    if (!diag && tid < kChunk) {
      const int64_t gj = cb + c0 + tid;
      if (gj < n) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < 4; ++w)
#pragma unroll
          for (int g = 0; g < 4; ++g) t += (double)csum[w][g][tid];
        pcol[(int64_t)blockIdx.y * n + gj] = t;
      }
    }
  }
  // row sums: reduce over the 16 column lanes of each row group
#pragma unroll
  for (int rt = 0; rt < kSymRT; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = racc[rt][r];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      const int64_t i = rb + wave * (16 * kSymRT) + rt * 16 + 4 * lg + r;
      if (lr == 0 && i < n) prow[(int64_t)blockIdx.y * n + i] = v;
    }
}

// Off-diagonal rounds on the matrix cores.  A workgroup keeps row block S
// (4 waves x kSymRT row tiles of 16) in registers for all the rounds of a
// launch and streams the column blocks (S + r) mod T through LDS, kRChunk
// columns at a time.  The Gram is augmented so that the matrix cores return
// the squared distance itself: rows carry (-2 a, |a|^2, 1) and columns
// (b, 1, |b|^2) in the coordinates k < d, k = d and k = d + 1 (so
// d + 2 <= KP; the padding k >= d + 2 is zero, written once).  Row sums:
// FP32 within a round (16 columns per lane), FP64 across rounds (reduced
// over the 16 column lanes at the end), one row partial per launch.  Column
// partials: one per round, as in the other symmetric kernels.
//
// BF16 x3 uses v_mfma_f32_16x16x32_bf16 when KP is a multiple of 32, else
// the 16x16x16 form.  These run beside the VALU, so the Gram of the next
// 16-column tile is issued between the kernel values of the current one
// (scheduling groups of one MFMA and a few VALU instructions).  FP32 MFMAs
// hold the VALU while they run; the same order costs nothing there.
//
// Workgroups are dealt to the 8 XCDs in turn; the row blocks are numbered so
// that each XCD takes a contiguous range of them, whose column blocks
// overlap (shared L2).
constexpr int kRChunk = 128;
constexpr int kRTiles = kRChunk / 16;
constexpr int kChunksPerRound = kSymBlk / kRChunk;

template <int KP, bool BF>
struct RoundsShape {
  static constexpr int KW = BF ? (KP % 32 == 0 ? 32 : 16) : 4;  // k per MFMA
  static constexpr int KT = KP / KW;                            // k steps of one Gram
  static constexpr int KE = KW / 4;                             // k per lane and step
  static constexpr int KH = KP / 2;                             // coordinates per staging thread
};

template <int KP, int NU2, bool BF>
__global__ __launch_bounds__(kT, 2) void mfma_rounds_kernel(const double* __restrict__ pts,
                                                            const double* __restrict__ x, int64_t n, int d, int T,
                                                            int round0, int nr, double zs, double* __restrict__ prow,
                                                            double* __restrict__ pcol) {
  using Sh = RoundsShape<KP, BF>;
  constexpr int KW = Sh::KW, KT = Sh::KT, KE = Sh::KE, KH = Sh::KH;
  using frag = typename std::conditional<KE == 8, s8, s4>::type;
  // column operands by k step: [KT][kRChunk][KW] (FP32, or BF16 hi and lo)
  constexpr int kOps = KT * kRChunk * KW;
  __shared__ __attribute__((aligned(16))) float cf[BF ? 4 : kOps];
  __shared__ __attribute__((aligned(16))) unsigned short chi[BF ? kOps : 8];
  __shared__ __attribute__((aligned(16))) unsigned short clo[BF ? kOps : 8];
  __shared__ double cx[kRChunk];
  __shared__ float csum[4][4][kRChunk];  // column partials per (wave, row group)
  __shared__ double ctr[32];
  auto op_index = [](int kk, int j) { return ((kk / KW) * kRChunk + j) * KW + (kk % KW); };
  int S;
  {
    const int b = (int)blockIdx.x, q = T / 8, rem = T % 8, xcd = b % 8;
    S = xcd * q + (xcd < rem ? xcd : rem) + b / 8;
  }
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t rb = (int64_t)S * kSymBlk;
  {
    int64_t ci = rb + kSymBlk / 2;
    if (ci >= n) ci = n - 1;
    if (tid < d) ctr[tid] = pts[ci * d + tid] * zs;
    for (int i = tid; i < kOps; i += kT) {
      if constexpr (BF) {
        chi[i] = 0;
        clo[i] = 0;
      } else {
        cf[i] = 0.0f;
      }
    }
  }
  __syncthreads();
  // row operands (-2 a, |a|^2, 1); lane l holds row l mod 16 of each row
  // tile and the k = KE (l / 16) + e of each step
  float af[BF ? 1 : kSymRT][BF ? 1 : KT];
  frag ahi[BF ? kSymRT : 1][BF ? KT : 1], alo[BF ? kSymRT : 1][BF ? KT : 1];
  float xr[kSymRT][4];
#pragma unroll
  for (int rt = 0; rt < kSymRT; ++rt) {
    const int64_t i0 = rb + wave * (16 * kSymRT) + rt * 16 + lr;
    const int64_t ia = i0 < n ? i0 : n - 1;
    float part = 0.0f;
#pragma unroll
    for (int t = 0; t < KT; ++t)
#pragma unroll
      for (int e = 0; e < KE; ++e) {
        const int k = KW * t + KE * lg + e;
        const float v = k < d ? (float)(pts[ia * d + k] * zs - ctr[k]) : 0.0f;
        if constexpr (!BF) {
          af[rt][t] = -2.0f * v;
          part = fmaf(v, v, part);
        } else {
          const __bf16 h = (__bf16)v;
          const __bf16 l = (__bf16)(v - (float)h);
          ahi[rt][t][e] = __builtin_bit_cast(short, (__bf16)(-2.0f * (float)h));  // exact
          alo[rt][t][e] = __builtin_bit_cast(short, (__bf16)(-2.0f * (float)l));
          const float vv = (float)h + (float)l;
          part = fmaf(vv, vv, part);
        }
      }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);  // |a|^2 of row lr
    const __bf16 nh = (__bf16)part, nl = (__bf16)(part - (float)nh);
#pragma unroll
    for (int t = 0; t < KT; ++t)
#pragma unroll
      for (int e = 0; e < KE; ++e) {
        const int k = KW * t + KE * lg + e;
        if constexpr (!BF) {
          if (k == d) af[rt][t] = part;
          if (k == d + 1) af[rt][t] = 1.0f;
        } else {
          if (k == d) {
            ahi[rt][t][e] = __builtin_bit_cast(short, nh);
            alo[rt][t][e] = __builtin_bit_cast(short, nl);
          }
          if (k == d + 1) {
            ahi[rt][t][e] = (short)0x3F80;  // 1.0
            alo[rt][t][e] = 0;
          }
        }
      }
    const float xa = i0 < n ? (float)x[i0] : 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) xr[rt][r] = __shfl(xa, 4 * lg + r, 64);
  }
  // rounds this block takes part in: in the half round (2 r = T, the last
  // round of all) the blocks S >= T/2 have no partner
  int nq = nr;
  if ((T % 2 == 0) && (2 * (round0 + nr - 1) == T) && S >= T / 2) --nq;
  const int nchunks = nq * kChunksPerRound;
  auto colbase = [&](int u) -> int64_t {
    const int rr = round0 + u / kChunksPerRound;
    return (int64_t)((S + rr) % T) * kSymBlk + (int64_t)(u % kChunksPerRound) * kRChunk;
  };
  // staging: two adjacent threads per column, thread sh takes the
  // coordinates kk = 2 k + sh
  const int sj = tid >> 1, sh = tid & 1;
  double pre[KH];
  double prex = 0.0;
  auto fetch = [&](int u) {
    // columns past n read point n - 1 (their x is 0, their partials are not written)
    const int64_t gj = colbase(u) + sj;
    const double* src = pts + (gj < n ? gj : n - 1) * d;
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      if (2 * k < d) {  // wave-uniform
        const int kk = 2 * k + sh;
        pre[k] = src[kk < d ? kk : d - 1];
      }
    }
    prex = (gj < n && sh == 0) ? x[gj] : 0.0;
  };
  // (b, 1, |b|^2) of column sj into LDS
  auto stage = [&]() {
    float part = 0.0f;
#pragma unroll
    for (int k = 0; k < KH; k += 2) {
      if (2 * k >= d) break;  // wave-uniform
      const int kk0 = 2 * k + sh, kk1 = kk0 + 2;
      const bool ok0 = kk0 < d, ok1 = kk1 < d;
      const float v0 = ok0 ? (float)(pre[k] * zs - ctr[kk0]) : 0.0f;
      const float v1 = ok1 ? (float)(pre[k + 1] * zs - ctr[kk1]) : 0.0f;
      if constexpr (!BF) {
        if (ok0) cf[op_index(kk0, sj)] = v0;
        if (ok1) cf[op_index(kk1, sj)] = v1;
        part = fmaf(v0, v0, fmaf(v1, v1, part));
      } else {
        const __bf16 h0 = (__bf16)v0, h1 = (__bf16)v1;
        const __bf16 l0 = (__bf16)(v0 - (float)h0), l1 = (__bf16)(v1 - (float)h1);
        if (ok0) {
          chi[op_index(kk0, sj)] = __builtin_bit_cast(unsigned short, h0);
          clo[op_index(kk0, sj)] = __builtin_bit_cast(unsigned short, l0);
        }
        if (ok1) {
          chi[op_index(kk1, sj)] = __builtin_bit_cast(unsigned short, h1);
          clo[op_index(kk1, sj)] = __builtin_bit_cast(unsigned short, l1);
        }
        const float w0 = (float)h0 + (float)l0, w1 = (float)h1 + (float)l1;
        part = fmaf(w0, w0, fmaf(w1, w1, part));
      }
    }
    part += __shfl_xor(part, 1, 64);  // the column's two staging threads are adjacent lanes
    // k = d holds 1, k = d + 1 holds |b|^2: one each for the two threads
    const int kk = (sh == (d & 1)) ? d : d + 1;
    if constexpr (!BF) {
      cf[op_index(kk, sj)] = kk == d ? 1.0f : part;
    } else {
      const __bf16 h = kk == d ? (__bf16)1.0f : (__bf16)part;
      const __bf16 l = kk == d ? (__bf16)0.0f : (__bf16)(part - (float)h);
      chi[op_index(kk, sj)] = __builtin_bit_cast(unsigned short, h);
      clo[op_index(kk, sj)] = __builtin_bit_cast(unsigned short, l);
    }
    if (sh == 0) cx[sj] = prex;
  };
  auto gram = [&](int tile, f4 (&gg)[kSymRT]) {
    const int jc = tile * 16 + lr;
#pragma unroll
    for (int rt = 0; rt < kSymRT; ++rt) gg[rt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (!BF) {
      float bf[KT];
#pragma unroll
      for (int t = 0; t < KT; ++t) bf[t] = cf[(t * kRChunk + jc) * 4 + lg];
#pragma unroll
      for (int t = 0; t < KT; ++t)
#pragma unroll
        for (int rt = 0; rt < kSymRT; ++rt) gg[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[rt][t], bf[t], gg[rt], 0, 0, 0);
    } else {
      frag bh[KT], bl[KT];
#pragma unroll
      for (int t = 0; t < KT; ++t) {
        const int o = (t * kRChunk + jc) * KW + KE * lg;
        bh[t] = *reinterpret_cast<const frag*>(&chi[o]);
        bl[t] = *reinterpret_cast<const frag*>(&clo[o]);
      }
#pragma unroll
      for (int t = 0; t < KT; ++t)
#pragma unroll
        for (int rt = 0; rt < kSymRT; ++rt) {
          if constexpr (KE == 8) {
            gg[rt] = mfma_bf16_k32(ahi[rt][t], bh[t], gg[rt]);
            gg[rt] = mfma_bf16_k32(ahi[rt][t], bl[t], gg[rt]);
            gg[rt] = mfma_bf16_k32(alo[rt][t], bh[t], gg[rt]);
          } else {
            gg[rt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi[rt][t], bh[t], gg[rt], 0, 0, 0);
            gg[rt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi[rt][t], bl[t], gg[rt], 0, 0, 0);
            gg[rt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo[rt][t], bh[t], gg[rt], 0, 0, 0);
          }
        }
    }
  };
  float rs[kSymRT][4];
#pragma unroll
  for (int rt = 0; rt < kSymRT; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) rs[rt][r] = 0.0f;
  auto values = [&](int tile, const f4 (&gg)[kSymRT]) {
    const int jc = tile * 16 + lr;
    const float xc = (float)cx[jc];
    float cp0 = 0.0f, cp1 = 0.0f;
#pragma unroll
    for (int rt = 0; rt < kSymRT; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float ph, unused;
        // |s|: a squared distance below zero is rounding of a near pair (free source modifier)
        pair_value_w<NU2, 1>(__builtin_amdgcn_sqrtf(fabsf(gg[rt][r])), ph, unused);
        rs[rt][r] = fmaf(ph, xc, rs[rt][r]);
        if (r & 1) cp1 = fmaf(ph, xr[rt][r], cp1);
        else cp0 = fmaf(ph, xr[rt][r], cp0);
      }
    csum[wave][lg][jc] = cp0 + cp1;
  };
  constexpr int kMfma = BF ? 3 * KT * kSymRT : KT * kSymRT;
  constexpr int kValu = 16 * (NU2 == 1 ? 5 : (NU2 == 3 ? 7 : 8)) + 4;
  constexpr int kValuPer = (kValu + kMfma - 1) / kMfma;
  auto interleave = [&]() {
    __builtin_amdgcn_sched_group_barrier(0x100, BF ? 2 * KT : KT, 0);
#pragma unroll
    for (int i = 0; i < kMfma; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, kValuPer, 0);
    }
  };
  double racc[kSymRT][4];
#pragma unroll
  for (int rt = 0; rt < kSymRT; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) racc[rt][r] = 0.0;
  if (nchunks > 0) fetch(0);
  for (int u = 0; u < nchunks; ++u) {
    if (u > 0) __syncthreads();  // the previous chunk's operands and column partials have been read
    stage();
    __syncthreads();
    if (u + 1 < nchunks) fetch(u + 1);
    f4 ga[kSymRT], gb[kSymRT];
    gram(0, ga);
#pragma unroll 1
    for (int tile = 0; tile < kRTiles - 2; tile += 2) {
      gram(tile + 1, gb);
      values(tile, ga);
      interleave();
      gram(tile + 2, ga);
      values(tile + 1, gb);
      interleave();
    }
    gram(kRTiles - 1, gb);
    values(kRTiles - 2, ga);
    interleave();
    values(kRTiles - 1, gb);
    if (u % kChunksPerRound == kChunksPerRound - 1) {
      // round done: the FP32 row sums (16 columns per lane) go to FP64
#pragma unroll
      for (int rt = 0; rt < kSymRT; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          racc[rt][r] += (double)rs[rt][r];
          rs[rt][r] = 0.0f;
        }
    }
    __syncthreads();
    if (tid < kRChunk) {
      const int64_t gj = colbase(u) + tid;
      if (gj < n) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < 4; ++w)
#pragma unroll
          for (int g = 0; g < 4; ++g) t += (double)csum[w][g][tid];
        pcol[(int64_t)(u / kChunksPerRound) * n + gj] = t;
      }
    }
  }
  // row sums: reduce over the 16 column lanes of each row group
#pragma unroll
  for (int rt = 0; rt < kSymRT; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = racc[rt][r];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      const int64_t i = rb + wave * (16 * kSymRT) + rt * 16 + 4 * lg + r;
      if (lr == 0 && i < n) prow[i] = v;
    }
}

template <int KP, int NU2, bool BF>
void launch_rounds(const PairArgs& a, double zs, int T, int r0, int nr, double* prow, double* pcol, hipStream_t s) {
  hipLaunchKernelGGL((mfma_rounds_kernel<KP, NU2, BF>), dim3(T), dim3(kT), 0, s, a.cols, a.x, a.n, a.d, T, r0, nr,
                     zs * 1.4426950408889634, prow, pcol);
}

using RoundsFn = void (*)(const PairArgs&, double, int, int, int, double*, double*, hipStream_t);

// the augmented Gram needs d + 2 <= KP
template <int NU2, bool BF>
RoundsFn pick_rounds_kp(int d) {
  if constexpr (BF) {
    if (d + 2 <= 16) return launch_rounds<16, NU2, true>;
    if (d + 2 <= 32) return launch_rounds<32, NU2, true>;
    if (d + 2 <= 64) return launch_rounds<64, NU2, true>;
  } else {
    if (d + 2 <= 12) return launch_rounds<12, NU2, false>;
    if (d + 2 <= 16) return launch_rounds<16, NU2, false>;
    if (d + 2 <= 20) return launch_rounds<20, NU2, false>;
    if (d + 2 <= 24) return launch_rounds<24, NU2, false>;
    if (d + 2 <= 28) return launch_rounds<28, NU2, false>;
    if (d + 2 <= 32) return launch_rounds<32, NU2, false>;
    if (d + 2 <= 36) return launch_rounds<36, NU2, false>;
  }
  return nullptr;
}

template <int KP, int NU2, bool BF>
void launch_sym(const PairArgs& a, double zs, void* work, int T, int r0, int nr, int diag, double* prow, double* pcol,
                hipStream_t s) {
  (void)work;
  // coordinates scaled by sqrt(2 nu)/rho log2(e): the kernel's distances are w = log2(e) z
  hipLaunchKernelGGL((mfma_sym_kernel<KP, NU2, BF>), dim3(T, nr), dim3(kT), 0, s, a.cols, a.x, a.n, a.d, T, r0, diag,
                     zs * 1.4426950408889634, prow, pcol);
}

using SymFn = void (*)(const PairArgs&, double, void*, int, int, int, int, double*, double*, hipStream_t);

template <int NU2, bool BF>
SymFn pick_sym_kp(int d) {
  if constexpr (BF) {
    if (d <= 16) return launch_sym<16, NU2, true>;
    if (d <= 32) return launch_sym<32, NU2, true>;
  } else {
    if (d <= 8) return launch_sym<8, NU2, false>;
    if (d <= 12) return launch_sym<12, NU2, false>;
    if (d <= 16) return launch_sym<16, NU2, false>;
    if (d <= 20) return launch_sym<20, NU2, false>;
    if (d <= 24) return launch_sym<24, NU2, false>;
    if (d <= 32) return launch_sym<32, NU2, false>;
  }
  return nullptr;
}

template <int KP, int NU2, bool BF>
void launch(const PairArgs& a, double zs, int S, int64_t cps, double* py, hipStream_t s) {
  dim3 grid((unsigned)((a.m + kRows - 1) / kRows), (unsigned)S);
  const int self = (a.rows == a.cols) ? 1 : 0;
  hipLaunchKernelGGL((mfma_kernel<KP, NU2, BF>), grid, dim3(kT), 0, s, a.rows, a.m, a.cols, a.n, a.d, a.x, py, zs, cps,
                     self);
}

template <int NU2, bool BF>
bool dispatch_kp(const PairArgs& a, double zs, int S, int64_t cps, double* py, hipStream_t s) {
  if constexpr (BF) {
    if (a.d <= 16) launch<16, NU2, true>(a, zs, S, cps, py, s);
    else if (a.d <= 32) launch<32, NU2, true>(a, zs, S, cps, py, s);
    else return false;
  } else {
    if (a.d <= 8) launch<8, NU2, false>(a, zs, S, cps, py, s);
    else if (a.d <= 12) launch<12, NU2, false>(a, zs, S, cps, py, s);
    else if (a.d <= 16) launch<16, NU2, false>(a, zs, S, cps, py, s);
    else if (a.d <= 20) launch<20, NU2, false>(a, zs, S, cps, py, s);
    else if (a.d <= 24) launch<24, NU2, false>(a, zs, S, cps, py, s);
    else if (a.d <= 32) launch<32, NU2, false>(a, zs, S, cps, py, s);
    else return false;
  }
  return true;
}

}  // namespace

int32_t mfma_splits(int64_t m, int64_t n) {
  const int64_t rb = (m + kRows - 1) / kRows;
  int64_t S = (4096 + rb - 1) / rb;
  const int64_t max_by_cols = (n + kChunk - 1) / kChunk;
  S = std::max<int64_t>(1, std::min<int64_t>({S, max_by_cols, 64}));
  return (int32_t)S;
}

bool mfma_applies(const PairArgs& a) {
  return (a.precision == MLBLUP_MFMA_FP32 || a.precision == MLBLUP_MFMA_BF16X3) && a.outputs == MLBLUP_VALUE &&
         a.d >= 8 && a.d <= 32 && a.nu2 > 0;
}

int mfma_sym_launch(const PairArgs& a, double zs, void* work, hipStream_t s) {
  const bool bf = a.precision == MLBLUP_MFMA_BF16X3;
  SymFn fn = nullptr;
  if (a.nu2 == 1) fn = bf ? pick_sym_kp<1, true>(a.d) : pick_sym_kp<1, false>(a.d);
  else if (a.nu2 == 3) fn = bf ? pick_sym_kp<3, true>(a.d) : pick_sym_kp<3, false>(a.d);
  else fn = bf ? pick_sym_kp<5, true>(a.d) : pick_sym_kp<5, false>(a.d);
  RoundsFn rfn = nullptr;
  if (a.nu2 == 1) rfn = bf ? pick_rounds_kp<1, true>(a.d) : pick_rounds_kp<1, false>(a.d);
  else if (a.nu2 == 3) rfn = bf ? pick_rounds_kp<3, true>(a.d) : pick_rounds_kp<3, false>(a.d);
  else rfn = bf ? pick_rounds_kp<5, true>(a.d) : pick_rounds_kp<5, false>(a.d);
  if (!fn || !rfn) return fail(MLBLUP_EINVAL, "matrix-core pair kernel: d > 32");
  // diagonal tiles: the tile kernel (exact differences on the self sub-tiles); rounds: one launch of
  // T workgroups per 16 rounds, one row partial per launch
  return sym_schedule(
      a, kSymBlk, work, s,
      [&](int T, int r0, int nr, int diag, double* prow, double* pcol, double*, double*) {
        if (diag) fn(a, zs, work, T, r0, nr, 1, prow, pcol, s);
        else rfn(a, zs, T, r0, nr, prow, pcol, s);
      },
      true);
}

int mfma_launch(const PairArgs& a, double zs, double* part, hipStream_t s) {
  const int S = mfma_splits(a.m, a.n);
  int64_t cps = (a.n + S - 1) / S;
  cps = (cps + kChunk - 1) / kChunk * kChunk;
  const bool bf = a.precision == MLBLUP_MFMA_BF16X3;
  bool ok;
  if (a.nu2 == 1) ok = bf ? dispatch_kp<1, true>(a, zs, S, cps, part, s) : dispatch_kp<1, false>(a, zs, S, cps, part, s);
  else if (a.nu2 == 3) ok = bf ? dispatch_kp<3, true>(a, zs, S, cps, part, s) : dispatch_kp<3, false>(a, zs, S, cps, part, s);
  else ok = bf ? dispatch_kp<5, true>(a, zs, S, cps, part, s) : dispatch_kp<5, false>(a, zs, S, cps, part, s);
  if (!ok) return fail(MLBLUP_EINVAL, "matrix-core pair kernel: d > 32");
  return hip_check(hipGetLastError(), "mfma pair kernel launch");
}

}  // namespace mlb
