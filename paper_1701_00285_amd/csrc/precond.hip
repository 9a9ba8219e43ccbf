// Preconditioner of the Krylov solve (preconditioner remark of Sec. 5.2):
// P_W = diag(C_W) (Jacobi), or the block form that keeps, for every cell,
// the whole block of C_W between that cell's own wavelets.
//
// The blocks are assembled bottom-up without ever forming C_W.  For a cell
// v with candidate vectors [Phi_L, Phi_R] (children's scaling vectors) the
// candidate Gram is
//     G_cand = [[G_L, X], [X^T, G_R]],  X = Phi_L^T K(S_L, S_R) Phi_R,
// G_c = Phi_c^T K(S_c, S_c) Phi_c the children's scaling Grams; for a leaf,
// G_cand = K(S_v, S_v).  With the cell's orthogonal block V = [V_s | V_w]:
//     G_v = V_s^T G_cand V_s   (passed up),   B_v = V_w^T G_cand V_w   (the block of C_W).
// Device work: the leaf kernel blocks and, per internal cell, the sibling
// cross term X, computed as y_i = sum_{j in S_R} phi_ij Phi_R[j,:] for rows
// i in S_L followed by the sum of Phi_L[i,:]^T y_i over the rows (about N^2/2
// pairs over all levels).  The scaling vectors' values on the points,
// Phi^(q), are produced level by level from Phi^(q+1) and the V blocks.
// Since this only preconditions, the pair values use FP32 sqrt/exp on FP64
// distances (relative error ~1e-7).
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.h"
#include "genu.h"
#include "precond.h"

namespace mlb {
namespace {

constexpr int kT = 256;
constexpr int kMaxD = 64;

// g32: the float value table of a general nu (genu.h), else unused
__device__ __forceinline__ double phi32(double s, int nu2, const float* __restrict__ g32) {
  if (nu2 == kNuGeneral) return (double)genu_f32(fmaxf((float)s, 1e-30f), g32);
  if (nu2 == 0) return (double)__builtin_amdgcn_exp2f(-0.72134752044448170f * (float)s);  // Gaussian e^{-s/2}
  const float z = __builtin_amdgcn_sqrtf((float)s);
  const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * z);
  float p = 1.0f;
  if (nu2 == 3) p = 1.0f + z;
  else if (nu2 == 5) p = fmaf(z, fmaf(z, 1.0f / 3.0f, 1.0f), 1.0f);
  return (double)(p * e);
}

__global__ __launch_bounds__(kT) void leaf_blocks(const int64_t* __restrict__ lbegin, const int32_t* __restrict__ lsize,
                                                  const int64_t* __restrict__ koff, const double* __restrict__ pts,
                                                  int d, double zs, int nu2, const float* __restrict__ g32,
                                                  double* __restrict__ K) {
  const int leaf = blockIdx.x;
  const int64_t b = lbegin[leaf];
  const int s = lsize[leaf];
  for (int e = threadIdx.x; e < s * s; e += kT) {
    const int i = e / s, j = e - i * s;
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
      const double t = (pts[(b + i) * d + k] - pts[(b + j) * d + k]) * zs;
      acc = fma(t, t, acc);
    }
    K[koff[leaf] + e] = phi32(acc, nu2, g32);
  }
}

// Phi^(q) from Phi^(q+1): one thread per point.  Level-q cells are listed in
// increasing `begin`; a point outside all of them (its leaf is shallower)
// is skipped.  P = row stride of the Phi buffers.
__global__ __launch_bounds__(kT) void scal_values(const PrecNode* __restrict__ nodes, const int32_t* __restrict__ lvl,
                                                  int32_t cnt, const double* __restrict__ V,
                                                  const double* __restrict__ phi_in, double* __restrict__ phi_out,
                                                  int P, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  int lo = 0, hi = cnt - 1, f = -1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const PrecNode& N = nodes[lvl[mid]];
    if (N.begin <= i) {
      f = mid;
      lo = mid + 1;
    } else {
      hi = mid - 1;
    }
  }
  if (f < 0) return;
  const PrecNode Nv = nodes[lvl[f]];
  if (i >= Nv.end) return;
  const double* B = V + Nv.v_off;
  const int m = Nv.m, a = Nv.a;
  double* out = phi_out + i * P;
  if (Nv.left < 0) {
    const int64_t r = i - Nv.begin;
    for (int c = 0; c < a; ++c) out[c] = B[r * m + c];
  } else {
    const PrecNode& L = nodes[Nv.left];
    const bool in_left = i < L.end;
    const int coff = in_left ? 0 : L.a;
    const int ac = in_left ? L.a : nodes[Nv.right].a;
    const double* in = phi_in + i * P;
    for (int c = 0; c < a; ++c) {
      double s = 0.0;
      for (int k = 0; k < ac; ++k) s = fma(in[k], B[(int64_t)(coff + k) * m + c], s);
      out[c] = s;
    }
  }
  for (int c = a; c < P; ++c) out[c] = 0.0;
}

__device__ __forceinline__ double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  return x;
}

// Sibling cross term partial: rows [r0, r1) of S_L, columns [c0, c1) of S_R.
template <int NR>
__global__ __launch_bounds__(kT) void cross_gram(const CrossTask* __restrict__ tasks, const double* __restrict__ pts,
                                                 int d, double zs, int nu2, const float* __restrict__ g32,
                                                 const double* __restrict__ phi, int P, double* __restrict__ part) {
  constexpr int TC = 64;
  __shared__ double cpts[TC * kMaxD];
  __shared__ double crhs[TC * NR];
  __shared__ double red[kT / 64][NR * NR];
  const CrossTask T = tasks[blockIdx.x];
  const int tid = threadIdx.x;
  const int64_t i = T.r0 + tid;
  const bool valid = i < T.r1;
  const int64_t ii = valid ? i : T.r0;
  double xr[kMaxD];
#pragma unroll
  for (int k = 0; k < kMaxD; ++k)
    if (k < d) xr[k] = pts[ii * d + k] * zs;
  double y[NR];
#pragma unroll
  for (int b = 0; b < NR; ++b) y[b] = 0.0;
  for (int64_t j0 = T.c0; j0 < T.c1; j0 += TC) {
    const int cnt = (int)((T.c1 - j0) < TC ? (T.c1 - j0) : TC);
    __syncthreads();
    for (int e = tid; e < TC * d; e += kT) {
      const int j = e / d, k = e - j * d;
      cpts[j * kMaxD + k] = j < cnt ? pts[(j0 + j) * d + k] * zs : 0.0;
    }
    for (int e = tid; e < TC * NR; e += kT) {
      const int j = e / NR, b = e - j * NR;
      crhs[e] = (j < cnt && b < P) ? phi[(j0 + j) * P + b] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxD; ++k)
        if (k < d) {
          const double t = xr[k] - cpts[j * kMaxD + k];
          s = fma(t, t, s);
        }
      const double f = phi32(s, nu2, g32);
#pragma unroll
      for (int b = 0; b < NR; ++b) y[b] = fma(f, crhs[j * NR + b], y[b]);
    }
  }
  // X partial = sum over this block's rows of Phi_L[i,:]^T y_i
  const int wave = tid >> 6, lane = tid & 63;
  for (int a = 0; a < NR; ++a) {
    const double pl = (valid && a < P) ? phi[ii * P + a] : 0.0;
    for (int b = 0; b < NR; ++b) {
      const double v = wave_sum(pl * y[b]);
      if (lane == 0) red[wave][a * NR + b] = v;
    }
  }
  __syncthreads();
  for (int e = tid; e < NR * NR; e += kT) {
    double s = 0.0;
    for (int w = 0; w < kT / 64; ++w) s += red[w][e];
    part[(int64_t)blockIdx.x * NR * NR + e] = s;
  }
}

__global__ __launch_bounds__(kT) void apply_blocks(const int64_t* __restrict__ w_off, const int32_t* __restrict__ mw,
                                                   const int64_t* __restrict__ boff, int32_t cnt,
                                                   const double* __restrict__ Binv, const double* __restrict__ r,
                                                   double* __restrict__ z) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t s = blockIdx.x * (kT / 64) + wave;
  if (s >= cnt) return;
  const int m = mw[s];
  const int64_t wo = w_off[s];
  const double* B = Binv + boff[s];
  for (int j = lane; j < m; j += 64) {
    double acc = 0.0;
    for (int i = 0; i < m; ++i) acc = fma(B[(int64_t)i * m + j], r[wo + i], acc);
    z[wo + j] = acc;
  }
}

__global__ __launch_bounds__(kT) void apply_diag(const double* __restrict__ inv, const double* __restrict__ r,
                                                 double* __restrict__ z, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) z[i] = inv[i] * r[i];
}

// out[i] = sum_j M[i][j] x[j] for an n x n row-major M stored in FP32 with
// rows of ld floats (ld a multiple of 4, zero padding): one wave per row,
// 16-byte loads of four entries per lane, products and sums in FP64, a
// fixed-order reduction across the wave; x has n entries.  tri = 1: M is
// lower triangular, tri = 2: upper triangular; the groups of four wholly
// in the zero triangle are not read (a lane's sum only skips exact zeros,
// so the result is the same as with tri = 0)
__global__ __launch_bounds__(kT) void gemv_rows(const float* __restrict__ M, int64_t n, int64_t ld,
                                               const double* __restrict__ x, double* __restrict__ out, int tri) {
  const int64_t i = (int64_t)blockIdx.x * (kT / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (i >= n) return;
  const float4* row = (const float4*)(M + i * ld);
  // groups [glo, ghi) hold the row's nonzeros
  const int64_t glo = tri == 2 ? i / 4 : 0, ghi = tri == 1 ? i / 4 + 1 : ld / 4;
  double acc = 0.0;
  int64_t c0 = lane;
  if (glo > lane) c0 += (glo - lane + 63) / 64 * 64;
  for (int64_t c = c0; c < ghi; c += 64) {
    const float4 v = row[c];
    const int64_t j = 4 * c;
    if (j + 3 < n) {
      acc = fma((double)v.x, x[j], acc);
      acc = fma((double)v.y, x[j + 1], acc);
      acc = fma((double)v.z, x[j + 2], acc);
      acc = fma((double)v.w, x[j + 3], acc);
    } else {
      if (j < n) acc = fma((double)v.x, x[j], acc);
      if (j + 1 < n) acc = fma((double)v.y, x[j + 1], acc);
      if (j + 2 < n) acc = fma((double)v.z, x[j + 2], acc);
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (lane == 0) out[i] = acc;
}

__global__ void fill0(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

}  // namespace

int prec_leaf_blocks(const int64_t* lbegin, const int32_t* lsize, const int64_t* koff, int32_t nleaves,
                     const double* pts, int d, double zs, int nu2, const float* g32, double* K, hipStream_t s) {
  if (nleaves <= 0) return MLBLUP_OK;
  hipLaunchKernelGGL(leaf_blocks, dim3(nleaves), dim3(kT), 0, s, lbegin, lsize, koff, pts, d, zs, nu2, g32, K);
  return hip_check(hipGetLastError(), "leaf_blocks launch");
}

int prec_scal_values(const PrecNode* nodes, const int32_t* lvl, int32_t cnt, const double* V, const double* phi_in,
                     double* phi_out, int P, int64_t n, hipStream_t s) {
  if (cnt <= 0) return MLBLUP_OK;
  hipLaunchKernelGGL(scal_values, dim3((unsigned)((n + kT - 1) / kT)), dim3(kT), 0, s, nodes, lvl, cnt, V, phi_in,
                     phi_out, P, n);
  return hip_check(hipGetLastError(), "scal_values launch");
}

int prec_zero(double* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill0, dim3(1024), dim3(256), 0, s, p, n);
  return hip_check(hipGetLastError(), "fill0 launch");
}

int prec_cross(const CrossTask* tasks, int32_t ntasks, int NR, const double* pts, int d, double zs, int nu2,
               const float* g32, const double* phi, int P, double* part, hipStream_t s) {
  if (ntasks <= 0) return MLBLUP_OK;
  if (d > kMaxD) return fail(MLBLUP_EINVAL, "preconditioner: d > 64");
  switch (NR) {
    case 8: hipLaunchKernelGGL(cross_gram<8>, dim3(ntasks), dim3(kT), 0, s, tasks, pts, d, zs, nu2, g32, phi, P, part); break;
    case 16: hipLaunchKernelGGL(cross_gram<16>, dim3(ntasks), dim3(kT), 0, s, tasks, pts, d, zs, nu2, g32, phi, P, part); break;
    case 24: hipLaunchKernelGGL(cross_gram<24>, dim3(ntasks), dim3(kT), 0, s, tasks, pts, d, zs, nu2, g32, phi, P, part); break;
    case 32: hipLaunchKernelGGL(cross_gram<32>, dim3(ntasks), dim3(kT), 0, s, tasks, pts, d, zs, nu2, g32, phi, P, part); break;
    default: return fail(MLBLUP_EINVAL, "preconditioner: trend dimension p > 32 not supported");
  }
  return hip_check(hipGetLastError(), "cross_gram launch");
}

int prec_apply_blocks(const int64_t* w_off, const int32_t* mw, const int64_t* boff, int32_t cnt, const double* Binv,
                      const double* r, double* z, hipStream_t s) {
  if (cnt <= 0) return MLBLUP_OK;
  hipLaunchKernelGGL(apply_blocks, dim3((unsigned)((cnt + 3) / 4)), dim3(kT), 0, s, w_off, mw, boff, cnt, Binv, r, z);
  return hip_check(hipGetLastError(), "apply_blocks launch");
}

int prec_gemv_rows(const float* M, int64_t n, int64_t ld, const double* x, double* out, hipStream_t s, int tri) {
  if (n <= 0) return MLBLUP_OK;
  if (ld < n || ld % 4) return fail(MLBLUP_EINVAL, "gemv_rows: row stride must be >= n and a multiple of 4");
  if (tri < 0 || tri > 2) return fail(MLBLUP_EINVAL, "gemv_rows: tri must be 0, 1 or 2");
  const int64_t g = (n + kT / 64 - 1) / (kT / 64);
  hipLaunchKernelGGL(gemv_rows, dim3((unsigned)g), dim3(kT), 0, s, M, n, ld, x, out, tri);
  return hip_check(hipGetLastError(), "gemv_rows launch");
}

int prec_apply_diag(const double* inv, const double* r, double* z, int64_t n, hipStream_t s) {
  int64_t g = (n + kT - 1) / kT;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(apply_diag, dim3((unsigned)(g > 0 ? g : 1)), dim3(kT), 0, s, inv, r, z, n);
  return hip_check(hipGetLastError(), "apply_diag launch");
}

}  // namespace mlb
