// Multilevel transform kernels (operators W and W^T, Sec. 3.1; steps (1)
// and (3) of the product chain, Sec. 6.2) and the Krylov vector kernels.
//
// Transform: launches of three tree levels each.  Analysis (v -> W v, L v)
// runs from the finest level to the root: a cell applies V^T to its
// candidate coefficients (leaf: its points' entries of v; internal: the
// children's scaling coefficients, stored contiguously); the first a results
// are its scaling coefficients (passed up; at the root they are L v), the
// rest its wavelet coefficients, written to their slot of W v.  Synthesis
// (W^T) runs root to leaves with V.  One 64-lane wave per cell.  V is
// stored in the compact WY form of the Householder reflectors it was built
// from, V = H_0 ... H_{K-1} = I - Y T Y^T (K = min(m, p) reflectors of length
// m and a K x K triangle), so a cell reads K m + K^2 doubles instead of m^2:
// the wave stages Y and T in LDS and applies them in three steps of serial
// dot products (wy_apply).  Cells with more than 256 candidates read the
// dense block instead.
//
// Reductions: every dot product is a fixed grid of kRedBlocks blocks, each
// reducing a fixed slice in a fixed tree order, then one block adding the
// kRedBlocks partials in a fixed order: results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "device.h"

namespace mlb {

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return MLBLUP_OK;
  return fail(MLBLUP_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

constexpr int kT = 256;
constexpr int kWavesPerBlock = 4;

// sum over the 64 lanes in a fixed order (a tree into lane 0), the same value on every lane
__device__ __forceinline__ double wave_allsum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  return __shfl(x, 0, 64);
}

constexpr int kPer = kTransformMaxM / 64;   // entries per lane of a cell's vector
constexpr int kHBuf = 2048;                 // doubles of LDS per wave

// x <- (I - Y T^T Y^T) x (analysis, V^T x) or (I - Y T Y^T) x (synthesis, V x) for one cell held by
// one wave (x: entries lane + 64 q).  Three steps of serial dot products from LDS, so no cross-lane
// reduction chain: w = Y^T x (64 / K lanes share row k of Y, then their sums are added), u = T^T w
// or T w (lane k: column or row k of the triangle against w), x -= Y u (lane i: column i of Y
// against u).  Y (row stride m | 1, odd, so that the lanes reading different rows hit different
// banks), T, the three vectors and the partial sums sit in the wave's LDS buffer.  A cell too large for the buffer applies its K reflectors
// one after the other from global memory instead, each a wave-wide dot product.
__device__ __forceinline__ void wy_apply(const double* __restrict__ Rg, int m, int K, int lane, bool analysis,
                                         double* __restrict__ buf, double (&x)[kPer]) {
  const int ys = m | 1;
  const int G = K > 0 && K <= 64 ? 64 / K : 1;   // lanes sharing one dot product of the first step
  const int64_t need = (int64_t)K * ys + (int64_t)K * K + m + 2 * K + (int64_t)G * K;
  const double* Tg = Rg + (int64_t)K * m;
  if (need <= kHBuf) {
    double* Ys = buf;
    double* Ts = Ys + K * ys;
    double* xs = Ts + K * K;
    double* ws = xs + m;
    double* us = ws + K;
    double* ps = us + K;
    for (int e = lane; e < K * m; e += 64) {
      const int k = e / m, i = e - k * m;
      Ys[k * ys + i] = Rg[e];
    }
    for (int e = lane; e < K * K; e += 64) Ts[e] = Tg[e];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = lane + 64 * q;
      if (i < m) xs[i] = x[q];
    }
    __builtin_amdgcn_wave_barrier();
    // w = Y^T x: G lanes per row k (lane l: k = l mod K, g = l / K) each sum every G-th entry from
    // k on (h_k is zero above k), then lane k adds the G partial sums in order
    if (G > 1) {
      const int k = lane % K, g = lane / K;
      if (g < G) {
        double s = 0.0;
#pragma unroll 4
        for (int i = k + g; i < m; i += G) s = fma(Ys[k * ys + i], xs[i], s);
        ps[g * K + k] = s;
      }
      __builtin_amdgcn_wave_barrier();
      if (lane < K) {
        double s = ps[lane];
        for (int q = 1; q < G; ++q) s += ps[q * K + lane];
        ws[lane] = s;
      }
    } else {
      for (int k = lane; k < K; k += 64) {
        double s = 0.0;
#pragma unroll 4
        for (int i = k; i < m; ++i) s = fma(Ys[k * ys + i], xs[i], s);
        ws[k] = s;
      }
    }
    __builtin_amdgcn_wave_barrier();
    for (int k = lane; k < K; k += 64) {
      double s = 0.0;
      if (analysis) {
        for (int j = 0; j <= k; ++j) s = fma(Ts[j * K + k], ws[j], s);
      } else {
        for (int j = k; j < K; ++j) s = fma(Ts[k * K + j], ws[j], s);
      }
      us[k] = s;
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = lane + 64 * q;
      if (i < m) {
        double s0 = x[q], s1 = 0.0;
        const int kmax = i < K ? i + 1 : K;   // h_k[i] = 0 for k > i
        int k = 0;
#pragma unroll 4
        for (; k + 1 < kmax; k += 2) {
          s0 = fma(-Ys[k * ys + i], us[k], s0);
          s1 = fma(-Ys[(k + 1) * ys + i], us[k + 1], s1);
        }
        if (k < kmax) s0 = fma(-Ys[k * ys + i], us[k], s0);
        x[q] = s0 + s1;
      }
    }
    __builtin_amdgcn_wave_barrier();
    return;
  }
  for (int st = 0; st < K; ++st) {
    const int k = analysis ? st : K - 1 - st;
    const double tk = Tg[(int64_t)k * K + k];
    if (tk == 0.0) continue;   // wave-uniform: an identity reflector
    const double* h = Rg + (int64_t)k * m;
    double hv[kPer];
    double d = 0.0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = lane + 64 * q;
      hv[q] = i < m ? h[i] : 0.0;
      d = fma(hv[q], x[q], d);
    }
    const double c = tk * wave_allsum(d);
#pragma unroll
    for (int q = 0; q < kPer; ++q) x[q] = fma(-c, hv[q], x[q]);
  }
}

// analysis of one cell: its candidate coefficients times V^T;
// the first a results are its scaling coefficients (to the parent's slot, or L v at the root),
// the rest its wavelet coefficients
__device__ __forceinline__ void analysis_node(const NodeDesc& D, int lane, const double* __restrict__ V,
                                              const double* __restrict__ H, double* __restrict__ buf,
                                              const double* __restrict__ v, double* __restrict__ scal,
                                              double* __restrict__ vw, double* __restrict__ vl) {
  const double* cin = D.leaf ? v + D.in_off : scal + D.in_off;
  const int m = D.m;
  auto put = [&](int j, double val) {
    if (j < D.a) {
      if (D.scal_off >= 0) scal[D.scal_off + j] = val;
      else if (vl) vl[j] = val;
    } else {
      vw[D.w_off + (j - D.a)] = val;
    }
  };
  if (m <= kTransformMaxM) {
    double x[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = lane + 64 * q;
      x[q] = i < m ? cin[i] : 0.0;
    }
    wy_apply(H + D.h_off, m, D.nref, lane, true, buf, x);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int j = lane + 64 * q;
      if (j < m) put(j, x[q]);
    }
    return;
  }
  const double* B = V + D.v_off;
  for (int j = lane; j < m; j += 64) {
    double acc = 0.0;
#pragma unroll 8
    for (int i = 0; i < m; ++i) acc = fma(B[(int64_t)i * m + j], cin[i], acc);
    put(j, acc);
  }
}

// synthesis of one cell: V times [scaling coefficients from the parent (zero at the root when
// vl is null); wavelet coefficients], to the children's slots or to v
__device__ __forceinline__ void synthesis_node(const NodeDesc& D, int lane, const double* __restrict__ V,
                                               const double* __restrict__ H, double* __restrict__ buf,
                                               const double* __restrict__ vw, const double* __restrict__ vl,
                                               double* __restrict__ scal, double* __restrict__ v) {
  const int m = D.m, a = D.a;
  const double* cs = D.scal_off >= 0 ? scal + D.scal_off : vl;  // may be null at the root
  const double* cw = vw + D.w_off - a;
  double* out = D.leaf ? v + D.in_off : scal + D.in_off;
  if (m <= kTransformMaxM) {
    double x[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = lane + 64 * q;
      x[q] = i < m ? (i < a ? (cs ? cs[i] : 0.0) : cw[i]) : 0.0;
    }
    wy_apply(H + D.h_off, m, D.nref, lane, false, buf, x);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = lane + 64 * q;
      if (i < m) out[i] = x[q];
    }
    return;
  }
  const double* B = V + D.v_off;
  for (int i = lane; i < m; i += 64) {
    double acc = 0.0;
    if (cs) {
#pragma unroll 8
      for (int j = 0; j < a; ++j) acc = fma(B[(int64_t)i * m + j], cs[j], acc);
    }
#pragma unroll 8
    for (int j = a; j < m; ++j) acc = fma(B[(int64_t)i * m + j], cw[j], acc);
    out[i] = acc;
  }
}

// Three levels per launch: a workgroup takes one cell at the group's top
// depth and the cells of its subtree one and two levels below (up to 2 and
// 4 cells, one per wave), with a workgroup barrier between the levels (the
// barrier orders this workgroup's global writes and reads).  The analysis
// runs a group from its deepest level up, the synthesis from its top down.
constexpr int kGroupLevels = 3;

// cell of the group for wave w at relative depth rel (0: the group's top
// cell r; 1: its children, waves 0-1; 2: its grandchildren, waves 0-3), or -1
__device__ __forceinline__ int32_t group_cell(const int32_t* __restrict__ children, int32_t n_nodes, int32_t r,
                                              int rel, int w) {
  if (rel == 0) return w == 0 ? r : -1;
  if (rel == 1) return w < 2 ? children[(int64_t)w * n_nodes + r] : -1;
  if (w >= 4) return -1;
  const int32_t c = children[(int64_t)(w >> 1) * n_nodes + r];
  return c >= 0 ? children[(int64_t)(w & 1) * n_nodes + c] : -1;
}

__global__ __launch_bounds__(kT) void analysis_group(const NodeDesc* __restrict__ desc,
                                                     const int32_t* __restrict__ children, int32_t n_nodes,
                                                     const int32_t* __restrict__ roots, int nlev,
                                                     const double* __restrict__ V, const double* __restrict__ H,
                                                     const double* __restrict__ v, double* __restrict__ scal,
                                                     double* __restrict__ vw, double* __restrict__ vl) {
  __shared__ double hbuf[kWavesPerBlock][kHBuf];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int32_t r = roots[blockIdx.x];
  for (int rel = nlev - 1; rel >= 0; --rel) {
    const int32_t u = group_cell(children, n_nodes, r, rel, wave);
    if (u >= 0) analysis_node(desc[u], lane, V, H, hbuf[wave], v, scal, vw, vl);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kT) void synthesis_group(const NodeDesc* __restrict__ desc,
                                                      const int32_t* __restrict__ children, int32_t n_nodes,
                                                      const int32_t* __restrict__ roots, int nlev,
                                                      const double* __restrict__ V, const double* __restrict__ H,
                                                      const double* __restrict__ vw, const double* __restrict__ vl,
                                                      double* __restrict__ scal, double* __restrict__ v) {
  __shared__ double hbuf[kWavesPerBlock][kHBuf];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int32_t r = roots[blockIdx.x];
  for (int rel = 0; rel < nlev; ++rel) {
    const int32_t u = group_cell(children, n_nodes, r, rel, wave);
    if (u >= 0) synthesis_node(desc[u], lane, V, H, hbuf[wave], vw, vl, scal, v);
    __syncthreads();
  }
}

// ---- reductions ----
__device__ __forceinline__ double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  return x;
}

// block sum over 256 threads, result valid in thread 0
__device__ __forceinline__ double block_sum(double x) {
  __shared__ double red[kT / 64];
  x = wave_sum(x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = x;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kT / 64; ++w) t += red[w];
  return t;
}

__global__ __launch_bounds__(kT) void dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                  int64_t n, double* __restrict__ part) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kT) s = fma(a[i], b[i], s);
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// sum of kRedBlocks partials in a fixed order by one block
__device__ double sum_partials(const double* part) {
  double s = 0.0;
  for (int k = threadIdx.x; k < kRedBlocks; k += kT) s += part[k];
  return block_sum(s);
}

__global__ __launch_bounds__(kT) void finish_dot(const double* __restrict__ part, double* __restrict__ out) {
  const double s = sum_partials(part);
  if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(kT) void finish_alpha(const double* __restrict__ part, double* __restrict__ sc) {
  const double pq = sum_partials(part);
  if (threadIdx.x == 0) {
    sc[S_PQ] = pq;
    const double rz = sc[S_RZ];
    const bool bad = !(pq > 0.0) || !isfinite(pq) || !isfinite(rz);
    sc[S_FLAG] = bad ? 1.0 : 0.0;
    sc[S_ALPHA] = bad ? 0.0 : rz / pq;
  }
}

__global__ __launch_bounds__(kT) void update_xr(double* __restrict__ x, double* __restrict__ r,
                                                const double* __restrict__ p, const double* __restrict__ q,
                                                int64_t n, double* __restrict__ part, const double* __restrict__ sc) {
  const double alpha = sc[S_ALPHA];
  double rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kT) {
    x[i] = fma(alpha, p[i], x[i]);
    const double ri = fma(-alpha, q[i], r[i]);
    r[i] = ri;
    rr = fma(ri, ri, rr);
  }
  rr = block_sum(rr);
  if (threadIdx.x == 0) part[blockIdx.x] = rr;
}

// rz_prev < 0: the previous r.z is sc[S_RZ]; else the one given
__global__ __launch_bounds__(kT) void finish_beta(const double* __restrict__ part, int has_diag, double rz_prev,
                                                  double* __restrict__ sc) {
  const double rr = sum_partials(part);
  double rz = rr;
  if (has_diag) {
    __syncthreads();
    rz = sum_partials(part + kRedBlocks);
  }
  if (threadIdx.x == 0) {
    sc[S_RR] = rr;
    const double beta = rz / (rz_prev < 0.0 ? sc[S_RZ] : rz_prev);
    sc[S_BETA] = beta;
    sc[S_RZ] = rz;
    if (!isfinite(rr) || !isfinite(rz)) sc[S_FLAG] = 1.0;
  }
}

__global__ __launch_bounds__(kT) void finish_start(const double* __restrict__ part, double* __restrict__ sc) {
  const double rz = sum_partials(part);
  if (threadIdx.x == 0) {
    sc[S_RZ] = rz;
    sc[S_FLAG] = isfinite(rz) ? 0.0 : 1.0;
  }
}

__global__ __launch_bounds__(kT) void update_p(double* __restrict__ p, const double* __restrict__ z, int64_t n,
                                               const double* __restrict__ sc) {
  const double beta = sc[S_BETA];
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    p[i] = fma(beta, p[i], z[i]);
}

__global__ __launch_bounds__(kT) void fcg_p(double* __restrict__ p, const double* __restrict__ z, int64_t n,
                                            const double* __restrict__ sc) {
  const double beta = -sc[S_DOT] / sc[S_PQ];
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    p[i] = fma(beta, p[i], z[i]);
}

__global__ __launch_bounds__(kT) void k_copy(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) b[i] = a[i];
}
__global__ __launch_bounds__(kT) void k_zero(double* __restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) a[i] = 0.0;
}
__global__ __launch_bounds__(kT) void k_sub_from(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) b[i] = a[i] - b[i];
}
__global__ __launch_bounds__(kT) void k_axpy(double alpha, const double* __restrict__ x, double* __restrict__ y,
                                             int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    y[i] = fma(alpha, x[i], y[i]);
}
__global__ __launch_bounds__(kT) void k_div(const double* __restrict__ r, const double* __restrict__ dg,
                                            double* __restrict__ z, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) z[i] = r[i] / dg[i];
}

__global__ __launch_bounds__(kT) void k_trend(const double* __restrict__ t, int64_t m, int d,
                                              const int32_t* __restrict__ E, int p, const double* __restrict__ c,
                                              double h, const double* __restrict__ beta, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= m) return;
  double s = 0.0;
  for (int b = 0; b < p; ++b) {
    double val = beta[b];
    for (int k = 0; k < d; ++k) {
      const int e = E[b * d + k];
      if (e) {
        const double u = (t[i * d + k] - c[k]) / h;
        for (int q = 0; q < e; ++q) val *= u;
      }
    }
    s += val;
  }
  out[i] += s;
}

unsigned grid_for(int64_t n) {
  int64_t g = (n + kT - 1) / kT;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// ---- instrumentation state ----
struct Prof {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> a, b;
  std::vector<int> bucket;
  std::vector<double> pairs;
};
Prof& prof() {
  static Prof p;
  return p;
}

}  // namespace

int transform_analysis(const TransformDev& T, const double* v, double* vw, double* vl, double* scal, hipStream_t s) {
  for (int qhi = T.levels - 1; qhi >= 0; qhi -= kGroupLevels) {
    const int qlo = qhi - (kGroupLevels - 1) > 0 ? qhi - (kGroupLevels - 1) : 0;
    const int32_t lb = T.lvl_begin_host[qlo], cnt = T.lvl_begin_host[qlo + 1] - lb;
    if (cnt <= 0) continue;
    hipLaunchKernelGGL(analysis_group, dim3((unsigned)cnt), dim3(kT), 0, s, T.desc, T.children, T.n_nodes,
                       T.level_nodes + lb, qhi - qlo + 1, T.V, T.H, v, scal, vw, vl);
  }
  return hip_check(hipGetLastError(), "analysis launch");
}

int transform_synthesis(const TransformDev& T, const double* vw, const double* vl, double* v, double* scal,
                        hipStream_t s) {
  for (int qlo = 0; qlo < T.levels; qlo += kGroupLevels) {
    const int qhi = qlo + kGroupLevels - 1 < T.levels - 1 ? qlo + kGroupLevels - 1 : T.levels - 1;
    const int32_t lb = T.lvl_begin_host[qlo], cnt = T.lvl_begin_host[qlo + 1] - lb;
    if (cnt <= 0) continue;
    hipLaunchKernelGGL(synthesis_group, dim3((unsigned)cnt), dim3(kT), 0, s, T.desc, T.children, T.n_nodes,
                       T.level_nodes + lb, qhi - qlo + 1, T.V, T.H, vw, vl, scal, v);
  }
  return hip_check(hipGetLastError(), "synthesis launch");
}

int vec_dot(const double* a, const double* b, int64_t n, double* part, double* out_dev, hipStream_t s) {
  hipLaunchKernelGGL(dot_partial, dim3(kRedBlocks), dim3(kT), 0, s, a, b, n, part);
  hipLaunchKernelGGL(finish_dot, dim3(1), dim3(kT), 0, s, part, out_dev);
  return hip_check(hipGetLastError(), "dot launch");
}

int vec_copy(const double* a, double* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(kT), 0, s, a, b, n);
  return hip_check(hipGetLastError(), "copy launch");
}
int vec_zero(double* a, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(grid_for(n)), dim3(kT), 0, s, a, n);
  return hip_check(hipGetLastError(), "zero launch");
}
int vec_sub_from(const double* a, double* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_from, dim3(grid_for(n)), dim3(kT), 0, s, a, b, n);
  return hip_check(hipGetLastError(), "sub launch");
}
int vec_axpy(double alpha, const double* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(kT), 0, s, alpha, x, y, n);
  return hip_check(hipGetLastError(), "axpy launch");
}
int vec_div(const double* r, const double* diag, double* z, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_div, dim3(grid_for(n)), dim3(kT), 0, s, r, diag, z, n);
  return hip_check(hipGetLastError(), "div launch");
}

int pcg_alpha(const double* p, const double* q, int64_t n, double* part, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(dot_partial, dim3(kRedBlocks), dim3(kT), 0, s, p, q, n, part);
  hipLaunchKernelGGL(finish_alpha, dim3(1), dim3(kT), 0, s, part, sc);
  return hip_check(hipGetLastError(), "alpha launch");
}

int pcg_update_xr(double* x, double* r, const double* p, const double* q, int64_t n, double* part, double* sc,
                  hipStream_t s) {
  hipLaunchKernelGGL(update_xr, dim3(kRedBlocks), dim3(kT), 0, s, x, r, p, q, n, part, sc);
  return hip_check(hipGetLastError(), "update launch");
}

int pcg_rz_partial(const double* r, const double* z, int64_t n, double* part, hipStream_t s) {
  hipLaunchKernelGGL(dot_partial, dim3(kRedBlocks), dim3(kT), 0, s, r, z, n, part + kRedBlocks);
  return hip_check(hipGetLastError(), "rz launch");
}

int pcg_finish_beta(double* part, bool has_z, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(finish_beta, dim3(1), dim3(kT), 0, s, part, has_z ? 1 : 0, -1.0, sc);
  return hip_check(hipGetLastError(), "beta launch");
}

int pcg_rr_partial(const double* r, int64_t n, double* part, hipStream_t s) {
  hipLaunchKernelGGL(dot_partial, dim3(kRedBlocks), dim3(kT), 0, s, r, r, n, part);
  return hip_check(hipGetLastError(), "rr launch");
}

int pcg_finish_beta_from(double* part, bool has_z, double rz_prev, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(finish_beta, dim3(1), dim3(kT), 0, s, part, has_z ? 1 : 0, rz_prev, sc);
  return hip_check(hipGetLastError(), "beta launch");
}

int pcg_update_p(double* p, const double* z, int64_t n, const double* sc, hipStream_t s) {
  hipLaunchKernelGGL(update_p, dim3(grid_for(n)), dim3(kT), 0, s, p, z, n, sc);
  return hip_check(hipGetLastError(), "update_p launch");
}

int fcg_update_p(double* p, const double* z, int64_t n, const double* sc, hipStream_t s) {
  hipLaunchKernelGGL(fcg_p, dim3(grid_for(n)), dim3(kT), 0, s, p, z, n, sc);
  return hip_check(hipGetLastError(), "fcg_p launch");
}

int pcg_start(const double* r, const double* z, int64_t n, double* part, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(dot_partial, dim3(kRedBlocks), dim3(kT), 0, s, r, z, n, part);
  hipLaunchKernelGGL(finish_start, dim3(1), dim3(kT), 0, s, part, sc);
  return hip_check(hipGetLastError(), "start launch");
}

int trend_add(const double* tgt, int64_t m, int32_t d, const int32_t* exps, int32_t p, const double* c, double h,
              const double* beta, double* out, hipStream_t s) {
  if (m <= 0) return MLBLUP_OK;
  hipLaunchKernelGGL(k_trend, dim3((unsigned)((m + kT - 1) / kT)), dim3(kT), 0, s, tgt, m, d, exps, p, c, h, beta,
                     out);
  return hip_check(hipGetLastError(), "trend launch");
}

namespace {
thread_local bool tl_profile_suppressed = false;
}

ProfileSuppress::ProfileSuppress() : prev_(tl_profile_suppressed) { tl_profile_suppressed = true; }
ProfileSuppress::~ProfileSuppress() { tl_profile_suppressed = prev_; }

bool profile_on() {
  return prof().on && !tl_profile_suppressed;
}

void profile_note(hipEvent_t a, hipEvent_t b, double pairs, int bucket) {
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.a.push_back(a);
  P.b.push_back(b);
  P.bucket.push_back(bucket);
  P.pairs.push_back(pairs);
}

}  // namespace mlb

extern "C" int mlblup_profile_enable(int32_t on) {
  mlb::clear_error();
  mlb::prof().on = on != 0;
  return MLBLUP_OK;
}

extern "C" int mlblup_profile_read(double* pair_ms, int64_t* launches, double* pairs) {
  mlb::clear_error();
  mlb::Prof& P = mlb::prof();
  std::lock_guard<std::mutex> g(P.mu);
  constexpr int NB = MLBLUP_PROF_BUCKETS;
  double ms_b[NB] = {0}, pairs_b[NB] = {0};
  int64_t n_b[NB] = {0};
  int st = MLBLUP_OK;
  for (size_t i = 0; i < P.a.size(); ++i) {
    float ms = 0.f;
    if (st == MLBLUP_OK) st = mlb::hip_check(hipEventSynchronize(P.b[i]), "hipEventSynchronize");
    if (st == MLBLUP_OK) st = mlb::hip_check(hipEventElapsedTime(&ms, P.a[i], P.b[i]), "hipEventElapsedTime");
    const int k = (P.bucket[i] >= 0 && P.bucket[i] < NB) ? P.bucket[i] : 0;
    ms_b[k] += ms;
    n_b[k] += 1;
    pairs_b[k] += P.pairs[i];
    (void)hipEventDestroy(P.a[i]);
    (void)hipEventDestroy(P.b[i]);
  }
  for (int k = 0; k < NB; ++k) {
    if (pair_ms) pair_ms[k] = ms_b[k];
    if (launches) launches[k] = n_b[k];
    if (pairs) pairs[k] = pairs_b[k];
  }
  P.a.clear();
  P.b.clear();
  P.bucket.clear();
  P.pairs.clear();
  return st;
}
