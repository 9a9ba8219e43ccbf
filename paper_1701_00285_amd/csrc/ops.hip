// Multilevel transform kernels (operators W and W^T, Sec. 3.1; steps (1)
// and (3) of the product chain, Sec. 6.2) and the Krylov vector kernels.
//
// Transform: one launch per tree level.  Analysis (v -> W v, L v) runs from
// the finest level to the root: a cell multiplies its candidate
// coefficients (leaf: its points' entries of v; internal: the children's
// scaling coefficients, stored contiguously) by V^T; the first a results
// are its scaling coefficients (passed up; at the root they are L v), the
// rest its wavelet coefficients, written to their slot of W v.  Synthesis
// (W^T) runs root to leaves with V.  One 64-lane wave per cell; lane j owns
// output j (and j+64, ...); the m x m block is read once, coalesced along
// the lanes (V for analysis, its transpose for synthesis), the m inputs are
// wave-uniform loads.  The work is HBM-bound: 8 m^2 bytes per cell.
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
constexpr int kMaxTopLevels = 24;
constexpr int kTopCells = 16;    // levels with at most this many cells go into the fused launch

__device__ __forceinline__ void analysis_node(const NodeDesc& D, int lane, const double* __restrict__ V,
                                              const double* __restrict__ v, double* __restrict__ scal,
                                              double* __restrict__ vw, double* __restrict__ vl) {
  const double* cin = D.leaf ? v + D.in_off : scal + D.in_off;
  const double* B = V + D.v_off;
  const int m = D.m;
  for (int j = lane; j < m; j += 64) {
    double acc = 0.0;
#pragma unroll 8
    for (int i = 0; i < m; ++i) acc = fma(B[(int64_t)i * m + j], cin[i], acc);
    if (j < D.a) {
      if (D.scal_off >= 0) scal[D.scal_off + j] = acc;
      else if (vl) vl[j] = acc;
    } else {
      vw[D.w_off + (j - D.a)] = acc;
    }
  }
}

__device__ __forceinline__ void synthesis_node(const NodeDesc& D, int lane, const double* __restrict__ Vt,
                                               const double* __restrict__ vw, const double* __restrict__ vl,
                                               double* __restrict__ scal, double* __restrict__ v) {
  const double* B = Vt + D.v_off;
  const int m = D.m, a = D.a;
  const double* cs = D.scal_off >= 0 ? scal + D.scal_off : vl;  // may be null at the root
  const double* cw = vw + D.w_off - a;
  double* out = D.leaf ? v + D.in_off : scal + D.in_off;
  for (int i = lane; i < m; i += 64) {
    double acc = 0.0;
    if (cs) {
#pragma unroll 8
      for (int j = 0; j < a; ++j) acc = fma(B[(int64_t)j * m + i], cs[j], acc);
    }
#pragma unroll 8
    for (int j = a; j < m; ++j) acc = fma(B[(int64_t)j * m + i], cw[j], acc);
    out[i] = acc;
  }
}

__global__ __launch_bounds__(kT) void analysis_level(const NodeDesc* __restrict__ desc,
                                                     const int32_t* __restrict__ lnodes, int32_t cnt,
                                                     const double* __restrict__ V, const double* __restrict__ v,
                                                     double* __restrict__ scal, double* __restrict__ vw,
                                                     double* __restrict__ vl) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t s = blockIdx.x * kWavesPerBlock + wave;
  if (s >= cnt) return;
  analysis_node(desc[lnodes[s]], lane, V, v, scal, vw, vl);
}

__global__ __launch_bounds__(kT) void synthesis_level(const NodeDesc* __restrict__ desc,
                                                      const int32_t* __restrict__ lnodes, int32_t cnt,
                                                      const double* __restrict__ Vt, const double* __restrict__ vw,
                                                      const double* __restrict__ vl, double* __restrict__ scal,
                                                      double* __restrict__ v) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t s = blockIdx.x * kWavesPerBlock + wave;
  if (s >= cnt) return;
  synthesis_node(desc[lnodes[s]], lane, Vt, vw, vl, scal, v);
}

// The whole synthesis in one launch: a wave per leaf walks its path from the
// root down.  At each cell on the path it forms only the scaling
// coefficients of the next cell (the cell's outputs that belong to that
// child), keeps them in LDS, and at the leaf writes the leaf's values.  An
// ancestor's few coefficients are recomputed by every leaf below it; the
// leaf blocks, which carry nearly all the bytes, are read once.  No
// workgroup waits for another.
constexpr int kPathMax = 64;   // tree depth bound of the fused form
constexpr int kCoefMax = 64;   // scaling coefficients per cell (p) bound of the fused form

__global__ __launch_bounds__(kT) void synthesis_fused(const NodeDesc* __restrict__ desc,
                                                      const int32_t* __restrict__ parent,
                                                      const int32_t* __restrict__ leaves, int32_t n_leaves,
                                                      const double* __restrict__ Vt, const double* __restrict__ vw,
                                                      const double* __restrict__ vl, double* __restrict__ v) {
  __shared__ int32_t path[kWavesPerBlock][kPathMax];
  __shared__ double cbuf[kWavesPerBlock][2][kCoefMax];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t g = blockIdx.x * kWavesPerBlock + wave;
  if (g >= n_leaves) return;
  // path leaf -> root
  int len = 0;
  if (lane == 0) {
    int32_t u = leaves[g];
    while (u >= 0 && len < kPathMax) {
      path[wave][len++] = u;
      u = parent[u];
    }
  }
  len = __shfl(len, 0, 64);
  __builtin_amdgcn_wave_barrier();
  // lane k holds the descriptor of the k-th cell of the path (one round trip
  // for the whole path); each step takes its fields from the step's lane
  int64_t p_voff = 0, p_woff = 0, p_inoff = 0, p_scal = 0;
  int p_m = 0, p_a = 0;
  if (lane < len) {
    const NodeDesc D = desc[path[wave][lane]];
    p_voff = D.v_off;
    p_woff = D.w_off;
    p_inoff = D.in_off;
    p_scal = D.scal_off;
    p_m = D.m;
    p_a = D.a;
  }
  auto from = [](int64_t x, int k) {
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)x, k);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), k);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
  };
  int cur = 0;
  for (int idx = len - 1; idx >= 0; --idx) {
    const double* B = Vt + from(p_voff, idx);
    const int m = __builtin_amdgcn_readlane(p_m, idx), a = __builtin_amdgcn_readlane(p_a, idx);
    const int64_t in_off = from(p_inoff, idx);
    const double* cs = idx == len - 1 ? vl : cbuf[wave][cur];  // the root's scaling part is L v (may be null)
    const double* cw = vw + from(p_woff, idx) - a;
    int lo = 0, cnt = m;
    if (idx > 0) {
      lo = (int)(from(p_scal, idx - 1) - in_off);  // 0 for the left child, a_left for the right
      cnt = __builtin_amdgcn_readlane(p_a, idx - 1);
    }
    for (int i = lo + lane; i < lo + cnt; i += 64) {
      double acc = 0.0;
      if (cs) {
        for (int j = 0; j < a; ++j) acc = fma(B[(int64_t)j * m + i], cs[j], acc);
      }
#pragma unroll 8
      for (int j = a; j < m; ++j) acc = fma(B[(int64_t)j * m + i], cw[j], acc);
      if (idx == 0) v[in_off + i] = acc;          // the leaf's values
      else cbuf[wave][cur ^ 1][i - lo] = acc;     // the next cell's scaling coefficients
    }
    __builtin_amdgcn_wave_barrier();
    cur ^= 1;
  }
}

// The small top levels (few cells each) in one launch of one workgroup:
// levels run in order with a workgroup barrier between them (the barrier
// orders this workgroup's global writes and reads).
struct TopLevels {
  int32_t begin[kMaxTopLevels + 1];  // level q occupies [begin[q], begin[q+1]) of level_nodes, q = 0..nlev-1
  int32_t nlev;
};

__global__ __launch_bounds__(kT) void analysis_top(const NodeDesc* __restrict__ desc,
                                                   const int32_t* __restrict__ lnodes, TopLevels L,
                                                   const double* __restrict__ V, const double* __restrict__ v,
                                                   double* __restrict__ scal, double* __restrict__ vw,
                                                   double* __restrict__ vl) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int q = L.nlev - 1; q >= 0; --q) {
    for (int32_t s = L.begin[q] + wave; s < L.begin[q + 1]; s += kWavesPerBlock)
      analysis_node(desc[lnodes[s]], lane, V, v, scal, vw, vl);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kT) void synthesis_top(const NodeDesc* __restrict__ desc,
                                                    const int32_t* __restrict__ lnodes, TopLevels L,
                                                    const double* __restrict__ Vt, const double* __restrict__ vw,
                                                    const double* __restrict__ vl, double* __restrict__ scal,
                                                    double* __restrict__ v) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int q = 0; q < L.nlev; ++q) {
    for (int32_t s = L.begin[q] + wave; s < L.begin[q + 1]; s += kWavesPerBlock)
      synthesis_node(desc[lnodes[s]], lane, Vt, vw, vl, scal, v);
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

// number of leading (shallow) levels small enough for the fused launch
int top_levels(const TransformDev& T) {
  int q = 0;
  while (q < T.levels && q < kMaxTopLevels && T.lvl_begin_host[q + 1] - T.lvl_begin_host[q] <= kTopCells) ++q;
  return q;
}

TopLevels make_top(const TransformDev& T, int nt) {
  TopLevels L{};
  for (int q = 0; q <= nt; ++q) L.begin[q] = T.lvl_begin_host[q];
  L.nlev = nt;
  return L;
}

}  // namespace

int transform_analysis(const TransformDev& T, const double* v, double* vw, double* vl, double* scal, hipStream_t s) {
  const int nt = top_levels(T);
  for (int q = T.levels - 1; q >= nt; --q) {
    const int32_t lb = T.lvl_begin_host[q], cnt = T.lvl_begin_host[q + 1] - lb;
    if (cnt <= 0) continue;
    const unsigned g = (unsigned)((cnt + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(analysis_level, dim3(g), dim3(kT), 0, s, T.desc, T.level_nodes + lb, cnt, T.V, v, scal, vw,
                       vl);
  }
  if (nt > 0)
    hipLaunchKernelGGL(analysis_top, dim3(1), dim3(kT), 0, s, T.desc, T.level_nodes, make_top(T, nt), T.V, v, scal, vw,
                       vl);
  return hip_check(hipGetLastError(), "analysis launch");
}

int transform_synthesis(const TransformDev& T, const double* vw, const double* vl, double* v, double* scal,
                        hipStream_t s) {
  if (T.leaves && T.n_leaves > 0 && T.levels <= kPathMax && T.p <= kCoefMax) {
    const unsigned g = (unsigned)((T.n_leaves + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(synthesis_fused, dim3(g), dim3(kT), 0, s, T.desc, T.parent, T.leaves, T.n_leaves, T.Vt, vw,
                       vl, v);
    return hip_check(hipGetLastError(), "synthesis launch");
  }
  const int nt = top_levels(T);
  if (nt > 0)
    hipLaunchKernelGGL(synthesis_top, dim3(1), dim3(kT), 0, s, T.desc, T.level_nodes, make_top(T, nt), T.Vt, vw, vl,
                       scal, v);
  for (int q = nt; q < T.levels; ++q) {
    const int32_t lb = T.lvl_begin_host[q], cnt = T.lvl_begin_host[q + 1] - lb;
    if (cnt <= 0) continue;
    const unsigned g = (unsigned)((cnt + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(synthesis_level, dim3(g), dim3(kT), 0, s, T.desc, T.level_nodes + lb, cnt, T.Vt, vw, vl,
                       scal, v);
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

bool profile_on() {
  return prof().on;
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
