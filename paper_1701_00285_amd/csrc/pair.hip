// Dense Matern covariance product y_i = sum_j sigma2 phi(|r_i - c_j|) x_j
// (step (2) of the three-step product of the predictor iteration, Sec. 6.2),
// plus the fused rho-derivative dy_i = sum_j rho dphi/drho x_j.
//
// Kernel form with z = sqrt(2 nu) r / rho (half-integer closed forms of the
// Matern family, Sec. 3.1 remark, written in z):
//   nu = 1/2:  phi = e^-z                   rho dphi/drho = z e^-z
//   nu = 3/2:  phi = (1 + z) e^-z           rho dphi/drho = z^2 e^-z
//   nu = 5/2:  phi = (1 + z + z^2/3) e^-z   rho dphi/drho = z^2 (1 + z)/3 e^-z
// Coordinates are multiplied by sqrt(2 nu)/rho once when staged, so z is
// the Euclidean distance of staged points.
//
// Layout of the work: a workgroup of 256 threads owns R rows per thread
// (row coordinates held in registers) and one contiguous column range (a
// "split"); column points and x stream through LDS in tiles of 128,
// point-major with stride d+1 so that every lane reads the same LDS address
// (broadcast, conflict-free).  Each split writes its own partial row sums;
// a second kernel adds the splits in fixed order, so results are bitwise
// reproducible (no atomics).  Distances always come from coordinate
// differences in FP64 (exact zero on the diagonal, no cancellation for near
// pairs).  MLBLUP_FP64 then evaluates sqrt/exp in FP64; MLBLUP_FP32 rounds
// the squared distance to FP32 and uses the hardware FP32 sqrt and exp2
// with FP32 per-tile sums folded into FP64 accumulators.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "device.h"
#include "pairmath.h"

namespace mlb {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 128;

// Copies the general-nu tables a kernel reads into LDS: the value table, and
// the derivative table when OUT asks for it; FP64 tables for the FP64
// kernels, their float copies for FP32T.  Returns the LDS address (for
// FP32T, of floats).  Only the used part of each table is copied.
template <int OUT, bool FP32T>
__device__ const double* stage_genu(const double* __restrict__ gtab) {
  constexpr int kTabs = (OUT & 2) ? 2 : 1;
  const int nd0 = kGenuOffPoly + (int)gtab[5] * (kGenuDeg + 1);
  const int nd1 = kGenuOffPoly + (int)gtab[kGenuOffDeriv + 5] * (kGenuDeg + 1);
  if constexpr (!FP32T) {
    __shared__ double gsh[kTabs * kGenuDoubles];
    for (int i = threadIdx.x; i < nd0; i += blockDim.x) gsh[i] = gtab[i];
    if constexpr (OUT & 2)
      for (int i = threadIdx.x; i < nd1; i += blockDim.x) gsh[kGenuOffDeriv + i] = gtab[kGenuOffDeriv + i];
    return gsh;
  } else {
    __shared__ float gshf[kTabs * kGenuDoubles];
    const float* src = reinterpret_cast<const float*>(gtab + kGenuOffF32);
    for (int i = threadIdx.x; i < nd0; i += blockDim.x) gshf[i] = src[i];
    if constexpr (OUT & 2)
      for (int i = threadIdx.x; i < nd1; i += blockDim.x) gshf[kGenuOffDeriv + i] = src[kGenuOffDeriv + i];
    return reinterpret_cast<const double*>(gshf);
  }
}

// D > 0: compile-time dimension, at least the points' dimension dd (the coordinates past dd are
// zero).  FP32T: FP32 transcendentals.
template <int D, int NU2, int OUT, int R, bool FP32T>
__global__ __launch_bounds__(kThreads) void pair_kernel(const double* __restrict__ rows, int64_t m,
                                                        const double* __restrict__ cols, int64_t n, int dd,
                                                        const double* __restrict__ x, double* __restrict__ py,
                                                        double* __restrict__ pdy, double zs, int64_t cps,
                                                        const double* __restrict__ gtab) {
  constexpr int SD = D + 1;
  __shared__ double tile[kTile * SD];
  __shared__ double tab[kExpTab];
  exp_table_fill(tab);
  // general nu: the tables in LDS (read by every pair)
  const double* gt = gtab;
  if constexpr (NU2 == kNuGeneralT) gt = stage_genu<OUT, FP32T>(gtab);
  const int tid = threadIdx.x;
  const int64_t rbase = (int64_t)blockIdx.x * (kThreads * R);
  double xr[R][D];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int64_t i = rbase + r * kThreads + tid;
    if (i >= m) i = m - 1;
#pragma unroll
    for (int k = 0; k < D; ++k) xr[r][k] = k < dd ? rows[i * dd + k] * zs : 0.0;
  }
  double acc[R], dacc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = dacc[r] = 0.0;

  const int64_t c0 = (int64_t)blockIdx.y * cps;
  const int64_t c1 = (c0 + cps < n) ? c0 + cps : n;
  for (int64_t j0 = c0; j0 < c1; j0 += kTile) {
    const int cnt = (int)((c1 - j0) < kTile ? (c1 - j0) : kTile);
    __syncthreads();
    for (int e = tid; e < kTile * D; e += kThreads) {
      const int j = e / D, k = e - j * D;
      tile[j * SD + k] = (j < cnt && k < dd) ? cols[(j0 + j) * dd + k] * zs : 0.0;
    }
    for (int j = tid; j < kTile; j += kThreads) tile[j * SD + D] = (j < cnt) ? x[j0 + j] : 0.0;
    __syncthreads();
#pragma unroll 2
    for (int j = 0; j < kTile; ++j) {
      double cj[D];
#pragma unroll
      for (int k = 0; k < D; ++k) cj[k] = tile[j * SD + k];
      const double aj = tile[j * SD + D];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double s = 1e-300;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const double t = xr[r][k] - cj[k];
          s = fma(t, t, s);
        }
        double f = 0.0, g = 0.0;
        pair_value<NU2, OUT, FP32T>(s, tab, f, g, gt);
        if constexpr (OUT & 1) acc[r] = fma(f, aj, acc[r]);
        if constexpr (OUT & 2) dacc[r] = fma(g, aj, dacc[r]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = rbase + r * kThreads + tid;
    if (i < m) {
      if constexpr (OUT & 1) py[(int64_t)blockIdx.y * m + i] = acc[r];
      if constexpr (OUT & 2) pdy[(int64_t)blockIdx.y * m + i] = dacc[r];
    }
  }
}

// Any dimension (runtime d): row coordinates re-read from memory; slow
// fallback for dimensions past the largest compiled one (32).
template <int NU2, int OUT, bool FP32T>
__global__ __launch_bounds__(kThreads) void pair_kernel_any(const double* __restrict__ rows, int64_t m,
                                                            const double* __restrict__ cols, int64_t n, int d,
                                                            const double* __restrict__ x, double* __restrict__ py,
                                                            double* __restrict__ pdy, double zs, int64_t cps,
                                                            const double* __restrict__ gtab) {
  __shared__ double tab[kExpTab];
  exp_table_fill(tab);
  // general nu: the tables in LDS (read by every pair)
  const double* gt = gtab;
  if constexpr (NU2 == kNuGeneralT) gt = stage_genu<OUT, FP32T>(gtab);
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t i = i0 < m ? i0 : m - 1;
  const int64_t c0 = (int64_t)blockIdx.y * cps;
  const int64_t c1 = (c0 + cps < n) ? c0 + cps : n;
  double acc = 0.0, dacc = 0.0;
  for (int64_t j = c0; j < c1; ++j) {
    double s = 1e-300;
    for (int k = 0; k < d; ++k) {
      const double t = (rows[i * d + k] - cols[j * d + k]) * zs;
      s = fma(t, t, s);
    }
    double f = 0.0, g = 0.0;
    pair_value<NU2, OUT, FP32T>(s, tab, f, g, gt);
    if constexpr (OUT & 1) acc = fma(f, x[j], acc);
    if constexpr (OUT & 2) dacc = fma(g, x[j], dacc);
  }
  if (i0 < m) {
    if constexpr (OUT & 1) py[(int64_t)blockIdx.y * m + i0] = acc;
    if constexpr (OUT & 2) pdy[(int64_t)blockIdx.y * m + i0] = dacc;
  }
}

__global__ __launch_bounds__(kThreads) void reduce_splits(const double* __restrict__ part, int S, int64_t m,
                                                          double scale, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= m) return;
  double s = 0.0;
  for (int k = 0; k < S; ++k) s += part[(int64_t)k * m + i];
  y[i] = scale * s;
}

__global__ void fill_zero(double* __restrict__ y, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) y[i] = 0.0;
}

constexpr int rows_per_thread(int D) { return D <= 10 ? 2 : 1; }

template <int D, int NU2, int OUT, bool F>
void launch_fixed(const PairArgs& a, double zs, int S, int64_t cps, double* py, double* pdy, hipStream_t s) {
  constexpr int R = rows_per_thread(D);
  dim3 grid((unsigned)((a.m + kThreads * R - 1) / (kThreads * R)), (unsigned)S);
  hipLaunchKernelGGL((pair_kernel<D, NU2, OUT, R, F>), grid, dim3(kThreads), 0, s, a.rows, a.m, a.cols, a.n, a.d,
                     a.x, py, pdy, zs, cps, a.gtab);
}

template <int NU2, int OUT, bool F>
void launch_any(const PairArgs& a, double zs, int S, int64_t cps, double* py, double* pdy, hipStream_t s) {
  dim3 grid((unsigned)((a.m + kThreads - 1) / kThreads), (unsigned)S);
  hipLaunchKernelGGL((pair_kernel_any<NU2, OUT, F>), grid, dim3(kThreads), 0, s, a.rows, a.m, a.cols, a.n, a.d,
                     a.x, py, pdy, zs, cps, a.gtab);
}

template <int NU2, int OUT, bool F>
void dispatch_d(const PairArgs& a, double zs, int S, int64_t cps, double* py, double* pdy, hipStream_t s) {
  switch (padded_dim(a.d)) {
    case 1: launch_fixed<1, NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
    case 2: launch_fixed<2, NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
    case 3: launch_fixed<3, NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
    case 4: launch_fixed<4, NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
    case 5: launch_fixed<5, NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
    case 6: launch_fixed<6, NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
    case 8: launch_fixed<8, NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
    case 10: launch_fixed<10, NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
    case 16: launch_fixed<16, NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
    case 20: launch_fixed<20, NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
    case 24: launch_fixed<24, NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
    case 28: launch_fixed<28, NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
    case 32: launch_fixed<32, NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
    default: launch_any<NU2, OUT, F>(a, zs, S, cps, py, pdy, s); break;
  }
}

template <int NU2, bool F>
void dispatch_out(const PairArgs& a, double zs, int S, int64_t cps, double* py, double* pdy, hipStream_t s) {
  switch (a.outputs) {
    case 1: dispatch_d<NU2, 1, F>(a, zs, S, cps, py, pdy, s); break;
    case 2: dispatch_d<NU2, 2, F>(a, zs, S, cps, py, pdy, s); break;
    default: dispatch_d<NU2, 3, F>(a, zs, S, cps, py, pdy, s); break;
  }
}

template <bool F>
void dispatch_nu(const PairArgs& a, double zs, int S, int64_t cps, double* py, double* pdy, hipStream_t s) {
  if (a.nu2 == kNuGeneral) {
    dispatch_out<kNuGeneralT, F>(a, zs, S, cps, py, pdy, s);
    return;
  }
  switch (a.nu2) {
    case 0: dispatch_out<0, F>(a, zs, S, cps, py, pdy, s); break;
    case 1: dispatch_out<1, F>(a, zs, S, cps, py, pdy, s); break;
    case 3: dispatch_out<3, F>(a, zs, S, cps, py, pdy, s); break;
    default: dispatch_out<5, F>(a, zs, S, cps, py, pdy, s); break;
  }
}

bool has_fixed(int d) { return padded_dim(d) > 0; }

}  // namespace

int32_t pair_splits(int64_t m, int64_t n, int32_t d, int32_t precision) {
  (void)precision;
  if (m <= 0 || n <= 0) return 1;
  const int R = has_fixed(d) ? rows_per_thread(padded_dim(d)) : 1;
  const int64_t row_blocks = (m + (int64_t)kThreads * R - 1) / ((int64_t)kThreads * R);
  // aim for >= 2048 workgroups (8 per CU on 256 CUs), at least one column tile per split
  int64_t S = (2048 + row_blocks - 1) / row_blocks;
  const int64_t max_by_cols = (n + kTile - 1) / kTile;
  if (S > max_by_cols) S = max_by_cols;
  if (S > 64) S = 64;
  if (S < 1) S = 1;
  return (int32_t)S;
}

int64_t pair_workspace_bytes(int64_t m, int64_t n, int32_t d, int32_t precision, int32_t outputs) {
  if (m <= 0 || n <= 0) return 0;
  const int64_t S = pair_splits(m, n, d, precision);
  const int64_t per = S * m * (int64_t)sizeof(double);
  const int64_t aligned = (per + 255) / 256 * 256;
  int64_t b = aligned * (((outputs & 1) ? 1 : 0) + ((outputs & 2) ? 1 : 0));
  if ((precision == MLBLUP_MFMA_FP32 || precision == MLBLUP_MFMA_BF16X3) && outputs == MLBLUP_VALUE)
    b = std::max(b, ((int64_t)mfma_splits(m, n) * m * (int64_t)sizeof(double) + 255) / 256 * 256);
  if (m == n && sym_worthwhile(n)) b = std::max(b, sym_workspace_bytes(n, outputs));
  // tail: the general-nu table
  return (b + 255) / 256 * 256 + kGenuBytes;
}

int pair_launch_body(const PairArgs& a, double zs, void* work, hipStream_t s);

// general-nu tables, built once per nu on the host and kept for the process
const double* genu_table_cached(double nu) {
  static std::mutex mu;
  static std::map<double, std::vector<double>> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(nu);
  if (it == cache.end()) {
    std::vector<double> tab;
    if (!genu_build(nu, tab)) return nullptr;
    it = cache.emplace(nu, std::move(tab)).first;
  }
  return it->second.data();
}

int pair_launch(const PairArgs& a, void* work, int64_t work_bytes, hipStream_t s) {
  if (a.m < 0 || a.n < 0 || a.d < 1 || a.d > 64) return fail(MLBLUP_EINVAL, "cov_matvec: bad m, n or d");
  if (a.outputs < 1 || a.outputs > 3) return fail(MLBLUP_EINVAL, "cov_matvec: outputs must be 1, 2 or 3");

  if (!(a.rho > 0) || !(a.sigma2 > 0) || !std::isfinite(a.rho) || !std::isfinite(a.sigma2))
    return fail(MLBLUP_EINVAL, "cov_matvec: rho and sigma2 must be finite and > 0");
  if (a.nu2 != 0 && a.nu2 != 1 && a.nu2 != 3 && a.nu2 != 5 && a.nu2 != kNuGeneral)
    return fail(MLBLUP_EINVAL, "cov_matvec: nu must be in (0, 8] or +inf (Gaussian)");
  if (a.precision < MLBLUP_FP64 || a.precision > MLBLUP_MFMA_BF16X3)
    return fail(MLBLUP_EINVAL, "cov_matvec: unknown precision");
  if (a.m == 0) return MLBLUP_OK;
  if (((a.outputs & 1) && !a.y) || ((a.outputs & 2) && !a.dy))
    return fail(MLBLUP_EINVAL, "cov_matvec: missing output pointer");
  if (a.n == 0) {
    const unsigned g = (unsigned)((a.m + 255) / 256);
    if (a.outputs & 1) hipLaunchKernelGGL(fill_zero, dim3(g), dim3(256), 0, s, a.y, a.m);
    if (a.outputs & 2) hipLaunchKernelGGL(fill_zero, dim3(g), dim3(256), 0, s, a.dy, a.m);
    return hip_check(hipGetLastError(), "fill_zero launch");
  }
  if (!a.rows || !a.cols || !a.x) return fail(MLBLUP_EINVAL, "cov_matvec: NULL input pointer");
  const int64_t need = pair_workspace_bytes(a.m, a.n, a.d, a.precision, a.outputs);
  if (!work || work_bytes < need)
    return fail(MLBLUP_EINVAL, "cov_matvec: workspace too small (need " + std::to_string(need) + " bytes)");
  const double zs = kernel_scale(a.nu2, a.nu, a.rho);  // sqrt(2 nu) / rho (Gaussian: 1 / rho)
  if (a.nu2 == kNuGeneral) {
    // the table goes to the workspace's tail; the host copy lives as long as the process
    const double* host = genu_table_cached(a.nu);
    if (!host) return fail(MLBLUP_EINVAL, "cov_matvec: nu out of range for the general-nu table");
    double* dev = (double*)((char*)work + (need - kGenuBytes));
    MLB_HIP(hipMemcpyAsync(dev, host, kGenuBytes, hipMemcpyHostToDevice, s));
    PairArgs b = a;
    b.gtab = dev;
    return pair_launch_body(b, zs, work, s);
  }
  return pair_launch_body(a, zs, work, s);
}

int pair_launch_body(const PairArgs& a, double zs, void* work, hipStream_t s) {
  if (mfma_applies(a)) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (profile_on()) {
      MLB_HIP(hipEventCreate(&e0));
      MLB_HIP(hipEventCreate(&e1));
      MLB_HIP(hipEventRecord(e0, s));
    }
    const bool square = a.rows == a.cols && a.m == a.n && sym_worthwhile(a.n);
    const int st = square ? mfma_sym_launch(a, zs, work, s) : mfma_launch(a, zs, (double*)work, s);
    if (st) return st;
    if (!square) {
      const unsigned g = (unsigned)((a.m + kThreads - 1) / kThreads);
      hipLaunchKernelGGL(reduce_splits, dim3(g), dim3(kThreads), 0, s, (const double*)work, mfma_splits(a.m, a.n),
                         a.m, a.sigma2, a.y);
    }
    if (profile_on()) {
      MLB_HIP(hipEventRecord(e1, s));
      profile_note(e0, e1, (double)a.m * (double)a.n, a.precision * 4 + a.outputs);
    }
    return hip_check(hipGetLastError(), "matrix-core pair kernel launch");
  }
  // general nu: the symmetric kernel takes FP64 values; other arithmetic and
  // the derivative run the row-tiled kernel
  const bool genu_sym = a.nu2 != kNuGeneral || (a.precision == MLBLUP_FP64 && a.outputs == MLBLUP_VALUE);
  if (a.rows == a.cols && a.m == a.n && genu_sym && sym_supported(a.d) && sym_worthwhile(a.n)) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (profile_on()) {
      MLB_HIP(hipEventCreate(&e0));
      MLB_HIP(hipEventCreate(&e1));
      MLB_HIP(hipEventRecord(e0, s));
    }
    const int st = sym_launch(a, zs, work, s);
    if (st) return st;
    if (profile_on()) {
      MLB_HIP(hipEventRecord(e1, s));
      profile_note(e0, e1, (double)a.m * (double)a.n, a.precision * 4 + a.outputs);
    }
    return MLBLUP_OK;
  }
  const int S = pair_splits(a.m, a.n, a.d, a.precision);
  int64_t cps = (a.n + S - 1) / S;
  cps = (cps + kTile - 1) / kTile * kTile;  // splits start on tile boundaries
  const int64_t per = ((S * a.m * (int64_t)sizeof(double)) + 255) / 256 * 256;
  double* py = (a.outputs & 1) ? (double*)work : nullptr;
  double* pdy = (a.outputs & 2) ? (double*)((char*)work + ((a.outputs & 1) ? per : 0)) : nullptr;
  // reduced precisions: the FP32-transcendental kernel (also for the
  // matrix-core precisions when their form does not apply: d < 8 or d > 32,
  // derivative outputs)
  const bool f32 = a.precision != MLBLUP_FP64;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (profile_on()) {
    MLB_HIP(hipEventCreate(&e0));
    MLB_HIP(hipEventCreate(&e1));
    MLB_HIP(hipEventRecord(e0, s));
  }
  if (f32) dispatch_nu<true>(a, zs, S, cps, py, pdy, s);
  else dispatch_nu<false>(a, zs, S, cps, py, pdy, s);
  MLB_HIP(hipGetLastError());
  if (profile_on()) {
    MLB_HIP(hipEventRecord(e1, s));
    profile_note(e0, e1, (double)a.m * (double)a.n, a.precision * 4 + a.outputs);
  }
  const unsigned g = (unsigned)((a.m + kThreads - 1) / kThreads);
  if (a.outputs & 1) hipLaunchKernelGGL(reduce_splits, dim3(g), dim3(kThreads), 0, s, py, S, a.m, a.sigma2, a.y);
  if (a.outputs & 2)
    hipLaunchKernelGGL(reduce_splits, dim3(g), dim3(kThreads), 0, s, pdy, S, a.m, a.sigma2, a.dy);
  return hip_check(hipGetLastError(), "reduce_splits launch");
}

// ---- products for callers that cannot allocate ------------------------------
// The workspace of mlblup_cov_matvec_noalloc is this file-scope array: every
// GPU the library runs on holds its own copy until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, once per device with that device current, and that
// address is what the launches receive.  The pair kernels write every
// partial they read in the same call, so nothing in it has to start at zero;
// calls that overlap on one GPU share the array and race.
namespace {
constexpr int kMaxScratchDevices = 64;
__device__ __align__(256) unsigned char scratch[MLBLUP_NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxScratchDevices] = {};

int scratch_address(void** out) {
  int dev = -1;
  MLB_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(MLBLUP_EINVAL, "cov_matvec_noalloc: device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_check(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return MLBLUP_OK;
}
}  // namespace

int pair_launch_noalloc(const PairArgs& a, hipStream_t s) {
  void* ptr = nullptr;
  const int st = scratch_address(&ptr);
  if (st) return st;
  // malformed arguments go to pair_launch, which reports them
  const bool sized = a.m > 0 && a.n > 0 && a.d >= 1 && a.d <= 64 && a.outputs >= 1 && a.outputs <= 3 &&
                     a.precision >= MLBLUP_FP64 && a.precision <= MLBLUP_MFMA_BF16X3;
  if (sized) {
    const int64_t need = pair_workspace_bytes(a.m, a.n, a.d, a.precision, a.outputs);
    if (need > MLBLUP_NOALLOC_SCRATCH_BYTES)
      return fail(MLBLUP_EINVAL, "cov_matvec_noalloc: this product needs " + std::to_string(need) +
                                     " bytes of scratch, above the static " +
                                     std::to_string((long long)MLBLUP_NOALLOC_SCRATCH_BYTES) +
                                     " (use mlblup_cov_matvec with a workspace)");
  }
  ProfileSuppress quiet;  // no timing events: they would be created here
  return pair_launch(a, ptr, MLBLUP_NOALLOC_SCRATCH_BYTES, s);
}

}  // namespace mlb
