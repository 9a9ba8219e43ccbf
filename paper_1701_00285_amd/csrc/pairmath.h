// Device arithmetic of one covariance pair: FP64 square root and e^{-z},
// the Matern closed forms in z, the FP32-transcendental variant.
#pragma once

#include <hip/hip_runtime.h>

namespace mlb {

// e^{-z} for 0 <= z, FP64, by the table-driven method of P. T. P. Tang
// ("Table-driven implementation of the exponential function in IEEE
// floating-point arithmetic", ACM TOMS 15(2), 1989): z = (32 m + j) ln2/32 + r,
// |r| <= ln2/64, e^{-z} = 2^{-m} 2^{-j/32} e^{-r}, with e^{-r} from its
// degree-6 Taylor polynomial (truncation < 4e-18 relative) and the 32
// values 2^{-j/32} from a table in LDS.  ln2/32 is split in two parts
// (Cody-Waite) so that n * L_HI is exact for n < 2^16; z is clamped to 708
// (e^{-708} is still a normal number), so m stays in range.  About 2 ulp.
constexpr double kExpInvL = 46.16624130844683;        // 32 / ln 2
constexpr double kExpLHi = 0.021660849392446835;      // ln 2 / 32, low 16 bits cleared
constexpr double kExpLLo = 5.145609244655338e-14;     // ln 2 / 32 - L_HI
constexpr int kExpTab = 32;

__device__ __forceinline__ void exp_table_fill(double* tab) {
  // 2^{-j/32}, j = 0..31, correctly rounded
  constexpr double t[kExpTab] = {
      1.0, 0.9785720620877001, 0.9576032806985737, 0.93708381705515, 0.9170040432046712,
      0.8973545375015536, 0.8781260801866497, 0.859309649061239, 0.8408964152537145,
      0.8228777390769825, 0.8052451659746271, 0.7879904225539432, 0.7711054127039704,
      0.7545822137967114, 0.7384130729697497, 0.7225904034885233, 0.7071067811865476,
      0.691954940981916, 0.6771277734684463, 0.6626183215798707, 0.6484197773255048,
      0.6345254785958666, 0.620928906036742, 0.6076236799902345, 0.5946035575013605,
      0.5818624293887887, 0.5693943173783458, 0.5571933712979462, 0.5452538663326288,
      0.5335702003384118, 0.5221368912137069, 0.5109485743270583};
  for (int j = threadIdx.x; j < kExpTab; j += blockDim.x) tab[j] = t[j];
}

__device__ __forceinline__ double exp_neg_f64(double z, const double* __restrict__ tab) {
  z = fmin(z, 708.0);
  // n = nearest integer to z 32/ln2: adding 1.5 * 2^52 leaves n in the low
  // mantissa bits (exact rounding by the FMA); subtracting it back gives n
  constexpr double kShift = 6755399441055744.0;  // 1.5 * 2^52
  const double t = fma(z, kExpInvL, kShift);
  const int ni = __double2loint(t);
  const double n = t - kShift;
  double r = fma(-n, kExpLHi, z);
  r = fma(-n, kExpLLo, r);
  const double u = -r;
  double p = fma(u, 1.0 / 720.0, 1.0 / 120.0);
  p = fma(u, p, 1.0 / 24.0);
  p = fma(u, p, 1.0 / 6.0);
  p = fma(u, p, 0.5);
  p = fma(u, p, 1.0);
  p = fma(u, p, 1.0);
  // 2^{-m} 2^{-j/32}: subtract m = n >> 5 from the exponent field of the
  // table value (m <= 1021 keeps the result a normal number)
  const double tj = tab[ni & (kExpTab - 1)];
  const double sc = __hiloint2double(__double2hiint(tj) - ((ni >> 5) << 20), __double2loint(tj));
  return p * sc;
}

// sqrt(s) for s > 0 (callers keep s away from 0 by a 1e-300 offset): the
// hardware reciprocal square root, one Goldschmidt step for g ~ sqrt(s),
// h ~ 1/(2 sqrt(s)), then one Newton correction of g.
__device__ __forceinline__ double sqrt_pos_f64(double s) {
  const double y = __builtin_amdgcn_rsq(s);
  double g = s * y;
  double h = 0.5 * y;
  const double e = fma(-g, h, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  const double d = fma(-g, g, s);
  return fma(d, h, g);
}

// Matern closed forms in z = sqrt(2 nu) r / rho (nu = NU2 / 2)
template <int NU2>
__device__ __forceinline__ double matern_poly(double z) {
  if constexpr (NU2 == 1) return 1.0;
  else if constexpr (NU2 == 3) return 1.0 + z;
  else return fma(z, fma(z, 1.0 / 3.0, 1.0), 1.0);
}
template <int NU2>
__device__ __forceinline__ double matern_dpoly(double z) {  // rho dphi/drho / e^{-z}
  if constexpr (NU2 == 1) return z;
  else if constexpr (NU2 == 3) return z * z;
  else return (z * z) * fma(z, 1.0 / 3.0, 1.0 / 3.0);
}
template <int NU2>
__device__ __forceinline__ float matern_polyf(float z) {
  if constexpr (NU2 == 1) return 1.0f;
  else if constexpr (NU2 == 3) return 1.0f + z;
  else return fmaf(z, fmaf(z, 1.0f / 3.0f, 1.0f), 1.0f);
}
template <int NU2>
__device__ __forceinline__ float matern_dpolyf(float z) {
  if constexpr (NU2 == 1) return z;
  else if constexpr (NU2 == 3) return z * z;
  else return (z * z) * fmaf(z, 1.0f / 3.0f, 1.0f / 3.0f);
}

// Kernel value (and rho-derivative) of one pair from its squared scaled
// distance s (FP64).  FP32T: FP32 sqrt and exp2 after rounding s to FP32.
template <int NU2, int OUT, bool FP32T>
__device__ __forceinline__ void pair_value(double s, const double* __restrict__ tab, double& f, double& g) {
  if constexpr (FP32T) {
    const float zf = __builtin_amdgcn_sqrtf((float)s);
    const float ef = __builtin_amdgcn_exp2f(-1.4426950408889634f * zf);
    if constexpr (OUT & 1) f = (double)(matern_polyf<NU2>(zf) * ef);
    if constexpr (OUT & 2) g = (double)(matern_dpolyf<NU2>(zf) * ef);
  } else {
    const double z = sqrt_pos_f64(s);
    const double e = exp_neg_f64(z, tab);
    if constexpr (OUT & 1) f = matern_poly<NU2>(z) * e;
    if constexpr (OUT & 2) g = matern_dpoly<NU2>(z) * e;
  }
}

// 64-lane rotation by one lane (DPP wave rotate); 64-bit value in two halves.
__device__ __forceinline__ double wave_rotate1(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x134, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x134, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ int wave_rotate1_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x134, 0xF, 0xF, false);
}

}  // namespace mlb
