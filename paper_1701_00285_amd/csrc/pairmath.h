// Device arithmetic of one covariance pair: FP64 square root and e^{-z},
// the Matern closed forms in z, the FP32-transcendental variant.
#pragma once

#include <hip/hip_runtime.h>

namespace mlb {

// e^{-z} for 0 <= z, FP64, by the table-driven method of P. T. P. Tang
// ("Table-driven implementation of the exponential function in IEEE
// floating-point arithmetic", ACM TOMS 15(2), 1989): with k the integer
// nearest to -z 64/ln2, -z = k ln2/64 + r, |r| <= ln2/128, and
// e^{-z} = 2^{k >> 6} 2^{(k & 63)/64} e^r.  e^r comes from its degree-5
// Taylor polynomial (truncation < 4e-17 relative), the 64 values
// 2^{j/64} from a table in LDS, and the power of two is added to the exponent
// field.  ln2/64 is
// split in two parts (Cody-Waite; the high part has 36 significant bits, so
// k L_HI is exact for |k| < 2^17); z is clamped to 700, which bounds |k|
// and keeps every scaled result a normal number.  About 2 ulp.
constexpr double kExpInvL = 92.33248261689366;         // 64 / ln 2
constexpr double kExpLHi = 0.010830424696223417;       // ln 2 / 64 to 36 bits
constexpr double kExpLLo = 2.572804622327669e-14;      // ln 2 / 64 - L_HI
constexpr int kExpTab = 64;

__device__ __forceinline__ void exp_table_fill(double* tab) {
  // 2^{j/64}, j = 0..63, correctly rounded
  constexpr double t[kExpTab] = {
      1.0, 1.0108892860517005, 1.0218971486541166, 1.0330248790212284,
      1.0442737824274138, 1.0556451783605572, 1.0671404006768237, 1.0787607977571199,
      1.0905077326652577, 1.102382583307841, 1.1143867425958924, 1.1265216186082418,
      1.1387886347566916, 1.1511892299529827, 1.1637248587775775, 1.1763969916502812,
      1.189207115002721, 1.202156731452703, 1.215247359980469, 1.22848053610687,
      1.241857812073484, 1.255380757024691, 1.2690509571917332, 1.2828700160787783,
      1.2968395546510096, 1.3109612115247644, 1.3252366431597413, 1.339667524053303,
      1.3542555469368927, 1.3690024229745905, 1.383909881963832, 1.3989796725383112,
      1.4142135623730951, 1.42961333839197, 1.4451808069770467, 1.460917794180647,
      1.4768261459394993, 1.4929077282912648, 1.5091644275934228, 1.5255981507445384,
      1.5422108254079407, 1.559004400237837, 1.5759808451078865, 1.593142151342267,
      1.6104903319492543, 1.6280274218573478, 1.645755478153965, 1.6636765803267364,
      1.681792830507429, 1.7001063537185235, 1.718619298122478, 1.7373338352737062,
      1.7562521603732995, 1.7753764925265212, 1.7947090750031072, 1.8142521755003989,
      1.8340080864093424, 1.8539791250833855, 1.8741676341103, 1.8945759815869656,
      1.9152065613971474, 1.9360617934922943, 1.9571441241754002, 1.978456026387951};
  for (int j = threadIdx.x; j < kExpTab; j += blockDim.x) tab[j] = t[j];
}

// e^{-z} = v 2^m: the mantissa part v in [~0.99, 2) and the exponent m, so
// that callers can multiply v by the Matern polynomial before scaling.
struct ExpParts {
  double v;
  int m;
};
__device__ __forceinline__ ExpParts exp_neg_parts(double z, const double* __restrict__ tab) {
  z = fmin(z, 700.0);
  // k = nearest integer to -z 64/ln2: adding 1.5 * 2^52 leaves k in the low
  // mantissa bits (exact rounding by the FMA); subtracting it back gives k
  constexpr double kShift = 6755399441055744.0;  // 1.5 * 2^52
  const double t = fma(-z, kExpInvL, kShift);
  const int k = __double2loint(t);
  const double kn = t - kShift;
  double r = fma(-kn, kExpLHi, -z);
  r = fma(-kn, kExpLLo, r);
  double p = fma(r, 1.0 / 120.0, 1.0 / 24.0);
  p = fma(r, p, 1.0 / 6.0);
  p = fma(r, p, 0.5);
  p = fma(r, p, 1.0);
  p = fma(r, p, 1.0);
  return {p * tab[k & (kExpTab - 1)], k >> 6};
}
// v 2^m for a normal v and a normal result: m added to the exponent field
__device__ __forceinline__ double scale_pow2(double v, int m) {
  return __hiloint2double(__double2hiint(v) + (m << 20), __double2loint(v));
}
__device__ __forceinline__ double exp_neg_f64(double z, const double* __restrict__ tab) {
  const ExpParts e = exp_neg_parts(z, tab);
  return scale_pow2(e.v, e.m);
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
// FP64: the polynomial multiplies the mantissa part of e^{-z} (for nu=3/2,
// (1+z) v is one FMA) before the power of two is applied.
template <int NU2, int OUT, bool FP32T>
__device__ __forceinline__ void pair_value(double s, const double* __restrict__ tab, double& f, double& g) {
  if constexpr (NU2 == 0) {
    // Gaussian: s = r^2 / rho^2, phi = e^{-s/2}, rho dphi/drho = s e^{-s/2}
    if constexpr (FP32T) {
      const float e = __builtin_amdgcn_exp2f(-0.72134752044448170f * (float)s);
      if constexpr (OUT & 1) f = (double)e;
      if constexpr (OUT & 2) g = (double)((float)s * e);
    } else {
      const ExpParts e = exp_neg_parts(0.5 * s, tab);
      if constexpr (OUT & 1) f = scale_pow2(e.v, e.m);
      if constexpr (OUT & 2) g = scale_pow2(s * e.v, e.m);
    }
  } else if constexpr (FP32T) {
    const float zf = __builtin_amdgcn_sqrtf((float)s);
    const float ef = __builtin_amdgcn_exp2f(-1.4426950408889634f * zf);
    if constexpr (OUT & 1) f = (double)(matern_polyf<NU2>(zf) * ef);
    if constexpr (OUT & 2) g = (double)(matern_dpolyf<NU2>(zf) * ef);
  } else {
    const double z = sqrt_pos_f64(s);
    const ExpParts e = exp_neg_parts(z, tab);
    if constexpr (OUT & 1) {
      double fv;
      if constexpr (NU2 == 1) fv = e.v;
      else if constexpr (NU2 == 3) fv = fma(z, e.v, e.v);
      else fv = fma(z * fma(z, 1.0 / 3.0, 1.0), e.v, e.v);
      f = scale_pow2(fv, e.m);
    }
    if constexpr (OUT & 2) g = scale_pow2(matern_dpoly<NU2>(z) * e.v, e.m);
  }
}

// FP32 kernel value (and rho-derivative) from w = log2(e) z, the distance
// scaled so that e^{-z} = 2^{-w}: FP32 exp2 and the Matern polynomial with
// its coefficients rescaled to w.
template <int NU2, int OUT>
__device__ __forceinline__ void pair_value_w(float w, float& f, float& g) {
  constexpr float l1 = 0.6931471805599453f;               // ln 2
  constexpr float l2 = 0.4804530139182014f;               // ln^2 2
  const float e = __builtin_amdgcn_exp2f(-w);
  if constexpr (OUT & 1) {
    if constexpr (NU2 == 1) f = e;
    else if constexpr (NU2 == 3) f = fmaf(w, l1, 1.0f) * e;
    else f = fmaf(w, fmaf(w, l2 / 3.0f, l1), 1.0f) * e;
  }
  if constexpr (OUT & 2) {
    // rho dphi/drho: z e^{-z}, z^2 e^{-z}, z^2 (1 + z) e^{-z} / 3
    if constexpr (NU2 == 1) g = (w * l1) * e;
    else if constexpr (NU2 == 3) g = (w * (w * l2)) * e;
    else g = (w * (w * (l2 / 3.0f))) * (fmaf(w, l1, 1.0f) * e);
  }
}

// FP32 kernels take coordinates scaled by the kernel scale times lp_scale:
// log2(e) for the Matern forms (the distance is then w = log2(e) z), and
// sqrt(log2(e)/2) for the Gaussian (the squared distance is then
// s' = log2(e) r^2 / (2 rho^2), so that phi = 2^{-s'})
template <int NU2>
constexpr double lp_scale() {
  return NU2 == 0 ? 0.84932180028801907 : 1.4426950408889634;
}
// FP32 kernel value (and rho-derivative) from the squared scaled distance
template <int NU2, int OUT>
__device__ __forceinline__ void pair_value_lp(float s, float& f, float& g) {
  if constexpr (NU2 == 0) {
    const float e = __builtin_amdgcn_exp2f(-s);
    if constexpr (OUT & 1) f = e;
    if constexpr (OUT & 2) g = (s * 1.3862943611198906f) * e;  // r^2/rho^2 = 2 ln2 s'
  } else {
    pair_value_w<NU2, OUT>(__builtin_amdgcn_sqrtf(s), f, g);
  }
}

// 64-lane rotation by one lane (DPP wave rotate); 64-bit value in two halves.
__device__ __forceinline__ double wave_rotate1(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x134, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x134, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float wave_rotate1_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x134, 0xF, 0xF, false));
}
__device__ __forceinline__ int wave_rotate1_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x134, 0xF, 0xF, false);
}

}  // namespace mlb
