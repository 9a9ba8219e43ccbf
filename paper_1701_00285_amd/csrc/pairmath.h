// Device arithmetic of one covariance pair: FP64 square root and e^{-z},
// the Matern closed forms in z, the FP32-transcendental variant.
#pragma once

#include <hip/hip_runtime.h>

#include "genu.h"

namespace mlb {

constexpr int kNuGeneralT = -2;  // template code of a general smoothness (see device.h)

// e^{-z} for 0 <= z, FP64, by the table-driven method of P. T. P. Tang
// ("Table-driven implementation of the exponential function in IEEE
// floating-point arithmetic", ACM TOMS 15(2), 1989): with k the integer
// nearest to -z 256/ln2, -z = (k + u) ln2/256 with |u| <= 1/2, and
// e^{-z} = 2^{k >> 8} 2^{(k & 255)/256} e^{u ln2/256}.  e^{u ln2/256} comes
// from its degree-4 Taylor polynomial in u (truncation < 4e-17 relative),
// the 256 values 2^{j/256} from a table in LDS, and the power of two is added
// to the exponent field.  u is one FMA, -z c - k with c = 256/ln2 rounded to
// FP64: the rounding of c (below 2^-45 relative) gives u an error below
// 3e-14 z, i.e. a relative error below 8e-17 z in the result (at most 3e-17
// absolute over all z), which the covariance products cannot see next to the
// rounding of their sums.  z is clamped to 700, which bounds |k| and keeps
// every scaled result a normal number.
constexpr double kExpInvL = 369.3299304675746;          // 256 / ln 2
constexpr double kExpL = 0.0027076061740622863;         // ln 2 / 256
constexpr int kExpTab = 256;
constexpr int kExpTabBits = 8;

__device__ __forceinline__ void exp_table_fill(double* tab) {
  // 2^{j/256}, j = 0..255, correctly rounded
  constexpr double t[kExpTab] = {
      1.0, 1.0027112750502025, 1.0054299011128027, 1.0081558981184175,
      1.0108892860517005, 1.0136300849514894, 1.016378314910953, 1.019133996077738,
      1.0218971486541166, 1.0246677928971357, 1.0274459491187637, 1.030231637686041,
      1.0330248790212284, 1.0358256936019572, 1.0386341019613787, 1.041450124688316,
      1.0442737824274138, 1.0471050958792898, 1.0499440858006872, 1.0527907730046264,
      1.0556451783605572, 1.0585073227945128, 1.061377227289262, 1.0642549128844645,
      1.0671404006768237, 1.0700337118202419, 1.0729348675259756, 1.075843889062791,
      1.0787607977571199, 1.0816856149932152, 1.0846183622133092, 1.0875590609177697,
      1.0905077326652577, 1.0934643990728858, 1.0964290818163769, 1.099401802630222,
      1.102382583307841, 1.1053714457017412, 1.1083684117236787, 1.1113735033448175,
      1.1143867425958924, 1.1174081515673693, 1.1204377524096067, 1.12347556733302,
      1.1265216186082418, 1.129575928566288, 1.1326385195987192, 1.1357094141578055,
      1.1387886347566916, 1.1418762039695616, 1.1449721444318042, 1.148076478840179,
      1.1511892299529827, 1.154310420590216, 1.1574400736337511, 1.1605782120274988,
      1.1637248587775775, 1.1668800369524817, 1.1700437696832502, 1.1732160801636373,
      1.1763969916502812, 1.1795865274628758, 1.182784710984341, 1.1859915656609938,
      1.189207115002721, 1.1924313825831512, 1.1956643920398273, 1.1989061670743806,
      1.202156731452703, 1.2054161090051239, 1.2086843236265816, 1.2119613992768012,
      1.215247359980469, 1.2185422298274085, 1.2218460329727576, 1.2251587936371455,
      1.22848053610687, 1.2318112847340759, 1.2351510639369334, 1.2384998981998165,
      1.241857812073484, 1.245224830175258, 1.2486009771892048, 1.2519862778663162,
      1.255380757024691, 1.2587844395497165, 1.2621973503942507, 1.2656195145788063,
      1.2690509571917332, 1.2724917033894028, 1.275941778396392, 1.2794012075056693,
      1.2828700160787783, 1.2863482295460256, 1.2898358734066657, 1.2933329732290895,
      1.2968395546510096, 1.3003556433796506, 1.3038812651919358, 1.3074164459346773,
      1.3109612115247644, 1.3145155879493546, 1.318079601266064, 1.3216532776031575,
      1.3252366431597413, 1.3288297242059544, 1.3324325470831615, 1.3360451382041458,
      1.339667524053303, 1.3432997311868353, 1.3469417862329458, 1.3505937158920345,
      1.3542555469368927, 1.3579273062129011, 1.3616090206382248, 1.365300717204012,
      1.3690024229745905, 1.3727141650876684, 1.3764359707545302, 1.380167867260238,
      1.383909881963832, 1.387662042298529, 1.3914243757719262, 1.3951969099662003,
      1.3989796725383112, 1.4027726912202048, 1.4065759938190154, 1.4103896082172707,
      1.4142135623730951, 1.4180478843204152, 1.4218926021691656, 1.4257477441054942,
      1.42961333839197, 1.433489413367789, 1.4373759974489824, 1.4412731191286257,
      1.4451808069770467, 1.449099089642035, 1.4530279958490526, 1.4569675544014438,
      1.460917794180647, 1.4648787441464057, 1.4688504333369818, 1.4728328908693675,
      1.4768261459394993, 1.4808302278224719, 1.4848451658727524, 1.488870989524397,
      1.4929077282912648, 1.4969554117672355, 1.5010140696264256, 1.5050837316234065,
      1.5091644275934228, 1.5132561874526098, 1.5173590411982147, 1.5214730189088146,
      1.5255981507445384, 1.529734466947287, 1.533881997840956, 1.5380407738316568,
      1.5422108254079407, 1.5463921831410214, 1.550584877685, 1.5547889397770887,
      1.559004400237837, 1.5632312899713576, 1.567469639965553, 1.5717194812923414,
      1.5759808451078865, 1.5802537626528246, 1.5845382652524937, 1.588834384317164,
      1.593142151342267, 1.597461597908627, 1.6017927556826934, 1.606135656416771,
      1.6104903319492543, 1.6148568142048607, 1.6192351351948637, 1.6236253270173289,
      1.6280274218573478, 1.632441451987275, 1.6368674497669644, 1.6413054476440063,
      1.645755478153965, 1.6502175739206177, 1.6546917676561943, 1.6591780921616162,
      1.6636765803267364, 1.6681872651305825, 1.6727101796415966, 1.6772453570178785,
      1.681792830507429, 1.6863526334483934, 1.6909247992693053, 1.6955093614893326,
      1.7001063537185235, 1.7047158096580513, 1.709337763100463, 1.713972247929926,
      1.718619298122478, 1.723278947746274, 1.7279512309618377, 1.732636182022311,
      1.7373338352737062, 1.7420442251551564, 1.746767386199169, 1.7515033530318782,
      1.7562521603732995, 1.761013843037584, 1.7657884359332727, 1.7705759740635547,
      1.7753764925265212, 1.7801900265154245, 1.785016611318935, 1.789856282321401,
      1.7947090750031072, 1.7995750249405351, 1.804454167806624, 1.809346539371032,
      1.8142521755003989, 1.8191711121586085, 1.8241033854070534, 1.8290490314048973,
      1.8340080864093424, 1.8389805867758937, 1.843966568958626, 1.8489660695104508,
      1.8539791250833855, 1.8590057724288205, 1.864046048397789, 1.8690999899412386,
      1.8741676341103, 1.8792490180565602, 1.8843441790323345, 1.8894531543909392,
      1.8945759815869656, 1.8997126981765553, 1.9048633418176741, 1.9100279502703899,
      1.9152065613971474, 1.9203992131630474, 1.925605943636125, 1.930826790987627,
      1.9360617934922943, 1.9413109895286405, 1.9465744175792332, 1.9518521162309783,
      1.9571441241754002, 1.9624504802089273, 1.9677712232331759, 1.9731063922552343,
      1.978456026387951, 1.9838201648502194, 1.9891988469672663, 1.9945921121709402};
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
  // k = nearest integer to -z 256/ln2: adding 1.5 * 2^52 leaves k in the low
  // mantissa bits (exact rounding by the FMA); subtracting it back gives k
  constexpr double kShift = 6755399441055744.0;  // 1.5 * 2^52
  const double t = fma(-z, kExpInvL, kShift);
  const int k = __double2loint(t);
  const double kn = t - kShift;
  const double u = fma(-z, kExpInvL, -kn);
  // e^{u L} = 1 + L u + (L u)^2/2 + (L u)^3/6 + (L u)^4/24, L = ln2/256
  constexpr double c2 = kExpL * kExpL / 2.0, c3 = c2 * kExpL / 3.0, c4 = c3 * kExpL / 4.0;
  double p = fma(u, c4, c3);
  p = fma(u, p, c2);
  p = fma(u, p, kExpL);
  p = fma(u, p, 1.0);
  // m = k >> 8 as a signed bitfield extract
  return {p * tab[k & (kExpTab - 1)], (int)__builtin_amdgcn_sbfe(k, kExpTabBits, 32 - kExpTabBits)};
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
// hardware reciprocal square root y (relative error below 2^-24 on gfx950,
// measured over [1e-6, 1e8]) and g = s y; with r = 1 - g y (one FMA, r of
// order 2^-23), sqrt(s) = g (1 - r)^(-1/2) = g (1 + r/2 + 3 r^2/8 + ...), and
// the series cut after r^2 leaves a relative error of about (5/16) r^3, below
// 2^-70: g + (g r)(1/2 + 3 r/8), 6 instructions (two Newton corrections of g
// with y/2 took 7)
__device__ __forceinline__ double sqrt_pos_f64(double s) {
  const double y = __builtin_amdgcn_rsq(s);
  const double g = s * y;
  const double r = fma(-g, y, 1.0);
  return fma(g * r, fma(0.375, r, 0.5), g);
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
__device__ __forceinline__ void pair_value(double s, const double* __restrict__ tab, double& f, double& g,
                                           const double* __restrict__ gtab = nullptr) {
  if constexpr (NU2 == kNuGeneralT) {
    // general nu (genu.h): FP64 from the value and derivative tables that
    // gtab points at, or FP32 from their float copies (then gtab points at
    // floats: the value table, the derivative table kGenuDoubles further on)
    if constexpr (FP32T) {
      const float* T = reinterpret_cast<const float*>(gtab);
      const float sf = fmaxf((float)s, 1e-30f);
      if constexpr (OUT & 1) f = (double)genu_f32(sf, T);
      if constexpr (OUT & 2) g = (double)genu_d32(sf, T + kGenuOffDeriv);
    } else {
      if constexpr (OUT & 1) f = genu_f(s, gtab);
      if constexpr (OUT & 2) g = genu_d(s, gtab);
    }
  } else if constexpr (NU2 == 0) {
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
