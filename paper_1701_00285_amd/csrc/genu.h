// Matern covariance for a general smoothness 0 < nu <= 8, FP64.
//
// phi(r) = sigma2 f(z), z = sqrt(2 nu) r / rho, with the Definition of
// Sec. 3.1: f(z) = c z^nu K_nu(z), c = 2^{1-nu} / Gamma(nu), f(0) = 1.
//
// Evaluation from s = z^2 (what the pair kernels compute), in two ranges:
//
//  * z < Z0: the series of K_nu at the origin (Abramowitz & Stegun 9.6.2,
//    9.6.10 for non-integer nu; 9.6.11 for integer nu), with w = z^2 / 4:
//      non-integer:  f = A(w) + s^nu C(w),
//        A_k = c pi 2^{nu}  / (2 sin(nu pi) k! Gamma(k+1-nu)),
//        C_k = -c pi 2^{-nu} / (2 sin(nu pi) k! Gamma(k+1+nu));
//      integer n:    f = A(w) + s^n (ln(z/2) B(w) + C(w)),
//        A_k = c 2^{n-1} (n-k-1)! (-1)^k / k!   (k < n),
//        B_k = c (-1)^{n+1} 2^{-n} / (k! (n+k)!),
//        C_k = c (-1)^n 2^{-n-1} (psi(k+1) + psi(n+k+1)) / (k! (n+k)!).
//    s^nu and ln(z/2) come from one FP64 logarithm of s (table-driven:
//    s = 2^e m, m near c_j = 1 + j/64, ln m = ln c_j + log1p(m/c_j - 1) with
//    a degree-8 series) and an FP64 exponential (genu_exp).  Near an integer
//    nu the two non-integer series cancel (1 / sin(nu pi)): within 0.001 of
//    an integer about 2e-12 relative remains.
//  * Z0 <= z < zcut: g(z) = f(z) e^z is smooth; it is tabulated as
//    degree-8 polynomials on intervals of width 1/4 (Chebyshev
//    interpolation on the host from std::cyl_bessel_k, stored as monomial
//    coefficients in t in [-1, 1]); f = g e^{-z}.
//  * z >= zcut, where f < 1e-18: f = 0.
//
// The table is a flat array of doubles built on the host (genu_build) and
// read by genu_f on the host or the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

namespace mlb {

constexpr int kGenuSer = 14;        // series terms (w <= 1: the next is below 1e-20 of the first)
constexpr int kGenuDeg = 8;         // polynomial degree per interval
constexpr int kGenuMaxInt = 256;    // intervals (z up to Z0 + 64)
constexpr int kGenuLogTab = 65;     // c_j = 1 + j/64, j = 0..64
constexpr double kGenuZ0 = 2.0;
constexpr double kGenuH = 0.25;
// layout: header, then A, B, C (kGenuSer each), the log table (1/c_j, ln c_j),
// the interval coefficients
constexpr int kGenuHdr = 8;
constexpr int kGenuOffA = kGenuHdr;
constexpr int kGenuOffB = kGenuOffA + kGenuSer;
constexpr int kGenuOffC = kGenuOffB + kGenuSer;
constexpr int kGenuOffLog = kGenuOffC + kGenuSer;
constexpr int kGenuOffPoly = kGenuOffLog + 2 * kGenuLogTab;
constexpr int kGenuDoubles = kGenuOffPoly + kGenuMaxInt * (kGenuDeg + 1);   // one table
// The device table of a general nu holds two tables and their FP32 copies:
//   [0, kGenuDoubles)                value f(z) = c z^nu K_nu(z), FP64;
//   [kGenuOffDeriv, +kGenuDoubles)   the derivative table, FP64: c z^mu K_mu(z)
//                                    with mu = |nu - 1|, so that (A&S 9.6.28,
//                                    K_{-mu} = K_mu) rho dphi/drho / sigma2 =
//                                    -z f'(z) = c z^{nu+1} K_{nu-1}(z) = s^e times it,
//                                    e = 1 for nu >= 1 and e = nu for nu < 1 (slot 2
//                                    of this table holds e);
//   from kGenuOffF32 (in doubles)    both tables again as floats, same layout.
constexpr int kGenuOffDeriv = kGenuDoubles;
constexpr int kGenuOffF32 = 2 * kGenuDoubles;
constexpr int kGenuSlotDexp = 2;
constexpr int64_t kGenuBytes = (int64_t)3 * kGenuDoubles * 8;

// Builds the device table for 0 < nu <= 8 (1/2, 3/2 and 5/2 use the closed
// forms instead, but are accepted); false if nu is out of range.
bool genu_build(double nu, std::vector<double>& tab);

// ln x for a normal x > 0 (FP64, a few ulp absolute near 1)
__host__ __device__ inline double genu_log(double x, const double* __restrict__ T) {
  const int hi = (int)(((uint64_t)__builtin_bit_cast(uint64_t, x)) >> 32);
  const uint32_t lo = (uint32_t)__builtin_bit_cast(uint64_t, x);
  int e = ((hi >> 20) & 0x7FF) - 1023;
  const uint64_t mb = ((uint64_t)(uint32_t)((hi & 0x000FFFFF) | 0x3FF00000) << 32) | lo;
  const double m = __builtin_bit_cast(double, mb);      // [1, 2)
  const int j = (int)((m - 1.0) * 64.0 + 0.5);           // nearest c_j
  const double u = fma(m, T[kGenuOffLog + 2 * j], -1.0);  // m / c_j - 1, |u| <= 1/128
  // log1p(u) = u - u^2/2 + ... + u^8/8 (next term < 2e-20)
  double p = fma(u, -1.0 / 8.0, 1.0 / 7.0);
  p = fma(u, p, -1.0 / 6.0);
  p = fma(u, p, 1.0 / 5.0);
  p = fma(u, p, -1.0 / 4.0);
  p = fma(u, p, 1.0 / 3.0);
  p = fma(u, p, -0.5);
  p = fma(u, p, 1.0);
  constexpr double kLn2Hi = 0.6931471805598903;           // ln 2 to 42 bits: e * hi exact for |e| < 2^11
  constexpr double kLn2Lo = 5.497923018708371e-14;
  return fma((double)e, kLn2Hi, fma((double)e, kLn2Lo, T[kGenuOffLog + 2 * j + 1] + u * p));
}

// e^x for |x| <= 708 (FP64, table-free): x = k ln2 + r, |r| <= ln2/2
// (Cody-Waite split of ln2), e^r by its degree-13 Taylor polynomial
// (truncation < 5e-18), 2^k in two exponent-field factors.
__host__ __device__ inline double genu_exp(double x) {
  x = fmin(fmax(x, -708.0), 708.0);
  const double k = rint(x * 1.4426950408889634);
  double r = fma(-k, 0.6931471805598903, x);
  r = fma(-k, 5.497923018708371e-14, r);
  double p = 1.0 / 6227020800.0;                         // 1/13!
  const double inv[13] = {1.0 / 479001600.0, 1.0 / 39916800.0, 1.0 / 3628800.0, 1.0 / 362880.0, 1.0 / 40320.0,
                          1.0 / 5040.0,      1.0 / 720.0,      1.0 / 120.0,     1.0 / 24.0,     1.0 / 6.0,
                          0.5,               1.0,              1.0};
  for (int i = 0; i < 13; ++i) p = fma(p, r, inv[i]);
  const int ki = (int)k;
  // 2^k in two factors so that k = -1074..1023 stays representable
  const int k1 = ki / 2, k2 = ki - k1;
  const double s1 = __builtin_bit_cast(double, (uint64_t)(k1 + 1023) << 52);
  const double s2 = __builtin_bit_cast(double, (uint64_t)(k2 + 1023) << 52);
  return p * s1 * s2;
}

// f(z) from s = z^2 (s > 0; callers add a tiny offset at s = 0)
__host__ __device__ inline double genu_f(double s, const double* __restrict__ T) {
  const double z = sqrt(s);
  if (z < kGenuZ0) {
    const double w = 0.25 * s;
    const int ns = (int)T[6];
    double a = 0.0, c = 0.0;
    for (int k = ns - 1; k >= 0; --k) {
      a = fma(a, w, T[kGenuOffA + k]);
      c = fma(c, w, T[kGenuOffC + k]);
    }
    const double ls = genu_log(s, T);
    const double pw = genu_exp(T[0] * ls);                // s^nu
    if (T[1] != 0.0) {
      double b = 0.0;
      for (int k = ns - 1; k >= 0; --k) b = fma(b, w, T[kGenuOffB + k]);
      const double lz = fma(0.5, ls, -0.6931471805599453);   // ln(z/2)
      return a + pw * fma(lz, b, c);
    }
    return a + pw * c;
  }
  if (z >= T[4]) return 0.0;
  const double q = (z - kGenuZ0) * (1.0 / kGenuH);
  int i = (int)q;
  const int nint = (int)T[5];
  if (i >= nint) i = nint - 1;
  const double t = 2.0 * (q - (double)i) - 1.0;
  const double* cf = T + kGenuOffPoly + i * (kGenuDeg + 1);
  double g = cf[kGenuDeg];
  for (int k = kGenuDeg - 1; k >= 0; --k) g = fma(g, t, cf[k]);
  return g * genu_exp(-z);
}

// rho dphi/drho / sigma2 = -z f'(z) from s = z^2 (s > 0); T is the value table
// of a device table (the derivative table follows it)
__host__ __device__ inline double genu_d(double s, const double* __restrict__ T) {
  const double* Td = T + kGenuOffDeriv;
  const double f = genu_f(s, Td);
  const double e = Td[kGenuSlotDexp];
  return e == 1.0 ? s * f : genu_exp(e * genu_log(s, Td)) * f;
}

// FP32 versions on the device (hardware sqrt, log2 and exp2), T the float copy
// of a table: relative error about 1e-6 (within 0.01 of an integer nu the
// series' two parts cancel and a few 1e-5 remain)
__device__ inline float genu_f32(float s, const float* __restrict__ T) {
  const float z = __builtin_amdgcn_sqrtf(s);
  if (z < (float)kGenuZ0) {
    const float w = 0.25f * s;
    const int ns = (int)T[6];
    float a = 0.0f, c = 0.0f;
    for (int k = ns - 1; k >= 0; --k) {
      a = fmaf(a, w, T[kGenuOffA + k]);
      c = fmaf(c, w, T[kGenuOffC + k]);
    }
    const float l2 = __builtin_amdgcn_logf(s);               // log2 s
    const float pw = __builtin_amdgcn_exp2f(T[0] * l2);        // s^nu
    if (T[1] != 0.0f) {
      float b = 0.0f;
      for (int k = ns - 1; k >= 0; --k) b = fmaf(b, w, T[kGenuOffB + k]);
      const float lz = 0.6931471805599453f * fmaf(0.5f, l2, -1.0f);   // ln(z/2)
      return a + pw * fmaf(lz, b, c);
    }
    return a + pw * c;
  }
  if (z >= T[4]) return 0.0f;
  const float q = (z - (float)kGenuZ0) * (float)(1.0 / kGenuH);
  int i = (int)q;
  const int nint = (int)T[5];
  if (i >= nint) i = nint - 1;
  const float t = 2.0f * (q - (float)i) - 1.0f;
  const float* cf = T + kGenuOffPoly + i * (kGenuDeg + 1);
  float g = cf[kGenuDeg];
  for (int k = kGenuDeg - 1; k >= 0; --k) g = fmaf(g, t, cf[k]);
  return g * __builtin_amdgcn_exp2f(-1.4426950408889634f * z);
}
// Td: the float copy of the derivative table
__device__ inline float genu_d32(float s, const float* __restrict__ Td) {
  const float f = genu_f32(s, Td);
  const float e = Td[kGenuSlotDexp];
  return e == 1.0f ? s * f : __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(s)) * f;
}

}  // namespace mlb
