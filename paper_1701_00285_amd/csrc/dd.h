// Double-double arithmetic (a value is hi + lo with |lo| <= ulp(hi)/2, about
// 32 significant digits), host and device.  The error-free transformations
// are Knuth's two-sum and the FMA two-product (Dekker's splitting is not
// needed with a fused multiply-add); the compound operations follow the
// double-double algorithms of Y. Hida, X. S. Li and D. H. Bailey
// ("Algorithms for quad-double precision floating point arithmetic",
// ARITH 15, 2001): accurate addition with two renormalisations, products
// with the cross terms folded into the error word.  The exponential reduces
// x = k ln2 + r, scales r by 2^-10, sums the Taylor series of e^r - 1 to
// degree 11 (|r| <= 3.4e-4, remainder below 1e-42) and undoes the scaling
// by ten squarings of (1 + s) written as s <- 2 s + s^2.
//
// Every function turns off floating-point contraction: a product fused into
// the following addition (a + b with a = x y computed as fma(x, y, b)) would
// break the error-free transformations.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace mlb {

struct dd {
  double hi, lo;
};

__host__ __device__ inline dd dd_make(double a) { return {a, 0.0}; }

__host__ __device__ inline dd two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__host__ __device__ inline dd quick_two_sum(double a, double b) {  // |a| >= |b|
#pragma clang fp contract(off)
  const double s = a + b;
  return {s, b - (s - a)};
}
__host__ __device__ inline dd two_prod(double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  return {p, fma(a, b, -p)};
}
__host__ __device__ inline dd dd_add(dd x, dd y) {
#pragma clang fp contract(off)
  dd s = two_sum(x.hi, y.hi);
  const dd t = two_sum(x.lo, y.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}
__host__ __device__ inline dd dd_neg(dd x) { return {-x.hi, -x.lo}; }
__host__ __device__ inline dd dd_sub(dd x, dd y) { return dd_add(x, dd_neg(y)); }
__host__ __device__ inline dd dd_add_d(dd x, double b) {
#pragma clang fp contract(off)
  dd s = two_sum(x.hi, b);
  s.lo += x.lo;
  return quick_two_sum(s.hi, s.lo);
}
__host__ __device__ inline dd dd_mul(dd x, dd y) {
#pragma clang fp contract(off)
  dd p = two_prod(x.hi, y.hi);
  p.lo += x.hi * y.lo + x.lo * y.hi;
  return quick_two_sum(p.hi, p.lo);
}
__host__ __device__ inline dd dd_mul_d(dd x, double b) {
#pragma clang fp contract(off)
  dd p = two_prod(x.hi, b);
  p.lo += x.lo * b;
  return quick_two_sum(p.hi, p.lo);
}
// x / b for a double b: one long-division step on the residual
__host__ __device__ inline dd dd_div_d(dd x, double b) {
#pragma clang fp contract(off)
  const double q1 = x.hi / b;
  const dd p = two_prod(q1, b);
  const double e = ((x.hi - p.hi) - p.lo + x.lo) / b;
  return quick_two_sum(q1, e);
}
// x / y: three quotient digits
__host__ __device__ inline dd dd_div(dd x, dd y) {
#pragma clang fp contract(off)
  const double q1 = x.hi / y.hi;
  dd r = dd_sub(x, dd_mul_d(y, q1));
  const double q2 = r.hi / y.hi;
  r = dd_sub(r, dd_mul_d(y, q2));
  const double q3 = r.hi / y.hi;
  const dd q = quick_two_sum(q1, q2);
  return dd_add_d(q, q3);
}
// sqrt(x) for x >= 0: the FP64 root q and one correction (x - q^2) / (2 q)
__host__ __device__ inline dd dd_sqrt(dd x) {
#pragma clang fp contract(off)
  if (!(x.hi > 0.0)) return {0.0, 0.0};
  const double q = sqrt(x.hi);
  const dd r = dd_sub(x, two_prod(q, q));
  return quick_two_sum(q, r.hi / (2.0 * q));
}
// 2^k x (exact while the result stays normal)
__host__ __device__ inline dd dd_ldexp(dd x, int k) { return {ldexp(x.hi, k), ldexp(x.lo, k)}; }

// e^x; x below -700 gives 0
__host__ __device__ inline dd dd_exp(dd x) {
#pragma clang fp contract(off)
  if (x.hi < -700.0) return {0.0, 0.0};
  const dd ln2 = {0.6931471805599453, 2.3190468138462996e-17};   // ln 2 = hi + lo
  const double k = nearbyint(x.hi / ln2.hi);
  dd r = dd_sub(x, dd_mul_d(ln2, k));
  r = dd_ldexp(r, -10);
  // e^r - 1 = r (1 + r/2 (1 + r/3 (... (1 + r/11))))
  dd s = dd_make(1.0);
  for (int j = 11; j >= 2; --j) s = dd_add_d(dd_mul(dd_div_d(r, (double)j), s), 1.0);
  s = dd_mul(r, s);
  for (int j = 0; j < 10; ++j) s = dd_add(dd_mul_d(s, 2.0), dd_mul(s, s));
  return dd_ldexp(dd_add_d(s, 1.0), (int)k);
}

}  // namespace mlb
