// Host construction of the general-nu Matern table (see genu.h for the
// representation and its sources).
#include "genu.h"

#include <algorithm>
#include <cmath>

namespace mlb {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.5772156649015329;

double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

// psi(m) for an integer m >= 1: -gamma + sum_{j < m} 1/j
double digamma_int(int m) {
  double s = -kEulerGamma;
  for (int j = 1; j < m; ++j) s += 1.0 / j;
  return s;
}

}  // namespace

namespace {

// One table of c z^nu K_nu(z) for an order 0 <= nu <= 8 and a given constant
// c (the Matern normalisation for the value table), cut where it falls below
// `cut`.
void build_one(double nu, double c, double cut, double* T) {
  std::fill(T, T + kGenuDoubles, 0.0);
  const bool integer = std::fabs(nu - std::round(nu)) < 1e-12;
  T[0] = integer ? std::round(nu) : nu;
  T[1] = integer ? 1.0 : 0.0;
  T[2] = kGenuZ0;
  T[3] = 1.0 / kGenuH;
  T[6] = kGenuSer;
  T[7] = c;
  if (!integer) {
    const double sn = std::sin(nu * kPi);
    for (int k = 0; k < kGenuSer; ++k) {
      T[kGenuOffA + k] = c * kPi * std::pow(2.0, nu) / (2.0 * sn * factorial(k) * std::tgamma(k + 1 - nu));
      T[kGenuOffC + k] = -c * kPi * std::pow(2.0, -nu) / (2.0 * sn * factorial(k) * std::tgamma(k + 1 + nu));
    }
  } else {
    const int n = (int)std::round(nu);
    for (int k = 0; k < kGenuSer; ++k) {
      if (k < n) T[kGenuOffA + k] = c * std::ldexp(1.0, n - 1) * factorial(n - k - 1) * ((k & 1) ? -1.0 : 1.0) /
                                    factorial(k);
      const double den = factorial(k) * factorial(n + k);
      T[kGenuOffB + k] = c * ((n + 1) % 2 ? -1.0 : 1.0) * std::ldexp(1.0, -n) / den;
      T[kGenuOffC + k] = c * (n % 2 ? -1.0 : 1.0) * std::ldexp(1.0, -n - 1) *
                         (digamma_int(k + 1) + digamma_int(n + k + 1)) / den;
    }
  }
  for (int j = 0; j < kGenuLogTab; ++j) {
    const double cj = 1.0 + j / 64.0;
    T[kGenuOffLog + 2 * j] = 1.0 / cj;
    T[kGenuOffLog + 2 * j + 1] = std::log(cj);
  }
  // g(z) = f(z) e^z on [Z0, zcut), zcut where f < cut
  auto f = [&](double z) { return c * std::pow(z, nu) * std::cyl_bessel_k(nu, z); };
  double zcut = kGenuZ0;
  while (zcut < kGenuZ0 + kGenuMaxInt * kGenuH && f(zcut) >= cut) zcut += kGenuH;
  const int nint = std::max(1, (int)std::lround((zcut - kGenuZ0) / kGenuH));
  T[4] = kGenuZ0 + nint * kGenuH;
  T[5] = nint;
  constexpr int N = kGenuDeg + 1;
  for (int i = 0; i < nint; ++i) {
    // Chebyshev interpolation at the N Chebyshev points of [-1, 1]
    double vals[N], ch[N];
    for (int l = 0; l < N; ++l) {
      const double t = std::cos(kPi * (l + 0.5) / N);
      const double z = kGenuZ0 + kGenuH * (i + 0.5 * (t + 1.0));
      vals[l] = f(z) * std::exp(z);
    }
    for (int k = 0; k < N; ++k) {
      double s = 0.0;
      for (int l = 0; l < N; ++l) s += vals[l] * std::cos(kPi * k * (l + 0.5) / N);
      ch[k] = (k == 0 ? 1.0 : 2.0) * s / N;
    }
    // Chebyshev -> monomial coefficients in t (T_{k+1} = 2 t T_k - T_{k-1})
    double mono[N] = {0}, tkm1[N] = {0}, tk[N] = {0}, tkp1[N];
    tkm1[0] = 1.0;  // T_0
    tk[1] = 1.0;    // T_1
    for (int j = 0; j < N; ++j) mono[j] += ch[0] * tkm1[j];
    if (N > 1)
      for (int j = 0; j < N; ++j) mono[j] += ch[1] * tk[j];
    for (int k = 2; k < N; ++k) {
      for (int j = 0; j < N; ++j) tkp1[j] = (j > 0 ? 2.0 * tk[j - 1] : 0.0) - tkm1[j];
      for (int j = 0; j < N; ++j) mono[j] += ch[k] * tkp1[j];
      std::copy(tk, tk + N, tkm1);
      std::copy(tkp1, tkp1 + N, tk);
    }
    for (int j = 0; j < N; ++j) T[kGenuOffPoly + i * N + j] = mono[j];
  }
}

}  // namespace

bool genu_build(double nu, std::vector<double>& T) {
  if (!(nu > 0.0) || nu > 8.0) return false;
  T.assign((size_t)(kGenuBytes / 8), 0.0);
  const double c = std::pow(2.0, 1.0 - nu) / std::tgamma(nu);
  build_one(nu, c, 1e-18, T.data());
  // derivative: -z f'(z) = c z^{nu+1} K_{nu-1}(z) = s^e c z^mu K_mu(z), mu = |nu - 1|
  // (the cut is lower: s^e grows to about 2e3 where the table ends)
  build_one(std::fabs(nu - 1.0), c, 1e-22, T.data() + kGenuOffDeriv);
  T[kGenuOffDeriv + kGenuSlotDexp] = nu >= 1.0 ? 1.0 : nu;
  float* f32 = reinterpret_cast<float*>(T.data() + kGenuOffF32);
  for (int i = 0; i < 2 * kGenuDoubles; ++i) f32[i] = (float)T[i];
  return true;
}

}  // namespace mlb
