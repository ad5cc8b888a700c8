// Host-side closed forms the estimators need (not used on the path).
#pragma once

#include <cmath>

namespace mcp {
namespace host {

inline double norm_cdf(double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); }

// Discounted call on e^Y, Y ~ N(m, s2).
inline double lognormal_call(double m, double s2, double K, double disc) {
  const double s = std::sqrt(s2);
  const double d2 = (m - std::log(K)) / s;
  return disc * (std::exp(m + 0.5 * s2) * norm_cdf(d2 + s) - K * norm_cdf(d2));
}

// Black-Scholes call (no dividends): S N(d1) - K e^{-rT} N(d2); K = 0 gives S.
inline double bs_call(double S, double K, double r, double sigma, double T) {
  if (K <= 0.0) return S;
  const double st = sigma * std::sqrt(T);
  const double d1 = (std::log(S / K) + (r + 0.5 * sigma * sigma) * T) / st;
  return S * norm_cdf(d1) - K * std::exp(-r * T) * norm_cdf(d1 - st);
}

// Geometric average of S at t_i = i T/n, i = 1..n, under GBM: ln G is normal
// with mean ln S0 + (r - sigma^2/2) T (n+1)/(2n) and variance
// sigma^2 T (n+1)(2n+1)/(6 n^2). The mean of the geometric-Asian control
// variate (Kemna-Vorst, discretely sampled).
inline double geo_asian_call(double S0, double K, double r, double sigma, double T, unsigned n) {
  const double nn = (double)n;
  const double m = std::log(S0) + (r - 0.5 * sigma * sigma) * T * (nn + 1.0) / (2.0 * nn);
  const double s2 = sigma * sigma * T * (nn + 1.0) * (2.0 * nn + 1.0) / (6.0 * nn * nn);
  const double disc = std::exp(-r * T);
  if (K <= 0.0) return disc * std::exp(m + 0.5 * s2);
  return lognormal_call(m, s2, K, disc);
}

// Lower Cholesky factor of the symmetric matrix C (row-major d x d):
// C = L L^T. Returns false when a pivot is not positive.
inline bool cholesky(int d, const double* C, double* L) {
  for (int i = 0; i < d * d; ++i) L[i] = 0.0;
  for (int j = 0; j < d; ++j) {
    double s = C[j * d + j];
    for (int k = 0; k < j; ++k) s -= L[j * d + k] * L[j * d + k];
    if (!(s > 0.0)) return false;
    const double ljj = std::sqrt(s);
    L[j * d + j] = ljj;
    for (int i = j + 1; i < d; ++i) {
      double t = C[i * d + j];
      for (int k = 0; k < j; ++k) t -= L[i * d + k] * L[j * d + k];
      L[i * d + j] = t / ljj;
    }
  }
  return true;
}

}  // namespace host
}  // namespace mcp
