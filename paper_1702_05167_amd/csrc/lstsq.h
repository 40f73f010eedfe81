// Small dense least squares on the host (the coefficients of Anderson mixing in the self-consistent
// loop): a few columns of length n, solved once per iteration.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace hsc {

// gamma = argmin || b - A gamma ||_2 for A (n x m, columns in `a`, column-major, overwritten) by
// Householder QR; false when R has a diagonal entry below 1e-12 of its largest (numerically singular)
// or when m > n (more columns than rows: dependent)
inline bool lstsq_householder(int64_t n, int m, std::vector<double>& a, std::vector<double>& b, double* gamma) {
  if ((int64_t)m > n) return false;
  std::vector<double> rdiag(m);
  for (int j = 0; j < m; ++j) {
    double* cj = a.data() + (size_t)j * n;
    double nrm = 0.0;
    for (int64_t i = j; i < n; ++i) nrm += cj[i] * cj[i];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) return false;
    const double alpha = cj[j] > 0.0 ? -nrm : nrm;
    cj[j] -= alpha;   // v = column below the diagonal with v_j = a_jj - alpha
    double vv = 0.0;
    for (int64_t i = j; i < n; ++i) vv += cj[i] * cj[i];
    auto reflect = [&](double* y) {
      double s = 0.0;
      for (int64_t i = j; i < n; ++i) s += cj[i] * y[i];
      s = 2.0 * s / vv;
      for (int64_t i = j; i < n; ++i) y[i] -= s * cj[i];
    };
    for (int k = j + 1; k < m; ++k) reflect(a.data() + (size_t)k * n);
    reflect(b.data());
    rdiag[j] = alpha;
  }
  double dmax = 0.0, dmin = INFINITY;
  for (double d : rdiag) { dmax = std::max(dmax, std::fabs(d)); dmin = std::min(dmin, std::fabs(d)); }
  if (!(dmin >= 1e-12 * dmax)) return false;
  for (int j = m - 1; j >= 0; --j) {   // R gamma = (Q^T b)[0:m]; R above the diagonal sits in a
    double s = b[j];
    for (int k = j + 1; k < m; ++k) s -= a[(size_t)k * n + j] * gamma[k];
    gamma[j] = s / rdiag[j];
  }
  return true;
}

}  // namespace hsc
