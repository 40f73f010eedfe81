// Closed-form orthonormal eigenbases of the 1D operators whose sum is the 7-point Poisson stencil on
// the device grid (host code; the Poisson solve uploads them once per grid).
#pragma once

#include <cmath>

namespace hsc {

// Q (N x N, row-major: Q[j * N + k] = mode k at point j) and lambda (N) of the operator
// (2 U_j - U_(j-1) - U_(j+1)) on N points:
//   dirichlet: the neighbours beyond both ends are fixed values (they move to the source);
//              Q[j][k] = sqrt(2 / (N + 1)) sin(pi (k + 1)(j + 1) / (N + 1)), lambda_k = 2 - 2 cos(pi (k + 1) / (N + 1));
//   otherwise (zero normal derivative): the neighbour beyond an end is the end point itself;
//              Q[j][k] = c_k cos(pi k (j + 1/2) / N), c_0 = sqrt(1 / N), c_k = sqrt(2 / N),
//              lambda_k = 2 - 2 cos(pi k / N).
inline void poisson_basis(int N, bool dirichlet, double* Q, double* lam) {
  const double pi = 3.14159265358979323846;
  for (int j = 0; j < N; ++j)
    for (int k = 0; k < N; ++k)
      Q[(long long)j * N + k] =
          dirichlet ? std::sqrt(2.0 / (N + 1)) * std::sin(pi * (k + 1) * (j + 1) / (N + 1))
                    : (k == 0 ? std::sqrt(1.0 / N) : std::sqrt(2.0 / N)) * std::cos(pi * k * (j + 0.5) / N);
  for (int k = 0; k < N; ++k)
    lam[k] = dirichlet ? 2.0 - 2.0 * std::cos(pi * (k + 1) / (N + 1)) : 2.0 - 2.0 * std::cos(pi * k / N);
}

}  // namespace hsc
