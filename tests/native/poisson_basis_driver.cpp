// Host driver for the Poisson solve's 1D eigenbases: reads "N dirichlet" pairs from stdin and prints
// N * N values of Q (row-major) and N eigenvalues per pair.
#include <cstdio>
#include <vector>

#include "../../paper_1702_05167_amd/csrc/poisson_basis.h"

int main() {
  int N = 0, dir = 0;
  while (std::scanf("%d %d", &N, &dir) == 2) {
    std::vector<double> Q((size_t)N * N), lam((size_t)N);
    hsc::poisson_basis(N, dir != 0, Q.data(), lam.data());
    for (double v : Q) std::printf("%.17g ", v);
    for (double v : lam) std::printf("%.17g ", v);
    std::printf("\n");
  }
  return 0;
}
