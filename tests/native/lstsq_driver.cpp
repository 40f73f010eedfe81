// Host driver for the least-squares routine of Anderson mixing: reads cases from stdin
// ("n m", then A column by column, then b) and prints "ok g_0 .. g_m-1" or "dependent" per case.
#include <cstdio>
#include <vector>

#include "../../paper_1702_05167_amd/csrc/lstsq.h"

int main() {
  long long n = 0;
  int m = 0;
  while (std::scanf("%lld %d", &n, &m) == 2) {
    std::vector<double> a((size_t)n * m), b((size_t)n), g((size_t)(m > 0 ? m : 1));
    for (double& v : a) if (std::scanf("%lf", &v) != 1) return 2;
    for (double& v : b) if (std::scanf("%lf", &v) != 1) return 2;
    if (hsc::lstsq_householder(n, m, a, b, g.data())) {
      std::printf("ok");
      for (int j = 0; j < m; ++j) std::printf(" %.17g", g[j]);
      std::printf("\n");
    } else {
      std::printf("dependent\n");
    }
  }
  return 0;
}
