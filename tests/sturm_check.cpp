// Host driver for the Sturm count of the bisection eigensolver (csrc/sturm.h).
// stdin: ncases, then per case: n, d[0..n-1], e2[0..n-1] (e2[j] couples rows
// j-1 and j; e2[0] unused), nx, x[0..nx-1].  stdout: the counts, one per line.
#include <cstdio>
#include <vector>

#include "../paper_1702_00339_amd/csrc/sturm.h"

int main() {
  int ncases = 0;
  if (std::scanf("%d", &ncases) != 1) return 1;
  for (int c = 0; c < ncases; ++c) {
    int n = 0, nx = 0;
    if (std::scanf("%d", &n) != 1 || n < 1) return 1;
    std::vector<double> d(n), e2(n);
    for (double& v : d) if (std::scanf("%lf", &v) != 1) return 1;
    for (double& v : e2) if (std::scanf("%lf", &v) != 1) return 1;
    if (std::scanf("%d", &nx) != 1) return 1;
    for (int i = 0; i < nx; ++i) {
      double x = 0;
      if (std::scanf("%lf", &x) != 1) return 1;
      std::printf("%d %d\n", lhf::sturm_count<true>(d.data(), e2.data(), n, x),
                  lhf::sturm_count<false>(d.data(), e2.data(), n, x));
    }
  }
  return 0;
}
