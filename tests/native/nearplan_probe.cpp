// Host-side probe of the near-target quadrature planner used by the field
// kernels.  Reads an arc (nodes, Chebyshev coefficients of its geometry,
// largest node spacing, largest speed, largest wavenumber) and targets on
// stdin; prints each target's class and, for near targets, the quadrature
// points, weights and cos(phi) values.  Built by the test suite with g++;
// it runs on the CPU only.
#include <cstdio>
#include <vector>
#include "../../paper_2507_05725_amd/csrc/nearfield.h"

int main() {
  int n = 0, np = 0;
  if (std::scanf("%d %d", &n, &np) != 2) return 1;
  std::vector<double> xy(2 * n), cgx(n), cgy(n), z(2 * np);
  for (int i = 0; i < n; ++i)
    if (std::scanf("%lf %lf", &xy[2 * i], &xy[2 * i + 1]) != 2) return 1;
  for (int i = 0; i < n; ++i)
    if (std::scanf("%lf %lf", &cgx[i], &cgy[i]) != 2) return 1;
  double hmax, smax, kmax;
  if (std::scanf("%lf %lf %lf", &hmax, &smax, &kmax) != 3) return 1;
  for (int p = 0; p < np; ++p)
    if (std::scanf("%lf %lf", &z[2 * p], &z[2 * p + 1]) != 2) return 1;
  fthms::NearPlanHost h;
  fthms::plan_near(n, xy.data(), cgx, cgy, hmax, smax, kmax, np, z.data(), nullptr, h);
  for (int p = 0; p < np; ++p) std::printf("C %d %d\n", p, (int)h.cls[p]);
  for (size_t t = 0; t < h.tgt.size(); ++t) {
    std::printf("T %d %d\n", h.tgt[t], h.qoff[t + 1] - h.qoff[t]);
    for (int q = h.qoff[t]; q < h.qoff[t + 1]; ++q)
      std::printf("%.17g %.17g %.17g %.17g\n", h.xq[2 * q], h.xq[2 * q + 1], h.wq[q], h.cq[q]);
  }
  return 0;
}
