// Host-side probe of the composite-panel set-up used by the library: the
// frequency-independent log table and the per-panel near-target plan.
// Reads from stdin
//   P n kmax np
//   P+1 breaks, P kinds           (printed back as a check only)
//   P*n node samples x y          (panel by panel)
//   np targets x y
// and prints "W" and the table row by row (W_ij, row i = target node), then
// "C p cls" per target and, per near target, "T p nq" and its quadrature
// points "x y w c panel".  Built by the test suite with g++; CPU only.
#include <cstdio>
#include <vector>
#include "../../paper_2507_05725_amd/csrc/panels.h"

int main() {
  int P = 0, n = 0, np = 0;
  double kmax = 0.0;
  if (std::scanf("%d %d %lf %d", &P, &n, &kmax, &np) != 4) return 1;
  std::vector<double> br(P + 1);
  std::vector<int> kinds(P);
  for (auto &b : br)
    if (std::scanf("%lf", &b) != 1) return 1;
  for (auto &k : kinds)
    if (std::scanf("%d", &k) != 1) return 1;
  const int N = P * n;
  std::vector<double> xy(2 * N), dxy(2 * N), z(2 * np);
  for (int i = 0; i < N; ++i)
    if (std::scanf("%lf %lf %lf %lf", &xy[2 * i], &xy[2 * i + 1], &dxy[2 * i], &dxy[2 * i + 1]) != 4)
      return 1;
  for (int p = 0; p < np; ++p)
    if (std::scanf("%lf %lf", &z[2 * p], &z[2 * p + 1]) != 2) return 1;
  const fthms::PanelGeom g =
      fthms::panel_geom_from_samples(P, n, xy.data(), dxy.data(), br.data(), kinds.data());
  std::vector<double> G;
  fthms::panel_log_table(g, xy, G);
  const double pi = 3.14159265358979323846264338327950288;
  std::printf("W\n");
  for (int i = 0; i < N; ++i) {
    for (int j = 0; j < N; ++j) std::printf("%.17g ", -2.0 * pi * G[(size_t)i + (size_t)j * N]);
    std::printf("\n");
  }
  // speeds |dx/ds| and spacing as the library forms them
  std::vector<double> smax(P, 0.0);
  for (int i = 0; i < N; ++i) {
    const int p = i / n;
    const double si = std::cos((2.0 * (i % n) + 1.0) * pi / (2.0 * n));
    double th, dth;
    fthms::cov_map(kinds[p], si, th, dth);
    const double sp = std::hypot(dxy[2 * i], dxy[2 * i + 1]) * std::fabs(0.5 * (br[p + 1] - br[p]) * dth);
    smax[p] = std::max(smax[p], sp);
  }
  double hmax = 0.0;  // along the arc: nodes of a panel run against t
  for (int p = 0; p < P; ++p)
    for (int j = 0; j + 1 < n; ++j) {
      const int a = p * n + j, b = a + 1;
      hmax = std::max(hmax, std::hypot(xy[2 * b] - xy[2 * a], xy[2 * b + 1] - xy[2 * a + 1]));
    }
  for (int p = 0; p + 1 < P; ++p) {
    const int a = p * n, b = (p + 1) * n + n - 1;
    hmax = std::max(hmax, std::hypot(xy[2 * b] - xy[2 * a], xy[2 * b + 1] - xy[2 * a + 1]));
  }
  fthms::NearPlanHost h;
  fthms::plan_near_panels(P, n, xy.data(), g.cx.data(), g.cy.data(), hmax, smax.data(), kmax, np,
                          z.data(), nullptr, h);
  for (int p = 0; p < np; ++p) std::printf("C %d %d\n", p, (int)h.cls[p]);
  for (size_t t = 0; t < h.tgt.size(); ++t) {
    std::printf("T %d %d\n", h.tgt[t], h.qoff[t + 1] - h.qoff[t]);
    for (int q = h.qoff[t]; q < h.qoff[t + 1]; ++q)
      std::printf("%.17g %.17g %.17g %.17g %d\n", h.xq[2 * q], h.xq[2 * q + 1], h.wq[q], h.cq[q],
                  h.pq[q]);
  }
  return 0;
}
