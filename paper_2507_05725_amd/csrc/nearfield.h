// Host planning of the near-target quadrature of the single-layer potential.
//
// A target z is "near" an arc when some node lies closer than ten times the
// largest node spacing h: there the Gauss-Chebyshev rule, whose error for a
// degree-(N-1) density decays like exp(-pi d / h), is not accurate to
// ~1e-14.  Near targets get the exact potential of the density interpolant,
//   U(z) = int_0^pi Phi_k(z, x(cos phi)) alpha_N(cos phi) dphi,
// with a composite 16-point Gauss-Legendre rule in phi:
//   * uniform base panels short enough for the density bandwidth (N) and the
//     kernel oscillation (k |x'|);
//   * geometric refinement (ratio 2) toward phi*, the parameter of the arc
//     point nearest z, down to half the distance a from phi* to the complex
//     log singularity of the kernel, a ~ d / max(|dx/dphi|, sqrt(2 d |x'|)).
// The geometry at quadrature points comes from the Chebyshev interpolant of
// the node samples.  A composite-panel arc gets one such rule per panel, in
// s = cos phi (weights times sin phi) on the panel's own interpolants.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

namespace fthms {

constexpr double kNearFactor = 10.0;

// 16-point Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on
// the Legendre recurrence.
inline void gauss_legendre16(double *x, double *w) {
  const int n = 16;
  const double pi = 3.14159265358979323846264338327950288;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

struct NearPlanHost {
  std::vector<unsigned char> cls;  // per point: 0 skip, 1 far, 2 near
  std::vector<int> tgt;            // point index of each near target
  std::vector<int> qoff;           // [ntgt + 1] quadrature offsets
  std::vector<double> xq;          // [nq][2]
  std::vector<double> wq, cq;      // [nq]
  std::vector<int> pq;             // [nq] panel of each point (composite-panel arcs only)
};

// x(cos phi) from Chebyshev coefficients (Clenshaw)
inline void geom_at(const double *cx, const double *cy, int n, double c, double &px,
                    double &py) {
  double bx1 = 0, bx2 = 0, by1 = 0, by2 = 0;
  for (int m = n - 1; m >= 1; --m) {
    const double nx = cx[m] + 2.0 * c * bx1 - bx2;
    const double ny = cy[m] + 2.0 * c * by1 - by2;
    bx2 = bx1;
    bx1 = nx;
    by2 = by1;
    by1 = ny;
  }
  px = cx[0] + c * bx1 - bx2;
  py = cy[0] + c * by1 - by2;
}

inline void geom_at(const std::vector<double> &cx, const std::vector<double> &cy, double c,
                    double &px, double &py) {
  geom_at(cx.data(), cy.data(), (int)cx.size(), c, px, py);
}

// The rule for one target z and one curve piece x(cos phi), phi in [0, pi]
// (n Chebyshev coefficients, largest speed smax, base panel length Lp):
// nearest parameter by dense samples and golden-section refinement, then
// geometric grading toward it.  With sin_measure the weights carry sin phi
// (integrals in s = cos phi); the points are appended to `out`.  sx, sy are
// the piece's points at phi = pi s / (8 n), s = 0..8n.
inline void rule_toward_nearest(const double *cgx, const double *cgy, int n, const double *sx,
                                const double *sy, double smax, double Lp, double zx, double zy,
                                bool sin_measure, int panel, NearPlanHost &out) {
  const double pi = 3.14159265358979323846264338327950288;
  double gx[16], gw[16];
  gauss_legendre16(gx, gw);
  const int nbase = (int)std::ceil(pi / Lp);
  const int S = 8 * n;
  int best = 0;
  double bd = 1e300;
  for (int s = 0; s <= S; ++s) {
    const double d = std::hypot(zx - sx[s], zy - sy[s]);
    if (d < bd) {
      bd = d;
      best = s;
    }
  }
  auto dist = [&](double ph) {
    double px, py;
    geom_at(cgx, cgy, n, std::cos(ph), px, py);
    return std::hypot(zx - px, zy - py);
  };
  double lo = pi * std::max(0, best - 1) / S, hi = pi * std::min(S, best + 1) / S;
  const double gr = 0.61803398874989484820;
  double a = hi - gr * (hi - lo), b = lo + gr * (hi - lo);
  double fa = dist(a), fb = dist(b);
  for (int it = 0; it < 80; ++it) {
    if (fa < fb) {
      hi = b;
      b = a;
      fb = fa;
      a = hi - gr * (hi - lo);
      fa = dist(a);
    } else {
      lo = a;
      a = b;
      fa = fb;
      b = lo + gr * (hi - lo);
      fb = dist(b);
    }
  }
  double phs = 0.5 * (lo + hi);
  double d = dist(phs);
  if (dist(0.0) <= d) {
    phs = 0.0;
    d = dist(0.0);
  }
  if (dist(pi) <= d) {
    phs = pi;
    d = dist(pi);
  }
  const double eps = 1e-6;
  double p1x, p1y, p2x, p2y;
  geom_at(cgx, cgy, n, std::cos(std::max(0.0, phs - eps)), p1x, p1y);
  geom_at(cgx, cgy, n, std::cos(std::min(pi, phs + eps)), p2x, p2y);
  const double sphi = std::hypot(p2x - p1x, p2y - p1y) /
                      (std::min(pi, phs + eps) - std::max(0.0, phs - eps));
  double aest = d / std::max(sphi, std::sqrt(2.0 * d * smax));
  aest = std::max(aest, 1e-14);
  std::vector<double> br;
  for (int i = 0; i <= nbase; ++i) br.push_back(pi * i / nbase);
  if (phs > 0.0 && phs < pi) br.push_back(phs);
  for (double h = 0.5 * Lp; h > 0.5 * aest && h > 1e-14; h *= 0.5) {
    if (phs - h > 0.0) br.push_back(phs - h);
    if (phs + h < pi) br.push_back(phs + h);
  }
  std::sort(br.begin(), br.end());
  std::vector<double> u;
  for (double v : br)
    if (u.empty() || v - u.back() > 1e-15) u.push_back(v);
  for (size_t i = 0; i + 1 < u.size(); ++i) {
    const double c0 = 0.5 * (u[i] + u[i + 1]), h = 0.5 * (u[i + 1] - u[i]);
    for (int g = 0; g < 16; ++g) {
      const double ph = c0 + h * gx[g];
      const double c = std::cos(ph);
      double px, py;
      geom_at(cgx, cgy, n, c, px, py);
      out.xq.push_back(px);
      out.xq.push_back(py);
      out.wq.push_back(sin_measure ? h * gw[g] * std::sin(ph) : h * gw[g]);
      out.cq.push_back(c);
      if (panel >= 0) out.pq.push_back(panel);
    }
  }
}

// Classify targets against the nodes; near ones get a rule per curve piece.
// One piece: the weighted single-panel arc (integral in phi).  P pieces:
// the panels of a composite arc (integrals in s), n nodes each.
inline void plan_near_impl(int P, int n, const double *node_xy, const double *cgx,
                           const double *cgy, double hmax, const double *smax, double kmax,
                           int np, const double *xy, const unsigned char *skip,
                           NearPlanHost &out) {
  const double pi = 3.14159265358979323846264338327950288;
  out.cls.assign(np, 0);
  out.tgt.clear();
  out.qoff.assign(1, 0);
  out.xq.clear();
  out.wq.clear();
  out.cq.clear();
  out.pq.clear();
  const double rad = kNearFactor * hmax;
  const int N = P * n;
  const int S = 8 * n;
  std::vector<double> sx((size_t)P * (S + 1)), sy((size_t)P * (S + 1));
  for (int q = 0; q < P; ++q)
    for (int s = 0; s <= S; ++s)
      geom_at(cgx + (size_t)q * n, cgy + (size_t)q * n, n, std::cos(pi * s / S),
              sx[(size_t)q * (S + 1) + s], sy[(size_t)q * (S + 1) + s]);
  for (int p = 0; p < np; ++p) {
    if (skip && skip[p]) continue;
    const double zx = xy[2 * p], zy = xy[2 * p + 1];
    double dmin = 1e300;
    for (int j = 0; j < N; ++j)
      dmin = std::min(dmin, std::hypot(zx - node_xy[2 * j], zy - node_xy[2 * j + 1]));
    if (!(dmin < rad)) {
      out.cls[p] = 1;
      continue;
    }
    out.cls[p] = 2;
    for (int q = 0; q < P; ++q) {
      const double Lp = std::min(pi / 4.0, 24.0 / (n + kmax * smax[q]));
      rule_toward_nearest(cgx + (size_t)q * n, cgy + (size_t)q * n, n,
                          sx.data() + (size_t)q * (S + 1), sy.data() + (size_t)q * (S + 1),
                          smax[q], Lp, zx, zy, P > 1, P > 1 ? q : -1, out);
    }
    out.tgt.push_back(p);
    out.qoff.push_back((int)out.wq.size());
  }
}

inline void plan_near(int n, const double *node_xy, const std::vector<double> &cgx,
                      const std::vector<double> &cgy, double hmax, double smax, double kmax,
                      int np, const double *xy, const unsigned char *skip, NearPlanHost &out) {
  plan_near_impl(1, n, node_xy, cgx.data(), cgy.data(), hmax, &smax, kmax, np, xy, skip, out);
}

// Composite-panel arc: P panels of n nodes, coefficients [P][n], per-panel
// largest speed |dx/ds|.
inline void plan_near_panels(int P, int n, const double *node_xy, const double *cgx,
                             const double *cgy, double hmax, const double *smax, double kmax,
                             int np, const double *xy, const unsigned char *skip,
                             NearPlanHost &out) {
  plan_near_impl(P, n, node_xy, cgx, cgy, hmax, smax, kmax, np, xy, skip, out);
}

}  // namespace fthms
