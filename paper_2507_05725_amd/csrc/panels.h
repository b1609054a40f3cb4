// Composite-panel arcs (Section 4.3, eqs. cov and psi-tilde): host set-up,
// once per arc and independent of the frequency.
//
// An arc x(t), t in [-1, 1], is cut at breakpoints t_0 = -1 < ... < t_P = 1
// into panels (the ends of the arc and of its truncated overlap are panel
// ends).  Panel p has its own variable theta in [-1, 1], t = t_p + (t_{p+1}
// - t_p)(1 + theta)/2, and theta = theta(s) is one of the cosine maps of
// eq. cov (none, both ends, the -1 end, the +1 end), chosen by where the
// density is singular.  In s: first-kind Chebyshev nodes s_i = cos(phi_i),
// phi_i = (2i+1) pi / (2n), and Fejer weights.  The unknown is the density
// per unit s, mu = psi |dx/ds|.
//
// Matrix: with Phi_k = -(1/2pi) J0(kr) log r + S(r), S smooth,
//     A_ij = -(1/2pi) J0(k r_ij) W_ij + w_j S(r_ij),
//     W_ij = int_{panel(j)} log|y_i - y(s)| l_j(s) ds   (l_j: Lagrange basis),
// i.e. the log part integrated exactly against the panel interpolant, the
// smooth part by the Fejer rule.  W is built here by composite 16-point
// Gauss-Legendre quadrature in phi (s = cos phi, ds = sin phi dphi) of the
// Chebyshev moments int log|y_i - y(s)| T_m(s) ds, graded geometrically
// toward the target (on its own panel) or toward the nearest panel point
// (on the others).  The geometry off the nodes is the panel interpolant of
// the node samples; near the target (on its own panel, or on a neighbouring
// panel next to the break they share, then via the break point) the
// differences y(s) - y(s_i) are integrals of the interpolated derivative,
// int_{s_i}^{s} x'(t(u)) t'(u) du (8-point Gauss-Legendre; t' analytic from
// eq. cov), which keeps them accurate in relative terms where the cosine
// maps cluster the nodes and differences of interpolated points would not.
#pragma once

#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "nearfield.h"

namespace fthms {

enum { kCovNone = 0, kCovBoth = 1, kCovLeft = 2, kCovRight = 3 };
constexpr int kMaxPanels = 16;

// eq. cov: theta(s) and theta'(s)
inline void cov_map(int kind, double s, double &th, double &dth) {
  const double pi = 3.14159265358979323846264338327950288;
  switch (kind) {
    case kCovBoth: {
      const double a = 0.5 * pi * (1.0 - s);
      th = std::cos(a);
      dth = 0.5 * pi * std::sin(a);
      return;
    }
    case kCovLeft: {
      const double a = 0.25 * pi * (1.0 + s);
      th = 1.0 - 2.0 * std::cos(a);
      dth = 0.5 * pi * std::sin(a);
      return;
    }
    case kCovRight: {
      const double a = 0.25 * pi * (1.0 - s);
      th = 2.0 * std::cos(a) - 1.0;
      dth = 0.5 * pi * std::sin(a);
      return;
    }
    default:
      th = s;
      dth = 1.0;
  }
}

// Fejer's first rule on s_i = cos(phi_i): w_i = int_{-1}^{1} l_i(s) ds
//   = (2/n) [1 - 2 sum_{m=1}^{n/2} cos(2 m phi_i) / (4 m^2 - 1)].
inline void fejer_weights(int n, std::vector<double> &w) {
  const double pi = 3.14159265358979323846264338327950288;
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    const double ph = (2.0 * i + 1.0) * pi / (2.0 * n);
    double acc = 0.0;
    for (int m = n / 2; m >= 1; --m) acc += std::cos(2.0 * m * ph) / (4.0 * m * m - 1.0);
    w[i] = (2.0 / n) * (1.0 - 2.0 * acc);
  }
}

struct PanelGeom {
  int P = 1, n = 0;
  std::vector<double> cx, cy;  // [P][n] Chebyshev coefficients of x(t(s)) per panel
  std::vector<double> dx, dy;  // [P][n] Chebyshev coefficients of x'(t(s)) (dx/dt)
  std::vector<double> breaks;  // [P + 1]
  std::vector<int> kinds;      // [P]
};

// Chebyshev coefficients of each panel's geometry and of dx/dt from the node
// samples xy, dxy [P n][2] (node i of a panel at phi_i = (2i+1) pi / (2n)):
//   c_m = ((2 - delta_m0) / n) sum_j x_j cos(m phi_j).
inline PanelGeom panel_geom_from_samples(int P, int n, const double *xy, const double *dxy,
                                         const double *breaks, const int *kinds) {
  const double pi = 3.14159265358979323846264338327950288;
  PanelGeom g;
  g.P = P;
  g.n = n;
  g.breaks.assign(breaks, breaks + P + 1);
  g.kinds.assign(kinds, kinds + P);
  g.cx.assign((size_t)P * n, 0.0);
  g.cy.assign((size_t)P * n, 0.0);
  g.dx.assign((size_t)P * n, 0.0);
  g.dy.assign((size_t)P * n, 0.0);
  for (int p = 0; p < P; ++p)
    for (int m = 0; m < n; ++m) {
      double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
      for (int j = 0; j < n; ++j) {
        const double cc = std::cos(m * (2.0 * j + 1.0) * pi / (2.0 * n));
        ax += xy[2 * (p * n + j)] * cc;
        ay += xy[2 * (p * n + j) + 1] * cc;
        bx += dxy[2 * (p * n + j)] * cc;
        by += dxy[2 * (p * n + j) + 1] * cc;
      }
      const double f = (m == 0 ? 1.0 : 2.0) / n;
      g.cx[(size_t)p * n + m] = f * ax;
      g.cy[(size_t)p * n + m] = f * ay;
      g.dx[(size_t)p * n + m] = f * bx;
      g.dy[(size_t)p * n + m] = f * by;
    }
  return g;
}

inline void panel_point(const PanelGeom &g, int p, double c, double &x, double &y) {
  const double *ax = g.cx.data() + (size_t)p * g.n, *ay = g.cy.data() + (size_t)p * g.n;
  double bx1 = 0, bx2 = 0, by1 = 0, by2 = 0;
  for (int m = g.n - 1; m >= 1; --m) {
    const double nx = ax[m] + 2.0 * c * bx1 - bx2;
    const double ny = ay[m] + 2.0 * c * by1 - by2;
    bx2 = bx1;
    bx1 = nx;
    by2 = by1;
    by1 = ny;
  }
  x = ax[0] + c * bx1 - bx2;
  y = ay[0] + c * by1 - by2;
}

// y_p(s) - y_p(s0) = int_{s0}^{s} x'(t(u)) t'(u) du, 8-point Gauss-Legendre
// (for |s - s0| up to a few tenths: the integrand is smooth on the panel)
inline void panel_diff(const PanelGeom &g, int p, double s, double s0, const double *g8x,
                       const double *g8w, double &dx, double &dy) {
  const int n = g.n;
  const double *ax = g.dx.data() + (size_t)p * n, *ay = g.dy.data() + (size_t)p * n;
  const double h = 0.5 * (g.breaks[p + 1] - g.breaks[p]);
  const double c0 = 0.5 * (s + s0), hw = 0.5 * (s - s0);
  double sx = 0.0, sy = 0.0;
  for (int q = 0; q < 8; ++q) {
    const double u = c0 + hw * g8x[q];
    double th, dth, px, py;
    cov_map(g.kinds[p], u, th, dth);
    geom_at(ax, ay, n, u, px, py);
    const double f = g8w[q] * h * dth;
    sx += f * px;
    sy += f * py;
  }
  dx = hw * sx;
  dy = hw * sy;
}

inline void gauss_legendre8(double *x, double *w) {
  const int n = 8;
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

// Frequency-independent table G = -W / (2 pi), column-major G[i + j N],
// N = P n, for nodes ordered panel by panel (node i of panel p at phi_i).
inline void panel_log_table(const PanelGeom &g, const std::vector<double> &node_xy,
                            std::vector<double> &G) {
  const double pi = 3.14159265358979323846264338327950288;
  const int P = g.P, n = g.n, N = P * n;
  G.assign((size_t)N * N, 0.0);
  double gx[16], gw[16], g8x[8], g8w[8];
  gauss_legendre16(gx, gw);
  gauss_legendre8(g8x, g8w);
  // C[m][j] = ((2 - delta_m0)/n) cos(m phi_j): l_j = sum_m C[m][j] T_m
  std::vector<double> C((size_t)n * n), phin(n);
  for (int j = 0; j < n; ++j) phin[j] = (2.0 * j + 1.0) * pi / (2.0 * n);
  for (int m = 0; m < n; ++m)
    for (int j = 0; j < n; ++j) C[(size_t)m * n + j] = (m ? 2.0 : 1.0) / n * std::cos(m * phin[j]);
  const int nbase = std::max(2, (int)std::ceil(pi * n / 12.0));
  // sampled panel points for nearest-point searches
  const int S = 8 * n;
  std::vector<double> spx((size_t)P * (S + 1)), spy((size_t)P * (S + 1));
  for (int p = 0; p < P; ++p)
    for (int q = 0; q <= S; ++q)
      panel_point(g, p, std::cos(pi * q / S), spx[(size_t)p * (S + 1) + q],
                  spy[(size_t)p * (S + 1) + q]);

  auto rows = [&](int i0, int i1) {
    std::vector<double> mom(n), br, u;
    for (int i = i0; i < i1; ++i) {
      const int pi_ = i / n;
      const double phi_i = phin[i % n], s_i = std::cos(phi_i);
      const double zx = node_xy[2 * i], zy = node_xy[2 * i + 1];
      for (int p = 0; p < P; ++p) {
        br.clear();
        for (int b = 0; b <= nbase; ++b) br.push_back(pi * b / nbase);
        double phs;
        bool grade = true;
        if (p == pi_) {
          phs = phi_i;
        } else {
          int best = 0;
          double bd = 1e300;
          for (int q = 0; q <= S; ++q) {
            const double d = std::hypot(zx - spx[(size_t)p * (S + 1) + q],
                                        zy - spy[(size_t)p * (S + 1) + q]);
            if (d < bd) {
              bd = d;
              best = q;
            }
          }
          auto dist = [&](double ph) {
            double px, py;
            panel_point(g, p, std::cos(ph), px, py);
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
          phs = 0.5 * (lo + hi);
          double d = dist(phs);
          if (dist(0.0) <= d) {
            phs = 0.0;
            d = dist(0.0);
          }
          if (dist(pi) <= d) {
            phs = pi;
            d = dist(pi);
          }
          // panel extent: chord between its ends
          double x0, y0, x1, y1;
          panel_point(g, p, 1.0, x0, y0);
          panel_point(g, p, -1.0, x1, y1);
          grade = d < 2.0 * std::hypot(x1 - x0, y1 - y0);
        }
        if (grade) {
          if (phs > 0.0 && phs < pi) br.push_back(phs);
          for (double h = 0.5 * pi / nbase; h > 1e-12 * pi; h *= 0.5) {
            if (phs - h > 0.0) br.push_back(phs - h);
            if (phs + h < pi) br.push_back(phs + h);
          }
        }
        std::sort(br.begin(), br.end());
        u.clear();
        for (double v : br)
          if (u.empty() || v - u.back() > 1e-15) u.push_back(v);
        std::fill(mom.begin(), mom.end(), 0.0);
        for (size_t e = 0; e + 1 < u.size(); ++e) {
          const double c0 = 0.5 * (u[e] + u[e + 1]), hw = 0.5 * (u[e + 1] - u[e]);
          for (int q = 0; q < 16; ++q) {
            const double ph = c0 + hw * gx[q];
            const double c = std::cos(ph);
            double dx, dy;
            // end of panel p shared with the target's panel (0: none)
            const double ep = (p == pi_ - 1) ? 1.0 : (p == pi_ + 1) ? -1.0 : 0.0;
            if (p == pi_ && std::fabs(c - s_i) < 0.25) {
              panel_diff(g, p, c, s_i, g8x, g8w, dx, dy);
            } else if (ep != 0.0 && std::fabs(c - ep) < 0.25 && std::fabs(s_i + ep) < 0.25) {
              // through the shared break: [y_p(s) - y_p(ep)] + [y_q(-ep) - y_q(s_i)]
              double ax, ay, bx, by;
              panel_diff(g, p, c, ep, g8x, g8w, ax, ay);
              panel_diff(g, pi_, -ep, s_i, g8x, g8w, bx, by);
              dx = ax + bx;
              dy = ay + by;
            } else {
              double px, py;
              panel_point(g, p, c, px, py);
              dx = px - zx;
              dy = py - zy;
            }
            const double r = std::hypot(dx, dy);
            const double f = hw * gw[q] * std::sin(ph) * std::log(std::max(r, 1e-300));
            // moments: T_m(c) by the Chebyshev recurrence
            double t0 = 1.0, t1 = c;
            mom[0] += f;
            if (n > 1) mom[1] += f * c;
            for (int m = 2; m < n; ++m) {
              const double t2 = 2.0 * c * t1 - t0;
              mom[m] += f * t2;
              t0 = t1;
              t1 = t2;
            }
          }
        }
        for (int j = 0; j < n; ++j) {
          double w = 0.0;
          for (int m = 0; m < n; ++m) w += mom[m] * C[(size_t)m * n + j];
          G[(size_t)i + (size_t)(p * n + j) * N] = -w / (2.0 * pi);
        }
      }
    }
  };
  unsigned hc = std::thread::hardware_concurrency();
  int nt = (int)std::min<unsigned>(std::max(1u, hc), 16u);
  nt = std::min(nt, N);
  std::vector<std::thread> th;
  const int per = (N + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int i0 = t * per, i1 = std::min(N, i0 + per);
    if (i0 < i1) th.emplace_back(rows, i0, i1);
  }
  for (auto &t : th) t.join();
}

}  // namespace fthms
