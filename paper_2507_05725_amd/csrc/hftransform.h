// High-frequency Fourier transforms of real time signals (Section 4.1, eqs.
// ft_appr, backwardFT1, int1, int2; the frequency set of Section 5).
//
// A real signal has G(-w) = conj G(w), so the truncated inverse transform
//   g(t) ~ (1/2pi) int_{-W}^{W} G(w) e^{-iwt} dw = (1/pi) Re [I_0^{w_c} + I_{w_c}^{W}]
// with
//   * I_0^{w_c}: graded points mu_j = w_c (j/P)^p (j = 1..P); on every
//     (mu_j, mu_{j+1}) the Clenshaw-Curtis points (n_cc of them, ends
//     shared with the neighbours), the polynomial through the samples
//     integrated against e^{-iwt} exactly (Filon) -- fixed cost for any t and
//     the logarithmic singularity of 2D fields at w = 0 resolved by the
//     grading; (0, mu_1), of length w_c P^{-p}, is left out;
//   * I_{w_c}^{W}: the samples on the uniform grid w_c + l (W - w_c)/L are
//     continued to a trigonometric polynomial of period b = 2 (W - w_c),
//     modes |k| <= L/4, by least squares (QR with column pivoting, columns
//     kept while |R_ii| > 1e-13 |R_00|), and integrated term by term.
// Both are linear in the samples: the host builds a weight matrix
// Wt[n][l], g(t_n) = (1/pi) Re sum_l Wt[n][l] G(w_l), and the device applies
// it (hf_apply_kernel).  The Filon moments int_{-1}^{1} T_k(x) e^{-ikx} dx
// come from Gauss-Legendre quadrature with enough points for the
// oscillation; the Chebyshev coefficients of the interpolant from the
// discrete cosine sums of the Clenshaw-Curtis samples.
#pragma once

#include <complex>

namespace fthms {

typedef std::complex<double> zd;

// The frequency set: Clenshaw-Curtis points of the graded intervals, then
// the uniform grid; sorted, each point once.
struct HfSet {
  double wc = 1.0, W = 20.0, p = 10.0;
  int P = 8, ncc = 11, L = 800;
  std::vector<double> mu;       // mu_1..mu_P
  std::vector<double> omega;    // the set
  std::vector<int> cc_index;    // [(P-1) * ncc]: position of each interval's points
  std::vector<int> uni_index;   // [L + 1]
};

static bool hf_set_build(HfSet &s) {
  if (!(s.wc > 0.0) || !(s.W > s.wc) || s.P < 2 || !(s.p >= 1.0) || s.ncc < 3 || s.ncc > 64 ||
      s.L < 8)
    return false;
  s.mu.resize(s.P);
  for (int j = 1; j <= s.P; ++j) s.mu[j - 1] = s.wc * std::pow((double)j / s.P, s.p);
  s.mu[s.P - 1] = s.wc;
  std::vector<double> pts;
  for (int j = 0; j + 1 < s.P; ++j) {
    const double a = s.mu[j], b = s.mu[j + 1];
    for (int i = 0; i < s.ncc; ++i) {
      // increasing: x_i = -cos(pi i / (ncc - 1))
      const double x = -std::cos(kPi * i / (s.ncc - 1));
      pts.push_back(i == 0 ? a : i == s.ncc - 1 ? b : 0.5 * (a + b) + 0.5 * (b - a) * x);
    }
  }
  for (int l = 0; l <= s.L; ++l)
    pts.push_back(l == 0 ? s.wc : l == s.L ? s.W : s.wc + (s.W - s.wc) * l / s.L);
  std::vector<double> srt = pts;
  std::sort(srt.begin(), srt.end());
  s.omega.clear();
  for (double v : srt)
    if (s.omega.empty() || v - s.omega.back() > 1e-14 * std::max(1.0, s.W)) s.omega.push_back(v);
  auto pos = [&](double v) {
    auto it = std::lower_bound(s.omega.begin(), s.omega.end(), v - 1e-13 * std::max(1.0, s.W));
    return (int)(it - s.omega.begin());
  };
  s.cc_index.resize((size_t)(s.P - 1) * s.ncc);
  for (size_t q = 0; q < s.cc_index.size(); ++q) s.cc_index[q] = pos(pts[q]);
  s.uni_index.resize(s.L + 1);
  for (int l = 0; l <= s.L; ++l) s.uni_index[l] = pos(pts[(size_t)(s.P - 1) * s.ncc + l]);
  return true;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n from the
// Chebyshev-like initial guesses).
static void gauss_legendre_rule(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) p0 = 1.0, p1 = z;
      pp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / pp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

// Filon-Clenshaw-Curtis weights of one interval [a, b] at time t: v[i] for
// the samples at the increasing Clenshaw-Curtis points.
static void hf_filon_weights(double a, double b, int n, double t, zd *v) {
  const double m = 0.5 * (a + b), r = 0.5 * (b - a), kap = r * t;
  // moments mu_k = int_{-1}^{1} T_k(x) e^{-i kap x} dx
  const int nq = (int)(n + 2.0 * std::fabs(kap) + 40.0);
  std::vector<double> gx, gw;
  gauss_legendre_rule(nq, gx, gw);
  std::vector<zd> mom(n, zd(0.0, 0.0));
  for (int q = 0; q < nq; ++q) {
    const zd e = gw[q] * std::exp(zd(0.0, -kap * gx[q]));
    double tkm = 1.0, tk = gx[q];  // T_0, T_1
    mom[0] += e;
    if (n > 1) mom[1] += e * tk;
    for (int k = 2; k < n; ++k) {
      const double tn = 2.0 * gx[q] * tk - tkm;
      tkm = tk;
      tk = tn;
      mom[k] += e * tn;
    }
  }
  // interpolant p(x) = sum_k c_k T_k(x) through f at x_i = -cos(pi i/(n-1))
  // (= cos(pi j/(n-1)) with j = n-1-i): c_k = (2/(n-1)) sum_j'' f cos(pi k j/(n-1)),
  // first and last k halved; the weight of sample i is sum_k mu_k dc_k/df_i
  const int N1 = n - 1;
  const zd ph = r * std::exp(zd(0.0, -m * t));
  for (int i = 0; i < n; ++i) {
    const int j = N1 - i;
    const double hj = (j == 0 || j == N1) ? 0.5 : 1.0;
    zd acc(0.0, 0.0);
    for (int k = 0; k < n; ++k) {
      const double hk = (k == 0 || k == N1) ? 0.5 : 1.0;
      acc += mom[k] * (hk * hj * (2.0 / N1) * std::cos(kPi * (double)((long long)k * j % (2 * N1)) / N1));
    }
    v[i] = ph * acc;
  }
}

// Least-squares Fourier continuation of the L+1 uniform samples on [0, D]:
// A[l][k] = exp(2 pi i k s_l / b), b = 2D, |k| <= K = L/4, factored
// A P = Q R by Householder QR with column pivoting (columns with
// |R_ii| > rtol |R_00| kept); weights of the samples for the integral over
// [w0, w0 + D] against e^{-iwt}: u = conj(Q_r) y with R_r^T y = P^T e(t).
struct HfFc {
  int m = 0, n = 0, r = 0;
  double D = 0.0, b = 0.0, w0 = 0.0;
  int K = 0;
  std::vector<zd> A;        // column-major m x n: R above the diagonal, v below
  std::vector<zd> beta;     // Householder scalars
  std::vector<zd> rdiag;    // R_ii
  std::vector<int> perm;    // column j of A P = column perm[j] of A
};

static void hf_fc_factor(HfFc &f, int L, double D, double w0, double rtol = 1e-13) {
  f.m = L + 1;
  f.K = L / 4;
  f.n = 2 * f.K + 1;
  f.D = D;
  f.b = 2.0 * D;
  f.w0 = w0;
  const int m = f.m, n = f.n;
  f.A.assign((size_t)m * n, zd(0.0, 0.0));
  for (int c = 0; c < n; ++c)
    for (int l = 0; l < m; ++l) {
      const double s = D * l / L;
      f.A[(size_t)c * m + l] = std::exp(zd(0.0, 2.0 * kPi * (c - f.K) * s / f.b));
    }
  f.perm.resize(n);
  for (int c = 0; c < n; ++c) f.perm[c] = c;
  f.beta.assign(n, zd(0.0, 0.0));
  f.rdiag.assign(n, zd(0.0, 0.0));
  const int steps = std::min(m, n);
  for (int j = 0; j < steps; ++j) {
    // pivot: the remaining column of largest norm (rows j..m-1)
    int best = j;
    double bn = -1.0;
    for (int c = j; c < n; ++c) {
      double s2 = 0.0;
      for (int l = j; l < m; ++l) s2 += std::norm(f.A[(size_t)c * m + l]);
      if (s2 > bn) {
        bn = s2;
        best = c;
      }
    }
    if (best != j) {
      for (int l = 0; l < m; ++l) std::swap(f.A[(size_t)j * m + l], f.A[(size_t)best * m + l]);
      std::swap(f.perm[j], f.perm[best]);
    }
    // Householder vector of column j below the diagonal
    zd *x = &f.A[(size_t)j * m];
    const double xn = std::sqrt(bn);
    const zd x0 = x[j];
    const zd alpha = -(std::abs(x0) > 0.0 ? x0 / std::abs(x0) : zd(1.0, 0.0)) * xn;
    x[j] = x0 - alpha;  // v = x - alpha e_j (v_j stored here, the rest in place)
    double vn2 = 0.0;
    for (int l = j; l < m; ++l) vn2 += std::norm(x[l]);
    const zd bt = vn2 > 0.0 ? zd(2.0 / vn2, 0.0) : zd(0.0, 0.0);
    f.beta[j] = bt;
    f.rdiag[j] = alpha;
    // apply H = I - beta v v^H to the later columns
    for (int c = j + 1; c < n; ++c) {
      zd *y = &f.A[(size_t)c * m];
      zd s(0.0, 0.0);
      for (int l = j; l < m; ++l) s += std::conj(x[l]) * y[l];
      s *= bt;
      for (int l = j; l < m; ++l) y[l] -= s * x[l];
    }
  }
  f.r = 0;
  const double r00 = std::abs(f.rdiag[0]);
  while (f.r < steps && std::abs(f.rdiag[f.r]) > rtol * r00) ++f.r;
}

// u[l], l <= L: weights of the uniform samples at time t
static void hf_fc_weights(const HfFc &f, double t, zd *u) {
  const int m = f.m, r = f.r;
  std::vector<zd> e(f.n), y(r), z(m, zd(0.0, 0.0));
  const zd ph = std::exp(zd(0.0, -f.w0 * t));
  for (int c = 0; c < f.n; ++c) {
    const double kap = 2.0 * kPi * (c - f.K) / f.b - t;
    zd v;
    if (std::fabs(kap * f.D) < 1e-8) v = zd(f.D, 0.5 * kap * f.D * f.D);
    else v = (std::exp(zd(0.0, kap * f.D)) - 1.0) / zd(0.0, kap);
    e[c] = ph * v;
  }
  // R_r^T y = (P^T e)_r  (forward substitution; R_ij above the diagonal
  // stored in A, R_ii in rdiag)
  for (int i = 0; i < r; ++i) {
    zd acc = e[f.perm[i]];
    for (int j = 0; j < i; ++j) acc -= f.A[(size_t)i * m + j] * y[j];
    y[i] = acc / f.rdiag[i];
  }
  // z = Q [conj(y); 0] = H_0 H_1 ... H_{r-1} [conj(y); 0]; u = conj(z)
  for (int i = 0; i < r; ++i) z[i] = std::conj(y[i]);
  for (int j = r - 1; j >= 0; --j) {
    const zd *v = &f.A[(size_t)j * m];
    zd s(0.0, 0.0);
    // v_j is stored in A[j][j]; rows below hold the rest of v
    for (int l = j; l < m; ++l) s += std::conj(v[l]) * z[l];
    s *= f.beta[j];
    for (int l = j; l < m; ++l) z[l] -= s * v[l];
  }
  for (int l = 0; l < m; ++l) u[l] = std::conj(z[l]);
}

// Wt[row][l] (row-major, ld = omega.size()) for the times t[row].
static void hf_weight_rows(const HfSet &s, const HfFc &fc, const double *t, int nt, zd *Wt) {
  const size_t J = s.omega.size();
  std::vector<zd> v(s.ncc), u(s.L + 1);
  for (int row = 0; row < nt; ++row) {
    zd *w = Wt + (size_t)row * J;
    for (size_t l = 0; l < J; ++l) w[l] = zd(0.0, 0.0);
    for (int j = 0; j + 1 < s.P; ++j) {
      hf_filon_weights(s.mu[j], s.mu[j + 1], s.ncc, t[row], v.data());
      for (int i = 0; i < s.ncc; ++i) w[s.cc_index[(size_t)j * s.ncc + i]] += v[i];
    }
    hf_fc_weights(fc, t[row], u.data());
    for (int l = 0; l <= s.L; ++l) w[s.uni_index[l]] += u[l];
  }
}

// out[t][p] (+)= (1/pi) Re sum_l W[t][l] U[l][p]  (written as complex with a
// zero imaginary part).  64 x 64 output tiles per block, 16 frequencies of
// W and U staged in LDS per step; each thread owns 4 x 4 outputs.
// REAL: out is double [nt][np] instead.
template <bool REAL>
__global__ __launch_bounds__(256) void hf_apply_kernel(const double2 *__restrict__ W, int nt,
                                                      int nk, const double2 *__restrict__ U,
                                                      int np, void *__restrict__ outp,
                                                      int accumulate) {
  __shared__ double2 sw[64][17];
  __shared__ double2 su[16][65];
  const int t0 = blockIdx.y * 64, p0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  for (int l0 = 0; l0 < nk; l0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int tt = e / 16, ll = e % 16;
      const int t = t0 + tt, l = l0 + ll;
      sw[tt][ll] = (t < nt && l < nk) ? W[(long long)t * nk + l] : make_double2(0.0, 0.0);
      const int ul = e / 64, up = e % 64;
      const int l2 = l0 + ul, p = p0 + up;
      su[ul][up] = (l2 < nk && p < np) ? U[(long long)l2 * np + p] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int ll = 0; ll < 16; ++ll) {
      double2 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sw[ty + 16 * i][ll];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = su[ll][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i].x * b[j].x - a[i].y * b[j].y;
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = t0 + ty + 16 * i, p = p0 + tx + 16 * j;
      if (t < nt && p < np) {
        const double v = acc[i][j] / kPi;
        if (REAL) {
          double *o = (double *)outp + (long long)t * np + p;
          *o = accumulate ? *o + v : v;
        } else {
          double2 *o = (double2 *)outp + (long long)t * np + p;
          *o = accumulate ? make_double2(o->x + v, 0.0) : make_double2(v, 0.0);
        }
      }
    }
}

}  // namespace fthms
