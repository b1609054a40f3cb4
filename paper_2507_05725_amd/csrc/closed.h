// Closed curves as single patches (Section 3.3, eqs. FDsolk-closed and
// FDBIEk-closed): the combined-field equation
//     (1/2 I + K - i eta V) Psi = G   on Gamma,   field (D - i eta S) Psi,
// eta = k, by the Nystrom method for 2pi-periodic kernels with a logarithmic
// singularity (the method the paper cites for closed curves).  N = 2n nodes
// tau_j = 2 pi j / N on a counter-clockwise parametrisation; with
// q = x2'(tau_j)(x1(t_i) - x1(tau_j)) - x1'(tau_j)(x2(t_i) - x2(tau_j)) and
// r = |x(t_i) - x(tau_j)|:
//   K  = (ik/4) H1(kr) q/r,       K1 = -(k/4pi) J1(kr) q/r,
//   V  = (i/4) H0(kr) |x'_j|,     V1 = -(1/4pi) J0(kr) |x'_j|,
//   K2 = K - K1 L_ij, V2 = V - V1 L_ij,  L_ij = log(4 sin^2((t_i - tau_j)/2)),
// diagonal K1 = 0, K2 = (x2' x1'' - x1' x2'') / (4 pi |x'|^2),
// V1 = -|x'|/(4pi), V2 = |x'| (i/4 - (log(k |x'|/2) + gamma)/(2pi));
//   A_ij = delta_ij / 2 + R_{i-j} (K1 - i eta V1) + (pi/n)(K2 - i eta V2),
// with the weights of the logarithmic quadrature
//   R_d = -(2pi/n) sum_{m=1}^{n-1} cos(m d pi/n)/m - (pi/n^2) cos(d pi)
// (they depend on (i - j) mod N only: one table of N values per curve, as
// are L_d).  The field is the trapezoid rule for (D - i eta S) Psi, valid
// for targets a few node spacings away; closer targets are refused.
#pragma once

#include "bessel.h"
#include "common.h"

namespace fthms {

// One block per 32x32 tile of the full matrix (not symmetric) and wavenumber.
template <bool W32>
__global__ __launch_bounds__(256) void cfie_assemble_kernel(
    const double2 *__restrict__ y, const double2 *__restrict__ dy,
    const double *__restrict__ Rw, const double *__restrict__ Lw,
    const double *__restrict__ kdiag, int N, const double *__restrict__ kvec,
    double2 *__restrict__ A64, float2 *__restrict__ A32, long long mstride) {
  const int b = blockIdx.z;
  const double k = kvec[b], eta = k;
  const int i = blockIdx.x * 32 + (threadIdx.x & 31);
  const double h = 2.0 * kPi / N;  // pi / n
  double2 *A = A64 + (long long)b * mstride;
  float2 *Af = W32 ? A32 + (long long)b * mstride : nullptr;
  if (i >= N) return;
  const double2 yi = y[i];
#pragma unroll
  for (int q4 = 0; q4 < 4; ++q4) {
    const int j = blockIdx.y * 32 + (threadIdx.x >> 5) + 8 * q4;
    if (j >= N) continue;
    const double2 dj = dy[j];
    const double sp = sqrt(dj.x * dj.x + dj.y * dj.y);
    int d = i - j;
    if (d < 0) d += N;
    double k1, v1, k2r, k2i, v2r, v2i;
    if (i == j) {
      k1 = 0.0;
      v1 = -sp / (4.0 * kPi);
      k2r = kdiag[i];
      k2i = 0.0;
      v2r = -sp * (log(0.5 * k * sp) + kEulerGamma) / (2.0 * kPi);
      v2i = 0.25 * sp;
    } else {
      const double2 yj = y[j];
      const double ex = yi.x - yj.x, ey = yi.y - yj.y;
      const double r = sqrt(ex * ex + ey * ey);
      const double q = dj.y * ex - dj.x * ey;
      double j0, y0, j1, y1;
      bessel_01(k * r, j0, y0, j1, y1);
      const double L = Lw[d];
      const double qr = q / r;
      k1 = -(k / (4.0 * kPi)) * j1 * qr;
      v1 = -(sp / (4.0 * kPi)) * j0;
      // K = (k/4)(-Y1 + i J1) q/r,  V = (|x'|/4)(-Y0 + i J0)
      k2r = -0.25 * k * y1 * qr - k1 * L;
      k2i = 0.25 * k * j1 * qr;
      v2r = -0.25 * sp * y0 - v1 * L;
      v2i = 0.25 * sp * j0;
    }
    const double R = Rw[d];
    // R (K1 - i eta V1) + h (K2 - i eta V2), K1, V1 real
    double ar = R * k1 + h * (k2r + eta * v2i);
    const double ai = -R * eta * v1 + h * (k2i - eta * v2r);
    if (i == j) ar += 0.5;
    const double2 v = make_double2(ar, ai);
    A[i + (long long)j * N] = v;
    if (W32) Af[i + (long long)j * N] = make_float2((float)v.x, (float)v.y);
  }
}

// (D - i eta S)[Psi] at targets by the trapezoid rule: one block per 256
// threads and wavenumber; nodes, tangents and density in LDS.
//   kernel = (k/4)(q/r)(-Y1 + i J1) + (eta |x'_j| / 4)(J0 + i Y0),
//   q = x2'_j (z1 - y1_j) - x1'_j (z2 - y2_j).
// With fewer targets than threads each target's node sum is shared by
// `split` threads (2, 4 or 8; nodes j = s, s + split, ...) whose partial sums
// are added in LDS in a fixed order; split = 1 is one thread per target.
__global__ __launch_bounds__(256) void closed_field_kernel(
    const double2 *__restrict__ ynodes, const double2 *__restrict__ dy, int N,
    const double *__restrict__ kvec, const double2 *__restrict__ psi, long long pstride,
    const double2 *__restrict__ pts, int np, const unsigned char *__restrict__ cls,
    double2 *__restrict__ U, long long ustride, int accumulate, int split) {
  __shared__ double2 sy[1024], sd[1024], sp[1024];
  __shared__ double2 red[256];
  const int b = blockIdx.y;
  for (int j = threadIdx.x; j < N; j += 256) {
    sy[j] = ynodes[j];
    sd[j] = dy[j];
    sp[j] = psi[(long long)b * pstride + j];
  }
  __syncthreads();
  const int tpb = 256 / split;  // targets per block
  const int pl = threadIdx.x % tpb, sl = threadIdx.x / tpb;
  const int p = blockIdx.x * tpb + pl;
  const bool active = p < np && (!cls || cls[p] == 1);
  const double k = kvec[b], eta = k;
  double accr = 0.0, acci = 0.0;
  if (active) {
    const double2 z = pts[p];
    for (int j = sl; j < N; j += split) {
      const double ex = z.x - sy[j].x, ey = z.y - sy[j].y;
      const double r = sqrt(ex * ex + ey * ey);
      const double q = sd[j].y * ex - sd[j].x * ey;
      const double s = sqrt(sd[j].x * sd[j].x + sd[j].y * sd[j].y);
      double j0, y0, j1, y1;
      bessel_01(k * r, j0, y0, j1, y1);
      const double a = 0.25 * k * q / r, c = 0.25 * eta * s;
      const double kr = -a * y1 + c * j0, ki = a * j1 + c * y0;
      const double2 w = sp[j];
      accr += kr * w.x - ki * w.y;
      acci += kr * w.y + ki * w.x;
    }
  }
  if (split > 1) {
    red[threadIdx.x] = make_double2(accr, acci);
    __syncthreads();
    if (sl != 0) return;
    for (int t = 1; t < split; ++t) {
      accr += red[pl + t * tpb].x;
      acci += red[pl + t * tpb].y;
    }
  }
  if (!active) return;
  const double h = 2.0 * kPi / N;
  double2 *u = U + (long long)b * ustride + p;
  if (accumulate) {
    const double2 o = *u;
    *u = make_double2(o.x + h * accr, o.y + h * acci);
  } else {
    *u = make_double2(h * accr, h * acci);
  }
}

// Near targets of a closed patch (closer than five node spacings): the same
// trapezoid rule on a grid kappa times finer, M = kappa N points
// tau_q = 2 pi q / M, with the density's trigonometric interpolant there,
//   psi_f(tau_q) = sum_j psi_j T(tau_q - tau_j),
//   T(t) = (1/N) sin(N t / 2) cot(t / 2), T(0) = 1
// (the interpolant of degree N/2 with the Nyquist term split evenly), and the
// geometry's (exact for curves that are trigonometric polynomials of lower
// degree, spectrally accurate otherwise).  The rule's error decays like
// exp(-2 pi d / h_fine) for a target at distance d from the curve; the host
// picks kappa so that d / h_fine >= 5.2.
//
// psif[b][q] = sum_j psi[b][j] T[(q - kappa j) mod M]: one block per 256 fine
// points and wavenumber, the density in LDS.
__global__ __launch_bounds__(256) void closed_upsample_kernel(const double2 *__restrict__ psi,
                                                              long long pstride, int N, int kappa,
                                                              const double *__restrict__ T,
                                                              double2 *__restrict__ psif) {
  __shared__ double2 sp[1024];
  const int b = blockIdx.y, M = kappa * N;
  for (int j = threadIdx.x; j < N; j += 256) sp[j] = psi[(long long)b * pstride + j];
  __syncthreads();
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= M) return;
  double ar = 0.0, ai = 0.0;
  int d = q;  // (q - kappa j) mod M for j = 0, 1, ...
  for (int j = 0; j < N; ++j) {
    const double t = T[d];
    ar += t * sp[j].x;
    ai += t * sp[j].y;
    d -= kappa;
    if (d < 0) d += M;
  }
  psif[(long long)b * M + q] = make_double2(ar, ai);
}

// U[b][p] (+)= (2 pi / M) sum_q kernel(z_p, yf_q, dyf_q) psif[b][q] for the
// near targets tgt[0 .. ntg) of one level; one block per (target,
// wavenumber), threads over the fine points, partial sums added in a fixed
// order.
__global__ __launch_bounds__(256) void closed_near_kernel(
    const double2 *__restrict__ yf, const double2 *__restrict__ dyf, int M,
    const double *__restrict__ kvec, const double2 *__restrict__ psif, const int *__restrict__ tgt,
    const double2 *__restrict__ pts, double2 *__restrict__ U, long long ustride, int accumulate) {
  __shared__ double2 red[256];
  const int b = blockIdx.y, p = tgt[blockIdx.x];
  const double k = kvec[b], eta = k;
  const double2 z = pts[p];
  double accr = 0.0, acci = 0.0;
  for (int q = threadIdx.x; q < M; q += 256) {
    const double2 y = yf[q], dy = dyf[q];
    const double ex = z.x - y.x, ey = z.y - y.y;
    const double r = sqrt(ex * ex + ey * ey);
    const double qn = dy.y * ex - dy.x * ey;
    const double s = sqrt(dy.x * dy.x + dy.y * dy.y);
    double j0, y0, j1, y1;
    bessel_01(k * r, j0, y0, j1, y1);
    const double a = 0.25 * k * qn / r, c = 0.25 * eta * s;
    const double kr = -a * y1 + c * j0, ki = a * j1 + c * y0;
    const double2 w = psif[(long long)b * M + q];
    accr += kr * w.x - ki * w.y;
    acci += kr * w.y + ki * w.x;
  }
  red[threadIdx.x] = make_double2(accr, acci);
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (threadIdx.x < h) {
      red[threadIdx.x].x += red[threadIdx.x + h].x;
      red[threadIdx.x].y += red[threadIdx.x + h].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double hw = 2.0 * kPi / M;
    double2 *u = U + (long long)b * ustride + p;
    const double2 v = make_double2(hw * red[0].x, hw * red[0].y);
    if (accumulate) *u = make_double2(u->x + v.x, u->y + v.y);
    else *u = v;
  }
}

// Stored cross operators of closed patches (multiple scattering between
// obstacles, each one combined-field patch): for every wavenumber b the
// matrix T[b] (S x S, row-major, S = total node count) with
//   T[b][i][l] = h_l kernel(y_i, y_l),  kernel as in closed_field_kernel,
// for nodes i and l on different patches, and 0 within a patch, so that
// the field of every other patch at the nodes of patch j is
// sum_l T[b][i][l] psi_l -- the trapezoid rule of closed_field_kernel with
// each target's terms stored once and applied at every step.
// pid[S]: patch of each node; hs[S]: its trapezoid weight 2 pi / N.
__global__ __launch_bounds__(256) void closed_cross_build_kernel(
    const double2 *__restrict__ y, const double2 *__restrict__ dy,
    const int *__restrict__ pid, const double *__restrict__ hs, int S,
    const double *__restrict__ kvec, double2 *__restrict__ T) {
  const int b = blockIdx.y;
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)S * S) return;
  const int i = (int)(e / S), l = (int)(e % S);
  double2 v = make_double2(0.0, 0.0);
  if (pid[i] != pid[l]) {
    const double k = kvec[b], eta = k;
    const double2 z = y[i], yl = y[l], d = dy[l];
    const double ex = z.x - yl.x, ey = z.y - yl.y;
    const double r = sqrt(ex * ex + ey * ey);
    const double q = d.y * ex - d.x * ey;
    const double sp = sqrt(d.x * d.x + d.y * d.y);
    double j0, y0, j1, y1;
    bessel_01(k * r, j0, y0, j1, y1);
    const double a = 0.25 * k * q / r, c = 0.25 * eta * sp;
    const double h = hs[l];
    v = make_double2(h * (-a * y1 + c * j0), h * (a * j1 + c * y0));
  }
  T[(long long)b * S * S + e] = v;
}

// out[b][i] = sum_l T[b][i][l] x[b][l] (complex, FP64): one block per 16
// rows of one wavenumber, 16 threads per row striding over the columns
// (coalesced), partial sums reduced with lane shuffles; x in LDS.
constexpr int kCrossMaxS = 4096;  // nodes of all patches (x in LDS: 64 KB)
__global__ __launch_bounds__(256) void cross_apply_kernel(const double2 *__restrict__ T, int S,
                                                         const double2 *__restrict__ x,
                                                         double2 *__restrict__ out) {
  __shared__ double2 sx[kCrossMaxS];
  const int b = blockIdx.y;
  const double2 *xb = x + (long long)b * S;
  for (int l = threadIdx.x; l < S; l += 256) sx[l] = xb[l];
  __syncthreads();
  const int row = blockIdx.x * 16 + (threadIdx.x >> 4), c0 = threadIdx.x & 15;
  double ar = 0.0, ai = 0.0;
  if (row < S) {
    const double2 *Tr = T + ((long long)b * S + row) * S;
    for (int l = c0; l < S; l += 16) {
      const double2 t = Tr[l], v = sx[l];
      ar += t.x * v.x - t.y * v.y;
      ai += t.x * v.y + t.y * v.x;
    }
  }
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) {
    ar += __shfl_xor(ar, off, 16);
    ai += __shfl_xor(ai, off, 16);
  }
  if (row < S && c0 == 0) out[(long long)b * S + row] = make_double2(ar, ai);
}

}  // namespace fthms
