// Nystrom matrix assembly and right-hand sides (FP64 VALU).
//
// Matrix of the first-kind open-arc operator V_Gamma (Section 3.2, eq.
// FDBIEk-interior) in the endpoint-weighted Chebyshev discretisation
// (Section 4.3, eq. singularity):
//
//   A_ij = W_ij L1_ij + (pi/N) L2_ij,   L1 = -J0(kr)/(2pi),
//   L2   = (i/4) H0^(1)(kr) + J0(kr) log|t_i - t_j| / (2pi),
//
// rewritten with the frequency-independent table (the kernel split of
// Section 4.2 that lets one table serve every frequency)
//
//   G_ij = ( -W_ij - (pi/N) log(r_ij / |t_i - t_j|) ) / (2pi),  i != j
//   G_ii = ( -W_ii - (pi/N) log s_i ) / (2pi),
//
// as  A_ij = J0(z)(G_ij - c_k) - (pi/4N) Y0hat(z) + i (pi/4N) J0(z),
//     z = k r_ij,  c_k = (gamma + log(k/2)) / (2N),
// and A_ii = G_ii - c_k + i pi/(4N).  Y0hat = Y0 - (2/pi)(log(z/2)+gamma) J0
// removes the log|t_i - t_j| cancellation near the diagonal exactly.
//
// Composite-panel arcs (Section 4.3, eqs. cov, psi-tilde) replace pi/N by
// the Fejer weight w_j of column j and G by -W/(2pi), W the product-
// integration table of log|y_i - y(s)| on the panels:
//   A_ij = J0(z)(G_ij - w_j c) - (w_j/4) Y0hat(z) + i (w_j/4) J0(z),
//   c = (gamma + log(k/2)) / (2pi);
// A is then no longer symmetric, but J0 and Y0hat of a node pair are.
//
// Large arguments (z >= 4, where the Bessel routines produce Y0 itself):
// since (2/pi)(log(z/2) + gamma) = (2/pi)(log(k/2) + gamma) + (2/pi) log r,
// the same entries are
//   A_ij = J0(z) Gl_ij - hq Y0(z) + i hq J0(z),   Gl_ij = G_ij + log(r_ij)/(2N)
// (hq = pi/(4N); composite panels: Gl_ij = G_ij + w_j log(r_ij)/(2pi) and
// w_j/4 for hq), with the frequency-independent table Gl stored after G:
// no logarithm per entry and frequency.
#pragma once

#include "bessel.h"
#include "common.h"

namespace fthms {

// Upper-triangular 32x32 tiles; each block computes one tile for one
// wavenumber and writes it and its mirror (A is complex symmetric; with
// column weights (WCOL) the mirror reuses the pair's Bessel values with its
// own table entry and weight).  With ylist / Glist (uneven batches) matrix b
// takes its own arc's nodes and table; otherwise every matrix uses y0 / G0.
// G0 / Glist[b]: the arc's tables G and Gl, n x n each, one after the other.
// lower (symmetric matrices only, not WCOL): write the lower block triangle
// only -- every 64 x 64 block on or below the diagonal, the diagonal blocks in
// full -- which is all the symmetric form of the LU and the symmetric
// residual of the refinement read (lu.h); the rest is left untouched.
template <bool W32, bool WCOL>
__global__ __launch_bounds__(256) void assemble_kernel(
    const double2 *__restrict__ y0, const double *__restrict__ G0, int N,
    const double *__restrict__ kvec, double2 *__restrict__ A64,
    float2 *__restrict__ A32, long long mstride, const double2 *const *ylist,
    const double *const *Glist, const double *__restrict__ wcol, int lower = 0) {
  __shared__ double2 tile[32][33];
  __shared__ unsigned char large[32][33];
  const int b = blockIdx.y;
  const double2 *__restrict__ y = ylist ? ylist[b] : y0;
  const double *__restrict__ G = Glist ? Glist[b] : G0;
  const double *__restrict__ Gl = G + (long long)N * N;
  const double k = kvec[b];
  const int t = blockIdx.x;
  int J = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= t) ++J;
  while (J * (J + 1) / 2 > t) --J;
  const int I = t - J * (J + 1) / 2;
  const int i0 = I * 32, j0 = J * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double ck = (kEulerGamma + log(0.5 * k)) / (2.0 * N);
  const double hq = kPi / (4.0 * N);
  double2 *A = A64 + (long long)b * mstride;
  float2 *Af = W32 ? A32 + (long long)b * mstride : nullptr;
  const int i = i0 + tx;
  double2 yi = make_double2(0.0, 0.0);
  if (i < N) yi = y[i];
  if (WCOL) {
    // tile holds (J0, Y) of each pair -- Y0hat with G below z = 4 (and on
    // the diagonal), Y0 with Gl above -- and `large` which one; both writes
    // form their own value
    const double c = (kEulerGamma + log(0.5 * k)) / (2.0 * kPi);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + ty + 8 * q;
      double2 jy = make_double2(1.0, 0.0);
      bool big = false;
      if (i < N && j < N) {
        double z = 0.0;
        if (i != j) {
          const double2 yj = y[j];
          const double dx = yi.x - yj.x, dy = yi.y - yj.y;
          z = k * sqrt(dx * dx + dy * dy);
        }
        big = z >= kBesselSeriesTo;
        const long long e = i + (long long)j * N;
        const double *tab = big ? Gl : G;  // one load from either table
        const double g = tab[e], w = wcol[j];
        if (big) bessel_modphase(z, jy.x, jy.y);
        else if (i != j) bessel_series(z, jy.x, jy.y);
        const double cc = big ? 0.0 : w * c;
        const double2 v = make_double2(jy.x * (g - cc) - 0.25 * w * jy.y, 0.25 * w * jy.x);
        A[e] = v;
        if (W32) Af[e] = make_float2((float)v.x, (float)v.y);
      }
      tile[ty + 8 * q][tx] = jy;
      large[ty + 8 * q][tx] = big;
    }
    if (I != J) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = j0 + tx, col = i0 + ty + 8 * q;
        if (row < N && col < N) {
          const double2 jy = tile[tx][ty + 8 * q];
          const bool big = large[tx][ty + 8 * q];
          const long long e = row + (long long)col * N;
          const double *tab = big ? Gl : G;
          const double g = tab[e], w = wcol[col];
          const double cc = big ? 0.0 : w * c;
          const double2 v = make_double2(jy.x * (g - cc) - 0.25 * w * jy.y, 0.25 * w * jy.x);
          A[e] = v;
          if (W32) Af[e] = make_float2((float)v.x, (float)v.y);
        }
      }
    }
    return;
  }
  // this tile lies above the diagonal (I < J); in the lower form it is
  // written only inside a diagonal 64 x 64 block
  const bool direct = !lower || (I >> 1) == (J >> 1);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = j0 + ty + 8 * q;
    double2 v = make_double2(0.0, 0.0);
    if (i < N && j < N) {
      const long long e = i + (long long)j * N;
      if (i == j) {
        v = make_double2(G[e] - ck, hq);
      } else {
        const double2 yj = y[j];
        const double dx = yi.x - yj.x, dy = yi.y - yj.y;
        const double r = sqrt(dx * dx + dy * dy), z = k * r;
        const bool big = z >= kBesselSeriesTo;
        const double *tab = big ? Gl : G;  // one load from either table
        const double g = tab[e];
        double j0v, yv;
        if (big) {
          // the arithmetic of assemble_mf_kernel at its first wavenumber, so
          // that both kernels give the same entries bit for bit there
          const double ir = 1.0 / r, ik = 1.0 / k;
          double P, Q, sz, cz;
          bessel_pq(z, ik * ir, P, Q);
          phase_sincos(k * r, sz, cz);
          bessel_combine(P, Q, cz, sz, sqrt((2.0 / kPi) * ir) * sqrt(ik), j0v, yv);
        } else {
          bessel_series(z, j0v, yv);
        }
        v = make_double2(j0v * (g - (big ? 0.0 : ck)) - hq * yv, hq * j0v);
      }
      if (direct) {
        A[e] = v;
        if (W32) Af[e] = make_float2((float)v.x, (float)v.y);
      }
    }
    tile[ty + 8 * q][tx] = v;
  }
  if (I != J) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = j0 + tx, col = i0 + ty + 8 * q;
      if (row < N && col < N) {
        const double2 v = tile[tx][ty + 8 * q];
        A[row + (long long)col * N] = v;
        if (W32) Af[row + (long long)col * N] = make_float2((float)v.x, (float)v.y);
      }
    }
  }
}

constexpr int kAsmF = 8;  // wavenumbers per block of assemble_mf_kernel

// assemble_kernel<W32, false> (Chebyshev arcs, one table pair G / Gl) for
// kAsmF consecutive wavenumbers per block: the geometry of a node pair
// (r, 1/r, sqrt(2/(pi r))) and its two table entries are formed once, the
// per-wavenumber constants (c_k, 1/k, sqrt(1/k)) once per block, and for
// z = k r >= 4 the modulus-phase form takes 1/z = (1/k)(1/r) and the
// amplitude sqrt(2/(pi r)) sqrt(1/k): a sine and cosine of z per entry, no
// division or square root.  The Bessel coefficients are read from LDS.
// assemble_kernel evaluates a single wavenumber with the same operations,
// so an entry does not depend on the wavenumbers launched with it.  Grid
// (tiles, ceil(count / kAsmF)).
template <bool W32>
__global__ __launch_bounds__(256) void assemble_mf_kernel(
    const double2 *__restrict__ y, const double *__restrict__ G, int N,
    const double *__restrict__ kvec, int count, double2 *__restrict__ A64,
    float2 *__restrict__ A32, long long mstride, int lower) {
  __shared__ double2 tile[32][33];
  __shared__ double2 btab[kBesselTabLen];
  __shared__ double wk[kAsmF][4];  // per wavenumber: k, c_k, 1/k, sqrt(1/k)
  const double *__restrict__ Gl = G + (long long)N * N;
  const int b0 = blockIdx.y * kAsmF, nf = min(kAsmF, count - b0);
  if (threadIdx.x < kBesselTabLen) bessel_tab_fill(btab, threadIdx.x);
  if (threadIdx.x >= 64 && threadIdx.x < 64 + nf) {
    const int f = threadIdx.x - 64;
    const double k = kvec[b0 + f], ik = 1.0 / k;
    wk[f][0] = k;
    wk[f][1] = (kEulerGamma + log(0.5 * k)) / (2.0 * N);
    wk[f][2] = ik;
    wk[f][3] = sqrt(ik);
  }
  const int t = blockIdx.x;
  int J = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= t) ++J;
  while (J * (J + 1) / 2 > t) --J;
  const int I = t - J * (J + 1) / 2;
  const int i0 = I * 32, j0 = J * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double hq = kPi / (4.0 * N);
  const int i = i0 + tx;
  double2 yi = make_double2(0.0, 0.0);
  if (i < N) yi = y[i];
  // per entry: distance, 1/r, sqrt(2/(pi r)), both table entries
  double r[4], ir[4], amp[4], g[4], gl[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = j0 + ty + 8 * q;
    r[q] = 0.0;
    ir[q] = amp[q] = g[q] = gl[q] = 0.0;
    if (i < N && j < N) {
      const long long e = i + (long long)j * N;
      g[q] = G[e];
      gl[q] = Gl[e];
      if (i != j) {
        const double2 yj = y[j];
        const double dx = yi.x - yj.x, dy = yi.y - yj.y;
        r[q] = sqrt(dx * dx + dy * dy);
        ir[q] = 1.0 / r[q];
        amp[q] = sqrt((2.0 / kPi) * ir[q]);
      }
    }
  }
  // this tile lies above the diagonal (I < J); in the lower form it is
  // written only inside a diagonal 64 x 64 block
  const bool direct = !lower || (I >> 1) == (J >> 1);
  for (int f = 0; f < nf; ++f) {
    const int b = b0 + f;
    double2 *A = A64 + (long long)b * mstride;
    float2 *Af = W32 ? A32 + (long long)b * mstride : nullptr;
    __syncthreads();  // the tables and the previous wavenumber's mirror reads are done
    const double k = wk[f][0], ck = wk[f][1], ik = wk[f][2], sk = wk[f][3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // the table's address is made opaque per entry so that its reads stay
      // with the entry rather than 104 constants held in registers
      int toff = 0;
      asm volatile("" : "+v"(toff));
      const double2 *tab = btab + toff;
      __builtin_amdgcn_sched_barrier(0);
      const int j = j0 + ty + 8 * q;
      double2 v = make_double2(0.0, 0.0);
      if (i < N && j < N) {
        if (i == j) {
          v = make_double2(g[q] - ck, hq);
        } else {
          const double z = k * r[q];
          double j0v, yv;
          if (z >= kBesselSeriesTo) {
            double P, Q, sz, cz;
            bessel_pq_tab(z, ik * ir[q], tab, P, Q);
            phase_sincos(k * r[q], sz, cz);
            bessel_combine(P, Q, cz, sz, amp[q] * sk, j0v, yv);
            v = make_double2(j0v * (gl[q] - 0.0) - hq * yv, hq * j0v);
          } else {
            bessel_series_tab(z, tab, j0v, yv);
            v = make_double2(j0v * (g[q] - ck) - hq * yv, hq * j0v);
          }
        }
        if (direct) {
          const long long e = i + (long long)j * N;
          A[e] = v;
          if (W32) Af[e] = make_float2((float)v.x, (float)v.y);
        }
      }
      tile[ty + 8 * q][tx] = v;
    }
    if (I != J) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = j0 + tx, col = i0 + ty + 8 * q;
        if (row < N && col < N) {
          const double2 v = tile[tx][ty + 8 * q];
          A[row + (long long)col * N] = v;
          if (W32) Af[row + (long long)col * N] = make_float2((float)v.x, (float)v.y);
        }
      }
    }
  }
}

struct IncidentDev {
  int kind;  // 0 plane, 1 gaussian plane, 2 point source
  double dx, dy, z0x, z0y, omega0, sigma, tau0;
};

// g(k) = exp(-(k - w0)^2 / sigma^2) exp(i k tau0)   (Section 5, u1 / u2)
__device__ __forceinline__ double2 gauss_factor(const IncidentDev &in, double k) {
  if (in.sigma <= 0.0) return make_double2(1.0, 0.0);
  const double a = exp(-((k - in.omega0) * (k - in.omega0)) / (in.sigma * in.sigma));
  double s, c;
  sincos(k * in.tau0, &s, &c);
  return make_double2(a * c, a * s);
}

__device__ __forceinline__ double2 incident_at(const IncidentDev &in, double k,
                                               double2 p) {
  if (in.kind == 2) {
    const double dx = p.x - in.z0x, dy = p.y - in.z0y;
    double j0v, y0v;
    bessel_j0_y0(k * sqrt(dx * dx + dy * dy), j0v, y0v);
    // (5i/2)(J0 + i Y0) = -5/2 Y0 + i 5/2 J0
    return cmul(make_double2(-2.5 * y0v, 2.5 * j0v), gauss_factor(in, k));
  }
  double s, c;
  sincos(k * (p.x * in.dx + p.y * in.dy), &s, &c);
  double2 u = make_double2(c, s);
  if (in.kind == 1) u = cmul(u, gauss_factor(in, k));
  return u;
}

// out[b][i] = scale * chi[i] * U^inc(p_i, k_b)   (chi == nullptr: 1)
__global__ __launch_bounds__(256) void incident_kernel(
    IncidentDev in, const double2 *__restrict__ p, const double *__restrict__ chi,
    int n, const double *__restrict__ kvec, double scale, double2 *__restrict__ out,
    long long ostride) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double2 u = incident_at(in, kvec[b], p[i]);
  const double s = chi ? scale * chi[i] : scale;
  out[(long long)b * ostride + i] = make_double2(s * u.x, s * u.y);
}

// Right-hand sides of an uneven batch: out[b][i] = -U^inc_b(y_b[i], k_b).
__global__ __launch_bounds__(256) void batch_rhs_kernel(const IncidentDev *__restrict__ inc,
                                                        const double2 *const *ylist,
                                                        const double *__restrict__ kvec, int n,
                                                        double2 *__restrict__ out,
                                                        long long ostride) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 u = incident_at(inc[b], kvec[b], ylist[b][i]);
  out[(long long)b * ostride + i] = make_double2(-u.x, -u.y);
}

}  // namespace fthms
