// Single-layer potential of a solved density and the frequency-to-time
// transform (FP64).
//
// Far targets (Section 3.2, eq. FDsolk-interior; Gauss-Chebyshev rule of the
// weighted density):  U(z) = (pi/N) sum_j Phi_k(z, y_j) alpha_j
//                          = (pi/4N) sum_j (i J0 - Y0)(k|z - y_j|) alpha_j;
// composite-panel arcs (Section 4.3) use their Fejer weights w_j in place of
// pi/N and integrate each panel's interpolant in s near the arc.
// Near targets: U(z) = sum_q w_q Phi_k(z, x_q) alpha_N(cos phi_q), the exact
// potential of the density interpolant alpha_N = sum_m a_m T_m, by a
// composite Gauss-Legendre rule in phi (t = cos phi) graded toward the point
// of the arc nearest the target; the rule and the geometry x_q are planned
// on the host once per target set (frequency independent).
//
// Time traces (eq. backwardFT, eq. TDsol-interior with one window):
//   u(x_p, t_n) = (1/2pi) sum_l w_l U(x_p, w_l) exp(-i w_l t_n).
#pragma once

#include "bessel.h"
#include "common.h"

namespace fthms {

constexpr int kFieldThreads = 256;

constexpr int kFieldF = 4;  // wavenumbers per block of field_far_mf_kernel

// Nodes per LDS chunk of field_far_mf_kernel (a multiple of every split).
constexpr int kFieldChunk = 256;

// Bytes of the dynamic LDS of field_far_mf_kernel: one chunk of nodes and
// their kFieldF weighted densities.
inline size_t field_mf_lds_bytes(int N) {
  return sizeof(double2) * (size_t)(1 + kFieldF) * (size_t)(N < kFieldChunk ? N : kFieldChunk);
}

// Far targets: up to 256 targets for kFieldF consecutive wavenumbers per
// block, nodes and weighted densities in LDS, kFieldChunk nodes at a time
// (about 26 KB of LDS per block: four blocks per CU, four waves per SIMD).  Composite-panel arcs pass
// their Fejer weights: U(z) = sum_j w_j Phi_k(z, y_j) mu_j; otherwise the
// weight is pi/N.  With up to 256 targets (split = 2, 4 or 8) each
// target's node sum is shared by `split` threads (nodes j = s, s + split,
// ...), whose partial sums are added in LDS in a fixed order; split = 1 is
// one thread per target.  A node's distance r to the target, 1/r and
// sqrt(2/(pi r)) are formed once for the block's wavenumbers; z = k r >= 4
// takes 1/z = (1/k)(1/r) and the amplitude sqrt(2/(pi r)) sqrt(1/k) (no
// division or square root per pair and wavenumber), and the Bessel
// coefficients are read from LDS.  A wavenumber's result does not depend on
// the others launched with it.
// Grid (target blocks, ceil(nk / kFieldF)); dynamic LDS field_mf_lds_bytes.
__global__ __launch_bounds__(kFieldThreads) __attribute__((amdgpu_waves_per_eu(4))) void field_far_mf_kernel(
    const double2 *__restrict__ ynodes, int N, const double *__restrict__ wnode,
    const double *__restrict__ kvec, int nk, const double2 *__restrict__ alpha,
    long long astride, const double2 *__restrict__ pts, int np,
    const unsigned char *__restrict__ cls, double2 *__restrict__ U, long long ustride,
    int accumulate, int split) {
  extern __shared__ double2 fdyn[];
  const int C = min(N, kFieldChunk);
  double2 *sy = fdyn, *sa = fdyn + C;  // sa[f C + j]: weighted density f at chunk node j
  __shared__ double2 red[kFieldThreads];
  __shared__ double2 btab[kBesselTabLen];
  __shared__ double wk[kFieldF][3];  // k, 1/k, sqrt(1/k)
  const int b0 = blockIdx.y * kFieldF, nf = min(kFieldF, nk - b0);
  if (threadIdx.x < kBesselTabLen) bessel_tab_fill(btab, threadIdx.x);
  if (threadIdx.x >= 64 && threadIdx.x < 64 + nf) {
    const int f = threadIdx.x - 64;
    const double k = kvec[b0 + f], ik = 1.0 / k;
    wk[f][0] = k;
    wk[f][1] = ik;
    wk[f][2] = sqrt(ik);
  }
  const int tpb = kFieldThreads / split;  // targets per block
  const int pl = threadIdx.x % tpb, sl = threadIdx.x / tpb;
  const int p = blockIdx.x * tpb + pl;
  const bool active = p < np && (!cls || cls[p] == 1);
  double ar[kFieldF], ai[kFieldF];
#pragma unroll
  for (int f = 0; f < kFieldF; ++f) ar[f] = ai[f] = 0.0;
  const double2 zt = active ? pts[p] : make_double2(0.0, 0.0);
  // the chunks in order, and in each a thread's nodes j0 + sl, j0 + sl +
  // split, ... (chunks are a multiple of split): every node in the order of
  // one pass over all of them
  for (int j0 = 0; j0 < N; j0 += C) {
    const int nc = min(C, N - j0);
    __syncthreads();  // the previous chunk is no longer read
    for (int j = threadIdx.x; j < nc; j += kFieldThreads) {
      sy[j] = ynodes[j0 + j];
      const double wj = wnode ? wnode[j0 + j] : 1.0;
#pragma unroll
      for (int f = 0; f < kFieldF; ++f) {
        double2 a = make_double2(0.0, 0.0);
        if (f < nf) a = alpha[(long long)(b0 + f) * astride + j0 + j];
        if (wnode) a = make_double2(wj * a.x, wj * a.y);
        sa[f * C + j] = a;
      }
    }
    __syncthreads();
    if (active) {
      for (int j = sl; j < nc; j += split) {
        const double2 yj = sy[j];
        const double dx = zt.x - yj.x, dy = zt.y - yj.y;
        const double r = sqrt(dx * dx + dy * dy), ir = 1.0 / r;
        const double amp = sqrt((2.0 / kPi) * ir);
        // the table's address is opaque per node so that its reads stay in
        // the loop rather than 104 constants held in registers
        int toff = 0;
        asm volatile("" : "+v"(toff));
        const double2 *tab = btab + toff;
#pragma unroll
        for (int f = 0; f < kFieldF; ++f) {
          if (f < nf) {
            const double k = wk[f][0], z = k * r;
            double j0v, y0v;
            if (z >= kBesselSeriesTo) {
              double P, Q, sz, cz;
              bessel_pq_tab(z, wk[f][1] * ir, tab, P, Q);
              phase_sincos(z, sz, cz);
              bessel_combine(P, Q, cz, sz, amp * wk[f][2], j0v, y0v);
            } else {
              double yh;
              bessel_series_tab(z, tab, j0v, yh);
              y0v = yh + bessel_logpart(z) * j0v;
            }
            // (i J0 - Y0) * a
            const double2 a = sa[f * C + j];
            ar[f] += -y0v * a.x - j0v * a.y;
            ai[f] += j0v * a.x - y0v * a.y;
          }
        }
      }
    }
  }
  if (split > 1) {
#pragma unroll
    for (int f = 0; f < kFieldF; ++f) {
      red[threadIdx.x] = make_double2(ar[f], ai[f]);
      __syncthreads();
      if (sl == 0) {
        for (int q = 1; q < split; ++q) {
          ar[f] += red[pl + q * tpb].x;
          ai[f] += red[pl + q * tpb].y;
        }
      }
      __syncthreads();
    }
    if (sl != 0) return;
  }
  if (!active) return;
  const double s = wnode ? 0.25 : kPi / (4.0 * N);
#pragma unroll
  for (int f = 0; f < kFieldF; ++f) {
    if (f < nf) {
      double2 *u = U + (long long)(b0 + f) * ustride + p;
      if (accumulate) {
        const double2 o = *u;
        *u = make_double2(o.x + s * ar[f], o.y + s * ai[f]);
      } else {
        *u = make_double2(s * ar[f], s * ai[f]);
      }
    }
  }
}

// Threads per target for field_far_mf_kernel and closed_field_kernel: the
// smallest power of two (at most 8) that gives at least four blocks' worth
// of threads, np x split >= 1024: 8 below 256 targets, 4 below 512, 2 below
// 1024, 1 from 1024 up.  At the headline's 256
// targets one thread per target left four waves per SIMD in all, too few to
// cover the latency of the Bessel evaluations' dependent chains (2.75 ms per
// step; 2.17 with two threads, 1.98 with four).  A function of the target
// count only, so a field does not depend on what else is launched.
inline int field_target_split(int np) {
  int split = 1;
  while (split < 8 && np * split < 4 * kFieldThreads) split *= 2;
  return split;
}

// Chebyshev coefficients of the density interpolant for each wavenumber,
// per panel of n = nper nodes (one panel: nper = N):
//   a_{p,m} = ((2 - delta_m0) / n) sum_j cos(m theta_j) alpha_{p n + j},
// cosT[j][m] = cos(m theta_j).  One block per wavenumber, threads over
// (p, m).
__global__ __launch_bounds__(kFieldThreads) void cheb_coeff_kernel(
    const double *__restrict__ cosT, int N, int nper, const double2 *__restrict__ alpha,
    long long astride, double2 *__restrict__ coef) {
  __shared__ double2 sa[1024];
  const int b = blockIdx.x;
  for (int j = threadIdx.x; j < N; j += kFieldThreads) sa[j] = alpha[(long long)b * astride + j];
  __syncthreads();
  for (int e = threadIdx.x; e < N; e += kFieldThreads) {
    const int p = e / nper, m = e - p * nper;
    const double2 *a = sa + p * nper;
    double ar = 0.0, ai = 0.0;
    for (int j = 0; j < nper; ++j) {
      const double c = cosT[(long long)j * nper + m];
      ar += c * a[j].x;
      ai += c * a[j].y;
    }
    const double f = (m == 0 ? 1.0 : 2.0) / nper;
    coef[(long long)b * N + e] = make_double2(f * ar, f * ai);
  }
}

// Clenshaw helpers of field_near_kernel: read a[m], ..., a[m-7] (m >= 7) and
// take the eight recurrence steps that use them.
__device__ __forceinline__ void clenshaw_read8(const double2 *a, int m, double2 *c) {
#pragma unroll
  for (int u = 0; u < 8; ++u) c[u] = a[m - u];
}

__device__ __forceinline__ void clenshaw_steps8(const double2 *c, double c2, double &b1r,
                                                double &b1i, double &b2r, double &b2i) {
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const double nr = fma(c2, b1r, c[u].x - b2r);
    const double ni = fma(c2, b1i, c[u].y - b2i);
    b2r = b1r;
    b2i = b1i;
    b1r = nr;
    b1i = ni;
  }
}

// Near targets: one block per (target, wavenumber).
//   U(z) = sum_q w_q (i/4) H0(k |z - x_q|) alpha_N(c_q),
//   alpha_N(c) = sum_m a_m T_m(c) by Clenshaw's recurrence, c_q = cos(phi_q),
// with the coefficients of point q's panel (pq[q]; none: one panel).
__global__ __launch_bounds__(kFieldThreads) void field_near_kernel(
    const int *__restrict__ tgt_index, const int *__restrict__ qoff,
    const double2 *__restrict__ xq, const double *__restrict__ wq,
    const double *__restrict__ cq, const int *__restrict__ pq, int N, int nper,
    const double2 *__restrict__ coef, const double *__restrict__ kvec,
    const double2 *__restrict__ pts, double2 *__restrict__ U, long long ustride,
    int accumulate) {
  __shared__ double2 sa[1024];
  __shared__ double red[2][kFieldThreads / 64];
  const int t = blockIdx.x, b = blockIdx.y;
  for (int j = threadIdx.x; j < N; j += kFieldThreads) sa[j] = coef[(long long)b * N + j];
  __syncthreads();
  const int p = tgt_index[t];
  const double2 z = pts[p];
  const double k = kvec[b];
  const int q0 = qoff[t], q1 = qoff[t + 1];
  double accr = 0.0, acci = 0.0;
  // the next quadrature point's data is read one point ahead (index clamped
  // to the target's last point; every near target has at least one point), so
  // its global loads overlap this point's sums
  const int qlast = q1 - 1;
  int qn = min(q0 + (int)threadIdx.x, qlast);
  double cn = cq[qn], wn = wq[qn];
  double2 xn = xq[qn];
  int pn = pq ? pq[qn] : 0;
  for (int q = q0 + threadIdx.x; q < q1; q += kFieldThreads) {
    const double c = cn, c2 = 2.0 * c, wcur = wn;
    const double2 x = xn;
    const double2 *a = sa + pn * nper;
    qn = min(q + kFieldThreads, qlast);
    cn = cq[qn];
    wn = wq[qn];
    xn = xq[qn];
    if (pq) pn = pq[qn];
    // Clenshaw: b_m = a_m + 2c b_{m+1} - b_{m+2}, written fma(2c, b_{m+1},
    // a_m - b_{m+2}) so one operation per step waits on b_{m+1}; the
    // coefficients are read from LDS eight at a time into two alternating
    // buffers, the next eight issued before the steps of the current ones.
    double b1r = 0.0, b1i = 0.0, b2r = 0.0, b2i = 0.0;
    int m = nper - 1;
    if (m >= 8) {
      double2 ca[8], cb[8];
      clenshaw_read8(a, m, ca);
      for (;;) {
        clenshaw_read8(a, max(m - 8, 7), cb);
        __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the steps
        clenshaw_steps8(ca, c2, b1r, b1i, b2r, b2i);
        m -= 8;
        if (m < 8) break;
        clenshaw_read8(a, max(m - 8, 7), ca);
        __builtin_amdgcn_sched_barrier(0);
        clenshaw_steps8(cb, c2, b1r, b1i, b2r, b2i);
        m -= 8;
        if (m < 8) break;
      }
    }
    for (; m >= 1; --m) {
      const double nr = fma(c2, b1r, a[m].x - b2r);
      const double ni = fma(c2, b1i, a[m].y - b2i);
      b2r = b1r;
      b2i = b1i;
      b1r = nr;
      b1i = ni;
    }
    const double dr = a[0].x + c * b1r - b2r;
    const double di = a[0].y + c * b1i - b2i;
    const double dx = z.x - x.x, dy = z.y - x.y;
    double j0v, y0v;
    bessel_j0_y0(k * sqrt(dx * dx + dy * dy), j0v, y0v);
    const double w = 0.25 * wcur;
    // (i/4)(J0 + i Y0) * d = w (-Y0 + i J0) * d
    accr += w * (-y0v * dr - j0v * di);
    acci += w * (j0v * dr - y0v * di);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    accr += __shfl_xor(accr, off);
    acci += __shfl_xor(acci, off);
  }
  if (lane == 0) {
    red[0][wave] = accr;
    red[1][wave] = acci;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sr = 0.0, si = 0.0;
    for (int w = 0; w < kFieldThreads / 64; ++w) {
      sr += red[0][w];
      si += red[1][w];
    }
    double2 *u = U + (long long)b * ustride + p;
    if (accumulate) {
      const double2 o = *u;
      *u = make_double2(o.x + sr, o.y + si);
    } else {
      *u = make_double2(sr, si);
    }
  }
}

// u[n][p] = (1/2pi) sum_l w_l U[l][p] e^{-i om_l t_n}; 64 x 64 output tile per
// block, 16 frequencies staged per step.
constexpr int kFtTile = 64;
constexpr int kFtChunk = 16;

// Frequencies [z lsplit, (z + 1) lsplit) for blockIdx.z = z: with part ==
// nullptr (one split) the block writes u directly, otherwise its unscaled
// partial sum to part[z][n][p], summed by freq_to_time_sum_kernel (a fixed
// order, so the result does not depend on scheduling).
__global__ __launch_bounds__(256) void freq_to_time_kernel(
    int nk, const double *__restrict__ om, const double *__restrict__ w, int np,
    const double2 *__restrict__ U, int nt, const double *__restrict__ t,
    double2 *__restrict__ u, int lsplit, double2 *__restrict__ part) {
  __shared__ double2 sE[kFtTile][kFtChunk + 1];
  __shared__ double2 sU[kFtChunk][kFtTile];
  const int n0 = blockIdx.y * kFtTile, p0 = blockIdx.x * kFtTile;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;  // 16 x 16 threads
  double2 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = make_double2(0.0, 0.0);
  const int lb = blockIdx.z * lsplit, le = min(nk, lb + lsplit);
  for (int l0 = lb; l0 < le; l0 += kFtChunk) {
    for (int e = threadIdx.x; e < kFtTile * kFtChunk; e += 256) {
      const int nn = e / kFtChunk, ll = e % kFtChunk;
      double2 v = make_double2(0.0, 0.0);
      if (n0 + nn < nt && l0 + ll < le) {
        double s, c;
        sincos(om[l0 + ll] * t[n0 + nn], &s, &c);
        const double ww = w[l0 + ll];
        v = make_double2(ww * c, -ww * s);
      }
      sE[nn][ll] = v;
    }
    for (int e = threadIdx.x; e < kFtTile * kFtChunk; e += 256) {
      const int ll = e / kFtTile, pp = e % kFtTile;
      sU[ll][pp] = (l0 + ll < le && p0 + pp < np) ? U[(long long)(l0 + ll) * np + p0 + pp]
                                                  : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int ll = 0; ll < kFtChunk; ++ll) {
      double2 e[4], v[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) e[a] = sE[ty + 16 * a][ll];
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = sU[ll][tx + 16 * c];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = cfma(acc[a][c], e[a], v[c]);
    }
    __syncthreads();
  }
  const double s = 1.0 / (2.0 * kPi);
  double2 *pz = part ? part + (long long)blockIdx.z * nt * np : nullptr;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int n = n0 + ty + 16 * a, p = p0 + tx + 16 * c;
      if (n < nt && p < np) {
        if (pz)
          pz[(long long)n * np + p] = acc[a][c];
        else
          u[(long long)n * np + p] = make_double2(s * acc[a][c].x, s * acc[a][c].y);
      }
    }
}

// u[i] = (1/2pi) sum_z part[z][i], z in order.
__global__ __launch_bounds__(256) void freq_to_time_sum_kernel(int nsplit, long long nn,
                                                               const double2 *__restrict__ part,
                                                               double2 *__restrict__ u) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= nn) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int z = 0; z < nsplit; ++z) {
    const double2 v = part[(long long)z * nn + i];
    acc.x += v.x;
    acc.y += v.y;
  }
  const double s = 1.0 / (2.0 * kPi);
  u[i] = make_double2(s * acc.x, s * acc.y);
}

// Device copy of a near-target quadrature plan (built on the host by
// plan_near): per point class, near target list, quadrature offsets, points,
// weights and cos(phi) values.
constexpr int kClosedLevels = 7;  // upsampling factors 2, 4, ..., 128

struct NearPlan {
  int np = 0, ntgt = 0, nq = 0;
  unsigned char *d_cls = nullptr;
  int *d_tgt = nullptr;
  int *d_qoff = nullptr;
  double2 *d_xq = nullptr;
  double *d_wq = nullptr;
  double *d_cq = nullptr;
  int *d_pq = nullptr;  // panel of each point (composite-panel arcs)
  // closed patches: near targets by the trapezoid rule on an upsampled grid,
  // one level per factor kappa = 2^(l+1) in use; the level's targets are
  // d_tgt[lev_first[l] .. lev_first[l + 1]); its fine geometry (kappa n
  // points) and periodic interpolation kernel (kappa n values)
  int np_nodes = 0;
  int lev_kappa[kClosedLevels] = {}, lev_first[kClosedLevels + 1] = {};
  double2 *d_yf[kClosedLevels] = {}, *d_dyf[kClosedLevels] = {};
  double *d_Tf[kClosedLevels] = {};
};

}  // namespace fthms
