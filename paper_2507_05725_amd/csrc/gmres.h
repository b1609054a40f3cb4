// Batched GMRES for the dense per-(arc, frequency) systems (FP64).
//
// The paper solves its frequency-domain integral equations with GMRES or
// direct solvers and uses GMRES iteration counts to show what splitting a
// trapping boundary into non-trapping patches buys (Section 5,
// Geometries 5).  Here: x0 = 0, Arnoldi with modified Gram-Schmidt, the
// Hessenberg least-squares problem kept triangular by complex Givens
// rotations (c real, s = (a/|a|) conj(b) / sqrt(|a|^2 + |b|^2)), stop at the
// first iteration with |residual estimate| <= tol |b| or at maxit; no
// restarts.
//
// One 256-thread workgroup per system.  The matrix is read once per
// iteration, column by column with consecutive threads on consecutive rows
// (coalesced; HBM-bound: 16 N^2 bytes per iteration); the Krylov basis
// lives in a global workspace [maxit + 1][N] per system, the current vector
// and the reductions in LDS; thread i owns rows i, i + 256, ...
#pragma once

#include "common.h"

namespace fthms {

constexpr int kGmresThreads = 256;
constexpr int kGmresMaxIt = 256;
constexpr int kGmresRows = 1024 / kGmresThreads;  // rows per thread at N <= 1024

__device__ __forceinline__ double2 gm_block_sum(double2 v, double2 *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    v.x += __shfl_xor(v.x, off);
    v.y += __shfl_xor(v.y, off);
  }
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int w = 0; w < kGmresThreads / 64; ++w) {
    s.x += red[w].x;
    s.y += red[w].y;
  }
  return s;
}

// work: per system (maxit + 1) N double2 for the basis, then maxit (maxit + 1)
// double2 for the triangular factor (column j holds R[0..j][j]).
//
// PREC: GMRES-IR -- right preconditioning by low-precision LU factors
// (LUbase / permbase, FP32 storage, as lu.h writes them): GMRES on
// A M^{-1} u = b with M = L U, x = M^{-1} u; every iteration applies the
// factors' triangular solves (FP64 accumulation) to the basis vector before
// the FP64 product with A, and the residual estimate is that of the original
// system.  status[sys] < 0 on entry (factors not usable) leaves the system
// alone; on exit it holds the iterations taken, or -1 when tol was not
// reached (the caller then solves that system in FP64).
template <bool PREC>
__global__ __launch_bounds__(kGmresThreads) void gmres_kernel(
    const double2 *__restrict__ Abase, long long mstride, int N, const double2 *__restrict__ bbase,
    long long bstride, double2 *__restrict__ xbase, long long xstride, int maxit, double tol,
    double2 *__restrict__ work, long long wstride, int *__restrict__ iters,
    double *__restrict__ relres, const float2 *__restrict__ LUbase = nullptr,
    const int *__restrict__ permbase = nullptr, int *__restrict__ status = nullptr) {
  __shared__ double2 sv[1024];
  __shared__ double2 red[kGmresThreads / 64];
  __shared__ double2 col[kGmresMaxIt + 1];
  __shared__ double2 g[kGmresMaxIt + 1];
  __shared__ double2 sn[kGmresMaxIt];
  __shared__ double cs[kGmresMaxIt];
  __shared__ int done;
  const int sys = blockIdx.x, tid = threadIdx.x;
  if (PREC && status[sys] < 0) return;
  const double2 *A = Abase + (long long)sys * mstride;
  const double2 *b = bbase + (long long)sys * bstride;
  double2 *x = xbase + (long long)sys * xstride;
  double2 *V = work + (long long)sys * wstride;
  double2 *R = V + (long long)(maxit + 1) * N;
  // this thread's rows tid + 256 q, clamped into the matrix
  int rowc[kGmresRows];
  double rmask[kGmresRows];  // 1 for a row of the matrix, 0 for a clamped one
#pragma unroll
  for (int q = 0; q < kGmresRows; ++q) {
    rowc[q] = min(tid + q * kGmresThreads, N - 1);
    rmask[q] = tid + q * kGmresThreads < N ? 1.0 : 0.0;
  }
  // v_0 = b / |b|
  double2 w[kGmresRows];
  double2 p = make_double2(0.0, 0.0);
#pragma unroll
  for (int q = 0; q < kGmresRows; ++q) {
    const int i = tid + q * kGmresThreads;
    w[q] = i < N ? b[i] : make_double2(0.0, 0.0);
    p.x += w[q].x * w[q].x + w[q].y * w[q].y;
  }
  const double beta = sqrt(gm_block_sum(p, red).x);
  if (beta == 0.0) {
    for (int i = tid; i < N; i += kGmresThreads) x[i] = make_double2(0.0, 0.0);
    if (tid == 0) {
      iters[sys] = 0;
      relres[sys] = 0.0;
      if (PREC) status[sys] = 0;
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < kGmresRows; ++q) {
    const int i = tid + q * kGmresThreads;
    if (i < N) V[i] = make_double2(w[q].x / beta, w[q].y / beta);
  }
  if (tid == 0) {
    g[0] = make_double2(beta, 0.0);
    done = 0;
  }
  int k = 0;
  double est = 1.0;
  for (int j = 0; j < maxit; ++j) {
    // current basis vector into LDS (written by this workgroup: a barrier
    // suffices between the global write and these reads)
    __syncthreads();
    for (int i = tid; i < N; i += kGmresThreads) sv[i] = V[(long long)j * N + i];
    __syncthreads();
    // z_j = M^{-1} v_j in place (its own barriers)
    if constexpr (PREC)
      lu_solve_lds<float>(LUbase + (long long)sys * mstride, permbase + (long long)sys * kMaxN, sv,
                          N);
    // w = A v_j, four columns per batch with all their loads in flight.
    // Rows are clamped into the matrix rather than tested (a load under a
    // divergent test is waited for before the next one is issued); the
    // clamped rows' sums are dropped after the sweep.
#pragma unroll
    for (int q = 0; q < kGmresRows; ++q) w[q] = make_double2(0.0, 0.0);
    int c = 0;
    for (; c + 4 <= N; c += 4) {
      double2 a[4][kGmresRows];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < kGmresRows; ++q) a[u][q] = A[(long long)(c + u) * N + rowc[q]];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 vc = sv[c + u];
#pragma unroll
        for (int q = 0; q < kGmresRows; ++q) {
          w[q].x += a[u][q].x * vc.x - a[u][q].y * vc.y;
          w[q].y += a[u][q].x * vc.y + a[u][q].y * vc.x;
        }
      }
    }
    for (; c < N; ++c) {
      const double2 vc = sv[c];
#pragma unroll
      for (int q = 0; q < kGmresRows; ++q) {
        const double2 a = A[(long long)c * N + rowc[q]];
        w[q].x += a.x * vc.x - a.y * vc.y;
        w[q].y += a.x * vc.y + a.y * vc.x;
      }
    }
#pragma unroll
    for (int q = 0; q < kGmresRows; ++q)
      if (tid + q * kGmresThreads >= N) w[q] = make_double2(0.0, 0.0);
    // modified Gram-Schmidt: h_i = <v_i, w>, w -= h_i v_i
    for (int i2 = 0; i2 <= j; ++i2) {
      const double2 *vi = V + (long long)i2 * N;
      double2 s = make_double2(0.0, 0.0);
      double2 vr[kGmresRows];
#pragma unroll
      for (int q = 0; q < kGmresRows; ++q) {
        // clamped rows are zeroed by a multiply (a select of a load would
        // be turned back into a branch); basis entries are finite
        const double2 v = vi[rowc[q]];
        vr[q] = make_double2(v.x * rmask[q], v.y * rmask[q]);
        // conj(v) w
        s.x += vr[q].x * w[q].x + vr[q].y * w[q].y;
        s.y += vr[q].x * w[q].y - vr[q].y * w[q].x;
      }
      const double2 h = gm_block_sum(s, red);
#pragma unroll
      for (int q = 0; q < kGmresRows; ++q) {
        w[q].x -= h.x * vr[q].x - h.y * vr[q].y;
        w[q].y -= h.x * vr[q].y + h.y * vr[q].x;
      }
      if (tid == 0) col[i2] = h;
    }
    p = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < kGmresRows; ++q) p.x += w[q].x * w[q].x + w[q].y * w[q].y;
    const double hn = sqrt(gm_block_sum(p, red).x);
    if (hn > 0.0) {
#pragma unroll
      for (int q = 0; q < kGmresRows; ++q) {
        const int i = tid + q * kGmresThreads;
        if (i < N) V[(long long)(j + 1) * N + i] = make_double2(w[q].x / hn, w[q].y / hn);
      }
    }
    if (tid == 0) {
      col[j + 1] = make_double2(hn, 0.0);
      // previous rotations on the new column
      for (int i = 0; i < j; ++i) {
        const double2 a = col[i], bb = col[i + 1];
        const double c = cs[i];
        const double2 s = sn[i];
        // (c a + s b, -conj(s) a + c b)
        col[i] = make_double2(c * a.x + s.x * bb.x - s.y * bb.y, c * a.y + s.x * bb.y + s.y * bb.x);
        col[i + 1] = make_double2(-(s.x * a.x + s.y * a.y) + c * bb.x,
                                  -(s.x * a.y - s.y * a.x) + c * bb.y);
      }
      // new rotation annihilating col[j + 1]
      const double2 a = col[j], bb = col[j + 1];
      const double aa = sqrt(a.x * a.x + a.y * a.y), ab = sqrt(bb.x * bb.x + bb.y * bb.y);
      double c;
      double2 s;
      if (ab == 0.0) {
        c = 1.0;
        s = make_double2(0.0, 0.0);
      } else if (aa == 0.0) {
        c = 0.0;
        s = make_double2(bb.x / ab, -bb.y / ab);
      } else {
        const double hh = sqrt(aa * aa + ab * ab);
        c = aa / hh;
        // (a/|a|) conj(b) / hh
        const double2 ua = make_double2(a.x / aa, a.y / aa);
        s = make_double2((ua.x * bb.x + ua.y * bb.y) / hh, (ua.y * bb.x - ua.x * bb.y) / hh);
      }
      cs[j] = c;
      sn[j] = s;
      col[j] = make_double2(c * a.x + s.x * bb.x - s.y * bb.y, c * a.y + s.x * bb.y + s.y * bb.x);
      const double2 gj = g[j];
      g[j + 1] = make_double2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
      g[j] = make_double2(c * gj.x, c * gj.y);
      for (int i = 0; i <= j; ++i) R[(long long)j * (maxit + 1) + i] = col[i];
      const double e = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y) / beta;
      relres[sys] = e;
      done = (e <= tol || hn == 0.0) ? 1 : 0;
    }
    __syncthreads();
    k = j + 1;
    if (done) break;
  }
  // y = R^{-1} g (back substitution, one thread), then x = V y
  __syncthreads();
  if (tid == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double2 s = g[i];
      for (int l = i + 1; l < k; ++l) {
        const double2 r = R[(long long)l * (maxit + 1) + i], y = col[l];
        s.x -= r.x * y.x - r.y * y.y;
        s.y -= r.x * y.y + r.y * y.x;
      }
      const double2 d = R[(long long)i * (maxit + 1) + i];
      const double dd = d.x * d.x + d.y * d.y;
      col[i] = make_double2((s.x * d.x + s.y * d.y) / dd, (s.y * d.x - s.x * d.y) / dd);
    }
    iters[sys] = k;
  }
  __syncthreads();
  for (int i = tid; i < N; i += kGmresThreads) {
    double2 acc = make_double2(0.0, 0.0);
    for (int l = 0; l < k; ++l) {
      const double2 v = V[(long long)l * N + i], y = col[l];
      acc.x += v.x * y.x - v.y * y.y;
      acc.y += v.x * y.y + v.y * y.x;
    }
    if (PREC) sv[i] = acc;
    else x[i] = acc;
  }
  if constexpr (PREC) {
    // x = M^{-1} V y
    __syncthreads();
    lu_solve_lds<float>(LUbase + (long long)sys * mstride, permbase + (long long)sys * kMaxN, sv,
                        N);
    for (int i = tid; i < N; i += kGmresThreads) x[i] = sv[i];
    if (tid == 0) status[sys] = relres[sys] <= tol ? k : -1;
  }
}

}  // namespace fthms
