// Batched dense complex LU with partial pivoting, triangular solves and
// FP64 iterative refinement; one 256-thread workgroup per matrix.
//
// The solve of the first-kind open-arc system (Section 3.2, eq.
// FDBIEk-interior; the paper states the subproblems are solved by direct
// linear algebra or GMRES) is a dense LU.  Layout: column-major, leading
// dimension N, interleaved complex (re, im).
//
// Right-looking blocked LU with two levels of blocking:
//   outer block NB = 64 columns: row swaps outside the block, blocked TRSM
//   for U12 and the trailing update A22 -= L21 U12 with K = 64;
//   inner panels of PW = 8 columns: register-resident factorisation with
//   partial pivoting (pivot choice |re| + |im|, first index on ties), then
//   the in-block TRSM and update with K = 8.
// Every update A -= B C runs on the matrix cores: complex products as four
// real 16x16x4 MFMA chains (f64 for the FP64 form, f32 with f32
// accumulation for the refined form).  Pivot search, pivot row, panel
// scaling and the triangular solves against the 8x8 diagonal blocks are
// done in FP64 in both forms.
#pragma once

#include "common.h"

namespace fthms {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
// Accumulator row of register r in lane group g = lane / 16 (column is
// lane % 16): interleaved for f64 (g + 4 r), blocked for f32 (4 g + r).
template <> struct Mma<double> {
  typedef v4d acc;
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int g, int r) { return g + 4 * r; }
};
template <> struct Mma<float> {
  typedef v4f acc;
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int g, int r) { return 4 * g + r; }
};

constexpr int kLuThreads = 256;
constexpr int kLuNB = 64;
constexpr int kLuPW = 8;

struct LuSmem {
  double red_v[4];
  int red_r[4];
  int piv[kLuNB];
  double2 bufp[kLuPW];
  double2 bufc[kLuPW];
  double2 L[kLuPW][kLuPW];
  int zero_pivot;
};

// C[m x n] -= A[m x K] * B[K x n]; operands are sub-blocks of column-major
// storage with leading dimension ld.  Each wave owns 32x32 output tiles
// (2x2 blocks of 16x16), streams A and B fragments from memory and keeps
// the tile in accumulator registers for the whole K loop.  No barrier.
//
// MFMA 16x16x4 operand layout: lane l holds A[l % 16][l / 16],
// B[l / 16][l % 16]; accumulator register r holds column l % 16 at row
// Mma<T>::crow(l / 16, r).
template <typename T>
__device__ void wg_gemm_sub(cplx_t<T> *C, const cplx_t<T> *A,
                            const cplx_t<T> *B, int ld, int m, int n, int K) {
  typedef typename Mma<T>::acc acc_t;
  if (m <= 0 || n <= 0 || K <= 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tm = (m + 31) >> 5, tn = (n + 31) >> 5;
  for (int t = wave; t < tm * tn; t += kLuThreads / 64) {
    const int ti = t % tm, tj = t / tm;
    acc_t cr[2][2], ci[2][2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const int col = tj * 32 + cb * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = ti * 32 + rb * 16 + Mma<T>::crow(lk, r);
          cplx_t<T> v = mk<T>(0, 0);
          if (row < m && col < n) v = C[row + (long long)col * ld];
          cr[rb][cb][r] = v.x;
          ci[rb][cb][r] = v.y;
        }
      }
    // fragments of the next k-step are loaded while the current one runs
    cplx_t<T> fa[2], fb[2];
    auto load_frag = [&](int k0) {
      const int kk = k0 + lk;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const int row = ti * 32 + rb * 16 + li;
        fa[rb] = (row < m && kk < K) ? A[row + (long long)kk * ld] : mk<T>(0, 0);
      }
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const int col = tj * 32 + cb * 16 + li;
        fb[cb] = (col < n && kk < K) ? B[kk + (long long)col * ld] : mk<T>(0, 0);
      }
    };
    load_frag(0);
#pragma unroll 1
    for (int k0 = 0; k0 < K; k0 += 4) {
      T ar[2], ai[2], pai[2], br[2], bi[2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        ar[rb] = -fa[rb].x;
        ai[rb] = -fa[rb].y;
        pai[rb] = fa[rb].y;
      }
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        br[cb] = fb[cb].x;
        bi[cb] = fb[cb].y;
      }
      if (k0 + 4 < K) load_frag(k0 + 4);
      // C - A B:  re += (-Ar) Br + Ai Bi ;  im += (-Ar) Bi + (-Ai) Br
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          cr[rb][cb] = Mma<T>::run(ar[rb], br[cb], cr[rb][cb]);
          ci[rb][cb] = Mma<T>::run(ar[rb], bi[cb], ci[rb][cb]);
        }
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          cr[rb][cb] = Mma<T>::run(pai[rb], bi[cb], cr[rb][cb]);
          ci[rb][cb] = Mma<T>::run(ai[rb], br[cb], ci[rb][cb]);
        }
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const int col = tj * 32 + cb * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = ti * 32 + rb * 16 + Mma<T>::crow(lk, r);
          if (row < m && col < n)
            C[row + (long long)col * ld] = mk<T>(cr[rb][cb][r], ci[rb][cb][r]);
        }
      }
  }
}

// Apply row interchanges spiv[0..cnt) (pivot of row r0 + i is spiv[i],
// absolute) in order to columns [c0, c1).
template <typename T>
__device__ void swap_rows(cplx_t<T> *A, int ld, const int *spiv, int r0, int cnt,
                          int c0, int c1) {
  for (int col = c0 + (int)threadIdx.x; col < c1; col += kLuThreads) {
    cplx_t<T> *a = A + (long long)col * ld;
    for (int i = 0; i < cnt; ++i) {
      const int p = spiv[i];
      if (p != r0 + i) {
        const cplx_t<T> t = a[r0 + i];
        a[r0 + i] = a[p];
        a[p] = t;
      }
    }
  }
}

// B := L^{-1} B for the unit lower pw x pw block at (r0, r0) and the rows
// r0..r0+pw of columns [c0, c1); FP64 arithmetic.
template <typename T>
__device__ void trsm_small(cplx_t<T> *A, int ld, int r0, int pw, int c0, int c1,
                           LuSmem &sm) {
  const int tid = threadIdx.x;
  if (tid < kLuPW * kLuPW) {
    const int i = tid % kLuPW, j = tid / kLuPW;
    sm.L[i][j] = (i < pw && j < pw) ? to_d2(A[(r0 + i) + (long long)(r0 + j) * ld])
                                    : make_double2(0.0, 0.0);
  }
  __syncthreads();
  // L is re-read from LDS for every column (volatile): hoisting the whole
  // block into registers would cost 112 VGPRs for a loop of a few trips.
  const volatile double *Lv = (const volatile double *)&sm.L[0][0];
  for (int col = c0 + tid; col < c1; col += kLuThreads) {
    cplx_t<T> *a = A + (long long)col * ld + r0;
    double2 x[kLuPW];
#pragma unroll
    for (int i = 0; i < kLuPW; ++i) x[i] = i < pw ? to_d2(a[i]) : make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 1; i < kLuPW; ++i)
#pragma unroll
      for (int j = 0; j < i; ++j) {
        const double2 l = make_double2(Lv[2 * (i * kLuPW + j)], Lv[2 * (i * kLuPW + j) + 1]);
        x[i] = cfms(x[i], l, x[j]);
      }
#pragma unroll
    for (int i = 0; i < kLuPW; ++i)
      if (i < pw) a[i] = from_d2<T>(x[i]);
  }
  __syncthreads();
}

// Factor the panel A[p0:N, p0:p0+pw] (pw <= PW) with partial pivoting.
// Rows p0 + tid + 256 q live in registers (FP64).  Pivots (absolute row
// indices) go to sm.piv[p0 - kb + c] and piv[p0 + c].
template <typename T, int R>
__device__ void panel_factor(cplx_t<T> *A, int ld, int N, int p0, int pw, int kb,
                             int *piv, LuSmem &sm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double2 v[R][kLuPW];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int row = p0 + tid + kLuThreads * q;
#pragma unroll
    for (int c = 0; c < kLuPW; ++c)
      v[q][c] = (row < N && c < pw) ? to_d2(A[row + (long long)(p0 + c) * ld])
                                    : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int c = 0; c < kLuPW; ++c) {
    if (c < pw) {
      const int col = p0 + c;
      double best = -1.0;
      int brow = N;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int row = p0 + tid + kLuThreads * q;
        if (row >= col && row < N) {
          const double a = cabs1(v[q][c]);
          if (a > best) {
            best = a;
            brow = row;
          }
        }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int orow = __shfl_xor(brow, off);
        if (ob > best || (ob == best && orow < brow)) {
          best = ob;
          brow = orow;
        }
      }
      if (lane == 0) {
        sm.red_v[wave] = best;
        sm.red_r[wave] = brow;
      }
      __syncthreads();
      best = sm.red_v[0];
      brow = sm.red_r[0];
#pragma unroll
      for (int w = 1; w < kLuThreads / 64; ++w) {
        const double ob = sm.red_v[w];
        const int orow = sm.red_r[w];
        if (ob > best || (ob == best && orow < brow)) {
          best = ob;
          brow = orow;
        }
      }
      // a column without any comparable entry (NaN) keeps its own row
      const int prow = (brow >= col && brow < N) ? brow : col;
      const int own_p = (prow - p0) & (kLuThreads - 1), q_p = (prow - p0) / kLuThreads;
      const int own_c = (col - p0) & (kLuThreads - 1), q_c = (col - p0) / kLuThreads;
      if (tid == own_p) {
#pragma unroll
        for (int q = 0; q < R; ++q)
          if (q == q_p)
#pragma unroll
            for (int c2 = 0; c2 < kLuPW; ++c2) sm.bufp[c2] = v[q][c2];
      }
      if (tid == own_c) {
#pragma unroll
        for (int q = 0; q < R; ++q)
          if (q == q_c)
#pragma unroll
            for (int c2 = 0; c2 < kLuPW; ++c2) sm.bufc[c2] = v[q][c2];
      }
      if (tid == 0) {
        sm.piv[p0 - kb + c] = prow;
        piv[col] = prow;
        if (!(best > 0.0) && sm.zero_pivot == 0) sm.zero_pivot = col + 1;
      }
      __syncthreads();
      double2 pr[kLuPW];
#pragma unroll
      for (int c2 = 0; c2 < kLuPW; ++c2) pr[c2] = sm.bufp[c2];
      if (prow != col) {
        if (tid == own_p) {
#pragma unroll
          for (int q = 0; q < R; ++q)
            if (q == q_p)
#pragma unroll
              for (int c2 = 0; c2 < kLuPW; ++c2) v[q][c2] = sm.bufc[c2];
        }
        if (tid == own_c) {
#pragma unroll
          for (int q = 0; q < R; ++q)
            if (q == q_c)
#pragma unroll
              for (int c2 = 0; c2 < kLuPW; ++c2) v[q][c2] = pr[c2];
        }
      }
      const double2 inv = best > 0.0 ? crcp(pr[c]) : make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int row = p0 + tid + kLuThreads * q;
        if (row > col && row < N) {
          const double2 l = cmul(v[q][c], inv);
          v[q][c] = l;
#pragma unroll
          for (int c2 = c + 1; c2 < kLuPW; ++c2)
            if (c2 < pw) v[q][c2] = cfms(v[q][c2], l, pr[c2]);
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int row = p0 + tid + kLuThreads * q;
    if (row < N)
#pragma unroll
      for (int c = 0; c < kLuPW; ++c)
        if (c < pw) A[row + (long long)(p0 + c) * ld] = from_d2<T>(v[q][c]);
  }
  __syncthreads();
}

// In-place LU of one N x N matrix by the calling workgroup.
template <typename T, int R>
__device__ void lu_factor(cplx_t<T> *A, int N, int *piv, LuSmem &sm) {
  const int ld = N;
  if (threadIdx.x == 0) sm.zero_pivot = 0;
  __syncthreads();
  for (int k0 = 0; k0 < N; k0 += kLuNB) {
    const int nb = min(kLuNB, N - k0);
    for (int p0 = k0; p0 < k0 + nb; p0 += kLuPW) {
      const int pw = min(kLuPW, k0 + nb - p0);
      panel_factor<T, R>(A, ld, N, p0, pw, k0, piv, sm);
      swap_rows<T>(A, ld, sm.piv + (p0 - k0), p0, pw, k0, p0);
      swap_rows<T>(A, ld, sm.piv + (p0 - k0), p0, pw, p0 + pw, k0 + nb);
      __syncthreads();
      if (p0 + pw < k0 + nb) {
        trsm_small<T>(A, ld, p0, pw, p0 + pw, k0 + nb, sm);
        wg_gemm_sub<T>(A + (p0 + pw) + (long long)(p0 + pw) * ld,
                       A + (p0 + pw) + (long long)p0 * ld,
                       A + p0 + (long long)(p0 + pw) * ld, ld, N - p0 - pw,
                       k0 + nb - p0 - pw, pw);
        __syncthreads();
      }
    }
    swap_rows<T>(A, ld, sm.piv, k0, nb, 0, k0);
    swap_rows<T>(A, ld, sm.piv, k0, nb, k0 + nb, N);
    __syncthreads();
    if (k0 + nb < N) {
      // U12 = L11^{-1} A12, blocked by PW rows
      for (int s0 = 0; s0 < nb; s0 += kLuPW) {
        const int sw = min(kLuPW, nb - s0);
        trsm_small<T>(A, ld, k0 + s0, sw, k0 + nb, N, sm);
        if (s0 + sw < nb) {
          wg_gemm_sub<T>(A + (k0 + s0 + sw) + (long long)(k0 + nb) * ld,
                         A + (k0 + s0 + sw) + (long long)(k0 + s0) * ld,
                         A + (k0 + s0) + (long long)(k0 + nb) * ld, ld,
                         nb - s0 - sw, N - k0 - nb, sw);
          __syncthreads();
        }
      }
      wg_gemm_sub<T>(A + (k0 + nb) + (long long)(k0 + nb) * ld,
                     A + (k0 + nb) + (long long)k0 * ld,
                     A + k0 + (long long)(k0 + nb) * ld, ld, N - k0 - nb,
                     N - k0 - nb, nb);
      __syncthreads();
    }
  }
}

template <typename T, int R>
__global__ __launch_bounds__(kLuThreads) void lu_kernel(cplx_t<T> *Abase, int N,
                                                        long long mstride, int *pivbase,
                                                        int *status) {
  __shared__ LuSmem sm;
  cplx_t<T> *A = Abase + (long long)blockIdx.x * mstride;
  int *piv = pivbase + (long long)blockIdx.x * N;
  lu_factor<T, R>(A, N, piv, sm);
  if (threadIdx.x == 0 && status) status[blockIdx.x] = sm.zero_pivot ? -2 : 0;
}

// ---------------------------------------------------------------------------
// triangular solves on a vector held in LDS (FP64 accumulation)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double2 ld2(const cplx_t<T> *p) {
  return to_d2(*p);
}

// y := U^{-1} L^{-1} P y for the factors in LU (column-major, ld = N).
template <typename T>
__device__ void lu_solve_lds(const cplx_t<T> *LU, const int *piv, double2 *y, int N) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) {
    for (int i = 0; i < N; ++i) {
      const int p = piv[i];
      if (p != i) {
        const double2 t = y[i];
        y[i] = y[p];
        y[p] = t;
      }
    }
  }
  __syncthreads();
  for (int jb = 0; jb < N; jb += 64) {
    const int nb = min(64, N - jb);
    if (wave == 0) {
      double2 yi = lane < nb ? y[jb + lane] : make_double2(0.0, 0.0);
      for (int c = 0; c < nb - 1; ++c) {
        const double2 yc = make_double2(__shfl(yi.x, c), __shfl(yi.y, c));
        if (lane > c && lane < nb)
          yi = cfms(yi, ld2<T>(LU + (jb + lane) + (long long)(jb + c) * N), yc);
      }
      if (lane < nb) y[jb + lane] = yi;
    }
    __syncthreads();
    for (int r = jb + nb + tid; r < N; r += kLuThreads) {
      double2 acc = y[r];
      for (int c = 0; c < nb; ++c)
        acc = cfms(acc, ld2<T>(LU + r + (long long)(jb + c) * N), y[jb + c]);
      y[r] = acc;
    }
    __syncthreads();
  }
  const int nblk = (N + 63) / 64;
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int jb = bi * 64;
    const int nb = min(64, N - jb);
    if (wave == 0) {
      double2 yi = lane < nb ? y[jb + lane] : make_double2(0.0, 0.0);
      for (int c = nb - 1; c >= 0; --c) {
        if (lane == c)
          yi = cmul(yi, crcp(ld2<T>(LU + (jb + c) + (long long)(jb + c) * N)));
        const double2 yc = make_double2(__shfl(yi.x, c), __shfl(yi.y, c));
        if (lane < c)
          yi = cfms(yi, ld2<T>(LU + (jb + lane) + (long long)(jb + c) * N), yc);
      }
      if (lane < nb) y[jb + lane] = yi;
    }
    __syncthreads();
    for (int r = tid; r < jb; r += kLuThreads) {
      double2 acc = y[r];
      for (int c = 0; c < nb; ++c)
        acc = cfms(acc, ld2<T>(LU + r + (long long)(jb + c) * N), y[jb + c]);
      y[r] = acc;
    }
    __syncthreads();
  }
}

constexpr int kMaxN = 1024;

// alpha = A^{-1} b from FP64 factors.
__global__ __launch_bounds__(kLuThreads) void lu_solve64_kernel(
    const double2 *LUbase, const int *pivbase, int N, long long mstride,
    const double2 *b, double2 *x, long long vstride) {
  __shared__ double2 y[kMaxN];
  const double2 *LU = LUbase + (long long)blockIdx.x * mstride;
  const int *piv = pivbase + (long long)blockIdx.x * N;
  for (int i = threadIdx.x; i < N; i += kLuThreads) y[i] = b[(long long)blockIdx.x * vstride + i];
  __syncthreads();
  lu_solve_lds<double>(LU, piv, y, N);
  for (int i = threadIdx.x; i < N; i += kLuThreads) x[(long long)blockIdx.x * vstride + i] = y[i];
}

__device__ double block_sum(double v, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kLuThreads / 64; ++w) s += red[w];
  return s;
}

// Refined solve: x0 from the FP32 factors, then repeat
//   r = b - A64 x (FP64), d = LU32^{-1} r, x += d
// and stop once the predicted error of the updated x, |d_k| * rho with
// rho = |d_k| / |d_{k-1}| (observed contraction), is below tol |x|.
// status[b] = steps taken, or -1 when the cap was hit or the iteration did
// not contract (the caller then redoes the solve in FP64).
__global__ __launch_bounds__(kLuThreads) void refine_kernel(
    const float2 *LUbase, const int *pivbase, const double2 *A64base, int N,
    long long mstride, const double2 *b, double2 *x, long long vstride, double tol,
    int max_iter, int *status, double *relres) {
  __shared__ double2 xs[kMaxN];
  __shared__ double2 rs[kMaxN];
  __shared__ double red[4];
  const long long mb = (long long)blockIdx.x;
  const float2 *LU = LUbase + mb * mstride;
  const int *piv = pivbase + mb * N;
  const double2 *A = A64base + mb * mstride;
  const double2 *bb = b + mb * vstride;
  const int tid = threadIdx.x;
  if (status && status[mb] == -2) {  // zero pivot: leave for the FP64 redo
    for (int i = tid; i < N; i += kLuThreads) x[mb * vstride + i] = make_double2(0.0, 0.0);
    return;
  }
  for (int i = tid; i < N; i += kLuThreads) xs[i] = bb[i];
  __syncthreads();
  lu_solve_lds<float>(LU, piv, xs, N);
  double prev = -1.0, last = 0.0;
  int it = 0, done = 0;
  for (; it < max_iter && !done; ++it) {
    // r = b - A x  (each thread owns rows; column sweep, coalesced)
    for (int r = tid; r < N; r += kLuThreads) {
      double2 acc = bb[r];
      for (int c = 0; c < N; ++c) acc = cfms(acc, A[r + (long long)c * N], xs[c]);
      rs[r] = acc;
    }
    __syncthreads();
    lu_solve_lds<float>(LU, piv, rs, N);
    double dn = 0.0, xn = 0.0;
    for (int i = tid; i < N; i += kLuThreads) {
      const double2 xi = cadd(xs[i], rs[i]);
      xs[i] = xi;
      dn += cnorm2(rs[i]);
      xn += cnorm2(xi);
    }
    dn = sqrt(block_sum(dn, red));
    xn = sqrt(block_sum(xn, red));
    last = xn > 0.0 ? dn / xn : 0.0;
    if (dn == 0.0) {
      done = 1;
    } else if (prev > 0.0) {
      const double rho = dn / prev;
      if (rho >= 1.0) break;  // not contracting
      if (rho * dn <= tol * xn) done = 1;
    }
    prev = dn;
    __syncthreads();
  }
  for (int i = tid; i < N; i += kLuThreads) x[mb * vstride + i] = xs[i];
  if (tid == 0) {
    if (status) status[mb] = done ? (it > 0 ? it : 1) : -1;
    if (relres) relres[mb] = last;
  }
}

// FP64 redo of the solves whose refined status is negative: factor the
// FP64 matrix in place and solve.
template <int R>
__global__ __launch_bounds__(kLuThreads) void fallback64_kernel(
    double2 *A64base, int *pivbase, int N, long long mstride, const double2 *b,
    double2 *x, long long vstride, int *status) {
  __shared__ LuSmem sm;
  __shared__ double2 y[kMaxN];
  const long long mb = (long long)blockIdx.x;
  if (status[mb] >= 0) return;
  double2 *A = A64base + mb * mstride;
  int *piv = pivbase + mb * N;
  lu_factor<double, R>(A, N, piv, sm);
  for (int i = threadIdx.x; i < N; i += kLuThreads) y[i] = b[mb * vstride + i];
  __syncthreads();
  lu_solve_lds<double>(A, piv, y, N);
  for (int i = threadIdx.x; i < N; i += kLuThreads) x[mb * vstride + i] = y[i];
  if (threadIdx.x == 0) status[mb] = sm.zero_pivot ? -2 : -1;
}

}  // namespace fthms
