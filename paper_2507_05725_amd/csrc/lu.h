// Batched dense complex LU with partial pivoting, triangular solves and
// FP64 iterative refinement; one 256-thread workgroup per matrix.
//
// The solve of the first-kind open-arc system (Section 3.2, eq.
// FDBIEk-interior; the paper states the subproblems are solved by direct
// linear algebra or GMRES) is a dense LU.  Layout: column-major, leading
// dimension N, interleaved complex (re, im).
//
// Right-looking blocked LU, two kernels per block of NB = 64 columns:
//
//   lu_panel_kernel  (one workgroup per matrix)  factors the m x 64 block
//     in inner panels of PW = 8 columns held in registers (FP64 partial
//     pivoting: pivot = largest |re| + |im|, first index on ties), with the
//     in-block triangular solves and updates in FP64 on the VALU, and
//     writes the block's net row permutation as (destination, source) pairs;
//   lu_strip_kernel  (one workgroup per 64-column strip of one matrix,
//     XCD-aware: all strips of a matrix land on the same XCD and share its
//     L2) applies the permutation to its columns as a gather, solves
//     U12 = L11^{-1} A12 for its 64 columns into LDS (FP64 arithmetic), and
//     updates the strip below, A22 -= L21 U12, on the matrix cores: complex
//     products as four real 16x16x4 MFMA chains (f64 for the FP64 form, f32
//     with f32 accumulation for the refined form), U12 as the LDS-resident
//     B operand, L21 fragments streamed from memory.
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

constexpr int kMaxN = 1024;
constexpr int kSwapMax = 2 * kLuNB;          // pairs per block
constexpr int kSwapStride = 1 + 2 * kSwapMax;  // ints per matrix

struct LuSmem {
  double red_v[4];
  int red_r[4];
  int piv[kLuNB];
  double2 bufp[kLuPW];
  double2 bufc[kLuPW];
  double2 L[kLuPW][kLuPW];
  int pr_row[2 * kLuPW], pr_src[2 * kLuPW];  // net permutation of one panel
  int npr;
  int count;
  int zero_pivot;
  union {  // phases of the panel kernel never overlap
    double2 U[kLuPW][kLuNB];           // in-block update
    double2 gat[kLuNB][2 * kLuPW];     // in-block row gather
    int src[kMaxN];                    // block permutation
    double2 Ld[kLuNB][kLuNB + 1];      // diagonal block for its inverse
  } big;
};

// Factor columns [p0, p0 + pw) of the rows p0 .. N-1 held in registers:
// v[q][c] is row p0 + tid + 256 q, column p0 + c.  On return v holds the
// factored rows (L below the diagonal, U on and above it) and sm.piv[p0 - k0
// + c] the absolute pivot rows.
template <int R>
__device__ __forceinline__ void panel_factor_regs(double2 (&v)[R][kLuPW], int N, int p0,
                                                  int pw, int k0, int *piv, LuSmem &sm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
        sm.piv[p0 - k0 + c] = prow;
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
}

// Factor the block of columns [k0, k0 + nb) of one matrix (all rows >= k0),
// record the pivots, and emit the block's net row permutation for the
// columns outside it: swp[0] = count, then count (dst, src) pairs meaning
// "new row dst = old row src".
template <typename T, int R>
__global__ __launch_bounds__(kLuThreads) void lu_panel_kernel(cplx_t<T> *Abase, int N,
                                                              long long mstride, int k0,
                                                              int *pivbase, int *swapbase,
                                                              cplx_t<T> *Linv, int *status,
                                                              int only_failed) {
  __shared__ LuSmem sm;
  const long long mb = blockIdx.x;
  if (only_failed && status[mb] >= 0) return;
  cplx_t<T> *A = Abase + mb * mstride;
  int *piv = pivbase + mb * N;
  int *swp = swapbase + mb * kSwapStride;
  const int tid = threadIdx.x;
  const int nb = min(kLuNB, N - k0);
  if (tid == 0) sm.zero_pivot = 0;
  __syncthreads();
  for (int p0 = k0; p0 < k0 + nb; p0 += kLuPW) {
    const int pw = min(kLuPW, k0 + nb - p0);
    double2 v[R][kLuPW];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int row = p0 + tid + kLuThreads * q;
#pragma unroll
      for (int c = 0; c < kLuPW; ++c)
        v[q][c] = (row < N && c < pw) ? to_d2(A[row + (long long)(p0 + c) * N])
                                      : make_double2(0.0, 0.0);
    }
    panel_factor_regs<R>(v, N, p0, pw, k0, piv, sm);
    // write the factored panel back; the diagonal block's unit-lower part
    // goes to LDS for the in-block triangular solve
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int row = p0 + tid + kLuThreads * q;
      if (row < N)
#pragma unroll
        for (int c = 0; c < kLuPW; ++c)
          if (c < pw) A[row + (long long)(p0 + c) * N] = from_d2<T>(v[q][c]);
    }
    if (tid < kLuPW) {
#pragma unroll
      for (int c = 0; c < kLuPW; ++c) sm.L[tid][c] = v[0][c];
    }
    // row swaps of this panel inside the block, left and right of it, as a
    // gather over the panel's net permutation (<= 16 rows)
    if (tid == 0) {
      int n = 0;
      for (int i = 0; i < pw; ++i) {
        const int r1 = p0 + i, r2 = sm.piv[p0 - k0 + i];
        int a = -1, b = -1;
        for (int e = 0; e < n; ++e) {
          if (sm.pr_row[e] == r1) a = e;
          if (sm.pr_row[e] == r2) b = e;
        }
        if (a < 0) { sm.pr_row[n] = r1; sm.pr_src[n] = r1; a = n++; }
        if (b < 0) { sm.pr_row[n] = r2; sm.pr_src[n] = r2; b = n++; }
        const int t = sm.pr_src[a];
        sm.pr_src[a] = sm.pr_src[b];
        sm.pr_src[b] = t;
      }
      sm.npr = n;
    }
    __syncthreads();
    const int wl = p0 - k0, wr = k0 + nb - p0 - pw;
    const int npr = sm.npr;
    for (int e = tid; e < (wl + wr) * npr; e += kLuThreads) {
      const int ce = e / npr, j = e % npr;
      const int col = ce < wl ? k0 + ce : p0 + pw + (ce - wl);
      sm.big.gat[ce][j] = to_d2(A[sm.pr_src[j] + (long long)col * N]);
    }
    __syncthreads();
    for (int e = tid; e < (wl + wr) * npr; e += kLuThreads) {
      const int ce = e / npr, j = e % npr;
      const int col = ce < wl ? k0 + ce : p0 + pw + (ce - wl);
      A[sm.pr_row[j] + (long long)col * N] = from_d2<T>(sm.big.gat[ce][j]);
    }
    __syncthreads();
    if (wr > 0) {
      // U rows of this panel for the rest of the block: L11^{-1} A12
      for (int e = tid; e < wr; e += kLuThreads) {
        const int col = p0 + pw + e;
        cplx_t<T> *a = A + (long long)col * N + p0;
        double2 x[kLuPW];
#pragma unroll
        for (int i = 0; i < kLuPW; ++i) x[i] = i < pw ? to_d2(a[i]) : make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 1; i < kLuPW; ++i)
#pragma unroll
          for (int j = 0; j < i; ++j) x[i] = cfms(x[i], sm.L[i][j], x[j]);
#pragma unroll
        for (int i = 0; i < kLuPW; ++i) {
          if (i < pw) a[i] = from_d2<T>(x[i]);
          sm.big.U[i][e] = x[i];
        }
      }
      __syncthreads();
      // rank-pw update of the rest of the block, rows below the panel; four
      // columns per batch with all loads issued before the stores
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int row = p0 + tid + kLuThreads * q;
        if (row >= p0 + pw && row < N) {
          cplx_t<T> *a = A + row + (long long)(p0 + pw) * N;
          for (int e0 = 0; e0 < wr; e0 += 4) {
            double2 acc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
              acc[u] = e0 + u < wr ? to_d2(a[(long long)(e0 + u) * N]) : make_double2(0.0, 0.0);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int i = 0; i < kLuPW; ++i)
                if (i < pw) acc[u] = cfms(acc[u], v[q][i], sm.big.U[i][e0 + u]);
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (e0 + u < wr) a[(long long)(e0 + u) * N] = from_d2<T>(acc[u]);
          }
        }
      }
      __syncthreads();
    }
  }
  // inverse of the block's unit-lower diagonal part, FP64, for the strips'
  // U12 = L11^{-1} A12 products: four lanes per column j solve L x = e_j,
  // lane s holding x[k] for k = s (mod 4)
  {
    for (int e = tid; e < kLuNB * kLuNB; e += kLuThreads) {
      const int i = e % kLuNB, j = e / kLuNB;
      sm.big.Ld[i][j] = (i < nb && j < nb) ? to_d2(A[(k0 + i) + (long long)(k0 + j) * N])
                                           : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int j = tid >> 2, sub = tid & 3;
    double2 x[kLuNB / 4];
#pragma unroll
    for (int m = 0; m < kLuNB / 4; ++m) x[m] = make_double2((4 * m + sub == j) ? 1.0 : 0.0, 0.0);
    for (int i = j + 1; i < nb; ++i) {
      double2 part = make_double2(0.0, 0.0);
#pragma unroll
      for (int m = 0; m < kLuNB / 4; ++m) {
        const int kk = 4 * m + sub;
        if (kk >= j && kk < i) part = cfma(part, sm.big.Ld[i][kk], x[m]);
      }
      part.x += __shfl_xor(part.x, 1);
      part.y += __shfl_xor(part.y, 1);
      part.x += __shfl_xor(part.x, 2);
      part.y += __shfl_xor(part.y, 2);
#pragma unroll
      for (int m = 0; m < kLuNB / 4; ++m)
        if (4 * m + sub == i) x[m] = make_double2(-part.x, -part.y);
    }
    cplx_t<T> *li = Linv + mb * (kLuNB * kLuNB);
#pragma unroll
    for (int m = 0; m < kLuNB / 4; ++m) li[(4 * m + sub) + kLuNB * j] = from_d2<T>(x[m]);
    __syncthreads();
  }
  // net permutation of the block for the columns outside it
  for (int r = k0 + tid; r < N; r += kLuThreads) sm.big.src[r] = r;
  if (tid == 0) sm.count = 0;
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < nb; ++i) {
      const int p = sm.piv[i];
      const int t = sm.big.src[k0 + i];
      sm.big.src[k0 + i] = sm.big.src[p];
      sm.big.src[p] = t;
    }
  }
  __syncthreads();
  for (int r = k0 + tid; r < N; r += kLuThreads) {
    const int s = sm.big.src[r];
    if (s != r) {
      const int e = atomicAdd(&sm.count, 1);
      swp[1 + 2 * e] = r;
      swp[2 + 2 * e] = s;
    }
  }
  __syncthreads();
  if (tid == 0) {
    swp[0] = sm.count;
    // status: 0 ok, -2 exact zero pivot; a redo (only_failed) stays negative
    // (-1: redone in FP64) so that its solve is redone too
    if (k0 == 0) status[mb] = sm.zero_pivot ? -2 : (only_failed ? -1 : 0);
    else if (sm.zero_pivot) status[mb] = -2;
  }
}

constexpr int kStripW = 64;

// One workgroup per (matrix, 64-column strip).  Strips left of the block
// only receive the block's row permutation; strips right of it also get
// U12 = L11^{-1} A12 and the update A22 -= L21 U12 down the whole strip.
template <typename T>
__global__ __launch_bounds__(kLuThreads) void lu_strip_kernel(
    cplx_t<T> *Abase, int N, long long mstride, int k0, const int *swapbase,
    const cplx_t<T> *Linv, int batch, int nleft, int nright, const int *status,
    int only_failed) {
  typedef cplx_t<T> T2;
  typedef typename Mma<T>::acc acc_t;
  __shared__ T2 sX[kLuNB][kStripW + 1];
  __shared__ int spair[2 * kSwapMax];
  // XCD-aware decode: block b runs on XCD b % 8; matrix m lives on XCD m % 8
  const int b = blockIdx.x, xcd = b & 7, idx = b >> 3;
  const int ns = nleft + nright;
  const int mat = xcd + 8 * (idx / ns), s = idx % ns;
  if (mat >= batch) return;
  if (only_failed && status[mat] >= 0) return;
  T2 *A = Abase + (long long)mat * mstride;
  const int *swp = swapbase + (long long)mat * kSwapStride;
  const int tid = threadIdx.x;
  const int nb = min(kLuNB, N - k0);
  const bool right = s >= nleft;
  const int c0 = right ? k0 + nb + (s - nleft) * kStripW : s * kStripW;
  const int cw = min(kStripW, (right ? N : k0) - c0);
  // ---- row permutation as a gather (read every source, then write), 32
  // columns at a time through LDS
  const int npair = swp[0];
  for (int e = tid; e < 2 * npair; e += kLuThreads) spair[e] = swp[1 + e];
  __syncthreads();
  T2 *tmpb = &sX[0][0];  // viewed as [32][kSwapMax + 2]
  for (int half = 0; half < 2; ++half) {
    const int cb0 = half * 32;
    for (int e = tid; e < 32 * npair; e += kLuThreads) {
      const int c = e & 31, j = e >> 5;
      if (cb0 + c < cw) tmpb[c * (kSwapMax + 2) + j] = A[spair[2 * j + 1] + (long long)(c0 + cb0 + c) * N];
    }
    __syncthreads();
    for (int e = tid; e < 32 * npair; e += kLuThreads) {
      const int c = e & 31, j = e >> 5;
      if (cb0 + c < cw) A[spair[2 * j] + (long long)(c0 + cb0 + c) * N] = tmpb[c * (kSwapMax + 2) + j];
    }
    __syncthreads();
  }
  if (!right) return;
  // ---- U12 for this strip: X = L11^{-1} A12 on the matrix cores, with
  // the inverse from the panel kernel; A12 in LDS as the B operand, the
  // product kept in registers, then written over it (and to memory)
  const int lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int kpad = (nb + 3) & ~3;
  for (int e = tid; e < kLuNB * kStripW; e += kLuThreads) {
    const int r = e / kStripW, c = e % kStripW;
    sX[r][c] = (r < nb && c < cw) ? A[(k0 + r) + (long long)(c0 + c) * N] : mk<T>(0, 0);
  }
  __syncthreads();
  {
    const T2 *lv = Linv + (long long)mat * (kLuNB * kLuNB);
    acc_t xr[4], xi[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        xr[cb][r] = 0;
        xi[cb][r] = 0;
      }
    const int arow = 16 * wave + li;
#pragma unroll 1
    for (int kk = 0; kk < kpad; kk += 4) {
      const T2 fa = lv[arow + kLuNB * (kk + lk)];
      const T ar = fa.x, ai = fa.y, nai = -fa.y;
      T br[4], bi[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const T2 bv = sX[kk + lk][cb * 16 + li];
        br[cb] = bv.x;
        bi[cb] = bv.y;
      }
      // X + Linv A12:  re += Ar Br - Ai Bi ;  im += Ar Bi + Ai Br
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        xr[cb] = Mma<T>::run(ar, br[cb], xr[cb]);
        xi[cb] = Mma<T>::run(ar, bi[cb], xi[cb]);
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        xr[cb] = Mma<T>::run(nai, bi[cb], xr[cb]);
        xi[cb] = Mma<T>::run(ai, br[cb], xi[cb]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * wave + Mma<T>::crow(lk, r), col = cb * 16 + li;
        const T2 v = mk<T>(xr[cb][r], xi[cb][r]);
        sX[row][col] = v;
        if (row < nb && col < cw) A[(k0 + row) + (long long)(c0 + col) * N] = v;
      }
    __syncthreads();
  }
  // ---- A22 -= L21 U12 down the strip: each wave owns 16 rows x 64 columns
  for (int r0 = k0 + nb; r0 < N; r0 += 64) {
    const int rw = r0 + 16 * wave;  // first row of this wave
    if (rw >= N) continue;
    acc_t cr[4], ci[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int col = cb * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rw + Mma<T>::crow(lk, r);
        T2 v = mk<T>(0, 0);
        if (row < N && col < cw) v = A[row + (long long)(c0 + col) * N];
        cr[cb][r] = v.x;
        ci[cb][r] = v.y;
      }
    }
    const int arow = rw + li;
    const T2 *ap = A + arow + (long long)k0 * N;
    T2 fa = (arow < N && lk < nb) ? ap[(long long)lk * N] : mk<T>(0, 0);
#pragma unroll 1
    for (int kk = 0; kk < kpad; kk += 4) {
      const T ar = -fa.x, ai = -fa.y, pai = fa.y;
      const int kn = kk + 4 + lk;
      if (kk + 4 < kpad) fa = (arow < N && kn < nb) ? ap[(long long)kn * N] : mk<T>(0, 0);
      T br[4], bi[4];
      const int krow = kk + lk;
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const T2 bv = krow < nb ? sX[krow][cb * 16 + li] : mk<T>(0, 0);
        br[cb] = bv.x;
        bi[cb] = bv.y;
      }
      // C - A B:  re += (-Ar) Br + Ai Bi ;  im += (-Ar) Bi + (-Ai) Br
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        cr[cb] = Mma<T>::run(ar, br[cb], cr[cb]);
        ci[cb] = Mma<T>::run(ar, bi[cb], ci[cb]);
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        cr[cb] = Mma<T>::run(pai, bi[cb], cr[cb]);
        ci[cb] = Mma<T>::run(ai, br[cb], ci[cb]);
      }
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int col = cb * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rw + Mma<T>::crow(lk, r);
        if (row < N && col < cw) A[row + (long long)(c0 + col) * N] = mk<T>(cr[cb][r], ci[cb][r]);
      }
    }
  }
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

// Solve for the matrices whose status is negative (FP64 redo after a
// refined solve that did not converge): x = A^{-1} b from FP64 factors.
__global__ __launch_bounds__(kLuThreads) void solve_failed64_kernel(
    const double2 *LUbase, const int *pivbase, int N, long long mstride, const double2 *b,
    double2 *x, long long vstride, const int *status) {
  __shared__ double2 y[kMaxN];
  const long long mb = blockIdx.x;
  if (status[mb] >= 0) return;
  const double2 *LU = LUbase + mb * mstride;
  const int *piv = pivbase + mb * N;
  for (int i = threadIdx.x; i < N; i += kLuThreads) y[i] = b[mb * vstride + i];
  __syncthreads();
  lu_solve_lds<double>(LU, piv, y, N);
  for (int i = threadIdx.x; i < N; i += kLuThreads) x[mb * vstride + i] = y[i];
}

}  // namespace fthms
