// Batched dense complex LU with partial pivoting, triangular solves and
// FP64 iterative refinement.
//
// The solve of the first-kind open-arc system (Section 3.2, eq.
// FDBIEk-interior; the paper states the subproblems are solved by direct
// linear algebra or GMRES) is a dense LU.  Layout: column-major, leading
// dimension N, interleaved complex (re, im).
//
// Right-looking blocked LU, two kernels per block of NB = 64 columns:
//
//   the panel  factors the m x 64 block with partial pivoting (pivot =
//     largest |re| + |im|, first index on ties) and writes L11^{-1} and the
//     block's net row permutation as (destination, source) pairs: either
//     lu_panel_reg_kernel (panel.h; the whole block in registers, one
//     1024-thread workgroup per matrix, used whenever the block fits) or
//     lu_panel_kernel (one 256-thread workgroup per matrix, inner panels of
//     PW = 8 columns in registers, in-block solves and updates in FP64 on
//     the VALU);
//   lu_strip_kernel  (one workgroup per 64-column strip of one matrix,
//     XCD-aware: all strips of a matrix land on the same XCD and share its
//     L2) applies the permutation to its columns as a gather, forms
//     U12 = L11^{-1} A12 for its 64 columns on the matrix cores into LDS, and
//     updates the strip below, A22 -= L21 U12: complex products as four real
//     16x16x4 MFMA chains (f64 for the FP64 form, f32 with f32 accumulation
//     for the refined form), U12 as the LDS-resident B operand, the L21
//     fragments and the C tile of each 64-row tile loaded in one round trip.
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

// readlane of FP32/FP64 values and complex pairs (lane index uniform)
__device__ __forceinline__ float rdlane(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double rdlane(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T2> __device__ __forceinline__ T2 rdlane2(T2 v, int l) {
  T2 r;
  r.x = rdlane(v.x, l);
  r.y = rdlane(v.y, l);
  return r;
}

// Integer register array version: v[idx] as a scalar / v[idx] = val.
template <int RL> __device__ __forceinline__ int iget(const int (&v)[RL], int idx) {
  const int s = idx >> 6, l = idx & 63;
  int y = __builtin_amdgcn_readlane(v[0], l);
#pragma unroll
  for (int i = 1; i < RL; ++i)
    if (i == s) y = __builtin_amdgcn_readlane(v[i], l);
  return y;
}
template <int RL> __device__ __forceinline__ void iset(int (&v)[RL], int idx, int val, int lane) {
  const int s = idx >> 6, l = idx & 63;
#pragma unroll
  for (int i = 0; i < RL; ++i) v[i] = (i == s && lane == l) ? val : v[i];
}

constexpr int kLuThreads = 256;
constexpr int kLuNB = 64;
constexpr int kLuPW = 8;

constexpr int kMaxN = 1024;

// Status words of a batched factorisation and what a redo pass factors.
// After the FP32 LU: 0, or -2 for an exactly zero pivot.  A refined solve
// writes its step count (>= 1) or, when it does not converge, -1 on the
// first solve with fresh factors and kStatusLateFail on a later solve with
// factors kept from earlier (multiple-scattering steps).  A redo pass
// (FP64 LU of A64 in place) then sets -1: the matrix is solved with FP64
// factors from then on.  Redo modes: kRedoNone factors every matrix,
// kRedoFailed those with status < 0 (first solves), kRedoLate those with
// status kStatusLateFail (later solves; the others, still FP32 or already
// FP64, are left alone).
constexpr int kStatusLateFail = -3;
constexpr int kRedoNone = 0, kRedoFailed = 1, kRedoLate = 2;
__device__ __forceinline__ bool redo_skips(int mode, const int *status, long long mb) {
  if (mode == kRedoFailed) return status[mb] >= 0;
  if (mode == kRedoLate) return status[mb] != kStatusLateFail;
  return false;
}
// status written by a panel at block 0 (k0 == 0): zero pivot, or the mode's
// "factored" value (a late redo keeps its marker until the whole
// factorisation is done, so that every block step still selects it)
__device__ __forceinline__ int panel_status(int mode, bool zero) {
  return zero ? -2 : mode == kRedoFailed ? -1 : mode == kRedoLate ? kStatusLateFail : 0;
}
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
  int src[kMaxN];  // cumulative row permutation of the block
  // running inverse of the block's unit-lower part, packed lower triangle:
  // element (r, c), c <= r, at r (r + 1) / 2 + c
  double2 li[kLuNB * (kLuNB + 1) / 2];
  union {          // phases of one inner panel never overlap
    struct {
      double2 top[kLuNB][kLuPW];  // rows k0..p0 of the panel columns
      double2 ut[kLuNB][kLuPW];   // U rows k0..p0 of the panel columns
    } a;
    double2 gat[kLuNB][2 * kLuPW];  // in-block row gather
    struct {
      double2 lrow[kLuPW][kLuNB];  // new rows of L11 (previous columns)
      double2 tm[kLuPW][kLuNB];    // their product with the running inverse
    } c;
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

__device__ __forceinline__ int tri(int r, int c) { return (r * (r + 1) >> 1) + c; }

// Factor the block of columns [k0, k0 + nb) of one matrix (all rows >= k0),
// left-looking inside the block: each 8-column inner panel first receives
// every earlier panel's contribution -- its U rows as U = L11inv A (the
// running inverse of the block's unit-lower part, kept in memory) and its
// lower rows as A -= L U with all loads of earlier L columns issued in
// batches -- and is then factored in registers.  The running inverse is
// extended by the panel's rows with the block-inverse formula
// [La 0; Lb Lpp]^-1 = [La^-1 0; -Lpp^-1 Lb La^-1  Lpp^-1], and is what the
// strip kernel multiplies by.  Outputs: factored block, pivots, L11inv
// (64 x 64, column-major, zero above the diagonal) and the block's net row
// permutation for the columns outside it: swp[0] = count, then (dst, src)
// pairs meaning "new row dst = old row src".
template <typename T, int R>
__global__ __launch_bounds__(kLuThreads) void lu_panel_kernel(cplx_t<T> *Abase, int N,
                                                              long long mstride, int k0,
                                                              int *pivbase, int *swapbase,
                                                              cplx_t<T> *Linv, int *status,
                                                              int only_failed) {
  typedef cplx_t<T> T2;
  __shared__ LuSmem sm;
  const long long mb = blockIdx.x;
  if (redo_skips(only_failed, status, mb)) return;
  T2 *A = Abase + mb * mstride;
  int *piv = pivbase + mb * N;
  int *swp = swapbase + mb * kSwapStride;
  T2 *Li = Linv + mb * (kLuNB * kLuNB);
  const int tid = threadIdx.x;
  const int nb = min(kLuNB, N - k0);
  if (tid == 0) sm.zero_pivot = 0;
  for (int r = k0 + tid; r < N; r += kLuThreads) sm.src[r] = r;
  __syncthreads();
  for (int p0 = k0; p0 < k0 + nb; p0 += kLuPW) {
    const int pw = min(kLuPW, k0 + nb - p0);
    const int lead = p0 - k0;
    if (lead > 0) {
      // U rows of the panel columns: U = L11inv(lead) A(rows k0..p0)
      for (int e = tid; e < lead * kLuPW; e += kLuThreads) {
        const int r = e / kLuPW, c = e % kLuPW;
        sm.big.a.top[r][c] = c < pw ? to_d2(A[(k0 + r) + (long long)(p0 + c) * N])
                                    : make_double2(0.0, 0.0);
      }
      __syncthreads();
      for (int e = tid; e < lead * kLuPW; e += kLuThreads) {
        const int r = e / kLuPW, c = e % kLuPW;
        double2 acc = make_double2(0.0, 0.0);
        for (int j = 0; j <= r; ++j) acc = cfma(acc, sm.li[tri(r, j)], sm.big.a.top[j][c]);
        sm.big.a.ut[r][c] = acc;
        if (c < pw) A[(k0 + r) + (long long)(p0 + c) * N] = from_d2<T>(acc);
      }
      __syncthreads();
    }
    // lower rows of the panel: load and apply every earlier panel at once.
    // All loads are issued before any value is converted (a conversion
    // right after each load, or a load under a bounds test, would wait for
    // it); out-of-range entries are clamped loads zeroed by a multiply.
    double2 v[R][kLuPW];
    {
      T2 raw[R][kLuPW];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int rowc = min(p0 + tid + kLuThreads * q, N - 1);
#pragma unroll
        for (int c = 0; c < kLuPW; ++c) raw[q][c] = A[rowc + (long long)(p0 + min(c, pw - 1)) * N];
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int row = p0 + tid + kLuThreads * q;
#pragma unroll
        for (int c = 0; c < kLuPW; ++c) {
          const double m = (row < N && c < pw) ? 1.0 : 0.0;
          const double2 d = to_d2(raw[q][c]);
          v[q][c] = make_double2(d.x * m, d.y * m);
        }
      }
    }
    // earlier L columns, 8 at a time (independent read-only loads)
    // (rows past N: clamped loads zeroed by a multiply, as above)
    double rmask[R];
#pragma unroll
    for (int q = 0; q < R; ++q) rmask[q] = p0 + tid + kLuThreads * q < N ? 1.0 : 0.0;
    for (int j0 = 0; j0 < lead; j0 += kLuPW) {
      T2 lv[R][kLuPW];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int rowc = min(p0 + tid + kLuThreads * q, N - 1);
#pragma unroll
        for (int t = 0; t < kLuPW; ++t) lv[q][t] = A[rowc + (long long)(k0 + j0 + t) * N];
      }
#pragma unroll
      for (int t = 0; t < kLuPW; ++t) {
        // keep the scheduler from hoisting all 64 LDS reads of U at once
        asm volatile("" ::: "memory");
        double2 u[kLuPW];
#pragma unroll
        for (int c = 0; c < kLuPW; ++c) u[c] = sm.big.a.ut[j0 + t][c];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const double2 ld = to_d2(lv[q][t]);
          const double2 l = make_double2(ld.x * rmask[q], ld.y * rmask[q]);
#pragma unroll
          for (int c = 0; c < kLuPW; ++c) v[q][c] = cfms(v[q][c], l, u[c]);
        }
      }
    }
    panel_factor_regs<R>(v, N, p0, pw, k0, piv, sm);
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
    // net permutation of this panel (<= 16 rows) by wave 0, one map entry
    // per lane; also folded into the block's cumulative permutation
    if (tid < 64) {
      const int lane = tid;
      int myrow = -1, mysrc = -1, n = 0;
      for (int i = 0; i < pw; ++i) {
        const int r1 = p0 + i, r2 = sm.piv[p0 - k0 + i];
        unsigned long long m1 = __ballot(myrow == r1);
        int a;
        if (m1 == 0ULL) {
          a = n++;
          if (lane == a) {
            myrow = r1;
            mysrc = r1;
          }
        } else {
          a = __ffsll((long long)m1) - 1;
        }
        unsigned long long m2 = __ballot(myrow == r2);
        int b;
        if (m2 == 0ULL) {
          b = n++;
          if (lane == b) {
            myrow = r2;
            mysrc = r2;
          }
        } else {
          b = __ffsll((long long)m2) - 1;
        }
        const int sa = __shfl(mysrc, a), sb = __shfl(mysrc, b);
        if (lane == a) mysrc = sb;
        if (lane == b) mysrc = sa;
      }
      if (lane < n) {
        sm.pr_row[lane] = myrow;
        sm.pr_src[lane] = mysrc;
      }
      if (lane == 0) {
        sm.npr = n;
        for (int i = 0; i < pw; ++i) {
          const int r1 = p0 + i, r2 = sm.piv[p0 - k0 + i];
          const int u = sm.src[r1];
          sm.src[r1] = sm.src[r2];
          sm.src[r2] = u;
        }
      }
    }
    __syncthreads();
    // the panel's row swaps for the other block columns, as a gather
    const int wl = p0 - k0, wr = k0 + nb - p0 - pw;
    const int npr = sm.npr;
    if ((wl + wr) * npr > 0) {
      // at most 56 columns x 16 rows: four entries per thread, loads first
      constexpr int kGi = (kLuNB * 2 * kLuPW + kLuThreads - 1) / kLuThreads;
      const int tot = (wl + wr) * npr;
      T2 raw[kGi];
#pragma unroll
      for (int it = 0; it < kGi; ++it) {
        const int e = min(tid + it * kLuThreads, tot - 1);
        const int ce = e / npr, j = e % npr;
        const int col = ce < wl ? k0 + ce : p0 + pw + (ce - wl);
        raw[it] = A[sm.pr_src[j] + (long long)col * N];
      }
#pragma unroll
      for (int it = 0; it < kGi; ++it) {
        const int e = tid + it * kLuThreads;
        if (e < tot) sm.big.gat[e / npr][e % npr] = to_d2(raw[it]);
      }
    }
    __syncthreads();
    for (int e = tid; e < (wl + wr) * npr; e += kLuThreads) {
      const int ce = e / npr, j = e % npr;
      const int col = ce < wl ? k0 + ce : p0 + pw + (ce - wl);
      A[sm.pr_row[j] + (long long)col * N] = from_d2<T>(sm.big.gat[ce][j]);
    }
    __syncthreads();
    // extend the running inverse by this panel's rows
    for (int e = tid; e < pw * lead; e += kLuThreads) {
      const int t = e / lead, j = e % lead;
      sm.big.c.lrow[t][j] = to_d2(A[(p0 + t) + (long long)(k0 + j) * N]);
    }
    __syncthreads();
    for (int e = tid; e < pw * lead; e += kLuThreads) {
      const int t = e / lead, cc = e % lead;
      double2 acc = make_double2(0.0, 0.0);
      for (int j = cc; j < lead; ++j) acc = cfma(acc, sm.big.c.lrow[t][j], sm.li[tri(j, cc)]);
      sm.big.c.tm[t][cc] = acc;
    }
    __syncthreads();
    if (tid < lead + pw) {
      const int cc = tid;
      double2 x[kLuPW];
#pragma unroll
      for (int t = 0; t < kLuPW; ++t) {
        if (cc < lead) {
          x[t] = t < pw ? make_double2(-sm.big.c.tm[t][cc].x, -sm.big.c.tm[t][cc].y)
                        : make_double2(0.0, 0.0);
        } else {
          x[t] = make_double2(t == cc - lead ? 1.0 : 0.0, 0.0);
        }
      }
#pragma unroll
      for (int t = 1; t < kLuPW; ++t)
#pragma unroll
        for (int j = 0; j < t; ++j) x[t] = cfms(x[t], sm.L[t][j], x[j]);
#pragma unroll
      for (int t = 0; t < kLuPW; ++t)
        if (t < pw && cc <= lead + t) sm.li[tri(lead + t, cc)] = x[t];
    }
    __syncthreads();
  }
  // the inverse for the strips: full 64 x 64, column-major, zero above the
  // diagonal and outside the block
  for (int e = tid; e < kLuNB * kLuNB; e += kLuThreads) {
    const int r = e % kLuNB, c = e / kLuNB;
    Li[e] = (c <= r && r < nb) ? from_d2<T>(sm.li[tri(r, c)]) : mk<T>(0, 0);
  }
  // net permutation of the block for the columns outside it
  if (tid == 0) sm.count = 0;
  __syncthreads();
  for (int r = k0 + tid; r < N; r += kLuThreads) {
    const int s = sm.src[r];
    if (s != r) {
      const int e = atomicAdd(&sm.count, 1);
      swp[1 + 2 * e] = r;
      swp[2 + 2 * e] = s;
    }
  }
  __syncthreads();
  if (tid == 0) {
    swp[0] = sm.count;
    // status: 0 ok, -2 exact zero pivot; a redo stays negative (-1: redone
    // in FP64) so that its solve is redone too
    if (k0 == 0) status[mb] = panel_status(only_failed, sm.zero_pivot != 0);
    else if (sm.zero_pivot) status[mb] = -2;
  }
}

constexpr int kStripW = 64;

// A strip's U12 block (nb x cw, staged in LDS) to rows k0.., columns c0..
// of the matrix, consecutive lanes down each column (whole cache lines).
template <typename T2>
__device__ __forceinline__ void u12_store(T2 *A, int N, int k0, int c0, int nb, int cw,
                                          const T2 (*sX)[kStripW + 1]) {
  constexpr int kSi = kLuNB * kStripW / kLuThreads;
#pragma unroll
  for (int it = 0; it < kSi; ++it) {
    const int e = threadIdx.x + it * kLuThreads, r = e % kLuNB, c = e / kLuNB;
    if (r < nb && c < cw) A[(k0 + r) + (c0 + c) * N] = sX[r][c];
  }
}

// One workgroup per (matrix, 64-column strip).  Strips left of the block
// only receive the block's row permutation; strips right of it also get
// U12 = L11^{-1} A12 and the update A22 -= L21 U12 down the whole strip.
// occupancy target: FP64 strips are LDS-bound at 2 workgroups per CU, FP32
// strips fit 4 (register budget 256 and 128 per lane)
//
// SYM: the symmetric form (complex symmetric A = A^T factored without row
// interchanges, the panel kernel checking that partial pivoting would have
// made none).  The reduced matrix stays symmetric, so that U12 = D1 L21^T
// (D1 the diagonal of U11) comes from the block's own L21 rows of the strip's
// columns, with no product and no row permutation, and only the tiles on and
// below the diagonal are updated: A22 -= L21 U12 for rows >= the strip's
// first column.  U12 is still stored, so that the factors take the usual LU
// form (unit lower L, upper U, identity permutation) for the solves; the
// part of the matrix strictly above the diagonal blocks is otherwise never
// read again and is left stale.
//
// H16 (T = float): the trailing update's products on the FP16 matrix cores
// (16x16x16 f16 MFMA, FP32 accumulation): L21 and U12 rounded to FP16 as
// they enter the products, the factors kept in FP32 -- the low-precision
// factorisation of GMRES-IR, whose FP64 GMRES recovers the accuracy.
template <typename T, bool SYM = false, bool H16 = false>
__global__ __launch_bounds__(kLuThreads, sizeof(T) == 8 ? 2 : 3)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 2 : 3, sizeof(T) == 8 ? 2 : 3))) void lu_strip_kernel(
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
  if (redo_skips(only_failed, status, mat)) return;
  T2 *A = Abase + (long long)mat * mstride;
  const int *swp = swapbase + (long long)mat * kSwapStride;
  const int tid = threadIdx.x;
  const int nb = min(kLuNB, N - k0);
  const bool right = s >= nleft;
  const int c0 = right ? k0 + nb + (s - nleft) * kStripW : s * kStripW;
  const int cw = min(kStripW, (right ? N : k0) - c0);
  // ---- row permutation as a gather (read every source, then write), 32
  // columns at a time.  No global access of this kernel sits under a bounds
  // branch: an access under a divergent branch is followed by a wait for it,
  // which serialises a whole loop of them on the memory latency.  Indices
  // are clamped into range instead; a clamped pair entry (pair npair - 1,
  // column cw - 1) copies exactly what that entry's own thread copies, so
  // its store is a duplicate of the same value.
  const int npair = SYM ? 0 : swp[0];
  for (int e = tid; e < 2 * npair; e += kLuThreads) spair[e] = swp[1 + e];
  if (!SYM) __syncthreads();
  if (npair > 0) {
    constexpr int kGi = 32 * kSwapMax / kLuThreads;  // entries per thread per half
    const int nit = (32 * npair + kLuThreads - 1) / kLuThreads;
    for (int half = 0; half < 2; ++half) {
      const int cb0 = half * 32;
      if (cb0 >= cw) break;
      // real and imaginary parts in scalar arrays, every element set
      // (entries past the last pair load duplicates of its row): both keep
      // the arrays in registers
      T gx[kGi], gy[kGi];
      int dst[kGi];  // destination element within the matrix
#pragma unroll
      for (int it = 0; it < kGi; ++it) {
        const int e = tid + it * kLuThreads;
        const int c = min(cb0 + (e & 31), cw - 1), j = min(e >> 5, npair - 1);
        const int col = (c0 + c) * N;
        const T2 v = A[spair[2 * j + 1] + col];
        gx[it] = v.x;
        gy[it] = v.y;
        dst[it] = spair[2 * j] + col;
      }
      __syncthreads();  // every source read before any row is overwritten
#pragma unroll
      for (int it = 0; it < kGi; ++it)
        if (it < nit) A[dst[it]] = mk<T>(gx[it], gy[it]);  // uniform test
      __syncthreads();
    }
  }
  if (!right) return;
  // a block with columns to its right is a full one (nb < 64 only for the
  // last block of a matrix); the update below relies on it
  if (nb < kLuNB) return;
  // ---- U12 for this strip: X = L11^{-1} A12 on the matrix cores, with
  // the inverse from the panel kernel; A12 in LDS as the B operand, the
  // product kept in registers, then written over it (and to memory)
  const int lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
  if constexpr (SYM) {
    // U12[r][c] = d_r L(c0 + c, k0 + r): the panel's rows c0.. of its
    // columns, contiguous in c for each r; kept in LDS as the update's B
    // operand and stored from there (the U part of the factors)
    constexpr int kSi = kLuNB * kStripW / kLuThreads;
    T2 lv[kSi], dv[kSi];
#pragma unroll
    for (int it = 0; it < kSi; ++it) {
      const int e = tid + it * kLuThreads, r = min(e / kStripW, nb - 1), c = e % kStripW;
      lv[it] = A[(c0 + min(c, cw - 1)) + (long long)(k0 + r) * N];
      dv[it] = A[(k0 + r) + (long long)(k0 + r) * N];
    }
#pragma unroll
    for (int it = 0; it < kSi; ++it) {
      const int e = tid + it * kLuThreads, r = e / kStripW, c = e % kStripW;
      const bool ok = r < nb && c < cw;
      const T2 d = dv[it], l = lv[it];
      const T2 v = ok ? mk<T>(d.x * l.x - d.y * l.y, d.x * l.y + d.y * l.x) : mk<T>(T(0), T(0));
      sX[r][c] = v;
    }
    __syncthreads();
    u12_store(A, N, k0, c0, nb, cw, sX);
  } else {
    constexpr int kSi = kLuNB * kStripW / kLuThreads;
    T gx[kSi], gy[kSi];
#pragma unroll
    for (int it = 0; it < kSi; ++it) {
      // consecutive lanes down a column of A12
      const int e = tid + it * kLuThreads, r = e % kLuNB, c = e / kLuNB;
      const T2 v = A[(k0 + min(r, nb - 1)) + (c0 + min(c, cw - 1)) * N];
      gx[it] = v.x;
      gy[it] = v.y;
    }
#pragma unroll
    for (int it = 0; it < kSi; ++it) {
      const int e = tid + it * kLuThreads, r = e % kLuNB, c = e / kLuNB;
      const bool ok = r < nb && c < cw;
      sX[r][c] = mk<T>(ok ? gx[it] : T(0), ok ? gy[it] : T(0));
    }
    __syncthreads();
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
    // every fragment of this wave's rows of L11^{-1} (64 x 64, always in
    // bounds) in flight at once
    T2 fl[kLuNB / 4];
#pragma unroll
    for (int st = 0; st < kLuNB / 4; ++st) fl[st] = lv[arow + kLuNB * (4 * st + lk)];
    __builtin_amdgcn_sched_barrier(0);
    // all 16 steps even for a partial last block (nb < 64): there the
    // inverse is zero outside the block and so are the staged rows >= nb,
    // and a loop without an exit lets every load above stay in flight
#pragma unroll
    for (int st = 0; st < kLuNB / 4; ++st) {
      const int kk = 4 * st;
      const T2 fa = fl[st];
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
        sX[row][col] = mk<T>(xr[cb][r], xi[cb][r]);
      }
    __syncthreads();
    u12_store(A, N, k0, c0, nb, cw, sX);
  }
  // ---- A22 -= L21 U12 down the strip: each wave owns 16 rows x 64 columns
  // (the symmetric form: from the strip's diagonal tile down).  The matrix
  // cores form the transposed tile, U12^T L21^T (U12 the A operand, L21 the
  // B operand), so that an accumulator's 16 columns are 16 consecutive rows
  // of the column-major matrix: lane (li, g) register r holds the entry at
  // row rw + li, column 16 cb + crow(g, r), and a C load or store
  // instruction touches whole cache lines (four in FP32, eight in FP64)
  // rather than a part of sixteen.  TR = false is the direct form.
  constexpr bool TR = true;
  for (int r0 = SYM ? c0 : k0 + nb; r0 < N; r0 += 64) {
    const int rw = r0 + 16 * wave;  // first row of this wave
    if (rw >= N) continue;
    // C tile and L21 fragments in one round trip, indices clamped (no
    // selects either: the compiler turns a select of a load back into a
    // branch).  Clamped C entries (rows >= N, columns >= cw) only feed
    // outputs that are never stored; the L21 columns need no clamp (the
    // block is a full one).  The products
    // accumulate from zero and C is added at the end, so that the C loads
    // have the whole product chain to arrive.
    // Issue order: the L21 fragments (needed first, in step order), then C;
    // memory returns count down in issue order, so step st waits for its
    // own fragment only.  The scheduling barrier keeps the compiler from
    // sinking the loads towards their uses.
    const int arow = min(rw + li, N - 1) + k0 * N;
    // fragment st: column 4 st + lk of the block (FP32/FP64 steps of k = 4);
    // with H16, steps of k = 16: fa[4 s + e] is column 16 s + 4 lk + e
    T2 fa[kLuNB / 4];
#pragma unroll
    for (int st = 0; st < kLuNB / 4; ++st) {
      const int kc = H16 ? 16 * (st >> 2) + 4 * lk + (st & 3) : 4 * st + lk;
      fa[st] = A[arow + kc * N];
    }
    T cx[4][4], cy[4][4];
    if constexpr (TR) {
      // 32-bit byte offsets from the matrix's (uniform) base: one register
      // per address instead of a 64-bit pointer
      const int rowc = min(rw + li, N - 1);  // clamped row of this lane
      // the strip's width, opaque per tile: its clamps are recomputed here
      // rather than sixteen column offsets held through the loop
      int cwt = cw;
      asm volatile("" : "+v"(cwt));
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int colc = c0 + min(cb * 16 + Mma<T>::crow(lk, r), cwt - 1);
          const unsigned off = (unsigned)(rowc + colc * N) * (unsigned)sizeof(T2);
          const T2 v = *(const T2 *)((const char *)A + off);
          cx[cb][r] = v.x;
          cy[cb][r] = v.y;
        }
    } else {
      const int ccl = c0 + min(li, cw - 1);  // clamped column of cb = 0
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int colc = min(ccl + cb * 16, c0 + cw - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = min(rw + Mma<T>::crow(lk, r), N - 1);
          const T2 v = A[row + colc * N];
          cx[cb][r] = v.x;
          cy[cb][r] = v.y;
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    acc_t cr[4], ci[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cr[cb][r] = 0;
        ci[cb][r] = 0;
      }
    if constexpr (H16) {
      // four steps of k = 16: lane (li, lk) holds k = 16 s + 4 lk + e of
      // row li (A) and of column li (B), e = 0..3
      typedef _Float16 h4 __attribute__((ext_vector_type(4)));
#pragma unroll
      for (int s4 = 0; s4 < kLuNB / 16; ++s4) {
        h4 ar, ai, pai;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const T2 f = fa[4 * s4 + e];
          ar[e] = (_Float16)(-f.x);
          ai[e] = (_Float16)(-f.y);
          pai[e] = (_Float16)f.y;
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          h4 br, bi;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const T2 bv = sX[16 * s4 + 4 * lk + e][cb * 16 + li];
            br[e] = (_Float16)bv.x;
            bi[e] = (_Float16)bv.y;
          }
          // C - A B:  re += (-Ar) Br + Ai Bi ;  im += (-Ar) Bi + (-Ai) Br
          cr[cb] = __builtin_amdgcn_mfma_f32_16x16x16f16(br, ar, cr[cb], 0, 0, 0);
          ci[cb] = __builtin_amdgcn_mfma_f32_16x16x16f16(bi, ar, ci[cb], 0, 0, 0);
          cr[cb] = __builtin_amdgcn_mfma_f32_16x16x16f16(bi, pai, cr[cb], 0, 0, 0);
          ci[cb] = __builtin_amdgcn_mfma_f32_16x16x16f16(br, ai, ci[cb], 0, 0, 0);
        }
      }
    } else if constexpr (sizeof(T) == 4) {
      // three real products per complex one (the FP32 factors, which the
      // refinement corrects): T1 = Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi), so that
      // Re AB = T1 - T2 and Im AB = T3 - T1 - T2; every step's three chains
      // accumulate from zero and are combined at the end
      acc_t c3[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) c3[cb][r] = 0;
#pragma unroll
      for (int st = 0; st < kLuNB / 4; ++st) {
        const T ar = fa[st].x, ai = fa[st].y, as = fa[st].x + fa[st].y;
        const int krow = 4 * st + lk;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          const T2 bv = sX[krow][cb * 16 + li];
          cr[cb] = Mma<T>::run(bv.x, ar, cr[cb]);
          ci[cb] = Mma<T>::run(bv.y, ai, ci[cb]);
          c3[cb] = Mma<T>::run(bv.x + bv.y, as, c3[cb]);
        }
      }
      // C - A B: cr = T1, ci = T2 -> (T2 - T1, T1 + T2 - T3)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const T t1 = cr[cb][r], t2 = ci[cb][r];
          cr[cb][r] = t2 - t1;
          ci[cb][r] = (t1 + t2) - c3[cb][r];
        }
    } else {
#pragma unroll
    // all 16 steps (zero fragments and rows beyond a partial block)
    for (int st = 0; st < kLuNB / 4; ++st) {
      const T ar = -fa[st].x, ai = -fa[st].y, pai = fa[st].y;
      T br[4], bi[4];
      const int krow = 4 * st + lk;
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const T2 bv = sX[krow][cb * 16 + li];
        br[cb] = bv.x;
        bi[cb] = bv.y;
      }
      // C - A B:  re += (-Ar) Br + Ai Bi ;  im += (-Ar) Bi + (-Ai) Br
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        cr[cb] = Mma<T>::run(br[cb], ar, cr[cb]);
        ci[cb] = Mma<T>::run(bi[cb], ar, ci[cb]);
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        cr[cb] = Mma<T>::run(bi[cb], pai, cr[cb]);
        ci[cb] = Mma<T>::run(br[cb], ai, ci[cb]);
      }
    }
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = TR ? rw + li : rw + Mma<T>::crow(lk, r);
        const int col = TR ? cb * 16 + Mma<T>::crow(lk, r) : cb * 16 + li;
        const T vx = cx[cb][r] + cr[cb][r], vy = cy[cb][r] + ci[cb][r];
        if (row < N && col < cw) {
          if constexpr (TR)
            *(T2 *)((char *)A + (unsigned)(row + (c0 + col) * N) * (unsigned)sizeof(T2)) = mk<T>(vx, vy);
          else
            A[row + (c0 + col) * N] = mk<T>(vx, vy);
        }
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

// acc -= sum_{c < n} col[c * stride] * y[c]: column sweep of one row with
// the next batch of 8 loads in flight while the current one is used (n >= 1).
// The loads take their column clamped to n - 1 instead of a test per load:
// such tests are loop-invariant masks the compiler keeps (and spills) across
// the sweep; the values past n are never accumulated.
template <typename P>
__device__ __forceinline__ double2 row_sweep(double2 acc, const P *col, long long stride,
                                             const double2 *y, int n) {
  constexpr int B = 8;
  P cur[B], nxt[B];
#pragma unroll
  for (int u = 0; u < B; ++u) nxt[u] = col[(long long)min(u, n - 1) * stride];
#pragma unroll 1
  for (int c0 = 0; c0 < n; c0 += B) {
#pragma unroll
    for (int u = 0; u < B; ++u) cur[u] = nxt[u];
#pragma unroll
    for (int u = 0; u < B; ++u) nxt[u] = col[(long long)min(c0 + B + u, n - 1) * stride];
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (c0 + u < n) acc = cfms(acc, to_d2(cur[u]), y[c0 + u]);
  }
  return acc;
}

// perm[i] = the original row of row i of P A, for the LAPACK-style row
// interchanges piv (row i swapped with row piv[i], i = 0, 1, ...), so that
// P y is the gather y[perm[i]].  One wave per matrix, the row indices in
// registers (S per lane, N <= 64 S); matrices with status >= 0 are skipped
// when only_failed is set.
template <int S>
__global__ __launch_bounds__(64) void perm_from_piv_kernel(const int *pivbase, int N, int *permbase,
                                                           const int *status, int only_failed) {
  const long long mb = blockIdx.x;
  if (redo_skips(only_failed, status, mb)) return;
  const int *piv = pivbase + mb * N;
  int *perm = permbase + mb * kMaxN;
  const int lane = threadIdx.x;
  int v[S], pv[S];
#pragma unroll
  for (int q = 0; q < S; ++q) {
    v[q] = lane + 64 * q;
    pv[q] = lane + 64 * q < N ? piv[lane + 64 * q] : 0;
  }
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const int nq = min(64, N - 64 * q);
    for (int l = 0; l < nq; ++l) {
      const int i = 64 * q + l;
      const int p = __builtin_amdgcn_readlane(pv[q], l);
      if (p != i) {
        const int x = __builtin_amdgcn_readlane(v[q], l);
        const int y = iget<S>(v, p);
        v[q] = lane == l ? y : v[q];
        iset<S>(v, p, x, lane);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < S; ++q)
    if (lane + 64 * q < N) perm[lane + 64 * q] = v[q];
}

// Diagonal-block solve on wave 0: y[jb, jb + nb) := L11^{-1} y (forward,
// unit lower) or U11^{-1} y (backward).  Lane i holds row jb + i; column c
// of the block is one coalesced load from the factors, issued eight columns
// ahead of its step.  A lane whose entry of column c is not used (rows
// c and above going forward, c and below going backward, rows past nb) loads
// the address of the nearest row that is, so the column costs only the cache
// lines of the triangle it contributes; such values are never applied.  Steps
// past the block are switched off per lane (column index clamped for the
// lane read), not by a branch.
template <typename T>
__device__ __forceinline__ void diag_block_solve(const cplx_t<T> *LU, int N, int jb, int nb,
                                                 bool fwd, double2 *y) {
  constexpr int B = 8;
  const int lane = threadIdx.x & 63;
  const int rl = min(lane, nb - 1);
  const cplx_t<T> *blk = LU + jb + (long long)jb * N;
  double2 yi = lane < nb ? y[jb + lane] : make_double2(0.0, 0.0);
  cplx_t<T> cur[B], nxt[B];
  if (fwd) {
    // column c (clamped to the block), row max(lane, c + 1) clamped to the block
    auto ld = [&](int c) {
      const int cc = min(c, nb - 1);
      return blk[max(rl, min(cc + 1, nb - 1)) + (long long)cc * N];
    };
#pragma unroll
    for (int u = 0; u < B; ++u) nxt[u] = ld(u);
#pragma unroll 1
    for (int c0 = 0; c0 < nb - 1; c0 += B) {
#pragma unroll
      for (int u = 0; u < B; ++u) cur[u] = nxt[u];
#pragma unroll
      for (int u = 0; u < B; ++u) nxt[u] = ld(c0 + B + u);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int c = c0 + u;
        const double2 yc = rdlane2(yi, min(c, 63));
        if (lane > c && c < nb - 1) yi = cfms(yi, to_d2(cur[u]), yc);
      }
    }
  } else {
    // column c (clamped at 0), row min(lane, c - 1) clamped at 0
    auto ld = [&](int c) {
      const int cc = max(c, 0);
      return blk[min(rl, max(cc - 1, 0)) + (long long)cc * N];
    };
    const double2 dinv =
        lane < nb ? crcp(to_d2(blk[rl + (long long)rl * N])) : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < B; ++u) nxt[u] = ld(nb - 1 - u);
#pragma unroll 1
    for (int c0 = nb - 1; c0 >= 0; c0 -= B) {
#pragma unroll
      for (int u = 0; u < B; ++u) cur[u] = nxt[u];
#pragma unroll
      for (int u = 0; u < B; ++u) nxt[u] = ld(c0 - B - u);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int c = c0 - u;
        if (lane == c) yi = cmul(yi, dinv);
        const double2 yc = rdlane2(yi, max(c, 0));
        if (lane < c) yi = cfms(yi, to_d2(cur[u]), yc);
      }
    }
  }
  if (lane < nb) y[jb + lane] = yi;
}

// y := (P A)^{-1} y = U^{-1} L^{-1} P y for the factors LU (column-major,
// stride N) and the gather permutation perm; y is in LDS.  Per 64-column
// block: the diagonal block on wave 0, then the rows below (forward) or above
// (backward) swept by the whole workgroup.
template <typename T>
__device__ __forceinline__ void lu_solve_lds(const cplx_t<T> *LU, const int *perm, double2 *y,
                                             int N) {
  const int tid = threadIdx.x, wave = tid >> 6;
  {
    // y := P y as a gather, four rows per thread (kMaxN = 4 x 256)
    static_assert(kMaxN == 4 * kLuThreads, "gather assumes four rows per thread");
    const int i0 = tid, i1 = tid + kLuThreads, i2 = tid + 2 * kLuThreads,
              i3 = tid + 3 * kLuThreads;
    const double2 g0 = y[i0 < N ? perm[i0] : 0], g1 = y[i1 < N ? perm[i1] : 0],
                  g2 = y[i2 < N ? perm[i2] : 0], g3 = y[i3 < N ? perm[i3] : 0];
    __syncthreads();
    if (i0 < N) y[i0] = g0;
    if (i1 < N) y[i1] = g1;
    if (i2 < N) y[i2] = g2;
    if (i3 < N) y[i3] = g3;
  }
  __syncthreads();
  const int nblk = (N + 63) / 64;
  for (int bi = 0; bi < 2 * nblk; ++bi) {
    const bool fwd = bi < nblk;
    const int jb = (fwd ? bi : 2 * nblk - 1 - bi) * 64;
    const int nb = min(64, N - jb);
    if (wave == 0) diag_block_solve<T>(LU, N, jb, nb, fwd, y);
    __syncthreads();
    // rows below (forward) or above (backward) the block
    const int r0 = fwd ? jb + nb : 0, r1 = fwd ? N : jb;
    for (int r = r0 + tid; r < r1; r += kLuThreads)
      y[r] = row_sweep(y[r], LU + r + (long long)jb * N, N, y + jb, nb);
    __syncthreads();
  }
}

// alpha = A^{-1} b from FP64 factors.
__global__ __launch_bounds__(kLuThreads, 2) void lu_solve64_kernel(
    const double2 *LUbase, const int *permbase, int N, long long mstride,
    const double2 *b, double2 *x, long long vstride) {
  __shared__ double2 y[kMaxN];
  const double2 *LU = LUbase + (long long)blockIdx.x * mstride;
  const int *piv = permbase + (long long)blockIdx.x * kMaxN;
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

// rs = bb - A xs for a complex symmetric A held as its lower block triangle
// (64 x 64 blocks (I, J) with I >= J, the diagonal blocks in full, as the
// symmetric form's assembly writes it; A_ij for j beyond i's diagonal block
// is A_ji), every stored element read once: each wave takes the blocks,
// J <= I, numbered row by row, t = wave, wave + 4, ...; lane i is row
// 64 I + i of the block, eight columns' loads in flight at a time (coalesced
// across the lanes).  Every element gives its row's term A_ij x_j (a
// per-lane sum) and, off the diagonal blocks, its column's term A_ij x_i
// (the transposed block's use): the eight columns' terms are summed over the
// 64 lanes in one transposing butterfly (lane pairs 32, 16 and 8 apart each
// halve the values held, then 4, 2, 1 apart add the last one), which leaves
// column u's sum in lane 8u.  The row and column sums go to the wave's own
// partial vector part[wave][N] in LDS, and rs = bb - the four partials
// added in a fixed order: no atomics, reproducible bit for bit.  (Reading
// the strictly lower blocks a second time, down their columns, for the
// transposed terms cost the refinement stage 20% more time.)
// xs, rs: N complex in LDS; part: 4N complex in LDS.  Ends with a barrier.
__device__ void sym_residual_fused(const double2 *__restrict__ A, int N,
                                   const double2 *__restrict__ bb, const double2 *xs,
                                   double2 *rs, double2 *part) {
  static_assert(kLuThreads == 256, "four waves, four partial vectors");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // waves 0..2 accumulate in part[0, 3N), wave 3 in rs itself (free until
  // the residual is formed): 40 KB of LDS in all at N = 512, four
  // workgroups per CU
  for (int e = tid; e < 3 * N; e += kLuThreads) part[e] = make_double2(0.0, 0.0);
  for (int e = tid; e < N; e += kLuThreads) rs[e] = make_double2(0.0, 0.0);
  __syncthreads();
  double2 *pw = wave < 3 ? part + (long long)wave * N : rs;
  const int nbk = (N + 63) >> 6, nblk = nbk * (nbk + 1) / 2;
  const int b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1;
  for (int t = wave; t < nblk; t += 4) {
    int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    const int J = t - I * (I + 1) / 2;
    const int i = 64 * I + lane, jb = 64 * J;
    const int ncol = min(64, N - jb);
    const double m = i < N ? 1.0 : 0.0;  // rows past N contribute nothing
    const double2 xi = xs[min(i, N - 1)];
    const double2 *arow = A + min(i, N - 1);
    double2 racc = make_double2(0.0, 0.0);
    for (int c0 = 0; c0 < 64; c0 += 8) {
      double2 a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = arow[(long long)(jb + min(c0 + u, ncol - 1)) * N];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        // columns past N (clamped loads) and rows past N: zero terms
        const double mu = c0 + u < ncol ? m : 0.0;
        a[u] = make_double2(a[u].x * mu, a[u].y * mu);
        racc = cfma(racc, a[u], xs[jb + min(c0 + u, ncol - 1)]);
      }
      if (I != J) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = cmul(a[u], xi);
        // lanes 32 apart: keep half of the eight, add the partner's half
        double2 w4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double2 snd = b5 ? v[k] : v[k + 4], kep = b5 ? v[k + 4] : v[k];
          w4[k] = make_double2(kep.x + __shfl_xor(snd.x, 32), kep.y + __shfl_xor(snd.y, 32));
        }
        double2 w2[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const double2 snd = b4 ? w4[k] : w4[k + 2], kep = b4 ? w4[k + 2] : w4[k];
          w2[k] = make_double2(kep.x + __shfl_xor(snd.x, 16), kep.y + __shfl_xor(snd.y, 16));
        }
        const double2 snd = b3 ? w2[0] : w2[1], kep = b3 ? w2[1] : w2[0];
        double2 w1 = make_double2(kep.x + __shfl_xor(snd.x, 8), kep.y + __shfl_xor(snd.y, 8));
#pragma unroll
        for (int off = 4; off >= 1; off >>= 1) {
          w1.x += __shfl_xor(w1.x, off);
          w1.y += __shfl_xor(w1.y, off);
        }
        // lane 8u holds the sum of column c0 + u (u = 4 b5 + 2 b4 + b3)
        if ((lane & 7) == 0) {
          const int c = c0 + (lane >> 3);
          if (c < ncol) pw[jb + c] = cadd(pw[jb + c], w1);
        }
      }
    }
    if (i < N) pw[i] = cadd(pw[i], racc);
  }
  __syncthreads();
  for (int r = tid; r < N; r += kLuThreads) {
    const double2 s = cadd(cadd(part[r], part[N + r]), cadd(part[2 * N + r], rs[r]));
    rs[r] = csub(bb[r], s);
  }
  __syncthreads();
}

// Bytes of the dynamic LDS of refine_kernel: x and r, and for the fused
// symmetric residual three more partial vectors (whose first doubles also
// hold the block sums' four wave totals, outside the residual); without it
// room for those four totals.
constexpr size_t refine_lds_bytes(int N, bool lower) {
  return lower ? sizeof(double2) * 5 * (size_t)N : sizeof(double2) * (2 * (size_t)N + 2);
}

// Refined solve: x0 from the FP32 factors, then repeat
//   r = b - A64 x (FP64), d = LU32^{-1} r, x += d
// and stop once the predicted error of the updated x, |d_k| * rho with
// rho = |d_k| / |d_{k-1}| (observed contraction; d_0 = x0), is below tol |x|.
// status[b] = steps taken, or -1 when the cap was hit or the iteration did
// not contract (the caller then redoes the solve in FP64).
// LOWER: A64 holds only its lower block triangle (the symmetric form's
// assembly), the residual by sym_residual_fused.  A template argument, so
// that the other form keeps its register budget.
template <bool LOWER>
__global__ __launch_bounds__(kLuThreads, 4) void refine_kernel(
    const float2 *LUbase, const int *permbase, const double2 *A64base, int N,
    long long mstride, const double2 *b, double2 *x, long long vstride, double tol,
    int max_iter, int *status, double *relres, int later) {
  // dynamic LDS (refine_lds_bytes, sized at launch): x and r, N complex128
  // each (16 KB at N = 512), then with the fused symmetric residual its
  // three partial vectors (40 KB in all at N = 512), else two double2; the
  // block sums' wave totals at refine_dyn + 2N (the partial vectors are
  // only in use inside the residual, between barriers)
  extern __shared__ double2 refine_dyn[];
  double2 *xs = refine_dyn, *rs = refine_dyn + N;
  double *red = (double *)(refine_dyn + 2 * N);
  const long long mb = (long long)blockIdx.x;
  const float2 *LU = LUbase + mb * mstride;
  const int *piv = permbase + mb * kMaxN;
  const double2 *A = A64base + mb * mstride;
  const double2 *bb = b + mb * vstride;
  const int tid = threadIdx.x;
  if (status && status[mb] == -2) {  // zero pivot: leave for the FP64 redo
    for (int i = tid; i < N; i += kLuThreads) x[mb * vstride + i] = make_double2(0.0, 0.0);
    return;
  }
  // a later solve of a matrix already redone in FP64: its FP64 solve follows
  if (later && status && status[mb] < 0) return;
  for (int i = tid; i < N; i += kLuThreads) xs[i] = bb[i];
  __syncthreads();
  lu_solve_lds<float>(LU, piv, xs, N);
  // the initial solve counts as the first correction (from x = 0), so the
  // contraction can be estimated, and the loop stopped, after one step
  double x0n = 0.0;
  for (int i = tid; i < N; i += kLuThreads) x0n += cnorm2(xs[i]);
  double prev = sqrt(block_sum(x0n, red)), last = 0.0;
  int it = 0, done = 0;
  for (; it < max_iter && !done; ++it) {
    // r = b - A x  (each thread owns rows; column sweep, coalesced)
    if constexpr (LOWER) {
      sym_residual_fused(A, N, bb, xs, rs, refine_dyn + 2 * N);
    } else {
      for (int r = tid; r < N; r += kLuThreads) rs[r] = row_sweep(bb[r], A + r, N, xs, N);
      __syncthreads();
    }
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
    if (status) status[mb] = done ? (it > 0 ? it : 1) : (later ? kStatusLateFail : -1);
    if (relres) relres[mb] = last;
  }
}

// Completes the upper block triangle of complex symmetric matrices held as
// their lower block triangle (A_IJ = A_JI^T for 64 x 64 blocks I < J), for
// the matrices the redo mode selects, before their FP64 redo with partial
// pivoting.  Grid: (64 x 64 blocks above the diagonal, count); 32 x 32
// quarters through LDS.
__global__ __launch_bounds__(256) void symmetrize_kernel(double2 *Abase, int N, long long mstride,
                                                          const int *status, int mode) {
  __shared__ double2 t[32][33];
  const long long mb = blockIdx.y;
  if (redo_skips(mode, status, mb)) return;
  const int nbk = (N + 63) / 64;
  // upper block (I, J), I < J, from the block index
  int I = 0, rem = blockIdx.x;
  while (rem >= nbk - 1 - I) {
    rem -= nbk - 1 - I;
    ++I;
  }
  const int J = I + 1 + rem;
  double2 *A = Abase + mb * mstride;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int qr = 0; qr < 2; ++qr)
    for (int qc = 0; qc < 2; ++qc) {
      // quarter of block (J, I) at rows 64J + 32qr, cols 64I + 32qc, read
      // down its columns, written transposed into block (I, J)
      const int r0 = 64 * J + 32 * qr, c0 = 64 * I + 32 * qc;
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = r0 + tx, c = c0 + ty + 8 * u;
        if (r < N && c < N) t[ty + 8 * u][tx] = A[r + (long long)c * N];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = c0 + tx, c = r0 + ty + 8 * u;  // element (r, c) = (c, r) of the source
        if (r < N && c < N) A[r + (long long)c * N] = t[tx][ty + 8 * u];
      }
    }
}

// refine_kernel for `count` matrices on stream st; lower: A64 holds its
// lower block triangle only.
inline void launch_refine(hipStream_t st, bool lower, int count, const float2 *LU,
                          const int *perm, const double2 *A64, int N, long long ms,
                          const double2 *b, double2 *x, long long vstride, double tol,
                          int max_iter, int *status, double *relres, int later) {
  if (lower)
    refine_kernel<true><<<count, kLuThreads, refine_lds_bytes(N, true), st>>>(
        LU, perm, A64, N, ms, b, x, vstride, tol, max_iter, status, relres, later);
  else
    refine_kernel<false><<<count, kLuThreads, refine_lds_bytes(N, false), st>>>(
        LU, perm, A64, N, ms, b, x, vstride, tol, max_iter, status, relres, later);
}

// After a late redo: the matrices factored in FP64 (status
// kStatusLateFail) are solved with FP64 factors from now on (-1).
__global__ void late_redo_done_kernel(int *status, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count && status[i] == kStatusLateFail) status[i] = -1;
}

// Solve for the matrices whose status is negative (FP64 redo after a
// refined solve that did not converge): x = A^{-1} b from FP64 factors.
__global__ __launch_bounds__(kLuThreads, 2) void solve_failed64_kernel(
    const double2 *LUbase, const int *permbase, int N, long long mstride, const double2 *b,
    double2 *x, long long vstride, const int *status) {
  __shared__ double2 y[kMaxN];
  const long long mb = blockIdx.x;
  if (status[mb] >= 0) return;
  const double2 *LU = LUbase + mb * mstride;
  const int *piv = permbase + mb * kMaxN;
  for (int i = threadIdx.x; i < N; i += kLuThreads) y[i] = b[mb * vstride + i];
  __syncthreads();
  lu_solve_lds<double>(LU, piv, y, N);
  for (int i = threadIdx.x; i < N; i += kLuThreads) x[mb * vstride + i] = y[i];
}

}  // namespace fthms
