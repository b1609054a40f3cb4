// Register-resident panel factorisation for the batched LU (one 1024-thread
// workgroup per matrix).
//
// The m x 64 column block at k0 (m = N - k0 <= 64 RL) is held entirely in
// registers: wave w owns columns 4w .. 4w+3, lane l the block rows l + 64 i
// (i < RL).  Right-looking partial pivoting inside the block with one
// workgroup barrier per column.  Rows are never moved during the
// factorisation: each lane keeps a mask of its rows already chosen as
// pivots, the pivot of column c is the largest |re| + |im| among the rows
// not yet chosen (lowest row index on ties), and the rows are written to
// their final positions when the block is stored.  The wave owning column c
// finds the pivot with a wave reduction, forms the multipliers, publishes
// them and the pivot row in LDS (double-buffered) and updates its own later
// columns; after the barrier the waves owning later columns fetch the pivot
// row's values with readlane and apply the rank-1 update.  Wave 0 keeps the
// row bookkeeping (position of every row, row at every position), from
// which the LAPACK-style pivot sequence and the block's net permutation
// follow.  The block is loaded once and stored once.
//
// Outputs match lu_panel_kernel (up to the choice among exactly tied pivot
// candidates): the factored block, absolute pivots, the
// block's net row permutation as (dst, src) pairs, and L11^{-1} (64 x 64,
// column-major, zero above the diagonal), computed at the end by forward
// substitution from L11 staged in LDS.
//
// Arithmetic is in the storage precision T.  Register budget: RL x 4
// complex values of T per lane; the launch bound of 1024 threads leaves 128
// VGPRs per lane, so FP32 blocks up to m = 512 and FP64 blocks up to m = 320
// take this path (larger ones use lu_panel_kernel).
#pragma once

#include "lu.h"

namespace fthms {

constexpr int kPrThreads = 1024;
constexpr int kPrWaves = kPrThreads / 64;  // 16 waves x 4 columns = 64

// Lane permutations for the pivot search, all without LDS: DPP quad
// permutations and row mirrors inside 16-lane rows, then the gfx950
// row-swap instructions across rows and across the two 32-lane halves.
// After each step a lane holds its own value and its partner's.
template <int CTRL> __device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ __forceinline__ float dpp_v(float x) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(x)));
}
template <int CTRL> __device__ __forceinline__ double dpp_v(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = dpp_i<CTRL>((int)(b & 0xffffffffLL)), hi = dpp_i<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T> __device__ __forceinline__ void swap_pair16(T &a, T &b);
template <> __device__ __forceinline__ void swap_pair16<int>(int &a, int &b) {
  const auto r = __builtin_amdgcn_permlane16_swap(a, a, false, false);
  a = r[0];
  b = r[1];
}
template <> __device__ __forceinline__ void swap_pair16<float>(float &a, float &b) {
  int x = __float_as_int(a), y;
  swap_pair16<int>(x, y);
  a = __int_as_float(x);
  b = __int_as_float(y);
}
template <> __device__ __forceinline__ void swap_pair16<double>(double &a, double &b) {
  const long long v = __double_as_longlong(a);
  int lo = (int)(v & 0xffffffffLL), hi = (int)(v >> 32), lo2, hi2;
  swap_pair16<int>(lo, lo2);
  swap_pair16<int>(hi, hi2);
  a = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  b = __longlong_as_double(((long long)hi2 << 32) | (unsigned int)lo2);
}
template <typename T> __device__ __forceinline__ void swap_pair32(T &a, T &b);
template <> __device__ __forceinline__ void swap_pair32<int>(int &a, int &b) {
  const auto r = __builtin_amdgcn_permlane32_swap(a, a, false, false);
  a = r[0];
  b = r[1];
}
template <> __device__ __forceinline__ void swap_pair32<float>(float &a, float &b) {
  int x = __float_as_int(a), y;
  swap_pair32<int>(x, y);
  a = __int_as_float(x);
  b = __int_as_float(y);
}
template <> __device__ __forceinline__ void swap_pair32<double>(double &a, double &b) {
  const long long v = __double_as_longlong(a);
  int lo = (int)(v & 0xffffffffLL), hi = (int)(v >> 32), lo2, hi2;
  swap_pair32<int>(lo, lo2);
  swap_pair32<int>(hi, hi2);
  a = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  b = __longlong_as_double(((long long)hi2 << 32) | (unsigned int)lo2);
}
// Wave-wide argmax of (best, brow): largest value, smallest row on ties;
// every lane ends with the result.  Two reductions: the wave's largest
// value, then the smallest row among the lanes holding it (each lane's brow
// is already its smallest row reaching its best, so this is the smallest
// row of the wave reaching the maximum).  Values are never NaN here.
template <typename T> __device__ __forceinline__ void wave_argmax(T &best, int &brow) {
  T m = best, m2;
  m = fmax(m, dpp_v<0xB1>(m));   // lane ^ 1
  m = fmax(m, dpp_v<0x4E>(m));   // lane ^ 2
  m = fmax(m, dpp_v<0x141>(m));  // mirror in 8
  m = fmax(m, dpp_v<0x140>(m));  // mirror in 16
  swap_pair16<T>(m, m2);
  m = fmax(m, m2);
  swap_pair32<T>(m, m2);
  m = fmax(m, m2);
  int r = best == m ? brow : 0x7fffffff, r2;
  r = min(r, dpp_i<0xB1>(r));
  r = min(r, dpp_i<0x4E>(r));
  r = min(r, dpp_i<0x141>(r));
  r = min(r, dpp_i<0x140>(r));
  swap_pair16<int>(r, r2);
  r = min(r, r2);
  swap_pair32<int>(r, r2);
  r = min(r, r2);
  best = m;
  brow = r;
}

template <typename T> __device__ __forceinline__ cplx_t<T> tmul(cplx_t<T> a, cplx_t<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a - b c
template <typename T>
__device__ __forceinline__ cplx_t<T> tfms(cplx_t<T> a, cplx_t<T> b, cplx_t<T> c) {
  return mk<T>(a.x - b.x * c.x + b.y * c.y, a.y - b.x * c.y - b.y * c.x);
}
// 1 / a from the hardware reciprocal (about 1 ulp; FP64 refined by two
// Newton steps), scaled by max(|re|, |im|) against over- and underflow.
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double hw_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}
template <typename T> __device__ __forceinline__ cplx_t<T> trcp(cplx_t<T> a) {
  const T s = fabs(a.x) > fabs(a.y) ? fabs(a.x) : fabs(a.y);
  const T rs = hw_rcp(s);
  const T ar = a.x * rs, ai = a.y * rs;
  const T rd = hw_rcp(ar * ar + ai * ai) * rs;
  return mk<T>(ar * rd, -ai * rd);
}

template <typename T, int RL> struct PanelRegSmem {
  cplx_t<T> lbuf[2][64 * RL];  // multipliers of the current column
  int pinfo[2];                // its pivot row (block row index)
  int ipiv[kLuNB];             // LAPACK-style pivots (block positions)
  int posv[64 * RL];           // final position of every block row
  int zero_pivot;
  int count;
  cplx_t<T> lt[kLuNB][kLuNB];  // L11 transposed: lt[s][r] = L(r, s)
};

// Value of row p (slot p >> 6, lane p & 63) of column J, as a scalar.  The
// slot is uniform; readlane is convergent, so the compiler keeps the slot
// test as a scalar branch rather than selecting across all slots.
template <typename T, int RL, int J>
__device__ __forceinline__ cplx_t<T> row_value(const cplx_t<T> (&a)[RL][4], int p) {
  const int sp = p >> 6, lp = p & 63;
  cplx_t<T> y = rdlane2(a[0][J], lp);
#pragma unroll
  for (int i = 1; i < RL; ++i)
    if (i == sp) y = rdlane2(a[i][J], lp);
  return y;
}

// One column c = 4 cw + J of the block.  used: bit i set if row lane + 64 i
// has been chosen as a pivot or lies past the block.  rowat/pos (wave 0): row at each position,
// position of each row.
template <typename T, int RL, int J, bool PIV>
__device__ __forceinline__ void panel_reg_column(cplx_t<T> (&a)[RL][4], int &used,
                                                 int (&rowat)[RL], int (&pos)[RL], int w, int cw,
                                                 int m, int &zero_col, int &would_pivot,
                                                 PanelRegSmem<T, RL> &sm) {
  typedef cplx_t<T> T2;
  const int lane = threadIdx.x & 63;
  const int c = 4 * cw + J, b = c & 1;
  int p;
  if (w == cw) {
    // the owner's work is the critical path: raise its issue priority
    __builtin_amdgcn_s_setprio(2);
    // magnitudes |re| + |im| are formed in FP64 whatever the storage
    // precision
    double best = -1.0;
    if constexpr (PIV) {
      // pivot search in column J over the rows not yet chosen; a NaN entry
      // ranks below every number so that a row is always found
      int brow = 0x7fffffff;
#pragma unroll
      for (int i = 0; i < RL; ++i) {
        const bool ok = ((used >> i) & 1) == 0;
        double mag = fabs((double)a[i][J].x) + fabs((double)a[i][J].y);
        mag = mag == mag ? mag : -0.5;
        const bool take = ok & (mag > best);
        best = take ? mag : best;
        brow = take ? lane + 64 * i : brow;
      }
      wave_argmax<double>(best, brow);
      p = __builtin_amdgcn_readfirstlane(brow);
    } else {
      p = c;
    }
    used |= lane == (p & 63) ? 1 << (p >> 6) : 0;
    if (PIV && lane == 0) sm.pinfo[b] = p;
    T2 u[4];
    u[0] = row_value<T, RL, 0>(a, p);
    u[1] = row_value<T, RL, 1>(a, p);
    u[2] = row_value<T, RL, 2>(a, p);
    u[3] = row_value<T, RL, 3>(a, p);
    if constexpr (!PIV) {
      // the diagonal is the pivot; partial pivoting would have taken another
      // row if one below is strictly larger (ties keep the first index):
      // flag that, lane by lane, with no reduction on the critical path
      best = fabs((double)u[J].x) + fabs((double)u[J].y);
#pragma unroll
      for (int i = 0; i < RL; ++i) {
        const bool ok = ((used >> i) & 1) == 0;
        const double mag = fabs((double)a[i][J].x) + fabs((double)a[i][J].y);
        would_pivot |= (ok & (mag > best)) ? 1 : 0;
      }
    }
    const bool nz = best > 0.0;
    // pivot reciprocal: FP64 factors in FP64; FP32 factors (which the
    // refinement corrects) from the FP32 hardware reciprocal, which keeps
    // the owner's step per column short
    T2 inv = mk<T>(T(0), T(0));
    if (nz) {
      if constexpr (sizeof(T) == 4) inv = trcp<T>(u[J]);
      else inv = trcp<double>(to_d2(u[J]));
    }
#pragma unroll
    for (int i = 0; i < RL; ++i) {
      const bool below = ((used >> i) & 1) == 0;
      const T2 l = below ? tmul<T>(a[i][J], inv) : mk<T>(T(0), T(0));
      if (below) a[i][J] = l;
      sm.lbuf[b][lane + 64 * i] = l;
#pragma unroll
      for (int j = J + 1; j < 4; ++j) a[i][j] = tfms<T>(a[i][j], l, u[j]);
    }
    // first exactly zero pivot of this wave's columns (1-based, 0: none)
    if (!nz && zero_col == 0) zero_col = c + 1;
    __builtin_amdgcn_s_setprio(0);
  }
  __syncthreads();
  if (w != cw) {
    if constexpr (PIV) p = __builtin_amdgcn_readfirstlane(sm.pinfo[b]);
    else p = c;
    used |= lane == (p & 63) ? 1 << (p >> 6) : 0;
    if (w > cw) {
      T2 u[4];
      u[0] = row_value<T, RL, 0>(a, p);
      u[1] = row_value<T, RL, 1>(a, p);
      u[2] = row_value<T, RL, 2>(a, p);
      u[3] = row_value<T, RL, 3>(a, p);
#pragma unroll
      for (int i = 0; i < RL; ++i) {
        const T2 l = sm.lbuf[b][lane + 64 * i];
#pragma unroll
        for (int j = 0; j < 4; ++j) a[i][j] = tfms<T>(a[i][j], l, u[j]);
      }
    }
  }
  if (PIV && w == 0) {
    // bookkeeping: row p moves to position c, the row there to p's position
    const int r = iget<RL>(pos, p);
    const int x = __builtin_amdgcn_readlane(rowat[0], c);
    iset<RL>(rowat, r, x, lane);
    iset<RL>(rowat, c, p, lane);
    iset<RL>(pos, x, r, lane);
    iset<RL>(pos, p, c, lane);
    if (lane == 0) sm.ipiv[c] = r;
  }
}

// PIV = false: the symmetric form of the batched LU (lu.h) -- no row
// interchanges (the diagonal is every column's pivot), no permutation and no
// L11^{-1}; a column where partial pivoting would have chosen another row
// makes the status -2 like a zero pivot, so that the caller solves that
// matrix with a pivoting factorisation instead.
template <typename T, int RL, bool PIV = true>
__global__ __launch_bounds__(kPrThreads) void lu_panel_reg_kernel(
    cplx_t<T> *Abase, int N, long long mstride, int k0, int *pivbase, int *swapbase,
    cplx_t<T> *Linv, int *status, int only_failed, int mrows = 1 << 30) {
  typedef cplx_t<T> T2;
  __shared__ PanelRegSmem<T, RL> sm;
  const long long mb = blockIdx.x;
  if (redo_skips(only_failed, status, mb)) return;
  T2 *A = Abase + mb * mstride;
  int *piv = pivbase + mb * N;
  int *swp = swapbase + mb * kSwapStride;
  T2 *Li = Linv + mb * (kLuNB * kLuNB);
  const int tid = threadIdx.x, lane = tid & 63;
  // wave index as a scalar, so that owner/follower branches are uniform
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  // mrows: factor only the top mrows rows of the column block (the
  // diagonal block of the symmetric form's two-launch panel)
  const int m = min(N - k0, mrows), nb = min(kLuNB, m);
  // this wave's first column, row k0 (a scalar base; lanes add row offsets)
  T2 *colp = A + k0 + (long long)(k0 + 4 * w) * N;
  // The block, loaded with row and column indices clamped into it: rows past
  // the block are marked used below (never pivots, zero multipliers, never
  // stored) and columns past a partial block are never factored or stored,
  // so their values do not matter; no per-slot mask is needed here.
  const T2 *blk = A + k0 + (long long)k0 * N;
  T2 a[RL][4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const long long coff = (long long)min(4 * w + j, nb - 1) * N;
#pragma unroll
    for (int i = 0; i < RL; ++i) a[i][j] = blk[min(lane + 64 * i, m - 1) + coff];
  }
  // used: bit i set if row lane + 64 i is a pivot already or lies past the
  // block (rows >= m are marked from the start, so that one bit test
  // excludes both and no per-slot row mask stays live across the loop)
  int used = 0, rowat[RL], pos[RL];
#pragma unroll
  for (int i = 0; i < RL; ++i) used |= lane < m - 64 * i ? 0 : 1 << i;
#pragma unroll
  for (int i = 0; i < RL; ++i) rowat[i] = pos[i] = lane + 64 * i;
  if (tid == 0) sm.zero_pivot = 0x7fffffff;
  int zero_col = 0, would_pivot = 0;
  __syncthreads();
  // the column loop touches no global memory, so its barriers wait on LDS only
  for (int cw = 0; 4 * cw < nb; ++cw) {
    // nb is a multiple of 4 except in a last, partial block
    panel_reg_column<T, RL, 0, PIV>(a, used, rowat, pos, w, cw, m, zero_col, would_pivot, sm);
    if (4 * cw + 1 < nb)
      panel_reg_column<T, RL, 1, PIV>(a, used, rowat, pos, w, cw, m, zero_col, would_pivot, sm);
    if (4 * cw + 2 < nb)
      panel_reg_column<T, RL, 2, PIV>(a, used, rowat, pos, w, cw, m, zero_col, would_pivot, sm);
    if (4 * cw + 3 < nb)
      panel_reg_column<T, RL, 3, PIV>(a, used, rowat, pos, w, cw, m, zero_col, would_pivot, sm);
  }
  if constexpr (!PIV) {
    // rows stay where they are; a flagged column counts as a zero pivot
    const bool flag = __builtin_amdgcn_ballot_w64(would_pivot != 0) != 0;
    if (lane == 0 && (flag || zero_col)) atomicMin(&sm.zero_pivot, 1);
    __syncthreads();
    if (tid < nb) piv[k0 + tid] = k0 + tid;
    const int nslot = (m - lane + 63) >> 6;
#pragma unroll
    for (int i = 0; i < RL; ++i) {
      if (i < nslot) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (4 * w + j < nb) colp[lane + 64 * i + (long long)j * N] = a[i][j];
      }
    }
    if (tid == 0) {
      swp[0] = 0;
      const bool bad = sm.zero_pivot != 0x7fffffff;
      if (k0 == 0) status[mb] = panel_status(only_failed, bad);
      else if (bad) status[mb] = -2;
    }
    return;
  }
  // wave 0 publishes the final positions and the block's net permutation
  // (pairs "new row dst = old row src"; at most 2 x 64 rows move)
  if (tid == 0) sm.count = 0;
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int i = 0; i < RL; ++i) {
      const int r = lane + 64 * i;
      if (r < m) {
        sm.posv[r] = pos[i];
        if (rowat[i] != r) {
          const int e = atomicAdd(&sm.count, 1);
          if (e < kSwapMax) {
            swp[1 + 2 * e] = k0 + r;
            swp[2 + 2 * e] = k0 + rowat[i];
          }
        }
      }
    }
  }
  if (lane == 0 && zero_col) atomicMin(&sm.zero_pivot, zero_col);
  __syncthreads();
  if (tid < nb) piv[k0 + tid] = k0 + sm.ipiv[tid];
  // store every row at its final position; stage L11 (strictly lower part)
  // transposed, by final position
  // this lane's rows in the block: slots i < nslot (written in a form of its
  // own, so that the compiler does not keep masks from the top of the kernel)
  const int nslot = (m - lane + 63) >> 6;
#pragma unroll
  for (int i = 0; i < RL; ++i) {
    if (i < nslot) {
      const int fp = sm.posv[lane + 64 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = 4 * w + j;
        if (col < nb) {
          colp[fp + (long long)j * N] = a[i][j];
          if (fp < kLuNB) sm.lt[col][fp] = fp > col ? a[i][j] : mk<T>(T(0), T(0));
        }
      }
    }
  }
  __syncthreads();
  // L11^{-1} by forward substitution, four columns per wave (lane = row)
  T2 x[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
    x[j] = mk<T>(lane == 4 * w + j ? T(1) : T(0), T(0));
  for (int s = 4 * w; s < nb - 1; ++s) {
    const T2 l = lane < nb ? sm.lt[s][lane] : mk<T>(T(0), T(0));
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = tfms<T>(x[j], l, rdlane2(x[j], s));
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int col = 4 * w + j;
    Li[lane + kLuNB * col] = (col < nb && lane < nb) ? x[j] : mk<T>(T(0), T(0));
  }
  if (tid == 0) {
    swp[0] = min(sm.count, kSwapMax);
    // status: 0 ok, -2 exact zero pivot; a redo (only_failed) stays negative
    // (-1: redone in FP64) so that its solve is redone too
    const bool zero = sm.zero_pivot != 0x7fffffff;
    if (k0 == 0) status[mb] = panel_status(only_failed, zero);
    else if (zero) status[mb] = -2;
  }
}

// The symmetric form's panel in two launches (the default in place of
// lu_panel_reg_kernel<T, RL, false> over the whole column block; same
// outputs, and the same test of partial pivoting, taken on the same updated
// entries): lu_panel_reg_kernel<T, 1, false> with mrows = 64 factors the
// diagonal block, A11 = L11 U11, then lu_rows_sym_kernel the rows below it.
// (A one-wave kernel for the diagonal block, its rows in registers and the
// pivot rows broadcast lane to lane, measured twice as slow: 64 dependent
// broadcast-update rounds per column block with two waves per SIMD.)
//
// lu_rows_sym_kernel: L21 = A21 U11^{-1} for the rows below the diagonal
// block (once that block is factored), one row per thread (so that every
// access to a column is coalesced), by forward substitution
//   s_c = a_c - sum_{j < c} l_j U11(j, c),   l_c = s_c / U11(c, c),
// in four passes of 16 columns; a pass reads the multipliers of the earlier
// passes back from the row it has written.  U11 sits in LDS, column c
// contiguous, read as broadcasts.  |s_c| > |U11(c, c)| (|re| + |im|) means
// partial pivoting would have taken this row: status -2.
// Grid: ((m - 64 + T - 1) / T, count) of T = 64, 128, 192 or 256 threads,
// m = N - k0 > 64.
template <typename T>
__global__ __launch_bounds__(256) void lu_rows_sym_kernel(cplx_t<T> *Abase, int N,
                                                          long long mstride, int k0,
                                                          int *status, int only_failed) {
  typedef cplx_t<T> T2;
  __shared__ T2 us[kLuNB][kLuNB];  // us[c][j] = U11(j, c) for j <= c, 0 below
  __shared__ T2 rinv[kLuNB];
  __shared__ double umag[kLuNB];
  const long long mb = blockIdx.y;
  if (redo_skips(only_failed, status, mb)) return;
  T2 *A = Abase + mb * mstride + k0 + (long long)k0 * N;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < kLuNB * kLuNB; e += nt) {
    const int j = e & 63, c = e >> 6;
    const T2 v = A[j + (long long)c * N];
    us[c][j] = j <= c ? v : mk<T>(T(0), T(0));
  }
  if (tid < kLuNB) {
    const T2 d = A[tid + (long long)tid * N];
    const double dm = fabs((double)d.x) + fabs((double)d.y);
    umag[tid] = dm;
    rinv[tid] = dm > 0.0 ? from_d2<T>(trcp<double>(to_d2(d))) : mk<T>(T(0), T(0));
  }
  __syncthreads();
  const int r = kLuNB + blockIdx.x * nt + tid;
  if (r >= N - k0) return;
  T2 *row = A + r;
  int bad = 0;
  for (int g = 0; g < kLuNB / 16; ++g) {
    T2 s[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) s[c] = row[(long long)(16 * g + c) * N];
    for (int h = 0; h < g; ++h) {
      T2 l[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) l[j] = row[(long long)(16 * h + j) * N];
      const T2 *ub = &us[16 * g][16 * h];
#pragma unroll
      for (int c = 0; c < 16; ++c)
#pragma unroll
        for (int j = 0; j < 16; ++j) s[c] = tfms<T>(s[c], l[j], ub[c * kLuNB + j]);
    }
    const T2 *ud = &us[16 * g][16 * g];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
#pragma unroll
      for (int j = 0; j < c; ++j) s[c] = tfms<T>(s[c], s[j], ud[c * kLuNB + j]);
      if (fabs((double)s[c].x) + fabs((double)s[c].y) > umag[16 * g + c]) bad = 1;
      s[c] = tmul<T>(s[c], rinv[16 * g + c]);
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) row[(long long)(16 * g + c) * N] = s[c];
  }
  if (bad) status[mb] = -2;
}

// The symmetric form's 64 x 64 diagonal block with one wave per matrix (in
// place of lu_panel_reg_kernel<float, 1, false> with mrows = 64; the same
// operations in the same order, so the same factors): lane r holds row r of
// the block in registers, the column steps unrolled so that every entry
// keeps its register.  Step c: lane c publishes its reduced row (from the
// diagonal on) in LDS, every lane reads it back as broadcasts, and lane
// r > c forms L(r, c) = A(r, c) / A(c, c) and updates A(r, j) -= L(r, c) A(c, j)
// for j > c -- one wave, so no workgroup barrier per column.  The tests are
// the register panel's: a row below the diagonal with a strictly larger
// |re| + |im| in column c (FP64 magnitudes), or a zero pivot, gives status
// -2.  (Publishing column c instead, one store per lane, the reduced matrix
// being symmetric in exact arithmetic: 0.4 ms less LU per step, but factors
// whose refinement needed 1.21 instead of 1.07 steps.)
// Grid: ceil(count / kDiagWaves) workgroups of kDiagWaves waves.
constexpr int kDiagWaves = 4;
__global__ __launch_bounds__(64 * kDiagWaves) void lu_diag_sym_kernel(
    float2 *Abase, int N, long long mstride, int k0, int *pivbase, int *swapbase, int *status,
    int count) {
  __shared__ float2 rowv[kDiagWaves][2][kLuNB];  // the published pivot rows
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long mb = (long long)blockIdx.x * kDiagWaves + wave;
  if (mb >= count) return;
  float2 *A = Abase + mb * mstride + k0 + (long long)k0 * N;
  const int nb = min(kLuNB, N - k0);
  // rows and columns past a partial block are clamped copies: they never
  // reach a stored entry or a test
  const int rl = min(lane, nb - 1);
  float2 a[kLuNB];
#pragma unroll
  for (int j = 0; j < kLuNB; ++j) a[j] = A[rl + (long long)min(j, nb - 1) * N];
  int bad = 0;
#pragma unroll
  for (int c = 0; c < kLuNB; ++c) {
    if (c < nb) {
      float2 *row = rowv[wave][c & 1];
      if (lane == c) {
#pragma unroll
        for (int j = c; j < kLuNB; ++j) row[j] = a[j];
      }
      __builtin_amdgcn_wave_barrier();
      const float2 p = row[c];
      const double pm = fabs((double)p.x) + fabs((double)p.y);
      const double mag = fabs((double)a[c].x) + fabs((double)a[c].y);
      if (lane > c && lane < nb && mag > pm) bad = 1;
      if (!(pm > 0.0)) bad = 1;
      float2 inv = make_float2(0.f, 0.f);
      if (pm > 0.0) inv = trcp<float>(p);
      const float2 l = lane > c ? tmul<float>(a[c], inv) : make_float2(0.f, 0.f);
      if (lane > c) a[c] = l;
#pragma unroll
      for (int j = c + 1; j < kLuNB; ++j) a[j] = tfms<float>(a[j], l, row[j]);
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (lane < nb) {
#pragma unroll
    for (int j = 0; j < kLuNB; ++j)
      if (j < nb) A[lane + (long long)j * N] = a[j];
    pivbase[mb * N + k0 + lane] = k0 + lane;
  }
  const bool flag = __builtin_amdgcn_ballot_w64(bad != 0) != 0;
  if (lane == 0) {
    swapbase[mb * kSwapStride] = 0;
    if (k0 == 0) status[mb] = panel_status(0, flag);
    else if (flag) status[mb] = -2;
  }
}

}  // namespace fthms
