// Blocked Cholesky factorisation of the Gram-Hadamard matrix V and the
// row-wise solve F = M V^{-1} of the ALS normal equations.
//
// V is Tp x Tp row-major (Tp = 64 nblk; padding rows/columns hold the
// identity).  Right-looking with two levels of blocking.  Block columns are
// 64 wide and grouped into panels of pw blocks (pw >= nblk: one level).
// Inside a panel, ONE launch per block step: step j updates the panel's
// tiles (i, k), k >= j+1, with block column j on the matrix cores and, for
// the tiles of column j+1, immediately factors the updated diagonal block --
// every workgroup of that column does so redundantly, so no workgroup ever
// waits on another -- and solves its own tile of the column.  In the
// one-level form the blocks beyond column j+2 take their updates in pairs
// (rank 128, every other step), and the backward solve is one dataflow
// launch (STEP_BWD_PAIR, two block columns per dependency hop, after its
// set-up launch STEP_BWD_PREP; or STEP_BWD_FLOW, one per hop; below).  After a panel, one GEMM applies its
// rank-(64 pw) update to the trailing matrix (and, in the forward
// solve, to the right-hand sides): the trailing matrix is read and written
// once per panel instead of once per block column.  The diagonal blocks of
// L are never written back to V (other workgroups of the same launch still
// read the unfactored block); the workgroup that owns one forms
// X = L_kk^{-T} and writes it to `ldiag`, so every forward and backward
// solve step with that block is a single MFMA product.
//
// The sequential parts keep a 64 x 64 tile in registers.  The diagonal
// factorisation uses the "strip" layout (thread t owns row t / 4 and the
// 16 columns (t % 4) + 4u, so the four threads of a row hold one 4-column
// block) and publishes four columns per barrier.  The solve of a panel tile
// with L_kk uses the "block-4" layout (4 rows x 4 columns per thread, the
// solved value broadcast inside a 16-lane DPP row), which needs a quarter
// of the strip layout's LDS reads.
#include <math.h>

#include "kernels.h"
#include "mfma.h"

namespace thccp {

// ---------------------------------------------------------- quad broadcast
template <int K>
__device__ __forceinline__ int qb_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, K * 0x55, 0xF, 0xF, false);
}
template <int K>
__device__ __forceinline__ double qb(double v) {
  union { double d; int i[2]; } a, b;
  a.d = v;
  b.i[0] = qb_int<K>(a.i[0]);
  b.i[1] = qb_int<K>(a.i[1]);
  return b.d;
}
template <int K>
__device__ __forceinline__ float qb(float v) {
  return __int_as_float(qb_int<K>(__float_as_int(v)));
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// ------------------------------------------------------ block-4 solves
// Block-4 layout: thread t owns rows 4g .. 4g+3 (g = t >> 4) and columns
// j + 16v (j = t & 15, v = 0..3) of a 64 x 64 tile, s[4 i + v] = S[4g+i][j+16v].
// The 16 threads of a row group form one 16-lane DPP row, so the solved
// value of column c is broadcast inside the group from lane c % 16
// (row_newbcast) and every thread reads only 4 values of L per column --
// a quarter of the LDS traffic of the strip layout.
template <int N>
__device__ __forceinline__ int rnb_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x150 + N, 0xF, 0xF, false);
}
template <int N>
__device__ __forceinline__ double rnb(double v) {
  union { double d; int i[2]; } a, b;
  a.d = v;
  b.i[0] = rnb_int<N>(a.i[0]);
  b.i[1] = rnb_int<N>(a.i[1]);
  return b.d;
}
template <int N>
__device__ __forceinline__ float rnb(float v) {
  return __int_as_float(rnb_int<N>(__float_as_int(v)));
}
template <typename T>
__device__ __forceinline__ void lds_to_b4(const T* S, T s[16], int g, int j) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) s[4 * i + v] = S[(4 * g + i) * LDT + j + 16 * v];
}
template <typename T>
__device__ __forceinline__ void store_b4(const T s[16], T* gp_, size_t ld, int nrows, int g, int j) {
  const gptr<T> gp = as_global(gp_);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = 4 * g + i;
    if (r < nrows) {
#pragma unroll
      for (int v = 0; v < 4; ++v) gp[(size_t)r * ld + j + 16 * v] = s[4 * i + v];
    }
  }
}
// One column step of the block-4 solves (template recursion keeps every
// register index a compile-time constant: a runtime index would put the
// tile in indexed registers).
//   FWD: S <- S L^{-T}  (solve X L^T = S, columns left to right)
//   BWD: S <- S L^{-1}  (solve X L = S, columns right to left)
// L in LDS row-major (stride LDT), invd[c] = 1 / L[c][c].  The LDS values a
// column needs (1 / L[c][c] and four entries of L) do not depend on the
// solve: each step reads those of the next column, so the reads stay off
// the dependent chain of the columns.
template <typename T, bool FWD, int C>
__device__ __forceinline__ void b4_col_values(const T* L, const T* invd, int j, T& ic, T lk[4]) {
  constexpr int vc = C >> 4, jc = C & 15;
  ic = invd[C];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    // FWD: L[k][C] for k = j + 16 v > C;  BWD: L[C][k] for k < C
    if (FWD ? v >= vc : v <= vc) {
      T x = FWD ? L[(j + 16 * v) * LDT + C] : L[C * LDT + j + 16 * v];
      if (v == vc) x = (FWD ? j > jc : j < jc) ? x : T(0);
      lk[v] = x;
    } else {
      lk[v] = T(0);
    }
  }
}
template <typename T, bool FWD, int C>
struct B4Solve {
  __device__ __forceinline__ static void run(T s[16], const T* L, const T* invd, int j, T ic, const T lk[4]) {
    if constexpr (C >= 0 && C < TB) {
      constexpr int vc = C >> 4, jc = C & 15;
      constexpr int CN = FWD ? C + 1 : C - 1;
      T icn = T(0), lkn[4] = {T(0), T(0), T(0), T(0)};
      if constexpr (CN >= 0 && CN < TB) b4_col_values<T, FWD, CN>(L, invd, j, icn, lkn);
      T x[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = rnb<jc>(s[4 * i + vc] * ic);
      const bool own = j == jc;
#pragma unroll
      for (int i = 0; i < 4; ++i) s[4 * i + vc] = own ? x[i] : s[4 * i + vc];
#pragma unroll
      for (int v = FWD ? vc : 0; v <= (FWD ? 3 : vc); ++v)
#pragma unroll
        for (int i = 0; i < 4; ++i) s[4 * i + v] -= x[i] * lk[v];
      B4Solve<T, FWD, CN>::run(s, L, invd, j, icn, lkn);
    }
  }
};
template <typename T>
__device__ __forceinline__ void b4_fwd(T s[16], const T* L, const T* invd, int j) {
  T ic, lk[4];
  b4_col_values<T, true, 0>(L, invd, j, ic, lk);
  B4Solve<T, true, 0>::run(s, L, invd, j, ic, lk);
}
template <typename T>
__device__ __forceinline__ void b4_bwd(T s[16], const T* L, const T* invd, int j) {
  T ic, lk[4];
  b4_col_values<T, false, TB - 1>(L, invd, j, ic, lk);
  B4Solve<T, false, TB - 1>::run(s, L, invd, j, ic, lk);
}

// Cholesky of the 64 x 64 block held in strip layout d (lower part used),
// four columns per barrier.  Column block b (columns 4b .. 4b+3) is exactly
// register d[b] of the four threads of a row (column offset q0).  Per
// block: every thread publishes d[b] = A[r][4b+q0] (updated by all earlier
// blocks) to cb[b & 1][r][q0] (row-major, so a row's four values are one
// 32-byte read); one barrier (the two buffers alternate); every thread then
// factors the 4 x 4 diagonal block D = Ld Ld^T from cb (redundantly), reads
// its row a_r = A[r][4b..4b+3] back from cb, forms y = a_r Ld^{-T} (row r of
// the block column of L) and w = y Ld^{-1} = a_r D^{-1}, and updates its
// trailing columns k = q0 + 4u, u > b, by d[u] -= w . A[k][4b..4b+3] (four
// fused multiply-adds, in the order of the four columns), the reads of
// A[k][.] running two columns ahead of the updates.  On return L is in LDS
// (row-major, stride LDT, zero above the diagonal) and invd[c] =
// 1 / L[c][c].  Returns false if a pivot was not positive (the factor is
// then finite garbage).
// PANEL: the thread also carries row r of a tile below the block in e[16]
// (same layout, published to cb[2 + (b & 1)]) through every column step,
// which solves it against L^T; the block's own L is then not kept (the
// values that the trailing updates use are the published A[k][.], so the
// tile comes out bitwise as it would beside the full factorisation).
// Keeps a value's computation at this point of the instruction stream (an
// empty asm statement that reads and writes it; such statements keep their
// source order).
template <typename T>
__device__ __forceinline__ void pin(T& x) {
  __asm__ volatile("" : "+v"(x));
}

// The deferred trailing updates of one column block, as a flat list of
// (column u, column q of the block) pairs, u = U0 .. 15 and q = 3 .. 0:
// pair i updates d[u] -= wp[q] A[k][c0 + q] (and e[u] with wtp), with
// k = q0 + 4u and A[k][.] the row k of the published buffer c, which is
// loaded into cr two columns ahead of its first pair.  The row offsets and
// the updated entries are pinned, so the loads and the updates stay in the
// gap of the chain they were placed in.
template <typename T, int U0, bool PANEL, int I0, int I1>
__device__ __forceinline__ void defer_pairs(T d[16], T e[16], T cr[16][4], const T* c, const T wp[4],
                                            const T wtp[4], int q0) {
#pragma unroll
  for (int i = I0; i < I1; ++i) {
    const int u = U0 + i / 4, q = 3 - i % 4;
    if (i % 4 == 0 && u + 2 < 16) {
      int off = (q0 + 4 * (u + 2)) * 4;
      pin(off);
#pragma unroll
      for (int m = 0; m < 4; ++m) cr[u + 2][m] = c[off + m];
    }
    d[u] = fma_t(-wp[q], cr[u][q], d[u]);
    pin(d[u]);
    if constexpr (PANEL) {
      e[u] = fma_t(-wtp[q], cr[u][q], e[u]);
      pin(e[u]);
    }
  }
}

// 1/sqrt of a pivot, one dependent step per call (so that the deferred
// updates can be placed between the steps): the hardware estimate
// (relative error below 2^-24 on gfx950) and one third-order correction,
// y (1 + e/2 + 3e^2/8) with e = 1 - x y^2, which leaves about one unit in
// the last place.  A pivot that is not positive and finite gives 1 and
// clears ok; that test runs beside the estimate, off the chain.
template <typename T>
struct PivotRsqrt {
  T x, y, t, e, p, qv;
  bool bad;
  __device__ __forceinline__ void s0(T xin, bool& ok) {
    x = xin;
    bad = !(x > T(0)) || !__builtin_isfinite(x);
    if (bad) ok = false;
    if constexpr (sizeof(T) == 8) y = __builtin_amdgcn_rsq(x);
    else y = T(1) / sqrtf(x);
    pin(y);
  }
  __device__ __forceinline__ void s1() {
    t = y * y;
    pin(t);
  }
  __device__ __forceinline__ void s2() {
    e = fma_t(-x, t, T(1));
    pin(e);
  }
  __device__ __forceinline__ void s3() {
    p = fma_t(e, T(0.375), T(0.5));
    qv = y * e;
    pin(p);
    pin(qv);
  }
  __device__ __forceinline__ T s4() {
    T r = fma_t(qv, p, y);
    r = bad ? T(1) : r;
    pin(r);
    return r;
  }
};

// Cholesky of the 64 x 64 block held in strip layout d (lower part used),
// four columns per barrier.  Column block b (columns c0 = 4b .. 4b+3) is
// exactly register d[b] of the four threads of a row (column offset q0).
// Per block: every thread publishes d[b] = A[r][c0+q0] (updated by all
// earlier blocks) to c_b = cb[b % 3][r][q0] (row-major, so a row's four
// values are one 32-byte read); one barrier; every thread then factors the
// 4 x 4 diagonal block D = Ld Ld^T from c_b (redundantly), reads its row
// a_r = A[r][c0..c0+3] back from c_b, forms y = a_r Ld^{-T} (row r of the
// block column of L) and w = y Ld^{-1} = a_r D^{-1}, and updates its
// trailing columns k = q0 + 4u, u > b, by d[u] -= w . A[k][c0..c0+3]
// (four fused multiply-adds, columns c0+3 down to c0).
// The chain from one barrier to the next is: the reads of D, the four
// pivots, the last substitution steps and the update of column b + 1,
// which the next block publishes.  It is written out one dependent step at
// a time (34 steps), and the updates of columns u >= b + 2 by the previous
// block, deferred to this block's window, are spread over the steps, a
// fixed share in each gap, so that they issue while a step waits for its
// operands.  Each entry takes its updates in block order.  Three published
// buffers rotate: c_b is read until the end of block b + 1, and the first
// write to it again (block b + 3) follows the barrier of block b + 2.  On
// return L is in LDS (row-major, stride LDT, zero above the diagonal) and
// invd[c] = 1 / L[c][c].  Returns false if a pivot was not positive (the
// factor is then finite garbage).
// PANEL: the thread also carries row r of a tile below the block in e[16]
// (same layout, published to cb[3 + (b & 1)]) through every column step,
// which solves it against L^T; the block's own L is then not kept (the
// values that the trailing updates use are the published A[k][.], so the
// tile comes out bitwise as it would beside the full factorisation).
template <typename T, int B, bool PANEL = false>
struct Potrf4 {
  __device__ __forceinline__ static void run(T d[16], T e[16], T* cb, T* invd, int r, int q0, bool& ok,
                                             const T wp[4], const T wtp[4]) {
    if constexpr (B < 16) {
      T* c = cb + (B % 3) * 4 * TB;
      T* ce = cb + (3 + (B & 1)) * 4 * TB;
      const T* cp = cb + ((B + 2) % 3) * 4 * TB;  // the previous block's values
      c[r * 4 + q0] = d[B];
      if constexpr (PANEL) ce[r * 4 + q0] = e[B];
      __syncthreads();
      constexpr int c0 = 4 * B;
      // deferred pairs of the previous block, spread over NG gaps
      constexpr int NP = B >= 1 ? (15 - B) * 4 : 0, NG = 34;
      T cr[16][4];
      T D[4][4], a[4], at[4], c1[4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q <= p; ++q) D[p][q] = c[(c0 + p) * 4 + q];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = c[r * 4 + q];
      if constexpr (PANEL) {
#pragma unroll
        for (int q = 0; q < 4; ++q) at[q] = ce[r * 4 + q];
      }
      if constexpr (B + 1 < 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) c1[q] = c[(q0 + 4 * (B + 1)) * 4 + q];
      }
      if constexpr (NP > 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) cr[B + 1][q] = cp[(q0 + 4 * (B + 1)) * 4 + q];
        if constexpr (B + 2 < 16) {
#pragma unroll
          for (int q = 0; q < 4; ++q) cr[B + 2][q] = cp[(q0 + 4 * (B + 2)) * 4 + q];
        }
      }
#define THCCP_GAP(g)                                                                               \
  do {                                                                                             \
    if constexpr (NP > 0)                                                                          \
      defer_pairs<T, B + 1, PANEL, (g) * NP / NG, ((g) + 1) * NP / NG>(d, e, cr, cp, wp, wtp, q0); \
  } while (0)
      PivotRsqrt<T> pv;
      // pivot 0
      pv.s0(D[0][0], ok);
      THCCP_GAP(0);
      pv.s1();
      THCCP_GAP(1);
      pv.s2();
      THCCP_GAP(2);
      pv.s3();
      THCCP_GAP(3);
      const T il0 = pv.s4();
      THCCP_GAP(4);
      T L10 = D[1][0] * il0, L20 = D[2][0] * il0, L30 = D[3][0] * il0;
      T y0 = a[0] * il0, yt0 = T(0);
      pin(L10);
      pin(L20);
      pin(L30);
      if constexpr (PANEL) yt0 = at[0] * il0;
      THCCP_GAP(5);
      T x1 = fma_t(-L10, L10, D[1][1]);
      T m21 = fma_t(-L20, L10, D[2][1]), m31 = fma_t(-L30, L10, D[3][1]);
      T m22 = fma_t(-L20, L20, D[2][2]), m32 = fma_t(-L30, L20, D[3][2]);
      T m33 = fma_t(-L30, L30, D[3][3]);
      T v1 = fma_t(-y0, L10, a[1]), v2 = fma_t(-y0, L20, a[2]), v3 = fma_t(-y0, L30, a[3]);
      T vt1 = T(0), vt2 = T(0), vt3 = T(0);
      if constexpr (PANEL) {
        vt1 = fma_t(-yt0, L10, at[1]);
        vt2 = fma_t(-yt0, L20, at[2]);
        vt3 = fma_t(-yt0, L30, at[3]);
      }
      pin(x1);
      // pivot 1
      pv.s0(x1, ok);
      THCCP_GAP(6);
      pv.s1();
      THCCP_GAP(7);
      pv.s2();
      THCCP_GAP(8);
      pv.s3();
      THCCP_GAP(9);
      const T il1 = pv.s4();
      THCCP_GAP(10);
      T L21 = m21 * il1, L31 = m31 * il1, y1 = v1 * il1, yt1 = T(0);
      pin(L21);
      pin(L31);
      if constexpr (PANEL) yt1 = vt1 * il1;
      THCCP_GAP(11);
      T x2 = fma_t(-L21, L21, m22);
      T m32b = fma_t(-L31, L21, m32), m33b = fma_t(-L31, L31, m33);
      T v2b = fma_t(-y1, L21, v2), v3b = fma_t(-y1, L31, v3);
      T vt2b = T(0), vt3b = T(0);
      if constexpr (PANEL) {
        vt2b = fma_t(-yt1, L21, vt2);
        vt3b = fma_t(-yt1, L31, vt3);
      }
      pin(x2);
      // pivot 2
      pv.s0(x2, ok);
      THCCP_GAP(12);
      pv.s1();
      THCCP_GAP(13);
      pv.s2();
      THCCP_GAP(14);
      pv.s3();
      THCCP_GAP(15);
      const T il2 = pv.s4();
      THCCP_GAP(16);
      T L32 = m32b * il2, y2 = v2b * il2, yt2 = T(0);
      pin(L32);
      if constexpr (PANEL) yt2 = vt2b * il2;
      THCCP_GAP(17);
      T x3 = fma_t(-L32, L32, m33b);
      T v3c = fma_t(-y2, L32, v3b), vt3c = T(0);
      if constexpr (PANEL) vt3c = fma_t(-yt2, L32, vt3b);
      pin(x3);
      // pivot 3
      pv.s0(x3, ok);
      THCCP_GAP(18);
      pv.s1();
      THCCP_GAP(19);
      pv.s2();
      THCCP_GAP(20);
      pv.s3();
      THCCP_GAP(21);
      const T il3 = pv.s4();
      THCCP_GAP(22);
      if (!PANEL && r == 0 && q0 == 0) {
        invd[c0] = il0;
        invd[c0 + 1] = il1;
        invd[c0 + 2] = il2;
        invd[c0 + 3] = il3;
      }
      T y3 = v3c * il3, yt3 = T(0);
      pin(y3);
      if constexpr (PANEL) {
        yt3 = vt3c * il3;
        pin(yt3);
      }
      // own entry of the block column: L[r][c0 + q0] = y[q0]
      if constexpr (!PANEL) d[B] = q0 == 0 ? y0 : q0 == 1 ? y1 : q0 == 2 ? y2 : y3;
      if constexpr (PANEL) e[B] = q0 == 0 ? yt0 : q0 == 1 ? yt1 : q0 == 2 ? yt2 : yt3;
      THCCP_GAP(23);
      // w = y Ld^{-1} from the last column back; column B + 1 is updated
      // with each w as it comes
      T wv[4], wt[4] = {T(0), T(0), T(0), T(0)};
      wv[3] = y3 * il3;
      pin(wv[3]);
      if constexpr (PANEL) {
        wt[3] = yt3 * il3;
        pin(wt[3]);
      }
      THCCP_GAP(24);
      T h2 = fma_t(-wv[3], L32, y2), h1 = fma_t(-wv[3], L31, y1), h0 = fma_t(-wv[3], L30, y0);
      T ht2 = T(0), ht1 = T(0), ht0 = T(0);
      if constexpr (B + 1 < 16) {
        d[B + 1] = fma_t(-wv[3], c1[3], d[B + 1]);
        pin(d[B + 1]);
      }
      if constexpr (PANEL) {
        ht2 = fma_t(-wt[3], L32, yt2);
        ht1 = fma_t(-wt[3], L31, yt1);
        ht0 = fma_t(-wt[3], L30, yt0);
        if constexpr (B + 1 < 16) {
          e[B + 1] = fma_t(-wt[3], c1[3], e[B + 1]);
          pin(e[B + 1]);
        }
      }
      pin(h2);
      THCCP_GAP(25);
      wv[2] = h2 * il2;
      pin(wv[2]);
      if constexpr (PANEL) {
        wt[2] = ht2 * il2;
        pin(wt[2]);
      }
      THCCP_GAP(26);
      h1 = fma_t(-wv[2], L21, h1);
      h0 = fma_t(-wv[2], L20, h0);
      if constexpr (B + 1 < 16) {
        d[B + 1] = fma_t(-wv[2], c1[2], d[B + 1]);
        pin(d[B + 1]);
      }
      if constexpr (PANEL) {
        ht1 = fma_t(-wt[2], L21, ht1);
        ht0 = fma_t(-wt[2], L20, ht0);
        if constexpr (B + 1 < 16) {
          e[B + 1] = fma_t(-wt[2], c1[2], e[B + 1]);
          pin(e[B + 1]);
        }
      }
      pin(h1);
      THCCP_GAP(27);
      wv[1] = h1 * il1;
      pin(wv[1]);
      if constexpr (PANEL) {
        wt[1] = ht1 * il1;
        pin(wt[1]);
      }
      THCCP_GAP(28);
      h0 = fma_t(-wv[1], L10, h0);
      if constexpr (B + 1 < 16) {
        d[B + 1] = fma_t(-wv[1], c1[1], d[B + 1]);
        pin(d[B + 1]);
      }
      if constexpr (PANEL) {
        ht0 = fma_t(-wt[1], L10, ht0);
        if constexpr (B + 1 < 16) {
          e[B + 1] = fma_t(-wt[1], c1[1], e[B + 1]);
          pin(e[B + 1]);
        }
      }
      pin(h0);
      THCCP_GAP(29);
      wv[0] = h0 * il0;
      pin(wv[0]);
      if constexpr (PANEL) {
        wt[0] = ht0 * il0;
        pin(wt[0]);
      }
      THCCP_GAP(30);
      if constexpr (B + 1 < 16) {
        d[B + 1] = fma_t(-wv[0], c1[0], d[B + 1]);
        if constexpr (PANEL) e[B + 1] = fma_t(-wt[0], c1[0], e[B + 1]);
      }
      THCCP_GAP(31);
      THCCP_GAP(32);
      THCCP_GAP(33);
#undef THCCP_GAP
      Potrf4<T, B + 1, PANEL>::run(d, e, cb, invd, r, q0, ok, wv, wt);
    }
  }
};
template <typename T>
__device__ __forceinline__ bool strip_potrf4(T d[16], T* L, T* invd, T* cb /* 3 x 64 x 4 */, int r, int q0) {
  bool ok = true;
  const T z[4] = {T(0), T(0), T(0), T(0)};
  Potrf4<T, 0>::run(d, d, cb, invd, r, q0, ok, z, z);
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int q = q0 + 4 * u;
    L[r * LDT + q] = q <= r ? d[u] : T(0);
  }
  __syncthreads();
  return ok;
}

// The factorisation of the diagonal block in d (as strip_potrf4, but L is
// left in d and not written to LDS) with row r of a tile below it carried in
// e: on return e holds that row of the tile solved against L^T, that is of
// A L^{-T}, in the strip layout.  The block's values are bitwise those of
// strip_potrf4.  Returns false if a pivot was not positive.
template <typename T>
__device__ __forceinline__ bool strip_potrf4_panel(T d[16], T e[16], T* invd, T* cb, int r, int q0) {
  bool ok = true;
  const T z[4] = {T(0), T(0), T(0), T(0)};
  Potrf4<T, 0, true>::run(d, e, cb, invd, r, q0, ok, z, z);
  return ok;
}

// ------------------------------------------------------- layout transfers
template <typename T>
__device__ __forceinline__ void acc_to_lds(const typename Acc4<T>::type acc[4], T* S, int lane, int w) {
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) S[acc_row<T>(lane, w, r) * LDT + acc_col(lane, tj)] = acc[tj][r];
}
// ... transposed: S[col][row] (the k-major A operand of tile_mma64).
template <typename T>
__device__ __forceinline__ void acc_to_lds_t(const typename Acc4<T>::type acc[4], T* S, int lane, int w) {
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) S[acc_col(lane, tj) * LDT + acc_row<T>(lane, w, r)] = acc[tj][r];
}
template <typename T>
__device__ __forceinline__ void lds_to_strip(const T* S, T s[16], int r, int q0) {
#pragma unroll
  for (int u = 0; u < 16; ++u) s[u] = S[r * LDT + q0 + 4 * u];
}
template <typename T>
__device__ __forceinline__ void load_acc(typename Acc4<T>::type acc[4], const T* g_, size_t ld, int nrows,
                                         int lane, int w) {
  const gptr<const T> g = as_global(g_);
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = acc_row<T>(lane, w, r);
      acc[tj][r] = row < nrows ? g[(size_t)row * ld + acc_col(lane, tj)] : T(0);
    }
}
template <typename T>
__device__ __forceinline__ void store_acc(const typename Acc4<T>::type acc[4], T* g_, size_t ld, int nrows,
                                          int lane, int w) {
  const gptr<T> g = as_global(g_);
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = acc_row<T>(lane, w, r);
      if (row < nrows) g[(size_t)row * ld + acc_col(lane, tj)] = acc[tj][r];
    }
}
// Register prefetch of a 64 x 64 row-major block (16 values per thread,
// element idx = tid + 256 e at (idx / 64, idx % 64)); rows >= nrows read 0.
template <typename T>
__device__ __forceinline__ void fetch_block(T v[16], const T* g_, size_t ld, int nrows, int tid) {
  const gptr<const T> g = as_global(g_);
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int idx = tid + 256 * e;
    v[e] = (idx >> 6) < nrows ? g[(size_t)(idx >> 6) * ld + (idx & 63)] : T(0);
  }
}
// ... written to LDS transposed (S[c][r]) or as is (S[r][c]).
template <typename T, bool TRANSPOSE>
__device__ __forceinline__ void put_block(T* S, const T v[16], int tid) {
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int idx = tid + 256 * e;
    if (TRANSPOSE) S[(idx & 63) * LDT + (idx >> 6)] = v[e];
    else S[(idx >> 6) * LDT + (idx & 63)] = v[e];
  }
}

// Maps a linear block id onto the lower-triangular tile (i, k) of the
// trailing matrix, i >= k >= k0; column k0 comes first.
__device__ __forceinline__ void tri_tile(int bid, int k0, int nblk, int& i, int& k) {
  k = k0;
  int len = nblk - k0;
  while (bid >= len) {
    bid -= len;
    ++k;
    --len;
  }
  i = k + bid;
}

// Block ranges of one launch.  Factorisation: step j (updates with block
// column j when j >= lo, factors column j + 1) covers columns j+1 .. kmax.
// Forward solve: same shape.  Backward solve: step js (updates with column
// js when js <= hi, solves column js - 1) covers columns kmin .. js-1.
// An empty range has kmax < j + 1 (kmin > js - 1).
__host__ __device__ inline void chol_range(int nblk, int pw, int pc, int tc, int& j, int& lo, int& kmax) {
  j = 0;
  lo = 0;
  kmax = -1;
  if (pc < 0 || tc < 0) return;
  lo = pw * pc;
  const int hi = nblk - 1 < lo + pw - 1 ? nblk - 1 : lo + pw - 1;
  j = lo - 1 + tc;
  if (j >= hi) {
    kmax = -1;
    return;
  }
  kmax = j < lo ? j + 1 : hi;
}
__host__ __device__ inline void bwd_range(int nblk, int pw, int pf, int tf, int& js, int& hi, int& kmin) {
  js = 0;
  hi = -1;
  kmin = 1;
  if (pf < 0 || tf < 0) return;
  const int lo = pw * pf;
  hi = nblk - 1 < lo + pw - 1 ? nblk - 1 : lo + pw - 1;
  js = hi + 1 - tf;
  if (lo > hi || js < lo + 1) {
    kmin = js;  // empty
    return;
  }
  kmin = js > hi ? js - 1 : lo;
}
// One level (pw >= nblk): the columns beyond j + 2 take their updates in
// pairs, at odd j (rank 128, columns j - 1 and j), and are left out of the
// launches of even j; columns j + 1 and j + 2 are always brought up to date,
// so a column is current when it becomes the next column to factor.  This
// halves the trailing-matrix traffic of the early, bandwidth-bound steps.
__host__ __device__ inline bool chol_paired(int nblk, int pw, int j) { return pw >= nblk && j >= 0; }
__host__ __device__ inline int chol_tiles(int nblk, int pw, int pc, int tc) {
  int j, lo, kmax;
  chol_range(nblk, pw, pc, tc, j, lo, kmax);
  if (chol_paired(nblk, pw, j) && !(j & 1) && kmax > j + 2) kmax = j + 2;
  int t = 0;
  for (int k = j + 1; k <= kmax; ++k) t += nblk - k;
  return t;
}
// The one-level triangular solves pair their far updates the same way:
// forward step js updates blocks beyond js + 2 only at odd js (with G_{js-1}
// and G_js); backward step js (s = hi - js steps from the end) updates
// blocks below js - 2 only at odd s (with F_{js+1} and F_js).
__host__ __device__ inline bool bwd_paired(int nblk, int pw, int js, int hi) { return pw >= nblk && js <= hi; }
__host__ __device__ inline int fwd_tiles(int nblk, int nrt, int pw, int pf, int tf) {
  int js, lo, kmax;
  chol_range(nblk, pw, pf, tf, js, lo, kmax);
  if (chol_paired(nblk, pw, js) && !(js & 1) && kmax > js + 2) kmax = js + 2;
  return kmax >= js + 1 ? nrt * (kmax - js) : 0;
}
__host__ __device__ inline int bwd_tiles(int nblk, int nrt, int pw, int pf, int tf) {
  int js, hi, kmin;
  bwd_range(nblk, pw, pf, tf, js, hi, kmin);
  if (bwd_paired(nblk, pw, js, hi) && !((hi - js) & 1) && kmin < js - 2) kmin = js - 2;
  return js - 1 >= kmin ? nrt * (js - kmin) : 0;
}

// One launch of the blocked factorisation / solve.
//   STEP_CHOL:     Cholesky step j (tiles of the trailing lower triangle).
//   STEP_FWD/BWD:  triangular-solve step j over (row tile, column block).
//                  Forward: G L^T = M; step j subtracts G_j L_kj^T from every
//                  block k > j, the blocks of column j+1 then solve with
//                  L_{j+1,j+1}.  Backward: F L = G, mirrored from the last
//                  column block down.
//   STEP_CHOL_FWD: Cholesky step j and forward step j-1 in one launch (the
//                  latter needs only panel columns <= j-1 and diagonal block
//                  j, all from earlier launches); no damped retry.
// (The bodies are written inline in the kernel: moving them into device
// functions doubles the register use and spills.)
template <typename T, int MODE>
__global__ __launch_bounds__(256) void step_kernel(const StepProb<T>* probs, const int* offs, int nprob,
                                                    StepCfg cfg, int retry_pass) {
  typedef typename Acc4<T>::type acc_t;
  __shared__ T S0[TB * LDT];
  __shared__ T S1[TB * LDT];
  __shared__ __attribute__((aligned(16))) T colbuf[12 * TB];  // 3 published column blocks
  __shared__ T invd[TB];
  int pid = 0;
  while (pid + 1 < nprob && (int)blockIdx.x >= offs[pid + 1]) ++pid;
  T* const V = probs[pid].V;
  T* const ldiag = probs[pid].ldiag;
  T* const diagL = probs[pid].diagL;
  T* const M = probs[pid].M;
  DevState* const st = probs[pid].st;
  const int nblk = probs[pid].nblk;
  const int n = probs[pid].n;
  int bid = blockIdx.x - offs[pid];
  const int nbid = offs[pid + 1] - offs[pid];
  if (st->done) return;
  // the forward solve of the damped-retry pass serves only the retried problems
  if (MODE == STEP_FWD && retry_pass && !st->retry_active) return;
  const int Tp = nblk * TB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int sr = tid >> 2, q0 = tid & 3;  // strip layout (diagonal factorisation)
  const int bg = tid >> 4, bj = tid & 15;  // block-4 layout (triangular solves)

  if constexpr (MODE == STEP_CHOL || MODE == STEP_CHOL_FWD) {
    if (MODE == STEP_CHOL_FWD ? st->chol_fail : (retry_pass ? !st->retry_active : st->chol_fail)) return;
    int j, jlo, kmax;
    chol_range(nblk, cfg.pw, cfg.pc, cfg.tc, j, jlo, kmax);
    const int nc = MODE == STEP_CHOL ? 1 << 30 : chol_tiles(nblk, cfg.pw, cfg.pc, cfg.tc);
    if (bid < nc) {
      const bool upd = j >= jlo;  // update with block column j (inside the panel)
      int i, k;
      // (no XCD remap here: the next column's tiles, the critical path,
      // must spread over all XCDs)
      tri_tile(bid, j + 1, nblk, i, k);
      // the next column's workgroups are the critical path: their waves
      // issue first on a compute unit shared with trailing updates
      if (k == j + 1) __builtin_amdgcn_s_setprio(3);
      T* tile = V + (size_t)i * TB * Tp + (size_t)k * TB;
      // a tile beyond column j + 1 at odd j also takes column j - 1
      const bool two = upd && chol_paired(nblk, cfg.pw, j) && (j & 1) && k >= j + 2;
      const int j0 = two ? j - 1 : j;
      // every global load of the step is issued up front
      acc_t acc[4];
      T ra[16], rb[16];
      load_acc<T>(acc, tile, Tp, TB, lane, w);
      if (upd) {
        fetch_block<T>(ra, V + (size_t)i * TB * Tp + (size_t)j0 * TB, Tp, TB, tid);
        fetch_block<T>(rb, V + (size_t)k * TB * Tp + (size_t)j0 * TB, Tp, TB, tid);
      }
      acc_t dd[4];
      const bool need_d = (k == j + 1) && (i != k);
      if (need_d) load_acc<T>(dd, V + (size_t)k * TB * Tp + (size_t)k * TB, Tp, TB, lane, w);
      if (upd) {
        // tile -= L_ij0 L_kj0^T (and, for a paired update, then L_ij L_kj^T)
        put_block<T, true>(S0, ra, tid);
        put_block<T, true>(S1, rb, tid);
        __syncthreads();
        if (two) {  // the second pair is fetched under the first product
          fetch_block<T>(ra, V + (size_t)i * TB * Tp + (size_t)j * TB, Tp, TB, tid);
          fetch_block<T>(rb, V + (size_t)k * TB * Tp + (size_t)j * TB, Tp, TB, tid);
        }
        acc_t p[4];
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) p[tj] = acc_t{0, 0, 0, 0};
        tile_mma64<T>(p, S0, S1, lane, w);
        if (two) {
          __syncthreads();  // every wave is past its reads of S0 / S1
          put_block<T, true>(S0, ra, tid);
          put_block<T, true>(S1, rb, tid);
          __syncthreads();
          tile_mma64<T>(p, S0, S1, lane, w);
        }
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) acc[tj] -= p[tj];
        if (k != j + 1) {
          store_acc<T>(acc, tile, Tp, TB, lane, w);
          return;
        }
      }
      // Column k = j + 1.  Updated diagonal block D = A_kk - L_kj L_kj^T,
      // staged through S1 (two tile buffers per workgroup keep two
      // workgroups resident per compute unit).
      T d[16];
      if (i == k) {
        __syncthreads();  // every wave is past its MMA reads of S0 / S1
        acc_to_lds<T>(acc, S1, lane, w);
      } else {
        if (upd) {
          acc_t p[4];
#pragma unroll
          for (int tj = 0; tj < 4; ++tj) p[tj] = acc_t{0, 0, 0, 0};
          tile_mma64<T>(p, S1, S1, lane, w);
#pragma unroll
          for (int tj = 0; tj < 4; ++tj) dd[tj] -= p[tj];
        }
        __syncthreads();
        acc_to_lds<T>(dd, S1, lane, w);
        acc_to_lds<T>(acc, S0, lane, w);
      }
      __syncthreads();
      lds_to_strip<T>(S1, d, sr, q0);
      __syncthreads();
      // S1 receives L_kk (every wave is past its last read of S1 here).
      const bool ok = strip_potrf4<T>(d, S1, invd, colbuf, sr, q0);
      if (i == k) {
        if (!ok && tid == 0) {
          if (retry_pass) atomicOr(&st->flags, (int)FLAG_NOT_SPD);
          else atomicExch(&st->chol_fail, 1);
        }
        if (tid < TB) as_global(diagL)[k * TB + tid] = S1[tid * LDT + tid];
        // X = L_kk^{-T} (the identity solved against L^T) replaces L_kk:
        // every later triangular solve with this block is one MFMA product
        T s[16];
#pragma unroll
        for (int ii = 0; ii < 4; ++ii)
#pragma unroll
          for (int v = 0; v < 4; ++v) s[4 * ii + v] = (4 * bg + ii == bj + 16 * v) ? T(1) : T(0);
        b4_fwd<T>(s, S1, invd, bj);
        store_b4<T>(s, ldiag + (size_t)k * TB * TB, TB, TB, bg, bj);
        return;
      }
      // Panel tile: L_ik = A'_ik L_kk^{-T}
      T s[16];
      lds_to_b4<T>(S0, s, bg, bj);
      b4_fwd<T>(s, S1, invd, bj);
      store_b4<T>(s, tile, Tp, TB, bg, bj);
      return;
    }
    bid -= nc;
  }
  if constexpr (MODE != STEP_CHOL) {
    constexpr bool FWD = MODE != STEP_BWD;
    int js, lim, kext;  // forward: lim = panel start; backward: lim = panel end
    if (FWD) chol_range(nblk, cfg.pw, cfg.pf, cfg.tf, js, lim, kext);
    else bwd_range(nblk, cfg.pw, cfg.pf, cfg.tf, js, lim, kext);
    const int nrt = (n + TB - 1) / TB;
    // the row blocks of one column share L_jk and the column's blocks of
    // one row share F_j: XCD-contiguous ranges keep both in one L2
    bid = xcd_remap(bid, MODE == STEP_CHOL_FWD ? nbid - chol_tiles(nblk, cfg.pw, cfg.pc, cfg.tc) : nbid);
    const int rt = bid % nrt;
    const int k = FWD ? js + 1 + bid / nrt : js - 1 - bid / nrt;
    const int r0 = rt * TB;
    const int nrows = min(TB, n - r0);
    T* tile = M + (size_t)r0 * Tp + (size_t)k * TB;
    const bool has_update = FWD ? (js >= lim) : (js <= lim);
    const bool solve = FWD ? (k == js + 1) : (k == js - 1);
    if (solve) __builtin_amdgcn_s_setprio(3);  // the solve chain, as above
    // a far block of a paired step also takes column js - 1 (forward) or
    // js + 1 (backward), first
    const bool two = has_update && (FWD ? chol_paired(nblk, cfg.pw, js) && (js & 1) && k >= js + 2
                                        : bwd_paired(nblk, cfg.pw, js, lim) && ((lim - js) & 1) && k <= js - 2);
    const int j0 = two ? (FWD ? js - 1 : js + 1) : js;
    // every global load of the step is issued up front
    acc_t acc[4];
    T ra[16], rb[16], rl[16];
    auto fetch_pair = [&](int jj) {
      fetch_block<T>(ra, M + (size_t)r0 * Tp + (size_t)jj * TB, Tp, nrows, tid);
      if (FWD) fetch_block<T>(rb, V + (size_t)k * TB * Tp + (size_t)jj * TB, Tp, TB, tid);  // L_kj
      else fetch_block<T>(rb, V + (size_t)jj * TB * Tp + (size_t)k * TB, Tp, TB, tid);     // L_jk
    };
    auto put_pair = [&]() {
      put_block<T, true>(S0, ra, tid);
      if (FWD) put_block<T, true>(S1, rb, tid);   // B = L_kj^T
      else put_block<T, false>(S1, rb, tid);      // B = L_jk
    };
    load_acc<T>(acc, tile, Tp, nrows, lane, w);
    if (has_update) fetch_pair(j0);
    if (solve) fetch_block<T>(rl, ldiag + (size_t)k * TB * TB, TB, TB, tid);
    if (has_update) {
      put_pair();
      __syncthreads();
      if (two) fetch_pair(js);  // under the first product
      acc_t p[4];
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) p[tj] = acc_t{0, 0, 0, 0};
      tile_mma64<T>(p, S0, S1, lane, w);
      if (two) {
        __syncthreads();  // every wave is past its reads of S0 / S1
        put_pair();
        __syncthreads();
        tile_mma64<T>(p, S0, S1, lane, w);
      }
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) acc[tj] -= p[tj];
    }
    if (!solve) {
      store_acc<T>(acc, tile, Tp, nrows, lane, w);
      return;
    }
    // Solve with the stored X = L_kk^{-T}: forward G = T X, backward T X^T.
    __syncthreads();
    acc_to_lds_t<T>(acc, S0, lane, w);
    if (FWD) put_block<T, false>(S1, rl, tid);
    else put_block<T, true>(S1, rl, tid);
    __syncthreads();
    acc_t p[4];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) p[tj] = acc_t{0, 0, 0, 0};
    tile_mma64<T>(p, S0, S1, lane, w);
    store_acc<T>(p, tile, Tp, nrows, lane, w);
  }
}

// ------------------------------------------------- dataflow backward solve
// The rows of F = G L^{-1} are independent, so each 64-row tile of F is its
// own chain over the block columns, from the last to the first:
//
//   F_k = (G_k - sum_{i > k} F_i L_ik) L_kk^{-1} = (...) X_k^T,
//
// (X_k = L_kk^{-T}, stored by the factorisation).  One launch holds every
// (row tile, block column) pair of every problem; the workgroup of (rt, k)
// takes the products with F_i as their ready flags appear, highest i
// first, and publishes its own F_k when it is stored.  Workgroups are
// numbered from each problem's last column down (flow_segments), so every
// wait is on a lower workgroup id: those are dispatched first and never
// wait on a higher one, hence the launch cannot deadlock.  A wait still
// gives up after spin_limit polls (setting
// FLAG_SOLVE_STALL, which every other wait of the problem sees and follows)
// so the grid always drains.
//
// The F tiles pass between workgroups through device-coherent accesses
// (agent-scope relaxed atomics, which bypass the per-XCD L2 state), so no
// L2-wide write-back or invalidation is needed: the producer waits for its
// stores to be acknowledged before it sets the flag, and the consumer's
// reads are issued after it has seen the flag.
constexpr int FLOW_SPIN_LIMIT = 1 << 20;
static int g_flow_spin_limit = FLOW_SPIN_LIMIT;  // host side, lowered only by a test hook

// Polls until *a >= want, and *b >= want when b is given.  Each poll
// issues the loads of both flags and of the problem's status word
// together, so it costs one memory round trip, and a second flag that is
// already set costs nothing more.  Gives up (setting FLAG_SOLVE_STALL, for
// every other wait of the problem to follow) once the problem has stalled
// or after spin_limit polls that found a flag unset.
__device__ __forceinline__ bool poll_flags(const int32_t* a, const int32_t* b, int32_t want, DevState* st,
                                           int spin_limit) {
  const auto pa = as_global(a), pb = as_global(b != nullptr ? b : a);
  const auto ps = as_global(&st->flags);
  for (int spins = 0;; ++spins) {
    const int32_t va = __hip_atomic_load(pa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t vb = __hip_atomic_load(pb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t fl = __hip_atomic_load(ps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (va >= want && vb >= want) return true;
    if ((fl & FLAG_SOLVE_STALL) || spins >= spin_limit) {
      __hip_atomic_fetch_or(ps, (int)FLAG_SOLVE_STALL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}
static int g_bwd_form = 0;  // host side: 0 block pairs, 1 one block column per hop
int set_bwd_form(int form) {
  const int prev = g_bwd_form;
  g_bwd_form = form == 1 ? 1 : 0;
  return prev;
}
int set_flow_spin_limit(int polls) {
  const int prev = g_flow_spin_limit;
  g_flow_spin_limit = polls < 0 ? FLOW_SPIN_LIMIT : polls;
  return prev;
}

template <typename T>
struct Bits;
template <>
struct Bits<double> {
  typedef unsigned long long type;
};
template <>
struct Bits<float> {
  typedef unsigned int type;
};
// (through global-address-space pointers: a generic pointer would make these
// FLAT accesses, which also count against the LDS wait counter)
template <typename T>
__device__ __forceinline__ T coherent_load(const T* p) {
  typedef typename Bits<T>::type U;
  const U u = __hip_atomic_load((gptr<const U>)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(T, u);
}
template <typename T>
__device__ __forceinline__ void coherent_store(T* p, T v) {
  typedef typename Bits<T>::type U;
  __hip_atomic_store((gptr<U>)p, __builtin_bit_cast(U, v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// fetch_block / store_acc through device-coherent accesses
template <typename T>
__device__ __forceinline__ void fetch_block_coherent(T v[16], const T* g, size_t ld, int nrows, int tid) {
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int idx = tid + 256 * e;
    v[e] = (idx >> 6) < nrows ? coherent_load<T>(g + (size_t)(idx >> 6) * ld + (idx & 63)) : T(0);
  }
}
// fetch_block_coherent through device-coherent 16-byte loads (FP64): load e
// of thread t brings the elements (r, c) and (r, c + 1) of pair p =
// t + 256 e, r = p / 32, c = 2 (p % 32), into v[2e], v[2e + 1]; rows at or
// past nrows read zero (the buffer's bound).  put_block2 writes that
// layout to LDS; other types keep the 8-byte element form.
template <typename T>
__device__ __forceinline__ void fetch_block2_coherent(T v[16], const T* g, size_t ld, int nrows, int tid) {
  if constexpr (sizeof(T) == 8) {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    constexpr int SC1 = 16;  // cache policy: device-coherent, as the agent-scope loads
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)g, (short)0, (int)((size_t)nrows * ld * sizeof(T)), 0x00020000);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int pr = tid + 256 * e;
      const u4 x = __builtin_amdgcn_raw_buffer_load_b128(
          rs, (int)(((pr >> 5) * ld + 2 * (pr & 31)) * sizeof(T)), 0, SC1);
      v[2 * e] = __builtin_bit_cast(T, (unsigned long long)x.x | ((unsigned long long)x.y << 32));
      v[2 * e + 1] = __builtin_bit_cast(T, (unsigned long long)x.z | ((unsigned long long)x.w << 32));
    }
  } else {
    fetch_block_coherent<T>(v, g, ld, nrows, tid);
  }
}
template <typename T, bool TRANSPOSE>
__device__ __forceinline__ void put_block2(T* S, const T v[16], int tid) {
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int pr = tid + 256 * e, r = pr >> 5, c = 2 * (pr & 31);
      if (TRANSPOSE) {
        S[c * LDT + r] = v[2 * e];
        S[(c + 1) * LDT + r] = v[2 * e + 1];
      } else {
        S[r * LDT + c] = v[2 * e];
        S[r * LDT + c + 1] = v[2 * e + 1];
      }
    }
  } else {
    put_block<T, TRANSPOSE>(S, v, tid);
  }
}
// A 64-column tile held in LDS (row-major, stride LDT) stored through
// device-coherent 16-byte stores, in the pair layout of fetch_block2_coherent
// (rows at or past nrows are dropped by the buffer's bound).  FP64 only.
__device__ __forceinline__ void store_block2_coherent(const double* S, double* g, size_t ld, int nrows, int tid) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  constexpr int SC1 = 16;  // cache policy: device-coherent, as the agent-scope stores
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)g, (short)0, (int)((size_t)nrows * ld * sizeof(double)), 0x00020000);
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int pr = tid + 256 * e, r = pr >> 5, c = 2 * (pr & 31);
    const unsigned long long x0 = __builtin_bit_cast(unsigned long long, S[r * LDT + c]);
    const unsigned long long x1 = __builtin_bit_cast(unsigned long long, S[r * LDT + c + 1]);
    const u4 v = {(unsigned)x0, (unsigned)(x0 >> 32), (unsigned)x1, (unsigned)(x1 >> 32)};
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)((r * ld + c) * sizeof(double)), 0, SC1);
  }
}
template <typename T>
__device__ __forceinline__ void store_acc_coherent(const typename Acc4<T>::type acc[4], T* g, size_t ld, int nrows,
                                                   int lane, int w) {
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = acc_row<T>(lane, w, r);
      if (row < nrows) coherent_store<T>(g + (size_t)row * ld + acc_col(lane, tj), acc[tj][r]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void flow_reset_kernel(const StepProb<T>* probs) {
  const StepProb<T>& q = probs[blockIdx.x];
  const int cnt = ((q.n + TB - 1) / TB) * q.nblk;
  const gptr<int32_t> f = as_global(q.flow);
  for (int e = threadIdx.x; e < cnt; e += 256) f[e] = 0;
}

// Segment of a grouped dataflow launch holding workgroup bx (see
// flow_segments): problem, block column, and the index inside the segment.
__device__ __forceinline__ void flow_segment(const int* seg, int nseg, int bx, int& pid, int& k, int& bid) {
  int lo = 0, hi = nseg - 1;  // the last segment starting at or before bx
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg[3 * mid] <= bx) lo = mid;
    else hi = mid - 1;
  }
  pid = seg[3 * lo + 1];
  k = seg[3 * lo + 2];
  bid = bx - seg[3 * lo];
}

template <typename T>
__global__ __launch_bounds__(256, 2) void bwd_flow_kernel(const StepProb<T>* probs, const int* seg, int nseg,
                                                       int spin_limit) {
  typedef typename Acc4<T>::type acc_t;
  __shared__ T S0[TB * LDT];
  __shared__ T S1[TB * LDT];
  __shared__ int stalled;
  int pid, k, rt;  // no XCD remap: the id order is the dependency order
  flow_segment(seg, nseg, blockIdx.x, pid, k, rt);
  const StepProb<T> q = probs[pid];
  DevState* const st = q.st;
  // uniform per problem and unchanged during the launch: all or none of a
  // problem's workgroups take part
  if (st->done) return;
  const int nblk = q.nblk, Tp = nblk * TB;
  const int r0 = rt * TB, nrows = min(TB, q.n - r0);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int32_t* const flag = q.flow + (size_t)rt * nblk;
  T* const tile = q.M + (size_t)r0 * Tp + (size_t)k * TB;
  acc_t acc[4];
  T rf[16], rl[16], rx[16];
  // the accumulators hold -G_k so that every product adds in place
  load_acc<T>(acc, tile, Tp, nrows, lane, w);
  fetch_block<T>(rx, q.ldiag + (size_t)k * TB * TB, TB, TB, tid);
  if (k + 1 < nblk) fetch_block<T>(rl, q.V + (size_t)(nblk - 1) * TB * Tp + (size_t)k * TB, Tp, TB, tid);
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) acc[tj] = -acc[tj];
  // Waits until F_i of this row tile is published; false (for every wave)
  // once a wait of the problem has stalled.  The barrier also means every
  // wave is past its reads of S0 / S1 for the previous product.
  auto wait_ready = [&](int i) -> bool {
    if (tid == 0) stalled = !poll_flags(flag + i, nullptr, 1, st, spin_limit);
    __syncthreads();
    return !stalled;
  };
  for (int i = nblk - 1; i > k + 1; --i) {
    if (!wait_ready(i)) return;
    fetch_block_coherent<T>(rf, q.M + (size_t)r0 * Tp + (size_t)i * TB, Tp, nrows, tid);
    put_block<T, false>(S1, rl, tid);  // L_ik
    fetch_block<T>(rl, q.V + (size_t)(i - 1) * TB * Tp + (size_t)k * TB, Tp, TB, tid);  // i - 1 > k
    put_block<T, true>(S0, rf, tid);  // F_i^T
    __syncthreads();
    tile_mma64<T>(acc, S0, S1, lane, w);  // acc += F_i L_ik
  }
  // f = acc X_k^T with the columns beyond k + 1; the last column then
  // enters as F_{k+1} P with P = L_{k+1,k} X_k^T formed while it is still
  // on its way, so one product follows the last wait.
  if (k + 1 < nblk) __syncthreads();  // every wave is past its reads of S0 / S1
  acc_to_lds_t<T>(acc, S0, lane, w);
  put_block<T, true>(S1, rx, tid);  // X_k^T
  __syncthreads();
  acc_t f[4];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) f[tj] = acc_t{0, 0, 0, 0};
  tile_mma64<T>(f, S0, S1, lane, w);
  if (k + 1 < nblk) {
    __syncthreads();
    put_block<T, true>(S0, rl, tid);  // L_{k+1,k}^T
    __syncthreads();
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] = acc_t{0, 0, 0, 0};
    tile_mma64<T>(acc, S0, S1, lane, w);  // P
    __syncthreads();
    acc_to_lds<T>(acc, S1, lane, w);  // B operand P
    if (!wait_ready(k + 1)) return;
    fetch_block_coherent<T>(rf, q.M + (size_t)r0 * Tp + (size_t)(k + 1) * TB, Tp, nrows, tid);
    put_block<T, true>(S0, rf, tid);  // F_{k+1}^T
    __syncthreads();
    tile_mma64<T>(f, S0, S1, lane, w);
  }
  // f = -(G_k - sum_{i > k} F_i L_ik) X_k^T = -F_k
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) f[tj] = -f[tj];
  store_acc_coherent<T>(f, tile, Tp, nrows, lane, w);
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores of F_k are acknowledged
  __syncthreads();
  if (tid == 0) __hip_atomic_store(as_global(flag + k), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------- backward solve in block pairs
// The recurrence F_k = (G_k - sum_{i>k} F_i L_ik) X_k^T (X_k = L_kk^{-T})
// taken two block columns per step: pair j holds b = nblk - 1 - 2j and
// a = b - 1 (none when b = 0), and depends on the pair before it, c = b + 1
// and d = b + 2, only through
//
//   F_b = -(R_b + F_c P_cb + F_d P_db),        R_b = acc_b X_b^T,
//   F_a = -(acc_a X_a^T - acc_b U + F_c Q_c + F_d Q_d),
//
// with acc_x = -G_x + sum_{i>=b+3} F_i L_ix (the columns beyond c and d),
// P_xb = L_xb X_b^T, S = L_ba X_a^T, U = X_b^T S and Q_x = L_xa X_a^T -
// P_xb S (substituting F_b into the equation of F_a).  P, U and Q depend on
// L alone: one launch forms them per pair into blocks of V's upper
// triangle, which the factorisation leaves unused ((b, c), (b, d), (a, b),
// (a, c), (a, d)).  The backward launch then has one workgroup per (pair,
// row tile, block): after the last wait each applies two products (F_c
// and F_d against its own P or Q), so the chain crosses a dependency hop
// once per two block columns.  The a workgroup needs acc_b: the b workgroup
// stores it in the a tile (which the a workgroup has read by then) and
// flags it.  Ready-flag values per (row tile, block): FL_GLOADED the a
// tile's G has been read, FL_ACCB acc_b is stored there, FL_F the block's
// F is stored.
constexpr int32_t FL_GLOADED = 1, FL_ACCB = 2, FL_F = 3;
__host__ __device__ inline int bwd_pair_count(int nblk) { return (nblk + 1) / 2; }
__host__ __device__ inline int bwd_prep_tiles(int nblk) { return 5 * bwd_pair_count(nblk); }

// acc += A B with A given as register fragments: a[m] = A[16 w + lane % 16][4 m + lane / 16]
template <typename T>
__device__ __forceinline__ void tile_mma64_ra(typename Acc4<T>::type acc[4], const T a[16], const T* Bk, int lane) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int k = 4 * m + (lane >> 4);
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] = mfma4(a[m], Bk[k * LDT + 16 * tj + (lane & 15)], acc[tj]);
  }
}
// the A fragments of rows 16 w.. of a row-major block written in this launch
template <typename T>
__device__ __forceinline__ void fetch_afrag_coherent(T a[16], const T* g, size_t ld, int nrows, int lane, int w) {
  const int row = 16 * w + (lane & 15);
#pragma unroll
  for (int m = 0; m < 16; ++m)
    a[m] = row < nrows ? coherent_load<T>(g + (size_t)row * ld + 4 * m + (lane >> 4)) : T(0);
}

// The same fragments through device-coherent 16-byte loads (FP64): product
// m of tile_mma64_ra2 takes k = 8 (m / 2) + 2 (lane / 16) + m % 2, so a
// lane's values of products 2 m2 and 2 m2 + 1 are adjacent in memory and
// come in one load.  Rows at or past nrows read zero (the buffer's bound).
__device__ __forceinline__ void fetch_afrag2_coherent(double a[16], const double* g, size_t ld, int nrows, int lane,
                                                      int w) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  constexpr int SC1 = 16;  // cache policy: device-coherent, as the agent-scope loads
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)g, (short)0, (int)((size_t)nrows * ld * sizeof(double)), 0x00020000);
  const int off = (int)(((16 * w + (lane & 15)) * ld + 2 * (lane >> 4)) * sizeof(double));
#pragma unroll
  for (int m2 = 0; m2 < 8; ++m2) {
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 64 * m2, 0, SC1);
    a[2 * m2] = __builtin_bit_cast(double, (unsigned long long)v.x | ((unsigned long long)v.y << 32));
    a[2 * m2 + 1] = __builtin_bit_cast(double, (unsigned long long)v.z | ((unsigned long long)v.w << 32));
  }
}
// acc += A B for fragments in that order
template <typename T>
__device__ __forceinline__ void tile_mma64_ra2(typename Acc4<T>::type acc[4], const T a[16], const T* Bk, int lane) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int k = 8 * (m >> 1) + 2 * (lane >> 4) + (m & 1);
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] = mfma4(a[m], Bk[k * LDT + 16 * tj + (lane & 15)], acc[tj]);
  }
}

// One product of the pair set-up per workgroup (output o of pair j): the
// result goes to an upper block of V.
template <typename T>
__global__ __launch_bounds__(256) void bwd_prep_kernel(const StepProb<T>* probs, const int* offs, int nprob) {
  typedef typename Acc4<T>::type acc_t;
  __shared__ T S0[TB * LDT];
  __shared__ T S1[TB * LDT];
  int pid = 0;
  while (pid + 1 < nprob && (int)blockIdx.x >= offs[pid + 1]) ++pid;
  const StepProb<T> q = probs[pid];
  if (q.st->done) return;  // as the backward launch that reads the results
  const int local = blockIdx.x - offs[pid], j = local / 5, o = local % 5;
  const int nblk = q.nblk, Tp = nblk * TB;
  const int b = nblk - 1 - 2 * j, a = b - 1, c = b + 1, d = b + 2;
  const bool has_a = a >= 0, has_q = j >= 1;
  if ((o < 2 && !has_q) || (o == 2 && !has_a) || (o > 2 && !(has_a && has_q))) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  auto blk = [&](int x, int y) { return q.V + (size_t)x * TB * Tp + (size_t)y * TB; };
  auto xk = [&](int k) { return q.ldiag + (size_t)k * TB * TB; };
  T ra[16], rb[16];
  acc_t acc[4], t[4], u[4];
  auto zero = [&](acc_t* x) {
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) x[tj] = acc_t{0, 0, 0, 0};
  };
  // x += L_{r,k} X_k^T
  auto l_xt = [&](acc_t* x, int r, int k) {
    fetch_block<T>(ra, blk(r, k), Tp, TB, tid);
    fetch_block<T>(rb, xk(k), TB, TB, tid);
    __syncthreads();  // every wave is past its reads of S0 / S1
    put_block<T, true>(S0, ra, tid);  // A = L_rk
    put_block<T, true>(S1, rb, tid);  // B = X_k^T
    __syncthreads();
    tile_mma64<T>(x, S0, S1, lane, w);
  };
  // x += y z (both accumulator tiles of this workgroup)
  auto prod = [&](acc_t* x, const acc_t* y, const acc_t* z) {
    __syncthreads();
    acc_to_lds_t<T>(y, S0, lane, w);
    acc_to_lds<T>(z, S1, lane, w);
    __syncthreads();
    tile_mma64<T>(x, S0, S1, lane, w);
  };
  zero(acc);
  T* dst;
  if (o < 2) {  // P_cb or P_db
    const int x = o == 0 ? c : d;
    l_xt(acc, x, b);
    dst = blk(b, x);
  } else {
    zero(t);
    l_xt(t, b, a);  // S
    if (o == 2) {  // U = X_b^T S
      fetch_block<T>(ra, xk(b), TB, TB, tid);
      __syncthreads();
      put_block<T, false>(S0, ra, tid);  // A = X_b^T
      acc_to_lds<T>(t, S1, lane, w);     // B = S
      __syncthreads();
      tile_mma64<T>(acc, S0, S1, lane, w);
      dst = blk(a, b);
    } else {  // Q_x = L_xa X_a^T - P_xb S
      const int x = o == 3 ? c : d;
      zero(u);
      l_xt(u, x, b);     // P_xb
      prod(acc, u, t);   // P_xb S
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) acc[tj] = -acc[tj];
      l_xt(acc, x, a);
      dst = blk(a, x);
    }
  }
  store_acc<T>(acc, dst, Tp, TB, lane, w);
}

template <typename T>
__global__ __launch_bounds__(256, 2) void bwd_pair_kernel(const StepProb<T>* probs, const int* seg, int nseg,
                                                       int spin_limit) {
  typedef typename Acc4<T>::type acc_t;
  __shared__ T S0[TB * LDT];
  __shared__ T S1[TB * LDT];
  __shared__ int stalled;
  int pid, j, bid;  // no XCD remap: the id order is the dependency order
  flow_segment(seg, nseg, blockIdx.x, pid, j, bid);
  const StepProb<T> q = probs[pid];
  DevState* const st = q.st;
  // uniform per problem and unchanged during the launch: all or none of a
  // problem's workgroups take part
  if (st->done) return;
  const int nblk = q.nblk, Tp = nblk * TB;
  const int hb = nblk - 1 - 2 * j, ha = hb - 1, c = hb + 1, d = hb + 2;
  const bool has_a = ha >= 0, has_q = j >= 1;
  const int per = has_a ? 2 : 1, rt = bid / per;
  const bool role_a = bid % per == 1;  // the b workgroup of a row tile comes first
  const int k = role_a ? ha : hb;
  const int r0 = rt * TB, nrows = min(TB, q.n - r0);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int32_t* const flag = q.flow + (size_t)rt * nblk;
  T* const rowp = q.M + (size_t)r0 * Tp;
  auto tile = [&](int x) { return rowp + (size_t)x * TB; };
  auto vblk = [&](int x, int y) { return q.V + (size_t)x * TB * Tp + (size_t)y * TB; };
  acc_t acc[4], f[4];
  T rf[16], rl[16], rx[16];
  // waits until flag i reaches want; false (for every wave) once a wait of
  // the problem has stalled.  The barrier also means every wave is past its
  // reads of S0 / S1.
  auto wait_flag = [&](int i, int32_t want) -> bool {
    if (tid == 0) stalled = !poll_flags(flag + i, nullptr, want, st, spin_limit);
    __syncthreads();
    return !stalled;
  };
  // ... for two flags polled together
  auto wait_flag2 = [&](int i, int i2, int32_t want) -> bool {
    if (tid == 0) stalled = !poll_flags(flag + i, flag + i2, want, st, spin_limit);
    __syncthreads();
    return !stalled;
  };
  auto set_flag = [&](int i, int32_t v) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores (and loads) are complete
    __syncthreads();
    if (tid == 0) __hip_atomic_store(as_global(flag + i), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  // the accumulators hold -G_k so that every product adds in place
  load_acc<T>(acc, tile(k), Tp, nrows, lane, w);
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) acc[tj] = -acc[tj];
  if (role_a) set_flag(ha, FL_GLOADED);  // the tile may now take acc_b
  fetch_block<T>(rx, q.ldiag + (size_t)k * TB * TB, TB, TB, tid);
  // acc += F_i L_ik for the columns beyond the previous pair
  const int ilo = has_q ? d + 1 : nblk;
  if (ilo < nblk) fetch_block<T>(rl, vblk(nblk - 1, k), Tp, TB, tid);
  for (int i = nblk - 1; i >= ilo; --i) {
    if (!wait_flag(i, FL_F)) return;
    fetch_block2_coherent<T>(rf, tile(i), Tp, nrows, tid);
    put_block<T, false>(S1, rl, tid);  // L_ik
    if (i > ilo) fetch_block<T>(rl, vblk(i - 1, k), Tp, TB, tid);
    put_block2<T, true>(S0, rf, tid);  // F_i^T
    __syncthreads();
    tile_mma64<T>(acc, S0, S1, lane, w);
  }
  if (!role_a && has_a) {
    // acc_b for the a workgroup, in its tile once its G has been read
    if (!wait_flag(ha, FL_GLOADED)) return;
    if constexpr (sizeof(T) == 8) {
      acc_to_lds<T>(acc, S0, lane, w);  // (the wait's barrier: every wave is past its reads of S0)
      __syncthreads();
      store_block2_coherent(S0, tile(ha), Tp, nrows, tid);
    } else {
      store_acc_coherent<T>(acc, tile(ha), Tp, nrows, lane, w);
    }
    set_flag(ha, FL_ACCB);
  }
  // f = acc X_k^T
  __syncthreads();  // every wave is past its reads of S0 / S1
  acc_to_lds_t<T>(acc, S0, lane, w);
  put_block<T, true>(S1, rx, tid);  // X_k^T
  __syncthreads();
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) f[tj] = acc_t{0, 0, 0, 0};
  tile_mma64<T>(f, S0, S1, lane, w);
  if (role_a) {
    // f -= acc_b U
    fetch_block<T>(rl, vblk(ha, hb), Tp, TB, tid);  // U
    if (!wait_flag(ha, FL_ACCB)) return;
    fetch_block2_coherent<T>(rf, tile(ha), Tp, nrows, tid);  // acc_b
    put_block<T, false>(S1, rl, tid);
    put_block2<T, true>(S0, rf, tid);
    __syncthreads();
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] = acc_t{0, 0, 0, 0};
    tile_mma64<T>(acc, S0, S1, lane, w);
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) f[tj] -= acc[tj];
  }
  if (has_q) {
    // f += F_c B_c + F_d B_d with B = P_cb, P_db (b) or Q_c, Q_d (a)
    fetch_block<T>(rl, role_a ? vblk(ha, c) : vblk(hb, c), Tp, TB, tid);
    fetch_block<T>(rx, role_a ? vblk(ha, d) : vblk(hb, d), Tp, TB, tid);
    __syncthreads();  // every wave is past its reads of S0 / S1
    put_block<T, false>(S0, rl, tid);
    put_block<T, false>(S1, rx, tid);
    if (!wait_flag2(c, d, FL_F)) return;
    __builtin_amdgcn_s_setprio(3);  // the chain
    T fc[16], fd[16];
    if constexpr (sizeof(T) == 8) {
      fetch_afrag2_coherent(fc, tile(c), Tp, nrows, lane, w);
      fetch_afrag2_coherent(fd, tile(d), Tp, nrows, lane, w);
      __builtin_amdgcn_sched_barrier(0);  // every load issued before the first product waits
      tile_mma64_ra2<T>(f, fc, S0, lane);
      tile_mma64_ra2<T>(f, fd, S1, lane);
    } else {
      fetch_afrag_coherent<T>(fc, tile(c), Tp, nrows, lane, w);
      fetch_afrag_coherent<T>(fd, tile(d), Tp, nrows, lane, w);
      tile_mma64_ra<T>(f, fc, S0, lane);
      tile_mma64_ra<T>(f, fd, S1, lane);
    }
  }
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) f[tj] = -f[tj];
  if constexpr (sizeof(T) == 8) {
    // through LDS into coalesced 16-byte stores
    __syncthreads();  // every wave is past its reads of S0 / S1
    acc_to_lds<T>(f, S0, lane, w);
    __syncthreads();
    store_block2_coherent(S0, tile(k), Tp, nrows, tid);
  } else {
    store_acc_coherent<T>(f, tile(k), Tp, nrows, lane, w);
  }
  set_flag(k, FL_F);
}

// ------------------------- dataflow factorisation with the forward solve
// One launch holds, block column by block column, the lower tiles (i, k) of
// the factorisation and the tiles (rt, k) of the forward solve G L^T = M:
//
//   L_ik = (A_ik - sum_{j<k} L_ij L_kj^T) L_kk^{-T},
//   G_k  = (M_k  - sum_{j<k} G_j  L_kj^T) X_k,        X_k = L_kk^{-T}.
//
// A workgroup takes the products of the earlier columns as their ready
// flags appear.  As in the per-step form, every workgroup of column k
// factors the diagonal block itself, so the chain from one column to the
// next is a single hop: the diagonal workgroup publishes D_k updated
// through column k - 2 early, and each workgroup applies column k - 1
// (the same product in every workgroup, so all hold the same L_kk) and
// factors D_k with its tile's rows carried through the same column steps,
// which solves the tile.  The diagonal workgroup also forms and
// publishes X_k for the forward solve.  Every wait is on a lower workgroup
// id (columns in order; in a column the diagonal tile first, the forward
// tiles last), so the launch cannot deadlock; waits are bounded as in the
// backward solve.
template <typename T>
__device__ __forceinline__ void load_acc_coherent(typename Acc4<T>::type acc[4], const T* g, size_t ld, int lane,
                                                  int w) {
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[tj][r] = coherent_load<T>(g + (size_t)acc_row<T>(lane, w, r) * ld + acc_col(lane, tj));
}
template <typename T>
__device__ __forceinline__ void store_b4_coherent(const T s[16], T* g, size_t ld, int g4, int j) {
#pragma unroll
  for (int ii = 0; ii < 4; ++ii)
#pragma unroll
    for (int v = 0; v < 4; ++v) coherent_store<T>(g + (size_t)(4 * g4 + ii) * ld + j + 16 * v, s[4 * ii + v]);
}
__host__ __device__ inline int chol_fwd_flow_tiles(int nblk, int nrt) { return nblk * (nblk + 1) / 2 + nrt * nblk; }

template <typename T>
__global__ __launch_bounds__(256) void cflow_reset_kernel(const StepProb<T>* probs) {
  const StepProb<T>& q = probs[blockIdx.x];
  const int nf = ((q.n + TB - 1) / TB) * q.nblk, nc = (q.nblk + 2) * q.nblk + CU_SLOTS;
  const gptr<int32_t> f = as_global(q.flow), c = as_global(q.cflow);
  for (int e = threadIdx.x; e < nf; e += 256) f[e] = 0;
  for (int e = threadIdx.x; e < nc; e += 256) c[e] = 0;
}

// D -= L L^T on the lower 16 x 16 tiles of a 64 x 64 block only (the
// factorisation reads no entry above the diagonal), spread over the waves
// so that none takes more than seven tile products together with the four
// of its rows of the tile update: wave W forms tiles (W, tj), tj <= W,
// except (3, 0), which wave 0 forms (into qx) for wave 3.  Lk is the block
// in k-major form, as tile_mma64 reads it; the products run over k in the
// same order, so each tile is bitwise the one tile_mma64 forms.
template <typename T, int W>
__device__ __forceinline__ void lower_llt(typename Acc4<T>::type q[4], typename Acc4<T>::type& qx, const T* Lk,
                                          int lane) {
#pragma unroll 4
  for (int kk = 0; kk < TB; kk += 4) {
    const T* row = Lk + (kk + (lane >> 4)) * LDT + (lane & 15);
    const T a = row[16 * W];
#pragma unroll
    for (int tj = (W == 3 ? 1 : 0); tj <= W; ++tj) q[tj] = mfma4(a, row[16 * tj], q[tj]);
    if constexpr (W == 0) qx = mfma4(row[48], row[0], qx);
  }
}

template <typename T>
__global__ __launch_bounds__(256, 2) void chol_fwd_flow_kernel(const StepProb<T>* probs, const int* seg,
                                                               int nseg, int spin_limit) {
  typedef typename Acc4<T>::type acc_t;
  __shared__ T S0[TB * LDT];
  __shared__ T S1[TB * LDT];
  __shared__ __attribute__((aligned(16))) T colbuf[20 * TB];  // 3 published column blocks, 2 tile blocks
  __shared__ T invd[TB];
  __shared__ int stalled;
  int pid, k, bid;
  flow_segment(seg, nseg, blockIdx.x, pid, k, bid);
  const StepProb<T> q = probs[pid];
  DevState* const st = q.st;
  // Uniform per problem and unchanged during the launch: all or none of a
  // problem's workgroups take part.  (chol_fail is not a valid gate here:
  // this launch sets it, and a workgroup that left on it would never
  // publish its flags.  A failed problem's tiles are discarded later.)
  if (st->done) return;
  const int nblk = q.nblk, Tp = nblk * TB, nrt = (q.n + TB - 1) / TB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wu = __builtin_amdgcn_readfirstlane(w);  // wave-uniform
  const int sr = tid >> 2, q0 = tid & 3;   // strip layout (diagonal factorisation)
  const int bg = tid >> 4, bj = tid & 15;  // block-4 layout (triangular solves)
  int32_t* const lfl = q.cflow;                // [i nblk + j]: L_ij stored
  int32_t* const dfl = q.cflow + nblk * nblk;  // [k]: D_k through column k - 2 stored
  int32_t* const xfl = dfl + nblk;             // [k]: X_k stored
  // waits for one or two flags; false (for every wave) once the problem has
  // stalled.  The barrier also means every wave is past its reads of S0 / S1.
  auto wait = [&](const int32_t* a, const int32_t* b) -> bool {
    if (tid == 0) stalled = !poll_flags(a, b, 1, st, spin_limit);
    __syncthreads();
    return !stalled;
  };
  // The compute unit this workgroup runs on, and its counter of the
  // chain's workgroups (a tile of the current block column between its
  // last wait and its publication) running there: their dependent FP64
  // steps slow down several times beside another wave's matrix
  // instructions on the same SIMD, so accumulating workgroups hold back
  // their next product while the counter is set (at most 64 polls of ~500
  // cycles: 16 gave 1.38 ms per launch at R = 4000, 32 1.36, 64 1.31, 128
  // 1.32).
  const unsigned hw_id = __builtin_amdgcn_s_getreg((31 << 11) | 4);    // HW_ID
  const unsigned xcc_id = __builtin_amdgcn_s_getreg((31 << 11) | 20);  // XCC_ID
  int32_t* const cu_busy = q.cflow + (nblk + 2) * nblk +
                           (int)(((xcc_id & 7u) << 8) | (((hw_id >> 13) & 7u) << 5) | (((hw_id >> 12) & 1u) << 4) |
                                 ((hw_id >> 8) & 15u));
  // a wait for one or two flags that then holds back while a chain
  // workgroup runs on this unit
  auto wait_acc = [&](const int32_t* a, const int32_t* b) -> bool {
    if (tid == 0) {
      stalled = !poll_flags(a, b, 1, st, spin_limit);
      for (int s = 0; s < 64 && __hip_atomic_load(as_global(cu_busy), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0;
           ++s)
        __builtin_amdgcn_s_sleep(8);
    }
    __syncthreads();
    return !stalled;
  };
  auto chain_begin = [&]() {
    if (tid == 0) __hip_atomic_fetch_add(as_global(cu_busy), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  auto chain_end = [&]() {
    if (tid == 0) __hip_atomic_fetch_add(as_global(cu_busy), -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  auto publish = [&](int32_t* f) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores are acknowledged
    __syncthreads();
    if (tid == 0) __hip_atomic_store(as_global(f), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  auto blk = [&](int i, int j) { return q.V + (size_t)i * TB * Tp + (size_t)j * TB; };
  acc_t acc[4], p[4];
  T ra[16], rb[16];

  if (bid < nblk - k) {
    // ---- factorisation tile (i, k)
    const int i = k + bid;
    const bool diag = i == k;
    T* const tile = blk(i, k);
    load_acc<T>(acc, tile, Tp, TB, lane, w);  // A_ik, written before the launch
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) p[tj] = acc_t{0, 0, 0, 0};
    for (int j = 0; j + 1 < k; ++j) {  // columns j <= k - 2
      if (!wait_acc(lfl + i * nblk + j, diag ? nullptr : lfl + k * nblk + j)) return;
      fetch_block2_coherent<T>(ra, blk(i, j), Tp, TB, tid);
      if (!diag) fetch_block2_coherent<T>(rb, blk(k, j), Tp, TB, tid);
      put_block2<T, true>(S0, ra, tid);
      if (!diag) put_block2<T, true>(S1, rb, tid);
      __syncthreads();
      tile_mma64<T>(p, S0, diag ? S0 : S1, lane, w);  // += L_ij L_kj^T
    }
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] -= p[tj];
    acc_t dd[4];
    if (diag) {
      if (k >= 2) {
        store_acc_coherent<T>(acc, q.dpart + (size_t)k * TB * TB, TB, TB, lane, w);
        publish(dfl + k);
      }
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) dd[tj] = acc[tj];
    } else if (k >= 2) {
      if (!wait(dfl + k, nullptr)) return;
      load_acc_coherent<T>(dd, q.dpart + (size_t)k * TB * TB, TB, lane, w);
    } else {
      load_acc<T>(dd, blk(k, k), Tp, TB, lane, w);  // A_kk: no earlier columns to apply
    }
    if (k >= 1) {
      // column k - 1: the own tile and D_k
      if (!wait(lfl + i * nblk + k - 1, diag ? nullptr : lfl + k * nblk + k - 1)) return;
      __builtin_amdgcn_s_setprio(3);  // the chain
      if (!diag) chain_begin();
      fetch_block2_coherent<T>(rb, blk(k, k - 1), Tp, TB, tid);
      if (!diag) fetch_block2_coherent<T>(ra, blk(i, k - 1), Tp, TB, tid);
      put_block2<T, true>(S1, rb, tid);
      if (!diag) put_block2<T, true>(S0, ra, tid);
      __syncthreads();
      if (!diag) {
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) p[tj] = acc_t{0, 0, 0, 0};
        tile_mma64<T>(p, S0, S1, lane, w);
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) acc[tj] -= p[tj];
      }
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) p[tj] = acc_t{0, 0, 0, 0};
      if (sizeof(T) == 8 && !diag) {
        // the chain: the lower tiles of D_k's update only, balanced
        acc_t qx = acc_t{0, 0, 0, 0};
        switch (wu) {
          case 0: lower_llt<T, 0>(p, qx, S1, lane); break;
          case 1: lower_llt<T, 1>(p, qx, S1, lane); break;
          case 2: lower_llt<T, 2>(p, qx, S1, lane); break;
          default: lower_llt<T, 3>(p, qx, S1, lane); break;
        }
        if (wu == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) colbuf[lane * 4 + r] = qx[r];  // tile (3, 0), read after the barrier
        }
      } else {
        tile_mma64<T>(p, S1, S1, lane, w);
      }
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) dd[tj] -= p[tj];  // zero for the tiles not formed here
    }
    __syncthreads();  // every wave is past its reads of S0 / S1
    if (sizeof(T) == 8 && !diag && k >= 1 && wu == 3) {
#pragma unroll
      for (int r = 0; r < 4; ++r) dd[0][r] -= colbuf[lane * 4 + r];
    }
    acc_to_lds<T>(dd, S1, lane, w);
    if (!diag) acc_to_lds<T>(acc, S0, lane, w);
    __syncthreads();
    T d[16];
    lds_to_strip<T>(S1, d, sr, q0);
    if constexpr (sizeof(T) == 8) {
      if (!diag) {
        // the tile's rows ride through the factorisation of D_k: L_ik comes
        // out of the same column steps, with no separate substitution
        // (FP64 only: the FP32 instance spills with the second strip)
        T e[16];
        lds_to_strip<T>(S0, e, sr, q0);
        strip_potrf4_panel<T>(d, e, invd, colbuf, sr, q0);
        // L_ik through LDS (S0 is free: every thread read its strip before
        // the factorisation's first barrier) into coalesced 16-byte stores
#pragma unroll
        for (int u = 0; u < 16; ++u) S0[sr * LDT + q0 + 4 * u] = e[u];
        __syncthreads();
        store_block2_coherent(S0, tile, Tp, TB, tid);
        publish(lfl + i * nblk + k);
        if (k >= 1) chain_end();
        return;
      }
    }
    __syncthreads();
    const bool ok = strip_potrf4<T>(d, S1, invd, colbuf, sr, q0);  // S1 = L_kk
    T s[16];
    if (!diag) {  // FP32: the tile by substitution with L_kk
      lds_to_b4<T>(S0, s, bg, bj);
      b4_fwd<T>(s, S1, invd, bj);
      store_b4_coherent<T>(s, tile, Tp, bg, bj);
      publish(lfl + i * nblk + k);
      if (k >= 1) chain_end();
      return;
    }
    // the diagonal workgroup: L_kk, and X_k = L_kk^{-T} for the forward solve
    if (!ok && tid == 0) atomicExch(&st->chol_fail, 1);
    if (tid < TB) as_global(q.diagL)[k * TB + tid] = S1[tid * LDT + tid];
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
      for (int v = 0; v < 4; ++v) s[4 * ii + v] = (4 * bg + ii == bj + 16 * v) ? T(1) : T(0);
    b4_fwd<T>(s, S1, invd, bj);  // X_k
    store_b4_coherent<T>(s, q.ldiag + (size_t)k * TB * TB, TB, bg, bj);
    publish(xfl + k);
    return;
  }

  // ---- forward-solve tile (rt, k)
  const int rt = bid - (nblk - k);
  const int r0 = rt * TB, nrows = min(TB, q.n - r0);
  int32_t* const gfl = q.flow + (size_t)rt * nblk;
  T* const tile = q.M + (size_t)r0 * Tp + (size_t)k * TB;
  load_acc<T>(acc, tile, Tp, nrows, lane, w);  // M_k, written before the launch
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) p[tj] = acc_t{0, 0, 0, 0};
  for (int j = 0; j < k; ++j) {
    if (!wait_acc(gfl + j, lfl + k * nblk + j)) return;
    fetch_block2_coherent<T>(ra, q.M + (size_t)r0 * Tp + (size_t)j * TB, Tp, nrows, tid);  // G_j
    fetch_block2_coherent<T>(rb, blk(k, j), Tp, TB, tid);                                 // L_kj
    put_block2<T, true>(S0, ra, tid);
    put_block2<T, true>(S1, rb, tid);
    __syncthreads();
    tile_mma64<T>(p, S0, S1, lane, w);  // += G_j L_kj^T
  }
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) acc[tj] -= p[tj];
  if (!wait(xfl + k, nullptr)) return;
  __builtin_amdgcn_s_setprio(3);
  fetch_block2_coherent<T>(ra, q.ldiag + (size_t)k * TB * TB, TB, TB, tid);
  acc_to_lds_t<T>(acc, S0, lane, w);
  put_block2<T, false>(S1, ra, tid);  // X_k
  __syncthreads();
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) p[tj] = acc_t{0, 0, 0, 0};
  tile_mma64<T>(p, S0, S1, lane, w);  // G_k
  if constexpr (sizeof(T) == 8) {
    __syncthreads();  // every wave is past its reads of S0 / S1
    acc_to_lds<T>(p, S0, lane, w);
    __syncthreads();
    store_block2_coherent(S0, tile, Tp, nrows, tid);
  } else {
    store_acc_coherent<T>(p, tile, Tp, nrows, lane, w);
  }
  publish(gfl + k);
}

std::vector<int> flow_segments(int mode, const std::vector<int>& nblk, const std::vector<int>& n) {
  std::vector<int> seg;
  int start = 0, cmax = 0;
  for (int b : nblk) cmax = b > cmax ? b : cmax;
  for (int c = 0; c < cmax; ++c)
    for (size_t p = 0; p < nblk.size(); ++p) {
      if (c >= nblk[p]) continue;
      const int nrt = (n[p] + TB - 1) / TB;
      if (mode == STEP_BWD_PAIR) {
        // segment (problem, pair c): per row tile the b workgroup, then the
        // a workgroup (the pair's lower block, if any)
        if (c >= bwd_pair_count(nblk[p])) continue;
        seg.push_back(start);
        seg.push_back((int)p);
        seg.push_back(c);
        start += nrt * (nblk[p] - 1 - 2 * c >= 1 ? 2 : 1);
        continue;
      }
      const int k = mode == STEP_BWD_FLOW ? nblk[p] - 1 - c : c;
      seg.push_back(start);
      seg.push_back((int)p);
      seg.push_back(k);
      start += mode == STEP_BWD_FLOW ? nrt : nblk[p] - k + nrt;
    }
  seg.push_back(start);
  seg.push_back(-1);
  seg.push_back(-1);
  return seg;
}

int step_tiles(int mode, int nblk, int n, StepCfg c) {
  const int nrt = (n + TB - 1) / TB;
  switch (mode) {
    case STEP_CHOL: return chol_tiles(nblk, c.pw, c.pc, c.tc);
    case STEP_FWD: return fwd_tiles(nblk, nrt, c.pw, c.pf, c.tf);
    case STEP_CHOL_FWD: return chol_tiles(nblk, c.pw, c.pc, c.tc) + fwd_tiles(nblk, nrt, c.pw, c.pf, c.tf);
    case STEP_FLOW_RESET: return 1;
    case STEP_BWD_FLOW: return nrt * nblk;
    case STEP_CFLOW_RESET: return 1;
    case STEP_CHOL_FWD_FLOW: return chol_fwd_flow_tiles(nblk, nrt);
    case STEP_BWD_PREP: return bwd_prep_tiles(nblk);
    case STEP_BWD_PAIR: return nrt * nblk;
    default: return bwd_tiles(nblk, nrt, c.pw, c.pf, c.tf);
  }
}

template <typename T>
void step_group(hipStream_t s, int mode, const StepProb<T>* probs, const int* offs, int nprob, int total_tiles,
                StepCfg cfg, int retry_pass) {
  if (total_tiles <= 0) return;
  dim3 grid(total_tiles), block(256);
  switch (mode) {
    case STEP_CHOL:
      hipLaunchKernelGGL((step_kernel<T, STEP_CHOL>), grid, block, 0, s, probs, offs, nprob, cfg, retry_pass);
      break;
    case STEP_FWD:
      hipLaunchKernelGGL((step_kernel<T, STEP_FWD>), grid, block, 0, s, probs, offs, nprob, cfg, retry_pass);
      break;
    case STEP_BWD:
      hipLaunchKernelGGL((step_kernel<T, STEP_BWD>), grid, block, 0, s, probs, offs, nprob, cfg, retry_pass);
      break;
    case STEP_FLOW_RESET:  // one workgroup per problem
      hipLaunchKernelGGL((flow_reset_kernel<T>), dim3(nprob), block, 0, s, probs);
      break;
    case STEP_BWD_FLOW:  // offs: segment table, nprob: its segment count
      hipLaunchKernelGGL((bwd_flow_kernel<T>), grid, block, 0, s, probs, offs, nprob, g_flow_spin_limit);
      break;
    case STEP_CFLOW_RESET:  // one workgroup per problem
      hipLaunchKernelGGL((cflow_reset_kernel<T>), dim3(nprob), block, 0, s, probs);
      break;
    case STEP_CHOL_FWD_FLOW:  // offs: segment table, nprob: its segment count
      hipLaunchKernelGGL((chol_fwd_flow_kernel<T>), grid, block, 0, s, probs, offs, nprob, g_flow_spin_limit);
      break;
    case STEP_BWD_PREP:
      hipLaunchKernelGGL((bwd_prep_kernel<T>), grid, block, 0, s, probs, offs, nprob);
      break;
    case STEP_BWD_PAIR:  // offs: segment table, nprob: its segment count
      hipLaunchKernelGGL((bwd_pair_kernel<T>), grid, block, 0, s, probs, offs, nprob, g_flow_spin_limit);
      break;
    default:
      hipLaunchKernelGGL((step_kernel<T, STEP_CHOL_FWD>), grid, block, 0, s, probs, offs, nprob, cfg,
                         retry_pass);
  }
}

template <typename T>
bool panel_gemm(int kind, const StepProb<T>& q, int pw, int p, GemmArgs<T>& g) {
  const int Tp = TB * q.nblk;
  const int lo = pw * p;
  const int hi = q.nblk - 1 < lo + pw - 1 ? q.nblk - 1 : lo + pw - 1;
  if (lo > hi) return false;
  const int K = TB * (hi - lo + 1);
  const int c0 = TB * (hi + 1);
  const int32_t* done = &q.st->done;
  T* const V = q.V;
  T* const M = q.M;
  switch (kind) {
    case PG_SYRK:
      if (c0 >= Tp) return false;
      g = GemmArgs<T>{Tp - c0, Tp - c0, K, V + (size_t)c0 * Tp + TB * lo, Tp, V + (size_t)c0 * Tp + TB * lo,
                      nullptr, Tp, V + (size_t)c0 * Tp + c0, Tp, nullptr, T(-1), T(1), done};
      g.lower = 1;
      return true;
    case PG_FWD:
      if (c0 >= Tp) return false;
      g = GemmArgs<T>{q.n, Tp - c0, K, M + TB * lo, Tp, V + (size_t)c0 * Tp + TB * lo, nullptr, Tp, M + c0, Tp,
                      nullptr, T(-1), T(1), done};
      return true;
    default:
      if (lo == 0) return false;
      g = GemmArgs<T>{q.n, TB * lo, K, M + TB * lo, Tp, V + (size_t)TB * lo * Tp, nullptr, Tp, M, Tp, nullptr,
                      T(-1), T(1), done};
      return true;
  }
}

std::vector<SolveItem> solve_schedule(int sched, int max_nblk, int pw) {
  std::vector<SolveItem> out;
  if (pw < 1) pw = 1;
  const int P = panel_count(max_nblk, pw);
  auto step = [&](int mode, int pc, int tc, int pf, int tf) {
    out.push_back(SolveItem{mode, StepCfg{pw, pc, tc, pf, tf}, {-1, -1}, {0, 0}});
  };
  auto gemm = [&](int k0, int p0, int k1, int p1) {
    if (k0 < 0 && k1 < 0) return;
    out.push_back(SolveItem{-1, StepCfg{pw, -1, 0, -1, 0}, {k0, k1}, {p0, p1}});
  };
  switch (sched) {
    case SCHED_CHOL:
      for (int p = 0; p < P; ++p) {
        for (int t = 0; t < pw; ++t) step(STEP_CHOL, p, t, -1, 0);
        if (p + 1 < P) gemm(PG_SYRK, p, -1, 0);
      }
      break;
    case SCHED_CHOL_FWD:
      if (P == 1) {
        // one level: one dataflow launch
        step(STEP_CFLOW_RESET, -1, 0, -1, 0);
        step(STEP_CHOL_FWD_FLOW, -1, 0, -1, 0);
        break;
      }
      for (int p = 0; p <= P; ++p) {
        for (int t = 0; t < pw; ++t) step(STEP_CHOL_FWD, p < P ? p : -1, t, p - 1, t);
        if (p < P) gemm(p + 1 < P ? PG_SYRK : -1, p, p >= 1 ? PG_FWD : -1, p - 1);
      }
      break;
    case SCHED_FWD:
      for (int p = 0; p < P; ++p) {
        for (int t = 0; t < pw; ++t) step(STEP_FWD, -1, 0, p, t);
        if (p + 1 < P) gemm(PG_FWD, p, -1, 0);
      }
      break;
    default:
      if (P == 1) {
        // one level: the whole solve as one dataflow launch, in block pairs
        // after their set-up launch, or one block column per hop
        step(STEP_FLOW_RESET, -1, 0, 0, 0);
        if (g_bwd_form == 0) {
          step(STEP_BWD_PREP, -1, 0, 0, 0);
          step(STEP_BWD_PAIR, -1, 0, 0, 0);
        } else {
          step(STEP_BWD_FLOW, -1, 0, 0, 0);
        }
        break;
      }
      for (int p = P - 1; p >= 0; --p) {
        for (int t = 0; t < pw; ++t) step(STEP_BWD, -1, 0, p, t);
        if (p > 0) gemm(PG_BWD, p, -1, 0);
      }
  }
  return out;
}

template void step_group<double>(hipStream_t, int, const StepProb<double>*, const int*, int, int, StepCfg, int);
template void step_group<float>(hipStream_t, int, const StepProb<float>*, const int*, int, int, StepCfg, int);
template bool panel_gemm<double>(int, const StepProb<double>&, int, int, GemmArgs<double>&);
template bool panel_gemm<float>(int, const StepProb<float>&, int, int, GemmArgs<float>&);

}  // namespace thccp
