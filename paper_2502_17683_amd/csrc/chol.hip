// Blocked Cholesky factorisation of the Gram-Hadamard matrix V and the
// row-wise solve F = M V^{-1} of the ALS normal equations.
//
// V is Tp x Tp row-major (Tp = 64 nblk; padding rows/columns hold the
// identity).  Right-looking, 64-wide blocks, ONE launch per block step:
// step j updates every trailing tile (i, k), k >= j+1, with panel j and,
// for the tiles of column j+1, immediately factors the (updated) diagonal
// block in LDS -- every workgroup of that column does so redundantly, so
// no workgroup ever waits on another -- and solves its own panel tile.
// The diagonal blocks of L are never written back to V (other workgroups
// of the same launch still read the unfactored block); their inverses go
// to `linv` and feed the triangular solves as small GEMMs.
#include <math.h>

#include "kernels.h"
#include "mfma.h"

namespace thccp {

// Unblocked Cholesky of the 64x64 block in LDS (row-major, stride LDT),
// outer-product form with deferred column scaling: one barrier per column.
// Returns false if a pivot was not positive (the block is then garbage
// but finite).
template <typename T>
__device__ bool lds_potrf64(T* D, int tid) {
  bool ok = true;
  const int r = tid >> 2, q0 = tid & 3;
  for (int c = 0; c < TB; ++c) {
    T piv = D[c * LDT + c];
    if (!(piv > T(0)) || !isfinite((double)piv)) { ok = false; piv = T(1); }
    const T inv = T(1) / piv;
    if (r > c) {
      const T lrc = D[r * LDT + c] * inv;
      for (int q = c + 1 + q0; q <= r; q += 4) D[r * LDT + q] -= lrc * D[q * LDT + c];
    }
    __syncthreads();
  }
  // D[c][c] still holds pivot c; scale the columns, clear the upper part.
  for (int e = tid; e < TB * TB; e += 256) {
    const int rr = e >> 6, cc = e & 63;
    if (cc < rr) {
      T pv = D[cc * LDT + cc];
      if (!(pv > T(0))) pv = T(1);
      D[rr * LDT + cc] /= sqrt(pv);
    }
  }
  __syncthreads();
  for (int e = tid; e < TB * TB; e += 256) {
    const int rr = e >> 6, cc = e & 63;
    if (cc > rr) D[rr * LDT + cc] = T(0);
    else if (cc == rr) {
      T pv = D[rr * LDT + rr];
      D[rr * LDT + rr] = sqrt(pv > T(0) ? pv : T(1));
    }
  }
  __syncthreads();
  return ok;
}

// Inverse of the lower-triangular 64x64 block L (LDS, row-major) written
// TRANSPOSED into XT (XT[c][r] = inv(L)[r][c]).  Forward substitution on
// the identity, outer-product form, one barrier per row.
template <typename T>
__device__ void lds_trtri64_t(const T* L, T* X, T* XT, int tid) {
  for (int e = tid; e < TB * TB; e += 256) {
    const int rr = e >> 6, cc = e & 63;
    X[rr * LDT + cc] = (rr == cc) ? T(1) : T(0);
  }
  __syncthreads();
  const int r = tid >> 2, q0 = tid & 3;
  for (int k = 0; k < TB; ++k) {
    // rows r > k: X[r][:] -= L[r][k] / L[k][k] * X[k][:]   (columns <= k)
    if (r > k) {
      const T f = L[r * LDT + k] / L[k * LDT + k];
      for (int q = q0; q <= k; q += 4) X[r * LDT + q] -= f * X[k * LDT + q];
    }
    __syncthreads();
  }
  for (int e = tid; e < TB * TB; e += 256) {
    const int rr = e >> 6, cc = e & 63;
    XT[cc * LDT + rr] = X[rr * LDT + cc] / L[rr * LDT + rr];
  }
  __syncthreads();
}

// Maps a linear block id onto the lower-triangular tile (i, k) of the
// trailing matrix, i >= k >= k0; column k0 comes first.
__device__ __forceinline__ void tri_tile(int bid, int k0, int nblk, int& i, int& k) {
  k = k0;
  int len = nblk - k0;
  while (bid >= len) { bid -= len; ++k; --len; }
  i = k + bid;
}

template <typename T>
__global__ __launch_bounds__(256) void chol_step_kernel(T* V, int nblk, int j, T* linv,
                                                         T* diagL, DevState* st, int retry_pass) {
  typedef typename Acc4<T>::type acc_t;
  __shared__ T S0[TB * LDT];
  __shared__ T S1[TB * LDT];
  __shared__ T S2[TB * LDT];
  if (st->done) return;
  if (retry_pass ? !st->retry_active : st->chol_fail) return;

  const int Tp = nblk * TB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int i, k;
  tri_tile(blockIdx.x, j + 1, nblk, i, k);
  T* tile = V + (size_t)i * TB * Tp + (size_t)k * TB;

  acc_t acc[4];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      acc[tj][r] = tile[(size_t)acc_row<T>(lane, w, r) * Tp + acc_col(lane, tj)];

  if (j >= 0) {
    // tile -= L_ij L_kj^T
    block_to_lds<T, true>(S0, V + (size_t)i * TB * Tp + (size_t)j * TB, Tp, TB, tid);
    block_to_lds<T, true>(S1, V + (size_t)k * TB * Tp + (size_t)j * TB, Tp, TB, tid);
    __syncthreads();
    acc_t p[4];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) p[tj] = acc_t{0, 0, 0, 0};
    tile_mma64<T>(p, S0, S1, lane, w);
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] -= p[tj];
    if (k != j + 1) {
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          tile[(size_t)acc_row<T>(lane, w, r) * Tp + acc_col(lane, tj)] = acc[tj][r];
      return;
    }
  }
  // Column k = j + 1: updated diagonal block D = A_kk - L_kj L_kj^T into S2.
  if (i == k) {
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) S2[acc_row<T>(lane, w, r) * LDT + acc_col(lane, tj)] = acc[tj][r];
  } else {
    const T* dblk = V + (size_t)k * TB * Tp + (size_t)k * TB;
    acc_t d[4];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) d[tj][r] = dblk[(size_t)acc_row<T>(lane, w, r) * Tp + acc_col(lane, tj)];
    if (j >= 0) {
      acc_t p[4];
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) p[tj] = acc_t{0, 0, 0, 0};
      tile_mma64<T>(p, S1, S1, lane, w);
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) d[tj] -= p[tj];
    }
    __syncthreads();  // S0 is reused below
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) S2[acc_row<T>(lane, w, r) * LDT + acc_col(lane, tj)] = d[tj][r];
  }
  __syncthreads();
  const bool ok = lds_potrf64<T>(S2, tid);
  // inverse of L_kk, transposed, into S1 (S0 is scratch)
  lds_trtri64_t<T>(S2, S0, S1, tid);
  if (i == k) {
    if (!ok && tid == 0) {
      if (retry_pass) atomicOr(&st->flags, (int)FLAG_NOT_SPD);
      else atomicExch(&st->chol_fail, 1);
    }
    T* out = linv + (size_t)k * TB * TB;
    for (int e = tid; e < TB * TB; e += 256) {
      const int rr = e >> 6, cc = e & 63;
      out[rr * TB + cc] = S1[cc * LDT + rr];
    }
    if (tid < TB) diagL[k * TB + tid] = S2[tid * LDT + tid];
    return;
  }
  // Panel tile: L_ik = A'_ik inv(L_kk)^T.  A operand from acc via LDS.
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) S0[acc_col(lane, tj) * LDT + acc_row<T>(lane, w, r)] = acc[tj][r];
  __syncthreads();
  // B[kk][c] = inv(L)[c][kk] = XT[kk][c]... S1 holds XT[c][r] = inv[r][c];
  // we need B[kk][c] = inv[c][kk] = S1[kk][c].
  acc_t o[4];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) o[tj] = acc_t{0, 0, 0, 0};
  tile_mma64<T>(o, S0, S1, lane, w);
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) tile[(size_t)acc_row<T>(lane, w, r) * Tp + acc_col(lane, tj)] = o[tj][r];
}

template <typename T>
void chol_factor(hipStream_t s, T* V, int nblk, T* linv, T* diagL, DevState* st, int retry_pass) {
  for (int j = -1; j <= nblk - 2; ++j) {
    const int t = nblk - 1 - j;
    const int tiles = (j < 0) ? nblk : t * (t + 1) / 2;  // step -1: column 0 only
    hipLaunchKernelGGL((chol_step_kernel<T>), dim3(tiles), dim3(256), 0, s, V, nblk, j, linv,
                       diagL, st, retry_pass);
  }
}

// ------------------------------------------------------------------ solves
// Row tiles of 64 rows of M (n x Tp).  Forward: G L^T = M; backward: F L = G.
template <typename T>
__global__ __launch_bounds__(256) void trsm_fwd_kernel(const T* V, int nblk, const T* linv, T* M,
                                                        int n, int j, DevState* st) {
  typedef typename Acc4<T>::type acc_t;
  __shared__ T S0[TB * LDT];
  __shared__ T S1[TB * LDT];
  if (st->done) return;
  const int Tp = nblk * TB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nrt = (n + TB - 1) / TB;
  const int rt = blockIdx.x % nrt;
  const int k = j + 1 + blockIdx.x / nrt;
  const int r0 = rt * TB;
  const int nrows = min(TB, n - r0);
  T* tile = M + (size_t)r0 * Tp + (size_t)k * TB;

  acc_t acc[4];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = acc_row<T>(lane, w, r);
      acc[tj][r] = row < nrows ? tile[(size_t)row * Tp + acc_col(lane, tj)] : T(0);
    }
  if (j >= 0) {
    // M_k -= G_j L_kj^T : A = G_j (rows x 64), B[kk][c] = L_kj[c][kk]
    block_to_lds<T, true>(S0, M + (size_t)r0 * Tp + (size_t)j * TB, Tp, nrows, tid);
    block_to_lds<T, true>(S1, V + (size_t)k * TB * Tp + (size_t)j * TB, Tp, TB, tid);
    __syncthreads();
    acc_t p[4];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) p[tj] = acc_t{0, 0, 0, 0};
    tile_mma64<T>(p, S0, S1, lane, w);
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] -= p[tj];
  }
  if (k == j + 1) {
    // G_k = M'_k inv(L_kk)^T : B[kk][c] = inv[c][kk]
    __syncthreads();
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) S0[acc_col(lane, tj) * LDT + acc_row<T>(lane, w, r)] = acc[tj][r];
    block_to_lds<T, true>(S1, linv + (size_t)k * TB * TB, TB, TB, tid);
    __syncthreads();
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] = acc_t{0, 0, 0, 0};
    tile_mma64<T>(acc, S0, S1, lane, w);
  }
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = acc_row<T>(lane, w, r);
      if (row < nrows) tile[(size_t)row * Tp + acc_col(lane, tj)] = acc[tj][r];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void trsm_bwd_kernel(const T* V, int nblk, const T* linv, T* M,
                                                        int n, int j, DevState* st) {
  typedef typename Acc4<T>::type acc_t;
  __shared__ T S0[TB * LDT];
  __shared__ T S1[TB * LDT];
  if (st->done) return;
  const int Tp = nblk * TB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nrt = (n + TB - 1) / TB;
  const int rt = blockIdx.x % nrt;
  const int k = j - 1 - blockIdx.x / nrt;  // k = j-1, j-2, ..., 0
  const int r0 = rt * TB;
  const int nrows = min(TB, n - r0);
  T* tile = M + (size_t)r0 * Tp + (size_t)k * TB;

  acc_t acc[4];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = acc_row<T>(lane, w, r);
      acc[tj][r] = row < nrows ? tile[(size_t)row * Tp + acc_col(lane, tj)] : T(0);
    }
  if (j < nblk) {
    // G_k -= F_j L_jk : A = F_j, B[kk][c] = L_jk[kk][c]
    block_to_lds<T, true>(S0, M + (size_t)r0 * Tp + (size_t)j * TB, Tp, nrows, tid);
    block_to_lds<T, false>(S1, V + (size_t)j * TB * Tp + (size_t)k * TB, Tp, TB, tid);
    __syncthreads();
    acc_t p[4];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) p[tj] = acc_t{0, 0, 0, 0};
    tile_mma64<T>(p, S0, S1, lane, w);
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] -= p[tj];
  }
  if (k == j - 1) {
    // F_k = G'_k inv(L_kk) : B[kk][c] = inv[kk][c]
    __syncthreads();
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) S0[acc_col(lane, tj) * LDT + acc_row<T>(lane, w, r)] = acc[tj][r];
    block_to_lds<T, false>(S1, linv + (size_t)k * TB * TB, TB, TB, tid);
    __syncthreads();
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] = acc_t{0, 0, 0, 0};
    tile_mma64<T>(acc, S0, S1, lane, w);
  }
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = acc_row<T>(lane, w, r);
      if (row < nrows) tile[(size_t)row * Tp + acc_col(lane, tj)] = acc[tj][r];
    }
}

template <typename T>
void chol_solve_rows(hipStream_t s, const T* V, int nblk, const T* linv, T* M, int n, DevState* st) {
  if (n <= 0) return;
  const int nrt = (n + TB - 1) / TB;
  for (int j = -1; j <= nblk - 2; ++j) {
    const int cols = (j < 0) ? 1 : nblk - 1 - j;
    hipLaunchKernelGGL((trsm_fwd_kernel<T>), dim3(nrt * cols), dim3(256), 0, s, V, nblk, linv, M, n,
                       j, st);
  }
  for (int j = nblk; j >= 1; --j) {
    const int cols = (j == nblk) ? 1 : j;
    hipLaunchKernelGGL((trsm_bwd_kernel<T>), dim3(nrt * cols), dim3(256), 0, s, V, nblk, linv, M, n,
                       j, st);
  }
}

template void chol_factor<double>(hipStream_t, double*, int, double*, double*, DevState*, int);
template void chol_factor<float>(hipStream_t, float*, int, float*, float*, DevState*, int);
template void chol_solve_rows<double>(hipStream_t, const double*, int, const double*, double*, int,
                                      DevState*);
template void chol_solve_rows<float>(hipStream_t, const float*, int, const float*, float*, int,
                                     DevState*);

}  // namespace thccp
