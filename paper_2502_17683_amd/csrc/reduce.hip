// Element-wise and reduction kernels of the CP-ALS sweep: the Gram-Hadamard
// normal matrix, the damped-retry bookkeeping, column normalisation with
// the CP weights (eq. cp4), and the matrix-free fit (Computational
// Details: fit = ||T - T~|| / ||T||).  All reductions run in a fixed order
// (no floating-point atomics), so repeated runs are bitwise identical.
#include <math.h>

#include "kernels.h"

namespace thccp {

// V = g0 o g1 o g2 on the R x R block, identity on the padding, plus mu I
// on the retry pass.
template <typename T>
__global__ __launch_bounds__(256) void form_V_kernel(T* V, int Tp, int R, const T* g0, const T* g1,
                                                      const T* g2, DevState* st, int retry_pass) {
  if (st->done) return;
  if (retry_pass && !st->retry_active) return;
  const T mu = retry_pass ? (T)st->mu : T(0);
  const size_t total = (size_t)Tp * Tp;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const int i = (int)(e / Tp), j = (int)(e % Tp);
    T v;
    if (i < R && j < R) {
      v = g0[e] * g1[e] * g2[e];
      if (i == j) v += mu;
    } else {
      v = (i == j) ? T(1) : T(0);
    }
    V[e] = v;
  }
}

template <typename T>
void form_normal_matrix(hipStream_t s, T* V, int Tp, int R, const T* g0, const T* g1, const T* g2,
                        DevState* st, int retry_pass) {
  const size_t total = (size_t)Tp * Tp;
  int grid = (int)((total + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL((form_V_kernel<T>), dim3(grid), dim3(256), 0, s, V, Tp, R, g0, g1, g2, st,
                     retry_pass);
}

// After the first factorisation pass: arm the damped retry (mu = 1e-12
// tr(V) / R, computed from the diagonals of the Grams) or flag failure.
template <typename T>
__global__ void retry_prepare_kernel(DevState* st, int allow_fallback, const T* g0, const T* g1,
                                     const T* g2, int R, int Tp) {
  __shared__ double part[256];
  if (st->done) return;
  const int tid = threadIdx.x;
  const int failed = st->chol_fail;
  double acc = 0.0;
  if (failed)
    for (int i = tid; i < R; i += 256) {
      const size_t d = (size_t)i * Tp + i;
      acc += (double)g0[d] * (double)g1[d] * (double)g2[d];
    }
  part[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    if (failed && allow_fallback) {
      st->retry_active = 1;
      st->fallbacks += 1;
      st->mu = 1e-12 * part[0] / (double)R;
    } else {
      st->retry_active = 0;
      if (failed) st->flags |= FLAG_NOT_SPD;
    }
    st->chol_fail = 0;
  }
}

template <typename T>
void retry_prepare_launch(hipStream_t s, DevState* st, int allow_fallback, const T* g0, const T* g1,
                          const T* g2, int R, int Tp) {
  hipLaunchKernelGGL((retry_prepare_kernel<T>), dim3(1), dim3(256), 0, s, st, allow_fallback, g0,
                     g1, g2, R, Tp);
}

// Column norms lambda_k of the solved factor, F = Msol / lambda, and (for
// the fit) the per-column partial sums of Msol o Msave.  One workgroup per
// 64 columns; 4 row groups reduced in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void normalise_kernel(const T* Msol, int n, int R, int ld, T* F,
                                                         T* lam, const T* Msave, double* inner_part,
                                                         DevState* st) {
  __shared__ double ss[4][64];
  __shared__ double si[4][64];
  if (st->done) return;
  const int tid = threadIdx.x, c = tid & 63, g = tid >> 6;
  const int col = blockIdx.x * 64 + c;
  double a = 0.0, b = 0.0;
  if (col < R)
    for (int s = g; s < n; s += 4) {
      const double v = (double)Msol[(size_t)s * ld + col];
      a += v * v;
      if (Msave) b += v * (double)Msave[(size_t)s * ld + col];
    }
  ss[g][c] = a;
  si[g][c] = b;
  __syncthreads();
  const double nrm = sqrt((ss[0][c] + ss[1][c]) + (ss[2][c] + ss[3][c]));
  if (col < R) {
    const double scale = nrm > 0.0 ? 1.0 / nrm : 1.0;
    for (int s = g; s < n; s += 4) {
      const size_t off = (size_t)s * ld + col;
      F[off] = (T)((double)Msol[off] * scale);
    }
    if (g == 0) {
      lam[col] = (T)nrm;
      if (inner_part) inner_part[col] = (si[0][c] + si[1][c]) + (si[2][c] + si[3][c]);
    }
  }
}

template <typename T>
void normalise_columns(hipStream_t s, const T* Msol, int n, int R, int ld, T* F, T* lam,
                       const T* Msave, double* inner_part, DevState* st) {
  hipLaunchKernelGGL((normalise_kernel<T>), dim3((R + 63) / 64), dim3(256), 0, s, Msol, n, R, ld, F,
                     lam, Msave, inner_part, st);
}

// ||G~||^2 = lambda^T (g0 o g1 o g2 o g3) lambda: per-row partials, then a
// single-workgroup final pass that also forms the fit and applies the
// stopping rule.
template <typename T>
__global__ __launch_bounds__(256) void model_norm_rows_kernel(const T* g0, const T* g1, const T* g2,
                                                              const T* g3, const T* lam, int R, int ld,
                                                              double* row_part, DevState* st) {
  __shared__ double part[256];
  if (st->done) return;
  const int i = blockIdx.x, tid = threadIdx.x;
  double acc = 0.0;
  for (int j = tid; j < R; j += 256) {
    const size_t e = (size_t)i * ld + j;
    acc += (double)g0[e] * (double)g1[e] * (double)g2[e] * (double)g3[e] * (double)lam[j];
  }
  part[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) row_part[i] = part[0] * (double)lam[i];
}

__global__ __launch_bounds__(256) void fit_final_kernel(const double* row_part, const double* inner_part,
                                                        int R, double* fit_hist, int hist_cap,
                                                        double tol, double fit_floor, DevState* st) {
  __shared__ double pa[256];
  __shared__ double pb[256];
  if (st->done) return;
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = tid; i < R; i += 256) {
    a += row_part[i];
    b += inner_part[i];
  }
  pa[tid] = a;
  pb[tid] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      pa[tid] += pa[tid + w];
      pb[tid] += pb[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double model2 = pa[0], inner = pb[0];
    double res2 = st->norm2 - 2.0 * inner + model2;
    if (res2 < 0.0) res2 = 0.0;
    const double fit = sqrt(res2) / sqrt(st->norm2);
    st->inner = inner;
    st->model2 = model2;
    if (!isfinite(fit)) st->flags |= FLAG_NONFINITE;
    const int k = st->sweeps;
    fit_hist[k % hist_cap] = fit;
    st->sweeps = k + 1;
    const double prev = st->fit_prev;
    if (fit <= fit_floor || (prev >= 0.0 && fabs(fit - prev) <= tol * prev) || !isfinite(fit) ||
        (st->flags & FLAG_NOT_SPD))
      st->done = 1;
    st->fit_prev = fit;
  }
}

template <typename T>
void fit_update(hipStream_t s, const T* const g[4], const T* lam, int R, int ld,
                const double* inner_part, double* scratch, double* fit_hist, int hist_cap, double tol,
                double fit_floor, DevState* st) {
  hipLaunchKernelGGL((model_norm_rows_kernel<T>), dim3(R), dim3(256), 0, s, g[0], g[1], g[2], g[3],
                     lam, R, ld, scratch, st);
  hipLaunchKernelGGL(fit_final_kernel, dim3(1), dim3(256), 0, s, scratch, inner_part, R, fit_hist,
                     hist_cap, tol, fit_floor, st);
}

// ------------------------------------------------------------------ set-up
__global__ void hadamard_inplace_kernel(double* A, const double* B, size_t count) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (size_t)gridDim.x * 256)
    A[e] *= B[e];
}
void hadamard_inplace_f64(hipStream_t s, double* A, const double* B, size_t count) {
  int grid = (int)((count + 255) / 256);
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(hadamard_inplace_kernel, dim3(grid), dim3(256), 0, s, A, B, count);
}

// sum_ij P[j][i] Q[i][j] over R x R (ld): 64x64 tiles through LDS, one
// partial per tile, then a fixed-order final sum.
__global__ __launch_bounds__(256) void tdot_tiles_kernel(const double* P, const double* Q, int R, int ld,
                                                         double* partials) {
  __shared__ double t[64][65];
  __shared__ double part[256];
  const int nt = (R + 63) / 64;
  const int bi = blockIdx.x / nt, bj = blockIdx.x % nt;
  const int tid = threadIdx.x;
  // t[c][r] = P[bj*64 + r][bi*64 + c]  (P block (bj, bi), transposed)
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const int gr = bj * 64 + r, gc = bi * 64 + c;
    t[c][r] = (gr < R && gc < R) ? P[(size_t)gr * ld + gc] : 0.0;
  }
  __syncthreads();
  double acc = 0.0;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const int gi = bi * 64 + r, gj = bj * 64 + c;
    if (gi < R && gj < R) acc += t[r][c] * Q[(size_t)gi * ld + gj];
  }
  part[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) partials[blockIdx.x] = part[0];
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double* partials, int count, double* out) {
  __shared__ double part[256];
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int i = tid; i < count; i += 256) acc += partials[i];
  part[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) *out = part[0];
}

void transposed_dot_f64(hipStream_t s, const double* P, const double* Q, int R, int ld,
                        double* partials, double* out) {
  const int nt = (R + 63) / 64;
  hipLaunchKernelGGL(tdot_tiles_kernel, dim3(nt * nt), dim3(256), 0, s, P, Q, R, ld, partials);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partials, nt * nt, out);
}

__global__ void fill_kernel(uint32_t* p, size_t words) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < words; e += (size_t)gridDim.x * 256)
    p[e] = 0u;
}
void fill_bytes(hipStream_t s, void* p, size_t bytes) {
  const size_t words = bytes / 4;
  int grid = (int)((words + 255) / 256);
  if (grid > 16384) grid = 16384;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, s, (uint32_t*)p, words);
}

__global__ void state_reset_kernel(DevState* st, const double* norm2_src) {
  if (threadIdx.x == 0) {
    st->norm2 = *norm2_src;
    st->fit_prev = -1.0;
    st->inner = 0.0;
    st->model2 = 0.0;
    st->mu = 0.0;
    st->done = 0;
    st->sweeps = 0;
    st->flags = 0;
    st->chol_fail = 0;
    st->fallbacks = 0;
    st->retry_active = 0;
    if (!(st->norm2 > 0.0) || !isfinite(st->norm2)) {
      st->flags |= FLAG_NONFINITE;
      st->done = 1;
    }
  }
}
void state_reset(hipStream_t s, DevState* st, double* norm2_src) {
  hipLaunchKernelGGL(state_reset_kernel, dim3(1), dim3(64), 0, s, st, norm2_src);
}

__global__ void cast_d2f_kernel(const double* a, float* b, size_t n) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256)
    b[e] = (float)a[e];
}
__global__ void cast_f2d_kernel(const float* a, double* b, size_t n) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256)
    b[e] = (double)a[e];
}
void cast_f64_to_f32(hipStream_t s, const double* a, float* b, size_t count) {
  int grid = (int)((count + 255) / 256);
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(cast_d2f_kernel, dim3(grid), dim3(256), 0, s, a, b, count);
}
void cast_f32_to_f64(hipStream_t s, const float* a, double* b, size_t count) {
  int grid = (int)((count + 255) / 256);
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(cast_f2d_kernel, dim3(grid), dim3(256), 0, s, a, b, count);
}

// dst (n x R, ld) = src (n x R, dense) with unit-norm columns.
__global__ __launch_bounds__(256) void init_norm_kernel(const double* src, int n, int R, int ld, double* dst) {
  __shared__ double ss[4][64];
  const int tid = threadIdx.x, c = tid & 63, g = tid >> 6;
  const int col = blockIdx.x * 64 + c;
  double a = 0.0;
  if (col < R)
    for (int s = g; s < n; s += 4) {
      const double v = src[(size_t)s * R + col];
      a += v * v;
    }
  ss[g][c] = a;
  __syncthreads();
  const double nrm = sqrt((ss[0][c] + ss[1][c]) + (ss[2][c] + ss[3][c]));
  if (col < R) {
    const double scale = nrm > 0.0 ? 1.0 / nrm : 1.0;
    for (int s = g; s < n; s += 4) dst[(size_t)s * ld + col] = src[(size_t)s * R + col] * scale;
  }
}
void copy_normalised_init(hipStream_t s, const double* src, int n, int R, int ld, double* dst) {
  hipLaunchKernelGGL(init_norm_kernel, dim3((R + 63) / 64), dim3(256), 0, s, src, n, R, ld, dst);
}

template void form_normal_matrix<double>(hipStream_t, double*, int, int, const double*, const double*,
                                         const double*, DevState*, int);
template void form_normal_matrix<float>(hipStream_t, float*, int, int, const float*, const float*,
                                        const float*, DevState*, int);
template void retry_prepare_launch<double>(hipStream_t, DevState*, int, const double*, const double*,
                                           const double*, int, int);
template void retry_prepare_launch<float>(hipStream_t, DevState*, int, const float*, const float*,
                                          const float*, int, int);
template void normalise_columns<double>(hipStream_t, const double*, int, int, int, double*, double*,
                                        const double*, double*, DevState*);
template void normalise_columns<float>(hipStream_t, const float*, int, int, int, float*, float*,
                                       const float*, double*, DevState*);
template void fit_update<double>(hipStream_t, const double* const*, const double*, int, int,
                                 const double*, double*, double*, int, double, double, DevState*);
template void fit_update<float>(hipStream_t, const float* const*, const float*, int, int,
                                const double*, double*, double*, int, double, double, DevState*);

}  // namespace thccp
