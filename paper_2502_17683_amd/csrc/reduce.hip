// Element-wise and reduction kernels of the CP-ALS sweep: the Gram-Hadamard
// normal matrix, the damped-retry bookkeeping, column normalisation with
// the CP weights (eq. cp4), and the matrix-free fit (Computational
// Details: fit = ||T - T~|| / ||T||).  All reductions run in a fixed order
// (no floating-point atomics), so repeated runs are bitwise identical.
#include <math.h>

#include "kernels.h"

namespace thccp {

// V = g0 o g1 o g2 on the R x R block, identity on the padding, plus mu I
// on the retry pass.  blockIdx.y selects the problem.  V is symmetric and
// the factorisation reads only its lower 64 x 64 blocks (diagonal blocks
// whole), so only those are formed; the Grams are computed on the lower
// tiles only, which cover them.  One workgroup per lower block (row-major
// order: block row r holds r + 1 blocks), two adjacent elements per thread
// and step.
template <typename T>
__global__ __launch_bounds__(256) void form_V_kernel(const FormVArgs<T>* tab, int retry_pass) {
  const FormVArgs<T> a = tab[blockIdx.y];
  DevState* st = a.st;
  if (st->done) return;
  if (retry_pass && !st->retry_active) return;
  const int nb = a.Tp / 64, b = blockIdx.x;
  if (b >= nb * (nb + 1) / 2) return;
  int r = (int)((sqrtf(8.f * (float)b + 1.f) - 1.f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= b) ++r;
  while (r * (r + 1) / 2 > b) --r;
  const int c = b - r * (r + 1) / 2;
  const T mu = retry_pass ? (T)st->mu : T(0);
  const int R = a.R;
  typedef T v2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int idx = threadIdx.x + 256 * e;
    const int i = 64 * r + (idx >> 5), j = 64 * c + 2 * (idx & 31);
    const size_t off = (size_t)i * a.Tp + j;
    v2 v;
    if (i < R && j + 1 < R) {
      const v2 x = *(const gptr<const v2>)(as_global(a.g0) + off);
      const v2 y = *(const gptr<const v2>)(as_global(a.g1) + off);
      const v2 z = *(const gptr<const v2>)(as_global(a.g2) + off);
      v = x * y * z;
      if (i == j) v.x += mu;
      if (i == j + 1) v.y += mu;
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int jj = j + h;
        T t;
        if (i < R && jj < R) {
          t = as_global(a.g0)[off + h] * as_global(a.g1)[off + h] * as_global(a.g2)[off + h];
          if (i == jj) t += mu;
        } else {
          t = (i == jj) ? T(1) : T(0);
        }
        v[h] = t;
      }
    }
    *(gptr<v2>)(as_global(a.V) + off) = v;
  }
}

template <typename T>
void form_v_group(hipStream_t s, const FormVArgs<T>* tab, int nprob, int max_Tp, int retry_pass) {
  const int nb = max_Tp / 64;
  hipLaunchKernelGGL((form_V_kernel<T>), dim3(nb * (nb + 1) / 2, nprob), dim3(256), 0, s, tab, retry_pass);
}

// After the first factorisation pass: arm the damped retry (mu = 1e-12
// tr(V) / R, computed from the diagonals of the Grams) or flag failure.
template <typename T>
__global__ void retry_prepare_kernel(const FormVArgs<T>* tab, int allow_fallback) {
  __shared__ double part[256];
  const FormVArgs<T> a = tab[blockIdx.x];
  DevState* st = a.st;
  if (st->done) return;
  const int tid = threadIdx.x;
  const int failed = st->chol_fail;
  double acc = 0.0;
  if (failed)
    for (int i = tid; i < a.R; i += 256) {
      const size_t d = (size_t)i * a.Tp + i;
      acc += (double)a.g0[d] * (double)a.g1[d] * (double)a.g2[d];
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
      st->mu = 1e-12 * part[0] / (double)a.R;
    } else {
      st->retry_active = 0;
      if (failed) st->flags |= FLAG_NOT_SPD;
    }
    st->chol_fail = 0;
  }
}

template <typename T>
void retry_prepare_group(hipStream_t s, const FormVArgs<T>* tab, int nprob, int allow_fallback) {
  hipLaunchKernelGGL((retry_prepare_kernel<T>), dim3(nprob), dim3(256), 0, s, tab, allow_fallback);
}

// Column norms lambda_k of the solved factor, F = Msol / lambda, and (for
// the fit) the per-column partial sums of Msol o Msave.  One workgroup per
// 16 columns (~R/16 workgroups, enough to keep HBM busy); 16 row groups
// reduced in a fixed order.  A thread's rows are read 16 at a time before
// they are summed (in row order), so that each thread has 16 loads in
// flight instead of waiting on one load per row.
template <typename T>
__global__ __launch_bounds__(256) void normalise_kernel(const NormArgs<T>* tab) {
  __shared__ double ss[16][16];
  __shared__ double si[16][16];
  const NormArgs<T> a = tab[blockIdx.y];
  if (a.st->done) return;
  const int tid = threadIdx.x, c = tid & 15, g = tid >> 4;
  const int col = blockIdx.x * 16 + c;
  if (blockIdx.x * 16 >= a.R) return;
  const int n = a.n, R = a.R, ld = a.ld;
  const gptr<const T> Msol = as_global(a.Msol), Msave = as_global(a.Msave);
  constexpr int NB = 16;
  double x = 0.0, y = 0.0;
  if (col < R) {
    for (int s0 = g; s0 < n; s0 += 16 * NB) {
      T v[NB], m[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int s = s0 + 16 * u;
        v[u] = s < n ? Msol[(size_t)s * ld + col] : T(0);
        m[u] = (a.Msave && s < n) ? Msave[(size_t)s * ld + col] : T(0);
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const double dv = (double)v[u];
        x += dv * dv;
        if (a.Msave) y += dv * (double)m[u];
      }
    }
  }
  ss[g][c] = x;
  si[g][c] = y;
  __syncthreads();
  double n2 = 0.0, ip = 0.0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    n2 += ss[r][c];
    ip += si[r][c];
  }
  const double nrm = sqrt(n2);
  if (col < R) {
    const double scale = nrm > 0.0 ? 1.0 / nrm : 1.0;
    for (int s0 = g; s0 < n; s0 += 16 * NB) {
      T v[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int s = s0 + 16 * u;
        v[u] = s < n ? Msol[(size_t)s * ld + col] : T(0);
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int s = s0 + 16 * u;
        if (s < n) as_global(a.F)[(size_t)s * ld + col] = (T)((double)v[u] * scale);
      }
    }
    if (g == 0) {
      a.lam[col] = (T)nrm;
      if (a.inner_part) a.inner_part[col] = ip;
    }
  }
}

template <typename T>
void normalise_group(hipStream_t s, const NormArgs<T>* tab, int nprob, int max_R) {
  hipLaunchKernelGGL((normalise_kernel<T>), dim3((max_R + 15) / 16, nprob), dim3(256), 0, s, tab);
}

// Tied model: inner_part[k] = lam[k] sum_s F3[s,k] M3[s,k] (the <G, G~>
// partials from the mode-3 MTTKRP of the tied factors; F3 is read through
// the Msol field, F is unused).
template <typename T>
__global__ __launch_bounds__(256) void tied_inner_kernel(const NormArgs<T>* tab) {
  __shared__ double si[16][16];
  const NormArgs<T> a = tab[blockIdx.y];
  if (a.st->done) return;
  const int tid = threadIdx.x, c = tid & 15, g = tid >> 4;
  const int col = blockIdx.x * 16 + c;
  if (blockIdx.x * 16 >= a.R) return;
  const gptr<const T> F3 = as_global(a.Msol), M3 = as_global(a.Msave);
  double y = 0.0;
  if (col < a.R) {
#pragma unroll 4
    for (int s = g; s < a.n; s += 16) y += (double)F3[(size_t)s * a.ld + col] * (double)M3[(size_t)s * a.ld + col];
  }
  si[g][c] = y;
  __syncthreads();
  if (g == 0 && col < a.R) {
    double ip = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) ip += si[r][c];
    a.inner_part[col] = (double)as_global(a.lam)[col] * ip;
  }
}
template <typename T>
void tied_inner_group(hipStream_t s, const NormArgs<T>* tab, int nprob, int max_R) {
  hipLaunchKernelGGL((tied_inner_kernel<T>), dim3((max_R + 15) / 16, nprob), dim3(256), 0, s, tab);
}
template void tied_inner_group<double>(hipStream_t, const NormArgs<double>*, int, int);
template void tied_inner_group<float>(hipStream_t, const NormArgs<float>*, int, int);

// ||G~||^2 = lambda^T (g0 o g1 o g2 o g3) lambda: per-row partials, then a
// single-workgroup final pass per problem that also forms the fit and
// applies the stopping rule.  The Grams are symmetric and only their lower
// triangles are computed: row i sums j < i twice and the diagonal once.
template <typename T>
__global__ __launch_bounds__(256) void model_norm_rows_kernel(const FitArgs<T>* tab) {
  __shared__ double part[256];
  const FitArgs<T> a = tab[blockIdx.y];
  if (a.st->done) return;
  const int i = blockIdx.x, tid = threadIdx.x;
  if (i >= a.R) return;
  double acc = 0.0;
  for (int j = tid; j <= i; j += 256) {
    const size_t e = (size_t)i * a.ld + j;
    const double w = j < i ? 2.0 : 1.0;
    acc += w * (double)as_global(a.g[0])[e] * (double)as_global(a.g[1])[e] * (double)as_global(a.g[2])[e] *
           (double)as_global(a.g[3])[e] * (double)as_global(a.lam)[j];
  }
  part[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) a.row_part[i] = part[0] * (double)a.lam[i];
}

// Precision guard of split-BF16 plans (guard != 0): a problem whose
// normal matrices became too ill-conditioned for the split-BF16 MTTKRP
// (cond estimate above cond_limit), that needed a damped retry, or whose
// fit rose, is promoted to the FP64 path; `promote` tells the host to
// replay the sweep.  The stopping rule is not applied in such a sweep.
__device__ __forceinline__ bool guard_trips(const DevState* st, double fit, double prev, double cond_limit) {
  if (st->path) return false;
  return st->cond_max > cond_limit || st->fallbacks > st->fallbacks_start ||
         (prev >= 0.0 && fit > prev * (1.0 + 1e-3)) || !(fit <= 1.0);
}

template <typename T>
__global__ __launch_bounds__(256) void fit_final_kernel(const FitArgs<T>* tab, int hist_cap, double tol,
                                                        double fit_floor, int guard, double cond_limit,
                                                        int rule_every) {
  __shared__ double pa[256];
  __shared__ double pb[256];
  const FitArgs<T> a = tab[blockIdx.x];
  DevState* st = a.st;
  if (st->done) return;
  const int tid = threadIdx.x;
  double x = 0.0, y = 0.0;
  for (int i = tid; i < a.R; i += 256) {
    x += a.row_part[i];
    y += a.inner_part[i];
  }
  pa[tid] = x;
  pb[tid] = y;
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
    a.fit_hist[k % hist_cap] = fit;
    st->sweeps = k + 1;
    const double prev = st->fit_prev;
    // Stopping rule, looked at on every rule_every-th sweep: the fit is at
    // or below the floor, or it changed by at most tol relative to the fit
    // of the previous rule sweep.  Failures stop the problem at once.
    const bool rule = (k + 1) % rule_every == 0;
    const double ref = st->fit_rule;
    if (guard && guard_trips(st, fit, prev, cond_limit)) {
      st->path = 1;
      st->promote = 1;
    } else if ((rule && (fit <= fit_floor || (ref >= 0.0 && fabs(fit - ref) <= tol * ref))) || !isfinite(fit) ||
               fit <= st->fit_target || (st->flags & (FLAG_NOT_SPD | FLAG_SOLVE_STALL))) {
      st->done = 1;
    }
    if (rule) st->fit_rule = fit;
    st->fit_prev = fit;
  }
}

template <typename T>
void fit_group(hipStream_t s, const FitArgs<T>* tab, int nprob, int max_R, int hist_cap, double tol,
               double fit_floor, int guard, double cond_limit, int rule_every) {
  if (rule_every < 1) rule_every = 1;
  hipLaunchKernelGGL((model_norm_rows_kernel<T>), dim3(max_R, nprob), dim3(256), 0, s, tab);
  hipLaunchKernelGGL((fit_final_kernel<T>), dim3(nprob), dim3(256), 0, s, tab, hist_cap, tol, fit_floor, guard,
                     cond_limit, rule_every);
}

__global__ void sweep_tick_kernel(DevState* const* st_tab, int guard, double cond_limit) {
  DevState* st = st_tab[blockIdx.x];
  if (threadIdx.x == 0 && !st->done) {
    st->sweeps += 1;
    if (st->flags & (FLAG_NOT_SPD | FLAG_SOLVE_STALL)) {
      st->done = 1;  // a failed solve ends the problem (later sweeps are no-ops)
    } else if (guard && guard_trips(st, 0.0, -1.0, cond_limit)) {
      st->path = 1;
      st->promote = 1;
    }
  }
}
void sweep_tick_group(hipStream_t s, DevState* const* st_tab, int nprob, int guard, double cond_limit) {
  hipLaunchKernelGGL(sweep_tick_kernel, dim3(nprob), dim3(64), 0, s, st_tab, guard, cond_limit);
}

template <typename T>
__global__ __launch_bounds__(256) void cond_track_kernel(const CondArgs<T>* tab) {
  __shared__ double lo[256];
  __shared__ double hi[256];
  const CondArgs<T> a = tab[blockIdx.x];
  if (a.st->done) return;
  const int tid = threadIdx.x;
  double l = INFINITY, h = 0.0;
  for (int i = tid; i < a.R; i += 256) {
    const double v = fabs((double)a.diagL[i]);
    l = fmin(l, v);
    h = fmax(h, v);
  }
  lo[tid] = l;
  hi[tid] = h;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      lo[tid] = fmin(lo[tid], lo[tid + w]);
      hi[tid] = fmax(hi[tid], hi[tid + w]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double c = lo[0] > 0.0 ? (hi[0] / lo[0]) * (hi[0] / lo[0]) : INFINITY;
    if (!(c <= a.st->cond_max)) a.st->cond_max = c;
  }
}
template <typename T>
void cond_track_group(hipStream_t s, const CondArgs<T>* tab, int nprob) {
  hipLaunchKernelGGL((cond_track_kernel<T>), dim3(nprob), dim3(256), 0, s, tab);
}
template void cond_track_group<double>(hipStream_t, const CondArgs<double>*, int);
template void cond_track_group<float>(hipStream_t, const CondArgs<float>*, int);

__global__ void guard_begin_kernel(DevState* const* st_tab) {
  DevState* st = st_tab[blockIdx.x];
  if (threadIdx.x == 0) {
    st->cond_max = 0.0;
    st->fallbacks_start = st->fallbacks;
    st->promote = 0;
  }
}
void guard_begin_group(hipStream_t s, DevState* const* st_tab, int nprob) {
  hipLaunchKernelGGL(guard_begin_kernel, dim3(nprob), dim3(64), 0, s, st_tab);
}

__global__ void set_path_kernel(DevState* const* st_tab, const int32_t* flags) {
  DevState* st = st_tab[blockIdx.x];
  if (threadIdx.x == 0 && flags[blockIdx.x]) {
    st->path = 1;
    st->promote = 0;
  }
}
void set_path_group(hipStream_t s, DevState* const* st_tab, int nprob, const int32_t* flags_dev) {
  hipLaunchKernelGGL(set_path_kernel, dim3(nprob), dim3(64), 0, s, st_tab, flags_dev);
}

// Factor checkpoint (dir 0: save, 1: restore).  The factor buffers are
// 256-byte aligned plan allocations, copied in 16-byte words (a 4-byte
// tail loop covers any remainder).
__global__ __launch_bounds__(256) void checkpoint_kernel(const CkptArgs* tab, int dir) {
  const CkptArgs c = tab[blockIdx.y];
  if (c.gate && *c.gate != c.want) return;
  const size_t t0 = (size_t)blockIdx.x * 256 + threadIdx.x, stride = (size_t)gridDim.x * 256;
  for (int m = 0; m < 4; ++m) {
    typedef uint32_t u4_t __attribute__((ext_vector_type(4)));
    const gptr<const u4_t> s16 = as_global((const u4_t*)(dir ? c.b[m] : c.a[m]));
    const gptr<u4_t> d16 = as_global((u4_t*)(dir ? c.a[m] : c.b[m]));
    const gptr<const uint32_t> s4 = as_global((const uint32_t*)(dir ? c.b[m] : c.a[m]));
    const gptr<uint32_t> d4 = as_global((uint32_t*)(dir ? c.a[m] : c.b[m]));
    const size_t n16 = c.bytes[m] / 16;
    for (size_t e = t0; e < n16; e += stride) d16[e] = s16[e];
    for (size_t e = n16 * 4 + t0; e < c.bytes[m] / 4; e += stride) d4[e] = s4[e];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && c.st && c.st_save) {  // (no state: a plain copy)
    if (dir) *c.st = *c.st_save;
    else *c.st_save = *c.st;
  }
}
void checkpoint_group(hipStream_t s, const CkptArgs* tab, int nprob, int dir) {
  hipLaunchKernelGGL(checkpoint_kernel, dim3(nprob > 4 ? 128 : 1024, nprob), dim3(256), 0, s, tab, dir);
}

// Laplace-transform scaling of the THC rows: out[p, :] = exp(sign eps_p t) X[p, :].
__global__ void lt_scale_kernel(const double* X, const double* eps, int n, int r, double t, double sign,
                                double* out) {
  const size_t total = (size_t)n * r;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const int p = (int)(e / r);
    out[e] = exp(sign * eps[p] * t) * X[e];
  }
}
void lt_scale_rows(hipStream_t s, const double* X, const double* eps, int n, int r, double t, double sign,
                   double* out) {
  size_t total = (size_t)n * r;
  int grid = (int)((total + 255) / 256);
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(lt_scale_kernel, dim3(grid), dim3(256), 0, s, X, eps, n, r, t, sign, out);
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

__global__ void state_reset_kernel(DevState* st, const double* norm2_src, double fit_target) {
  if (threadIdx.x == 0) {
    st->norm2 = *norm2_src;
    st->fit_target = fit_target;
    st->fit_prev = -1.0;
    st->fit_rule = -1.0;
    st->inner = 0.0;
    st->model2 = 0.0;
    st->mu = 0.0;
    st->done = 0;
    st->sweeps = 0;
    st->flags = 0;
    st->chol_fail = 0;
    st->fallbacks = 0;
    st->retry_active = 0;
    st->path = 0;
    st->promote = 0;
    st->fallbacks_start = 0;
    st->cond_max = 0.0;
    if (!(st->norm2 > 0.0) || !isfinite(st->norm2)) {
      st->flags |= FLAG_NONFINITE;
      st->done = 1;
    }
  }
}
void state_reset(hipStream_t s, DevState* st, double* norm2_src, double fit_target) {
  hipLaunchKernelGGL(state_reset_kernel, dim3(1), dim3(64), 0, s, st, norm2_src, fit_target);
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

template void form_v_group<double>(hipStream_t, const FormVArgs<double>*, int, int, int);
template void form_v_group<float>(hipStream_t, const FormVArgs<float>*, int, int, int);
template void retry_prepare_group<double>(hipStream_t, const FormVArgs<double>*, int, int);
template void retry_prepare_group<float>(hipStream_t, const FormVArgs<float>*, int, int);
template void normalise_group<double>(hipStream_t, const NormArgs<double>*, int, int);
template void normalise_group<float>(hipStream_t, const NormArgs<float>*, int, int);
template void fit_group<double>(hipStream_t, const FitArgs<double>*, int, int, int, double, double, int, double,
                                int);
template void fit_group<float>(hipStream_t, const FitArgs<float>*, int, int, int, double, double, int, double,
                               int);

}  // namespace thccp
