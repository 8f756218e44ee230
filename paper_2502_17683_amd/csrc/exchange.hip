// Robust CPD+THC LT-MP2 exchange energy (Section 2.2: the single-CPD term
// eq. cpd_single_k, the double-CPD term after it, and their robust
// combination eq. rob_K) for one system over all its Laplace points.
//
// Tensors are in the (i, a, j, b) mode order: the THC (ia|jb) from X_occ,
// X_virt and Z, and its CPD (F0 on i, F1 on a, F2 on j, F3 on b, weights
// lam).  The exchange pairing is K(T, S) = sum T[i,a,j,b] S[i,b,j,a].
//
// The Laplace scaling exp(-D t) factors into row scalings, and for the
// exchange pairing it may sit on either tensor (the paper's symmetry
// remark).  Here it goes onto the CPD factors, one column block per point:
//   Fs_m[p, k R + r] = exp(+-eps_p t_k) F_m[p, r].
// All points then share a few wide products that read X, Z and F once:
//   W0 = X_occ^T F0s   W1 = X_virt^T F3s   W2 = X_occ^T F2s   W3 = X_virt^T F1s
//   Y  = Z (W2 o W3)                                  (R_thc x n_t R_cp each)
//   (W2 o W3 is formed in place before the product)
//   k_single[k] = sum_{P, r} lam_r W0 W1 Y [P, k R + r]
// The LT-scaled CPD gives the double-CPD overlaps from the same stacks:
//   C0 = F0^T F0s   C2 = F2^T F2s   C13 = F1^T F3s    (R_cp x n_t R_cp)
//   k_double[k] = sum_{r, r'} lam_r lam_r' C0 C2 C13 [r, k R + r'] C13[r', k R + r]
// and E_K = - sum_k w_k (2 k_single[k] - k_double[k]).
// Given separate CPDs E_k of the scaled tensors instead (per_point), their
// factors are stacked and the double term takes four plain overlaps,
//   Cm = Es_m^T F_{pm}  (L x R; pm = 0, 3, 2, 1),
//   k_double[k] = sum_{r, r'} lam_e[kR + r] lam_r' C0 C1 C2 C3 [kR + r, r'].
//
// The same file holds the THC LT-MP2 Coulomb and exchange terms and the
// LT-MP2 energy (below).
//
// Products run on the FP64 matrix cores (gemm_f64); the stacks and the two
// dot products are HBM-bound element-wise kernels.  Every reduction has a
// fixed order (per-block partials, then a fixed tree per point), so
// repeated calls are bitwise identical.
#include <math.h>
#include <stdint.h>

#include "../../include/thccp.h"
#include "common.h"
#include "kernels.h"

namespace thccp {

namespace {

struct LtQuad {
  int n;
  double t[CPD_LT_MAX_POINTS];
  double w[CPD_LT_MAX_POINTS];
};

struct StackArgs {
  const double* F[4];
  const double* eps[4];
  double* out[4];
  int rows[4];
};

constexpr int kDotRows = 16;  // rows of W per single-term block
constexpr int kTile = 64;     // double-term tile edge

// Fs_m[p, k R + r] = exp(sign_m eps_p t_k) F_m[p, r]; blockIdx.y = m
// (sign +1 for the occupied modes 0 and 2, -1 for the virtual modes 1, 3).
__global__ __launch_bounds__(256) void lt_stack_kernel(StackArgs a, LtQuad q, int R) {
  const int m = blockIdx.y;
  const double sign = (m & 1) ? -1.0 : 1.0;
  const int n = a.rows[m];
  const size_t L = (size_t)q.n * R;
  const size_t total = (size_t)n * L;
  auto F = as_global(a.F[m]);
  auto eps = as_global(a.eps[m]);
  auto out = as_global(a.out[m]);
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const size_t p = e / L;
    const size_t c = e - p * L;
    const int k = (int)(c / R);
    const int r = (int)(c - (size_t)k * R);
    out[e] = exp(sign * eps[p] * q.t[k]) * F[p * R + r];
  }
}

// partials[k * chunks + c] = sum over rows [c kDotRows, ...) and columns r
// of lam_r W0 W1 Y at column k R + r.  grid (chunks, n_t).
__global__ __launch_bounds__(256) void single_dot_kernel(const double* W0, const double* W1, const double* Y,
                                                         const double* lam, int Rt, int R, size_t L,
                                                         double* partials) {
  __shared__ double part[256];
  const int c = blockIdx.x, k = blockIdx.y, tid = threadIdx.x;
  const int p0 = c * kDotRows;
  const int p1 = p0 + kDotRows < Rt ? p0 + kDotRows : Rt;
  auto w0 = as_global(W0);
  auto w1 = as_global(W1);
  auto y = as_global(Y);
  double acc = 0.0;
  for (int r = tid; r < R; r += 256) {
    const double l = lam ? as_global(lam)[r] : 1.0;
    double s = 0.0;
    for (int p = p0; p < p1; ++p) {
      const size_t e = (size_t)p * L + (size_t)k * R + r;
      s += w0[e] * w1[e] * y[e];
    }
    acc += l * s;
  }
  part[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) as_global(partials)[(size_t)k * gridDim.x + c] = part[0];
}

// partials[k * nt^2 + (bi nt + bj)]: the (bi, bj) 64 x 64 tile of point k,
// rows r in tile bi, columns r' in tile bj:
//   sum lam_r lam_r' C0[r, kR + r'] C2[r, kR + r'] C13[r, kR + r'] C13[r', kR + r].
// The transposed C13 tile is staged through LDS (odd row stride, so the
// column-wise reads do not conflict).  grid (nt^2, n_t).
__global__ __launch_bounds__(256) void double_dot_kernel(const double* C0, const double* C2, const double* C13,
                                                         const double* lam, int R, size_t L, double* partials) {
  __shared__ double tt[kTile][kTile + 1];
  __shared__ double part[256];
  const int nt = (R + kTile - 1) / kTile;
  const int bi = blockIdx.x / nt, bj = blockIdx.x % nt, k = blockIdx.y, tid = threadIdx.x;
  const size_t col0 = (size_t)k * R;
  auto c0 = as_global(C0);
  auto c2 = as_global(C2);
  auto c13 = as_global(C13);
  // tt[r'_l][r_l] = C13[bj 64 + r'_l, kR + bi 64 + r_l]
  for (int e = tid; e < kTile * kTile; e += 256) {
    const int rl = e & (kTile - 1), rpl = e >> 6;
    const int r = bi * kTile + rl, rp = bj * kTile + rpl;
    tt[rpl][rl] = (r < R && rp < R) ? c13[(size_t)rp * L + col0 + r] : 0.0;
  }
  __syncthreads();
  double acc = 0.0;
  for (int e = tid; e < kTile * kTile; e += 256) {
    const int rpl = e & (kTile - 1), rl = e >> 6;
    const int r = bi * kTile + rl, rp = bj * kTile + rpl;
    if (r < R && rp < R) {
      const size_t g = (size_t)r * L + col0 + rp;
      const double lr = lam ? as_global(lam)[r] * as_global(lam)[rp] : 1.0;
      acc += lr * c0[g] * c2[g] * c13[g] * tt[rpl][rl];
    }
  }
  part[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) as_global(partials)[(size_t)k * gridDim.x + blockIdx.x] = part[0];
}

// Point k's separate CPD into the stacks: Es_m[:, kR : kR + R] = E_m and
// lame[kR : kR + R] = lam_e (ones for NULL).  blockIdx.y = m (4: weights).
struct GatherArgs {
  const double* E[4];
  const double* lam;
  double* out[4];
  double* lam_out;
  int rows[4];
};
__global__ __launch_bounds__(256) void gather_point_kernel(GatherArgs g, int k, int R, size_t L) {
  const int m = blockIdx.y;
  if (m == 4) {
    for (int r = blockIdx.x * 256 + threadIdx.x; r < R; r += gridDim.x * 256)
      as_global(g.lam_out)[(size_t)k * R + r] = g.lam ? as_global(g.lam)[r] : 1.0;
    return;
  }
  const size_t total = (size_t)g.rows[m] * R;
  auto src = as_global(g.E[m]);
  auto dst = as_global(g.out[m]);
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const size_t p = e / R;
    const int r = (int)(e - p * R);
    dst[p * L + (size_t)k * R + r] = src[e];
  }
}

// Separate per-point CPDs: partials[k * dchunks + c] = sum over rows
// r in chunk c of point k and all r' of
//   lame[kR + r] lam[r'] C0 C1 C2 C3 [kR + r, r']   (each L x R).
// grid (dchunks, n_t).
__global__ __launch_bounds__(256) void double_dot_sep_kernel(const double* C0, const double* C1, const double* C2,
                                                             const double* C3, const double* lame,
                                                             const double* lam, int R, double* partials) {
  __shared__ double part[256];
  const int c = blockIdx.x, k = blockIdx.y, tid = threadIdx.x;
  const int r0 = c * kDotRows;
  const int r1 = r0 + kDotRows < R ? r0 + kDotRows : R;
  auto c0 = as_global(C0);
  auto c1 = as_global(C1);
  auto c2 = as_global(C2);
  auto c3 = as_global(C3);
  double acc = 0.0;
  for (int rp = tid; rp < R; rp += 256) {
    const double lf = lam ? as_global(lam)[rp] : 1.0;
    double s = 0.0;
    for (int r = r0; r < r1; ++r) {
      const size_t row = (size_t)k * R + r;
      const size_t e = row * R + rp;
      s += as_global(lame)[row] * c0[e] * c1[e] * c2[e] * c3[e];
    }
    acc += lf * s;
  }
  part[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) as_global(partials)[(size_t)k * gridDim.x + c] = part[0];
}

// One workgroup of 16 waves: wave j reduces points j, j + 16, ...; each lane
// sums a strided subset of the point's partials, then the wave's 64 sums
// are combined in a fixed shuffle tree.  Thread 0 then forms
// E_K = - sum_k w_k (2 k_single[k] - k_double[k]) in point order.
constexpr int kFinishWaves = 16;
__global__ __launch_bounds__(64 * kFinishWaves) void exchange_finish_kernel(const double* p1, int n1,
                                                                            const double* p2, int n2, LtQuad q,
                                                                            double* k1, double* k2, double* ek) {
  __shared__ double s1[CPD_LT_MAX_POINTS], s2[CPD_LT_MAX_POINTS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = wave; k < q.n; k += kFinishWaves) {
    double a = 0.0, b = 0.0;
    for (int c = lane; c < n1; c += 64) a += as_global(p1)[(size_t)k * n1 + c];
    for (int c = lane; c < n2; c += 64) b += as_global(p2)[(size_t)k * n2 + c];
    for (int w = 32; w > 0; w >>= 1) {
      a += __shfl_down(a, w);
      b += __shfl_down(b, w);
    }
    if (lane == 0) {
      s1[k] = a;
      s2[k] = b;
      as_global(k1)[k] = a;
      as_global(k2)[k] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double e = 0.0;
    for (int j = 0; j < q.n; ++j) e += q.w[j] * (2.0 * s1[j] - s2[j]);
    as_global(ek)[0] = -e;
  }
}

struct ExchangeLayout {
  size_t fs[4], w[4], y, c[4], es[4], lame, p1, p2, total;
  int chunks, tiles, dchunks;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// per_point: separate CPDs of the scaled tensors (the E stacks, their
// weights and a fourth overlap) instead of the LT-scaled bare CPD.
ExchangeLayout exchange_layout(int o, int v, int Rt, int R, int n, bool per_point) {
  ExchangeLayout l{};
  const size_t L = (size_t)n * R, d = sizeof(double);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align256(bytes);
    return at;
  };
  const int rows[4] = {o, v, o, v};
  for (int m = 0; m < 4; ++m) l.fs[m] = take((size_t)rows[m] * L * d);
  for (int m = 0; m < 4; ++m) l.w[m] = take((size_t)Rt * L * d);
  l.y = take((size_t)Rt * L * d);
  for (int m = 0; m < (per_point ? 4 : 3); ++m) l.c[m] = take((size_t)R * L * d);
  if (per_point) {
    for (int m = 0; m < 4; ++m) l.es[m] = take((size_t)rows[m] * L * d);
    l.lame = take(L * d);
  }
  l.chunks = (Rt + kDotRows - 1) / kDotRows;
  const int nt = (R + kTile - 1) / kTile;
  l.tiles = nt * nt;
  l.dchunks = (R + kDotRows - 1) / kDotRows;
  l.p1 = take((size_t)n * l.chunks * d);
  l.p2 = take((size_t)n * (per_point ? l.dchunks : l.tiles) * d);
  l.total = off;
  return l;
}

bool exchange_sizes_ok(int o, int v, int Rt, int R, int n) {
  if (o <= 0 || v <= 0 || Rt <= 0 || R <= 0 || n <= 0 || n > CPD_LT_MAX_POINTS) return false;
  // the products index columns with int
  return (int64_t)n * R <= INT32_MAX && (int64_t)Rt * Rt <= ((int64_t)1 << 40);
}


// ----------------------------------------------------------------------
// THC LT-MP2 Coulomb and exchange terms (eq. thc_Ej, eq. thc_Ek, eq.
// LT-Emp2).
//
// Coulomb: with the occupied and virtual factors scaled per point (stacks
// Xs_o, Xs_v, one R_thc block per point), M_k = (X_o^T Xs_o)_k o
// (X_v^T Xs_v)_k is symmetric, and
//   J[k] = sum_{P,S} M_k[P,S] (Z M_k Z^T)[P,S] = sum_{P,T} A_k[P,T] B_k[T,P]
// with A = Z M and B = Z^T M (B = A for a symmetric Z): one or two wide
// products over all points, then a transposed dot per point.
//
// Exchange (for a symmetric Z only the blocks i >= j, see below): the
// (ia|jb) matrix G = Bp Z Bp^T with Bp[(i,a), P] =
// X_o[i,P] X_v[a,P] ((o v) x (o v), o^2 v^2 R_thc flops: the THC exchange
// costs a power of N more than the Coulomb term), the swapped product
// Pm[(i,a),(j,b)] = G[(i,a),(j,b)] G[(i,b),(j,a)], the virtual Laplace
// factors H^T = U^T Pm_flat^T with U[b,k] = exp(-eps_b t_k) and Pm_flat the
// (o v o) x v view of Pm, and
//   K[k] = sum_{i,a,j} exp((eps_i + eps_j - eps_a) t_k) H^T[k, (i,a,j)].

// partials[k * nt^2 + (bi nt + bj)] = sum over the (bi, bj) tile of point
// k of A[r, kR + c] B[c, kR + r] (B tile transposed through LDS).
__global__ __launch_bounds__(256) void tdot_blocks_kernel(const double* A, const double* B, int R, size_t L,
                                                          double* partials) {
  __shared__ double tt[kTile][kTile + 1];
  __shared__ double part[256];
  const int nt = (R + kTile - 1) / kTile;
  const int bi = blockIdx.x / nt, bj = blockIdx.x % nt, k = blockIdx.y, tid = threadIdx.x;
  const size_t col0 = (size_t)k * R;
  auto a = as_global(A);
  auto b = as_global(B);
  // tt[c_l][r_l] = B[bj 64 + c_l, kR + bi 64 + r_l]
  for (int e = tid; e < kTile * kTile; e += 256) {
    const int rl = e & (kTile - 1), cl = e >> 6;
    const int r = bi * kTile + rl, c = bj * kTile + cl;
    tt[cl][rl] = (r < R && c < R) ? b[(size_t)c * L + col0 + r] : 0.0;
  }
  __syncthreads();
  double acc = 0.0;
  for (int e = tid; e < kTile * kTile; e += 256) {
    const int cl = e & (kTile - 1), rl = e >> 6;
    const int r = bi * kTile + rl, c = bj * kTile + cl;
    if (r < R && c < R) acc += a[(size_t)r * L + col0 + c] * tt[cl][rl];
  }
  part[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) as_global(partials)[(size_t)k * gridDim.x + blockIdx.x] = part[0];
}

// Bp[(i v + a), P] = X_o[i, P] X_v[a, P]
__global__ __launch_bounds__(256) void pair_rows_kernel(const double* Xo, const double* Xv, int o, int v, int Rt,
                                                        double* Bp) {
  const size_t total = (size_t)o * v * Rt;
  auto xo = as_global(Xo);
  auto xv = as_global(Xv);
  auto out = as_global(Bp);
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const size_t row = e / Rt;
    const int P = (int)(e - row * Rt);
    const int i = (int)(row / v), a = (int)(row - (size_t)i * v);
    out[e] = xo[(size_t)i * Rt + P] * xv[(size_t)a * Rt + P];
  }
}

// Pm[(i,a),(j,b)] = G[(i,a),(j,b)] G[(i,b),(j,a)]: block (i, j) of G is
// v x v; the swapped factor is the transposed block, read through LDS.
// grid o^2 nv^2 (flat), nv = ceil(v / 64); block = (i, j, tile row, tile col).
__global__ __launch_bounds__(256) void swap_product_kernel(const double* G, int o, int v, double* Pm) {
  __shared__ double tt[kTile][kTile + 1];
  const int nv = (v + kTile - 1) / kTile;
  const int tile = blockIdx.x % (nv * nv), pair = blockIdx.x / (nv * nv);
  const int ta = tile / nv, tb = tile % nv;
  const int i = pair / o, j = pair % o;
  const size_t ld = (size_t)o * v;
  const size_t base = (size_t)i * v * ld + (size_t)j * v;  // block (i, j)
  auto g = as_global(G);
  auto out = as_global(Pm);
  const int tid = threadIdx.x;
  // tt[b_l][a_l] = G[(i, tb 64 + b_l), (j, ta 64 + a_l)]
  for (int e = tid; e < kTile * kTile; e += 256) {
    const int al = e & (kTile - 1), bl = e >> 6;
    const int a = ta * kTile + al, b = tb * kTile + bl;
    tt[bl][al] = (a < v && b < v) ? g[base + (size_t)b * ld + a] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < kTile * kTile; e += 256) {
    const int bl = e & (kTile - 1), al = e >> 6;
    const int a = ta * kTile + al, b = tb * kTile + bl;
    if (a < v && b < v) {
      const size_t idx = base + (size_t)a * ld + b;
      out[idx] = g[idx] * tt[bl][al];
    }
  }
}

// Symmetric Z: (ia|jb) = (jb|ia), and both factors of a swapped product
// lie in the same block (i, j), whose contribution equals that of (j, i).
// Only the blocks i >= j are formed, and pair p = i (i + 1) / 2 + j is
// stored compactly: Pc[(p v + a), b] = G[(i,a),(j,b)] G[(i,b),(j,a)].
__device__ __forceinline__ void pair_decode(int p, int& i, int& j) {
  i = (int)((sqrtf(8.f * (float)p + 1.f) - 1.f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= p) ++i;
  while (i * (i + 1) / 2 > p) --i;
  j = p - i * (i + 1) / 2;
}
// grid npairs nv^2 (flat); block = (pair, tile row, tile col).
__global__ __launch_bounds__(256) void swap_product_lower_kernel(const double* G, int o, int v, double* Pc) {
  __shared__ double tt[kTile][kTile + 1];
  const int nv = (v + kTile - 1) / kTile;
  const int tile = blockIdx.x % (nv * nv), pair = blockIdx.x / (nv * nv);
  const int ta = tile / nv, tb = tile % nv;
  int i, j;
  pair_decode(pair, i, j);
  const size_t ld = (size_t)o * v;
  const size_t base = (size_t)i * v * ld + (size_t)j * v;  // block (i, j)
  const size_t obase = (size_t)pair * v * v;
  auto g = as_global(G);
  auto out = as_global(Pc);
  const int tid = threadIdx.x;
  for (int e = tid; e < kTile * kTile; e += 256) {
    const int al = e & (kTile - 1), bl = e >> 6;
    const int a = ta * kTile + al, b = tb * kTile + bl;
    tt[bl][al] = (a < v && b < v) ? g[base + (size_t)b * ld + a] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < kTile * kTile; e += 256) {
    const int bl = e & (kTile - 1), al = e >> 6;
    const int a = ta * kTile + al, b = tb * kTile + bl;
    if (a < v && b < v) out[obase + (size_t)a * v + b] = g[base + (size_t)a * ld + b] * tt[bl][al];
  }
}

// U^T[k, b] = exp(-eps_b t_k)  (n x v)
__global__ __launch_bounds__(256) void virt_factor_kernel(const double* eps_v, int v, LtQuad q, double* Ut) {
  const int total = q.n * v;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
    const int k = e / v, b = e - k * v;
    as_global(Ut)[e] = exp(-as_global(eps_v)[b] * q.t[k]);
  }
}

// partials[k * chunks + c] = sum over rows r = (i, a, j) of chunk c of
// exp((eps_i + eps_j - eps_a) t_k) Ht[k, r].  grid (chunks, n).
constexpr int kRowsPerBlock = 4096;
__global__ __launch_bounds__(256) void occ_weight_dot_kernel(const double* Ht, const double* eps_o,
                                                             const double* eps_v, int o, int v, LtQuad q,
                                                             double* partials) {
  __shared__ double part[256];
  const int c = blockIdx.x, k = blockIdx.y, tid = threadIdx.x;
  const size_t rows = (size_t)o * v * o;
  const size_t r0 = (size_t)c * kRowsPerBlock;
  const size_t r1 = r0 + kRowsPerBlock < rows ? r0 + kRowsPerBlock : rows;
  const double tk = q.t[k];
  auto h = as_global(Ht);
  auto eo = as_global(eps_o);
  auto ev = as_global(eps_v);
  double acc = 0.0;
  for (size_t r = r0 + tid; r < r1; r += 256) {
    const int j = (int)(r % o);
    const size_t ia = r / o;
    const int a = (int)(ia % v), i = (int)(ia / v);
    acc += exp((eo[i] + eo[j] - ev[a]) * tk) * h[(size_t)k * rows + r];
  }
  part[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) as_global(partials)[(size_t)k * gridDim.x + c] = part[0];
}

// Compact lower-block rows r = p v + a (pair p = (i, j), i >= j):
// partials[k * chunks + c] = sum over the chunk of
// m_ij exp((eps_i + eps_j - eps_a) t_k) Ht[k, r], m_ij = 1 (i = j) or 2.
__global__ __launch_bounds__(256) void occ_weight_dot_lower_kernel(const double* Ht, const double* eps_o,
                                                                   const double* eps_v, int o, int v, LtQuad q,
                                                                   double* partials) {
  __shared__ double part[256];
  const int c = blockIdx.x, k = blockIdx.y, tid = threadIdx.x;
  const size_t rows = (size_t)o * (o + 1) / 2 * v;
  const size_t r0 = (size_t)c * kRowsPerBlock;
  const size_t r1 = r0 + kRowsPerBlock < rows ? r0 + kRowsPerBlock : rows;
  const double tk = q.t[k];
  auto h = as_global(Ht);
  auto eo = as_global(eps_o);
  auto ev = as_global(eps_v);
  double acc = 0.0;
  for (size_t r = r0 + tid; r < r1; r += 256) {
    const int p = (int)(r / v), a = (int)(r - (size_t)p * v);
    int i, j;
    pair_decode(p, i, j);
    const double m = i == j ? 1.0 : 2.0;
    acc += m * exp((eo[i] + eo[j] - ev[a]) * tk) * h[(size_t)k * rows + r];
  }
  part[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) as_global(partials)[(size_t)k * gridDim.x + c] = part[0];
}

// One workgroup of 16 waves: per-point sums of both partial sets in a fixed
// tree (as exchange_finish_kernel), then e[0] = E_J = 2 sum_k w_k J[k],
// e[1] = E_K = - sum_k w_k K[k] (0 without the exchange term), e[2] = E_J + E_K.
__global__ __launch_bounds__(64 * kFinishWaves) void mp2_finish_kernel(const double* pj, int nj, const double* pk,
                                                                       int nk, LtQuad q, double* J, double* K,
                                                                       double* e) {
  __shared__ double sj[CPD_LT_MAX_POINTS], sk[CPD_LT_MAX_POINTS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = wave; k < q.n; k += kFinishWaves) {
    double a = 0.0, b = 0.0;
    for (int c = lane; c < nj; c += 64) a += as_global(pj)[(size_t)k * nj + c];
    for (int c = lane; c < nk; c += 64) b += as_global(pk)[(size_t)k * nk + c];
    for (int w = 32; w > 0; w >>= 1) {
      a += __shfl_down(a, w);
      b += __shfl_down(b, w);
    }
    if (lane == 0) {
      sj[k] = a;
      sk[k] = b;
      as_global(J)[k] = a;
      if (K) as_global(K)[k] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ej = 0.0, ek = 0.0;
    for (int k = 0; k < q.n; ++k) {
      ej += q.w[k] * sj[k];
      ek += q.w[k] * sk[k];
    }
    as_global(e)[0] = 2.0 * ej;
    as_global(e)[1] = -ek;
    as_global(e)[2] = 2.0 * ej - ek;
  }
}

struct Mp2Layout {
  size_t xs[2], om, vm, a, b, pj;  // Coulomb
  size_t bp, c1, g, pm, ut, ht, pk;  // exchange
  size_t total;
  int jtiles, kchunks;
};

Mp2Layout mp2_layout(int o, int v, int Rt, int n, bool with_k, bool z_sym) {
  Mp2Layout l{};
  const size_t L = (size_t)n * Rt, d = sizeof(double);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align256(bytes);
    return at;
  };
  l.xs[0] = take((size_t)o * L * d);
  l.xs[1] = take((size_t)v * L * d);
  l.om = take((size_t)Rt * L * d);
  l.vm = take((size_t)Rt * L * d);
  l.a = take((size_t)Rt * L * d);
  l.b = z_sym ? l.a : take((size_t)Rt * L * d);
  const int nt = (Rt + kTile - 1) / kTile;
  l.jtiles = nt * nt;
  l.pj = take((size_t)n * l.jtiles * d);
  if (with_k) {
    // symmetric Z: the lower block triangle, pairs stored compactly
    const size_t ov = (size_t)o * v, rows = z_sym ? (size_t)o * (o + 1) / 2 * v : ov * o;
    l.bp = take(ov * Rt * d);
    l.c1 = take(ov * Rt * d);
    l.g = take(ov * ov * d);
    l.pm = take(rows * v * d);
    l.ut = take((size_t)n * v * d);
    l.ht = take((size_t)n * rows * d);
    l.kchunks = (int)((rows + kRowsPerBlock - 1) / kRowsPerBlock);
    l.pk = take((size_t)n * l.kchunks * d);
  }
  l.total = off;
  return l;
}

bool mp2_sizes_ok(int o, int v, int Rt, int n, bool with_k) {
  if (o <= 0 || v <= 0 || Rt <= 0 || n <= 0 || n > CPD_LT_MAX_POINTS) return false;
  if ((int64_t)n * Rt > INT32_MAX) return false;
  // the exchange products index (o v) and (o v o) rows with int
  if (with_k && ((int64_t)o * v * o > INT32_MAX || (int64_t)o * v > 46340)) return false;
  return true;
}
}  // namespace

}  // namespace thccp

using namespace thccp;

extern "C" {

size_t cpd_lt_exchange_workspace(int32_t n_occ, int32_t n_virt, int32_t r_thc, int32_t r_cp, int32_t n_points,
                                 int32_t per_point_cpds) {
  if (!exchange_sizes_ok(n_occ, n_virt, r_thc, r_cp, n_points)) return 0;
  return exchange_layout(n_occ, n_virt, r_thc, r_cp, n_points, per_point_cpds != 0).total;
}

cpd_status cpd_lt_exchange(int32_t n_occ, int32_t n_virt, int32_t r_thc, int32_t r_cp, int32_t n_points,
                           const double* X_occ, const double* X_virt, const double* Z, const double* eps_occ,
                           const double* eps_virt, const double* t_host, const double* w_host, const double* F0,
                           const double* F1, const double* F2, const double* F3, const double* lam,
                           const double* const* E_host, const double* const* lam_e_host, double* k_single,
                           double* k_double, double* e_k, void* workspace, size_t workspace_bytes,
                           void* stream) {
  if (!exchange_sizes_ok(n_occ, n_virt, r_thc, r_cp, n_points)) return CPD_ERR_INVALID_ARG;
  if (!X_occ || !X_virt || !Z || !eps_occ || !eps_virt || !t_host || !w_host || !F0 || !F1 || !F2 || !F3 ||
      !k_single || !k_double || !e_k)
    return CPD_ERR_INVALID_ARG;
  const bool per_point = E_host != nullptr;
  if (per_point)
    for (int e = 0; e < 4 * n_points; ++e)
      if (!E_host[e]) return CPD_ERR_INVALID_ARG;
  LtQuad q{};
  q.n = n_points;
  for (int k = 0; k < n_points; ++k) {
    if (!isfinite(t_host[k]) || !isfinite(w_host[k])) return CPD_ERR_INVALID_ARG;
    q.t[k] = t_host[k];
    q.w[k] = w_host[k];
  }
  const ExchangeLayout l = exchange_layout(n_occ, n_virt, r_thc, r_cp, n_points, per_point);
  if (!workspace || workspace_bytes < l.total) return CPD_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  auto buf = [&](size_t off) { return (double*)(ws + off); };
  const int o = n_occ, v = n_virt, Rt = r_thc, R = r_cp;
  const int L = n_points * R;

  StackArgs sa{};
  const double* Fm[4] = {F0, F1, F2, F3};
  const double* em[4] = {eps_occ, eps_virt, eps_occ, eps_virt};
  const int rows[4] = {o, v, o, v};
  for (int m = 0; m < 4; ++m) {
    sa.F[m] = Fm[m];
    sa.eps[m] = em[m];
    sa.out[m] = buf(l.fs[m]);
    sa.rows[m] = rows[m];
  }
  {
    const size_t most = (size_t)(o > v ? o : v) * L;
    int grid = (int)((most + 255) / 256);
    if (grid > 2048) grid = 2048;
    hipLaunchKernelGGL(lt_stack_kernel, dim3(grid, 4), dim3(256), 0, s, sa, q, R);
  }
  // projections (A = X^T, stored n x R_thc) and the double-term overlaps
  // (A = F^T, stored n x R_cp), all against the scaled stacks
  auto proj = [&](const double* A, int lda, int M, int K, const double* B, double* C) {
    GemmF64 g{M, L, K, A, lda, true, B, nullptr, L, false, C, L, nullptr, 1.0, 0.0, nullptr};
    gemm_f64(s, g);
  };
  proj(X_occ, Rt, Rt, o, buf(l.fs[0]), buf(l.w[0]));   // W0 = X_occ^T F0s
  proj(X_virt, Rt, Rt, v, buf(l.fs[3]), buf(l.w[1]));  // W1 = X_virt^T F3s
  proj(X_occ, Rt, Rt, o, buf(l.fs[2]), buf(l.w[2]));   // W2 = X_occ^T F2s
  proj(X_virt, Rt, Rt, v, buf(l.fs[1]), buf(l.w[3]));  // W3 = X_virt^T F1s
  {
    // Y = Z (W2 o W3), the Hadamard product formed in place first: the plain
    // product's k-step is twice that of the paired-operand form (about 20%
    // faster at R_thc = 1920), which outweighs one element-wise pass
    hadamard_inplace_f64(s, buf(l.w[2]), buf(l.w[3]), (size_t)Rt * L);
    GemmF64 g{Rt, L, Rt, Z, Rt, false, buf(l.w[2]), nullptr, L, false, buf(l.y), L, nullptr, 1.0, 0.0, nullptr};
    gemm_f64(s, g);
  }
  hipLaunchKernelGGL(single_dot_kernel, dim3(l.chunks, n_points), dim3(256), 0, s, buf(l.w[0]), buf(l.w[1]),
                     buf(l.y), lam, Rt, R, (size_t)L, buf(l.p1));
  if (!per_point) {
    proj(F0, R, R, o, buf(l.fs[0]), buf(l.c[0]));  // C0 = F0^T F0s
    proj(F2, R, R, o, buf(l.fs[2]), buf(l.c[1]));  // C2 = F2^T F2s
    proj(F1, R, R, v, buf(l.fs[3]), buf(l.c[2]));  // C13 = F1^T F3s
    hipLaunchKernelGGL(double_dot_kernel, dim3(l.tiles, n_points), dim3(256), 0, s, buf(l.c[0]), buf(l.c[1]),
                       buf(l.c[2]), lam, R, (size_t)L, buf(l.p2));
  } else {
    // separate CPDs E_k of the scaled tensors: stack them, then the four
    // overlaps (E0^T F0)(E1^T F3)(E2^T F2)(E3^T F1) of every point at once
    for (int k = 0; k < n_points; ++k) {
      GatherArgs g{};
      for (int m = 0; m < 4; ++m) {
        g.E[m] = E_host[4 * k + m];
        g.out[m] = buf(l.es[m]);
        g.rows[m] = rows[m];
      }
      g.lam = lam_e_host ? lam_e_host[k] : nullptr;
      g.lam_out = buf(l.lame);
      const size_t most = (size_t)(o > v ? o : v) * R;
      int grid = (int)((most + 255) / 256 < 1024 ? (most + 255) / 256 : 1024);
      hipLaunchKernelGGL(gather_point_kernel, dim3(grid, 5), dim3(256), 0, s, g, k, R, (size_t)L);
    }
    const double* partner[4] = {F0, F3, F2, F1};
    for (int m = 0; m < 4; ++m) {
      // C_m = Es_m^T partner_m  (L x R)
      GemmF64 g{L, R, rows[m], buf(l.es[m]), L, true, partner[m], nullptr, R, false, buf(l.c[m]), R, nullptr,
                1.0, 0.0, nullptr};
      gemm_f64(s, g);
    }
    hipLaunchKernelGGL(double_dot_sep_kernel, dim3(l.dchunks, n_points), dim3(256), 0, s, buf(l.c[0]),
                       buf(l.c[1]), buf(l.c[2]), buf(l.c[3]), buf(l.lame), lam, R, buf(l.p2));
  }
  hipLaunchKernelGGL(exchange_finish_kernel, dim3(1), dim3(64 * kFinishWaves), 0, s, buf(l.p1), l.chunks,
                     buf(l.p2), per_point ? l.dchunks : l.tiles, q, k_single, k_double, e_k);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}


size_t cpd_lt_mp2_workspace(int32_t n_occ, int32_t n_virt, int32_t r_thc, int32_t n_points, int32_t thc_exchange,
                            int32_t z_symmetric) {
  if (!mp2_sizes_ok(n_occ, n_virt, r_thc, n_points, thc_exchange != 0)) return 0;
  return mp2_layout(n_occ, n_virt, r_thc, n_points, thc_exchange != 0, z_symmetric != 0).total;
}

cpd_status cpd_lt_mp2(int32_t n_occ, int32_t n_virt, int32_t r_thc, int32_t n_points, const double* X_occ,
                      const double* X_virt, const double* Z, const double* eps_occ, const double* eps_virt,
                      const double* t_host, const double* w_host, int32_t thc_exchange, int32_t z_symmetric,
                      double* J, double* K, double* energies, void* workspace, size_t workspace_bytes,
                      void* stream) {
  const bool with_k = thc_exchange != 0, z_sym = z_symmetric != 0;
  if (!mp2_sizes_ok(n_occ, n_virt, r_thc, n_points, with_k)) return CPD_ERR_INVALID_ARG;
  if (!X_occ || !X_virt || !Z || !eps_occ || !eps_virt || !t_host || !w_host || !J || !energies ||
      (with_k && !K))
    return CPD_ERR_INVALID_ARG;
  LtQuad q{};
  q.n = n_points;
  for (int k = 0; k < n_points; ++k) {
    if (!isfinite(t_host[k]) || !isfinite(w_host[k])) return CPD_ERR_INVALID_ARG;
    q.t[k] = t_host[k];
    q.w[k] = w_host[k];
  }
  const Mp2Layout l = mp2_layout(n_occ, n_virt, r_thc, n_points, with_k, z_sym);
  if (!workspace || workspace_bytes < l.total) return CPD_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  auto buf = [&](size_t off) { return (double*)(ws + off); };
  const int o = n_occ, v = n_virt, Rt = r_thc;
  const int L = n_points * Rt;

  // Coulomb term
  StackArgs sa{};
  sa.F[0] = X_occ;
  sa.eps[0] = eps_occ;
  sa.out[0] = buf(l.xs[0]);
  sa.rows[0] = o;
  sa.F[1] = X_virt;
  sa.eps[1] = eps_virt;
  sa.out[1] = buf(l.xs[1]);
  sa.rows[1] = v;
  {
    const size_t most = (size_t)(o > v ? o : v) * L;
    int grid = (int)((most + 255) / 256);
    if (grid > 2048) grid = 2048;
    hipLaunchKernelGGL(lt_stack_kernel, dim3(grid, 2), dim3(256), 0, s, sa, q, Rt);
  }
  auto gemm = [&](int M, int N, int Kd, const double* A, int lda, bool at, const double* B, int ldb, bool bt,
                  double* C, int ldc) {
    GemmF64 g{M, N, Kd, A, lda, at, B, nullptr, ldb, bt, C, ldc, nullptr, 1.0, 0.0, nullptr};
    gemm_f64(s, g);
  };
  gemm(Rt, L, o, X_occ, Rt, true, buf(l.xs[0]), L, false, buf(l.om), L);   // O = X_o^T Xs_o
  gemm(Rt, L, v, X_virt, Rt, true, buf(l.xs[1]), L, false, buf(l.vm), L);  // V = X_v^T Xs_v
  hadamard_inplace_f64(s, buf(l.om), buf(l.vm), (size_t)Rt * L);             // M = O o V
  gemm(Rt, L, Rt, Z, Rt, false, buf(l.om), L, false, buf(l.a), L);          // A = Z M
  if (!z_sym) gemm(Rt, L, Rt, Z, Rt, true, buf(l.om), L, false, buf(l.b), L);  // B = Z^T M
  hipLaunchKernelGGL(tdot_blocks_kernel, dim3(l.jtiles, n_points), dim3(256), 0, s, buf(l.a), buf(l.b), Rt,
                     (size_t)L, buf(l.pj));

  // THC exchange term
  if (with_k) {
    const int ov = o * v;
    {
      const size_t total = (size_t)ov * Rt;
      int grid = (int)((total + 255) / 256);
      if (grid > 8192) grid = 8192;
      hipLaunchKernelGGL(pair_rows_kernel, dim3(grid), dim3(256), 0, s, X_occ, X_virt, o, v, Rt, buf(l.bp));
    }
    gemm(ov, Rt, Rt, buf(l.bp), Rt, false, Z, Rt, false, buf(l.c1), Rt);  // C1 = Bp Z
    const int nv = (v + kTile - 1) / kTile;
    int rows;
    if (z_sym) {
      // the block rows in at most 8 panels, each up to its last diagonal
      // block (blocks above the diagonal inside a panel are formed and not
      // read): about (P + 1) / (2 P) of the full product in P launches.
      // Below o v = 4096 one full product is faster than several small
      // ones (0.23 vs 0.76 ms for the whole exchange term at o v = 2000).
      const int P = ov < 4096 ? 1 : (o < 8 ? o : 8);
      for (int pn = 0; pn < P; ++pn) {
        const int i0 = pn * o / P, i1 = (pn + 1) * o / P;
        if (i1 <= i0) continue;
        gemm((i1 - i0) * v, i1 * v, Rt, buf(l.c1) + (size_t)i0 * v * Rt, Rt, false, buf(l.bp), Rt, true,
             buf(l.g) + (size_t)i0 * v * ov, ov);
      }
      const int npairs = o * (o + 1) / 2;
      hipLaunchKernelGGL(swap_product_lower_kernel, dim3(nv * nv * npairs), dim3(256), 0, s, buf(l.g), o, v,
                         buf(l.pm));
      rows = npairs * v;
    } else {
      gemm(ov, ov, Rt, buf(l.c1), Rt, false, buf(l.bp), Rt, true, buf(l.g), ov);  // G = C1 Bp^T
      hipLaunchKernelGGL(swap_product_kernel, dim3(nv * nv * o * o), dim3(256), 0, s, buf(l.g), o, v, buf(l.pm));
      rows = ov * o;
    }
    {
      int grid = (n_points * v + 255) / 256;
      hipLaunchKernelGGL(virt_factor_kernel, dim3(grid), dim3(256), 0, s, eps_virt, v, q, buf(l.ut));
    }
    gemm(n_points, rows, v, buf(l.ut), v, false, buf(l.pm), v, true, buf(l.ht), rows);  // H^T = U^T Pm^T
    if (z_sym)
      hipLaunchKernelGGL(occ_weight_dot_lower_kernel, dim3(l.kchunks, n_points), dim3(256), 0, s, buf(l.ht),
                         eps_occ, eps_virt, o, v, q, buf(l.pk));
    else
      hipLaunchKernelGGL(occ_weight_dot_kernel, dim3(l.kchunks, n_points), dim3(256), 0, s, buf(l.ht), eps_occ,
                         eps_virt, o, v, q, buf(l.pk));
  }
  hipLaunchKernelGGL(mp2_finish_kernel, dim3(1), dim3(64 * kFinishWaves), 0, s, buf(l.pj), l.jtiles,
                     with_k ? buf(l.pk) : buf(l.pj), with_k ? l.kchunks : 0, q, J, with_k ? K : nullptr,
                     energies);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

}  // extern "C"
