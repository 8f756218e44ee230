// Learned warm start for CP-ALS (gfx950).
//
// With a diagonal core the THC form is already an exact CP decomposition
// whose columns are the grid columns X_m[:, P] (eq. THC), so an initial CP
// is built from R_cp selected grid columns, each scaled.  A three-layer
// network scores every grid point from eight features of (X0, Z, S) and
// predicts a log-scale; the top-R_cp grid points by score become the
// initial factor columns.  The paper notes that the sweep count depends
// strongly on the initial guess (Results) and leaves better guesses open.
//
//   features   per grid point P: log Z_PP, log sum_Q |Z_PQ|, log S_PP,
//              log sum_Q S_PQ^2, log max_p |X0_pP|, participation ratio
//              (sum x^2)^2 / (n sum x^4), log sum_Q S_PQ^2 |Z_PQ|,
//              log Z_PP S_PP^2; standardised over the grid points.
//   selection  rank of every grid point by score (ties: smaller P first),
//              F_m[:, k] = exp(ell_P) (X_m[:, P] + sigma ||X_m[:, P]|| R^_m[:, k])
//              for rank k < R_cp, R^ the unit columns of the caller's
//              random guess (the positive, strongly overlapping grid
//              columns alone make a nearly degenerate start).
//   labels     greedy one-to-one matching of a converged CPD's mode-0
//              columns to grid columns by |cosine|, largest first.
//   network    8 -> 256 -> 256 -> 2 with SiLU; FP32 training (the 256 x 256
//              layer and its gradients on the FP32 matrix cores through the
//              GEMM kernel, the rest in fused element-wise and fixed-order
//              reduction kernels, Adam); BF16 inference in one fused kernel
//              (the 256 x 256 layer on the BF16 matrix cores, FP32
//              accumulation).
// Every reduction has a fixed order: results are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <mutex>

#include "../../include/thccp.h"
#include "common.h"
#include "kernels.h"

using namespace thccp;

namespace {

constexpr int D_IN = 8, WIDTH = 256, D_OUT = 2;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + D_IN * WIDTH;
constexpr int OFF_W2 = OFF_B1 + WIDTH;
constexpr int OFF_B2 = OFF_W2 + WIDTH * WIDTH;
constexpr int OFF_W3 = OFF_B2 + WIDTH;
constexpr int OFF_B3 = OFF_W3 + WIDTH * D_OUT;
constexpr int NPARAM = OFF_B3 + D_OUT;

// Packed inference weights: FP32 W1, b1, b2, W3, b3, then W2 transposed in
// BF16 (n-major, so one lane's eight k values are one 16-byte load).
constexpr int PK_W1 = 0;
constexpr int PK_B1 = PK_W1 + D_IN * WIDTH;
constexpr int PK_B2 = PK_B1 + WIDTH;
constexpr int PK_W3 = PK_B2 + WIDTH;
constexpr int PK_B3 = PK_W3 + WIDTH * D_OUT;
constexpr size_t PK_W2T_BYTES = ((size_t)(PK_B3 + D_OUT) * 4 + 255) & ~(size_t)255;
constexpr size_t PK_BYTES = PK_W2T_BYTES + (size_t)WIDTH * WIDTH * 2;

constexpr int CHUNK = 256;  // rows per partial sum of the reductions over rows
constexpr double TINY = 1e-300;

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }
int grid_of(size_t n) {
  size_t g = (n + 255) / 256;
  return (int)(g > 16384 ? 16384 : (g < 1 ? 1 : g));
}

#define WSCHK(x)                             \
  do {                                       \
    if ((x) != hipSuccess) return CPD_ERR_HIP; \
  } while (0)

struct Carve {
  char* p;
  size_t used = 0;
  template <typename T>
  T* take(size_t count) {
    T* r = (T*)(p + used);
    used += al(sizeof(T) * count);
    return r;
  }
};

// log(max(v, 1e-300)), NaN propagating like the definition's max.
__device__ __forceinline__ double lg(double v) { return v != v ? v : log(v > TINY ? v : TINY); }
__device__ __forceinline__ float sigm(float a) { return 1.f / (1.f + expf(-a)); }
__device__ __forceinline__ float silu(float a) { return a * sigm(a); }
__device__ __forceinline__ float silu_grad(float a) {
  const float g = sigm(a);
  return g * (1.f + a * (1.f - g));
}

// Fixed-order tree reduction over the 256 threads of a block.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  T r = sh[0];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------ features
__global__ __launch_bounds__(256) void feat_rows_kernel(const double* Z, const double* S, int R, double* raw) {
  __shared__ double sh[256];
  const int P = blockIdx.x;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int Q = threadIdx.x; Q < R; Q += 256) {
    const double z = fabs(Z[(size_t)P * R + Q]);
    const double s = S[(size_t)P * R + Q];
    a += z;
    b += s * s;
    c += s * s * z;
  }
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  c = block_sum(c, sh);
  if (threadIdx.x == 0) {
    const double zd = Z[(size_t)P * R + P], sd = S[(size_t)P * R + P];
    double* f = raw + (size_t)P * D_IN;
    f[0] = lg(zd);
    f[1] = lg(a);
    f[2] = lg(sd);
    f[3] = lg(b);
    f[6] = lg(c);
    f[7] = lg(zd * sd * sd);
  }
}

__global__ void feat_cols_kernel(const double* X0, int n, int R, double* raw) {
  const int P = blockIdx.x * 256 + threadIdx.x;
  if (P >= R) return;
  double mx = 0.0, x2 = 0.0, x4 = 0.0;
  for (int p = 0; p < n; ++p) {
    const double x = X0[(size_t)p * R + P];
    if (fabs(x) > mx || x != x) mx = fabs(x);  // NaN sticks
    x2 += x * x;
    x4 += (x * x) * (x * x);
  }
  raw[(size_t)P * D_IN + 4] = lg(mx);
  raw[(size_t)P * D_IN + 5] = x4 > 0.0 ? x2 * x2 / ((double)n * x4) : 0.0;
}

__global__ __launch_bounds__(256) void feat_standardise_kernel(const double* raw, int R, float* feat, double* heur) {
  __shared__ double sh[256];
  const int f = blockIdx.x;
  double s = 0.0;
  for (int P = threadIdx.x; P < R; P += 256) s += raw[(size_t)P * D_IN + f];
  const double mu = block_sum(s, sh) / R;
  double v = 0.0;
  for (int P = threadIdx.x; P < R; P += 256) {
    const double d = raw[(size_t)P * D_IN + f] - mu;
    v += d * d;
  }
  const double sd = sqrt(block_sum(v, sh) / R);
  const bool ok = sd > 1e-9 * fmax(1.0, fabs(mu));
  for (int P = threadIdx.x; P < R; P += 256) {
    const double x = raw[(size_t)P * D_IN + f];
    feat[(size_t)P * D_IN + f] = ok ? (float)((x - mu) / sd) : 0.f;
    if (f == 7 && heur) heur[P] = x;
  }
}

// ------------------------------------------------------------ selection
template <typename S>
__global__ void rank_kernel(const S* s, int stride, int R, int Rc, int* perm) {
  const int P = blockIdx.x * 256 + threadIdx.x;
  if (P >= R) return;
  const S sp = s[(size_t)P * stride];
  int cnt = 0;
  for (int Q = 0; Q < R; ++Q) {
    const S sq = s[(size_t)Q * stride];
    cnt += (sq > sp) || (sq == sp && Q < P);
  }
  if (cnt < Rc) perm[cnt] = P;
}

struct ScatterArgs {
  const double* X[4];
  const double* noise[4];  // nullable: no blend
  double* F[4];
  int n[4];
};
// Column norms for the blend: xn[m][P] of X_m (r_thc per mode) and
// rn[m][k] of noise_m (r_cp per mode), laid out as 4 x (R + Rc).
__global__ void blend_norms_kernel(ScatterArgs a, int R, int Rc, double* norms) {
  const int m = blockIdx.y, z = blockIdx.z;
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int cols = z ? Rc : R;
  if (c >= cols) return;
  const double* A = z ? a.noise[m] : a.X[m];
  double s = 0.0;
  for (int p = 0; p < a.n[m]; ++p) {
    const double v = A[(size_t)p * cols + c];
    s += v * v;
  }
  norms[(size_t)m * (R + Rc) + (z ? R : 0) + c] = sqrt(s);
}
// F_m[p, k] = exp(ell_P) (X_m[p, P] + sigma ||X_m[:, P]|| R_m[p, k] / ||R_m[:, k]||),
// P = perm[k].  Every element is read and written by one thread, so noise
// may alias F.
__global__ void scatter_kernel(ScatterArgs a, int R, int Rc, const int* perm, const float* ell, int stride,
                               double sigma, const double* norms) {
  const int m = blockIdx.y;
  const size_t total = (size_t)a.n[m] * Rc;
  const double* xn = norms + (size_t)m * (R + Rc);
  const double* rn = xn + R;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const int p = (int)(e / Rc), k = (int)(e % Rc);
    const int P = perm[k];
    const double sc = ell ? exp((double)ell[(size_t)P * stride]) : 1.0;
    double v = a.X[m][(size_t)p * R + P];
    if (a.noise[m]) {
      const double unit = rn[k] > 0.0 ? a.noise[m][e] / rn[k] : 0.0;
      v = v + (sigma * xn[P]) * unit;
    }
    a.F[m][e] = v * sc;
  }
}

template <typename S>
__global__ void finite_kernel(const S* v, size_t count, int* bad) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (size_t)gridDim.x * 256)
    if (!isfinite((double)v[e])) *bad = 1;
}

// ------------------------------------------------------------ labels
__global__ void col_norms_kernel(const double* A, int rows, int cols, double* out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int r = 0; r < rows; ++r) {
    const double v = A[(size_t)r * cols + c];
    s += v * v;
  }
  out[c] = sqrt(s);
}

__global__ void abs_cos_kernel(double* C, const double* fn, const double* xn, int Rc, int R) {
  const size_t total = (size_t)Rc * R;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const int k = (int)(e / R), P = (int)(e % R);
    const double den = fn[k] * xn[P];
    C[e] = den > 0.0 ? fabs(C[e]) / den : 0.0;
  }
}

// Better of two (value, index) candidates: larger value, then smaller index.
__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i >= 0 && (bi < 0 || i < bi));
}

__global__ __launch_bounds__(256) void row_argmax_kernel(const double* C, int R, double* rowmax, int* rowarg) {
  __shared__ double sv[256];
  __shared__ int si[256];
  const int k = blockIdx.x, tid = threadIdx.x;
  double bv = -1.0;
  int bi = -1;
  for (int P = tid; P < R; P += 256) {
    const double v = C[(size_t)k * R + P];
    if (better(v, P, bv, bi)) { bv = v; bi = P; }
  }
  sv[tid] = bv;
  si[tid] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w && better(sv[tid + w], si[tid + w], sv[tid], si[tid])) {
      sv[tid] = sv[tid + w];
      si[tid] = si[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    rowmax[k] = sv[0];
    rowarg[k] = si[0];
  }
}

// Greedy matching in one workgroup: each round takes the largest remaining
// entry (ties: smaller row, then smaller column), then rescans the rows
// whose best column was just taken.
__global__ __launch_bounds__(1024) void greedy_kernel(const double* C, int Rc, int R, double* rowmax, int* rowarg,
                                                      int* rowused, int* colused, int* match) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  const int tid = threadIdx.x;
  for (int k = tid; k < Rc; k += 1024) {
    rowused[k] = 0;
    match[k] = -1;
  }
  for (int P = tid; P < R; P += 1024) colused[P] = 0;
  __syncthreads();
  const int rounds = Rc < R ? Rc : R;
  for (int round = 0; round < rounds; ++round) {
    double bv = -1.0;
    int bk = -1;
    for (int k = tid; k < Rc; k += 1024) {
      if (rowused[k] || rowarg[k] < 0) continue;
      if (better(rowmax[k], k, bv, bk)) { bv = rowmax[k]; bk = k; }
    }
    sv[tid] = bv;
    si[tid] = bk;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (tid < w && better(sv[tid + w], si[tid + w], sv[tid], si[tid])) {
        sv[tid] = sv[tid + w];
        si[tid] = si[tid + w];
      }
      __syncthreads();
    }
    const int ks = si[0];
    if (ks < 0) break;  // uniform: every thread read the same value
    const int Ps = rowarg[ks];
    __syncthreads();
    if (tid == 0) {
      match[ks] = Ps;
      rowused[ks] = 1;
      colused[Ps] = 1;
    }
    __syncthreads();
    for (int k = tid; k < Rc; k += 1024) {
      if (rowused[k] || rowarg[k] != Ps) continue;
      double v = -1.0;
      int b = -1;
      for (int P = 0; P < R; ++P) {
        if (colused[P]) continue;
        const double c = C[(size_t)k * R + P];
        if (better(c, P, v, b)) { v = c; b = P; }
      }
      rowmax[k] = v;
      rowarg[k] = b;
    }
    __syncthreads();
  }
}

struct LabelArgs {
  const double* X[4];
  const double* F[4];
  int n[4];
};
__global__ __launch_bounds__(256) void label_targets_kernel(LabelArgs a, const double* lam, const int* match, int R,
                                                            int Rc, float* y, float* ell, float* mask) {
  __shared__ double sh[256];
  const int k = blockIdx.x;
  const int P = match[k];
  if (P < 0) return;
  const double w = pow(fabs(lam[k]), 0.25);
  double acc = 0.0;
  bool ok = true;
  for (int m = 0; m < 4; ++m) {
    double xx = 0.0, d = 0.0;
    for (int p = threadIdx.x; p < a.n[m]; p += 256) {
      const double x = a.X[m][(size_t)p * R + P];
      xx += x * x;
      d += a.F[m][(size_t)p * Rc + k] * x;
    }
    xx = block_sum(xx, sh);
    d = block_sum(d, sh);
    if (!(xx > 0.0)) {
      ok = false;
      break;
    }
    acc += lg(fabs(w * d / xx));
  }
  if (threadIdx.x == 0) {
    y[P] = 1.f;
    ell[P] = ok ? (float)(acc / 4.0) : 0.f;
    mask[P] = ok ? 1.f : 0.f;
  }
}

__global__ void zero_f32(float* a, size_t n) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) a[e] = 0.f;
}

// ------------------------------------------------------------ network, FP32
__global__ __launch_bounds__(256) void l1_fwd_kernel(const float* prm, const float* x, const int* idx, int rows,
                                                     float* a1, float* h1) {
  const int r = blockIdx.x, j = threadIdx.x;
  const int src = idx ? idx[r] : r;
  float a = prm[OFF_B1 + j];
#pragma unroll
  for (int i = 0; i < D_IN; ++i) a += x[(size_t)src * D_IN + i] * prm[OFF_W1 + i * WIDTH + j];
  a1[(size_t)r * WIDTH + j] = a;
  h1[(size_t)r * WIDTH + j] = silu(a);
}

__global__ void bias_act_kernel(float* a, const float* b, float* h, size_t total) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const float v = a[e] + b[e % WIDTH];
    a[e] = v;
    h[e] = silu(v);
  }
}

// out = h2 W3 + b3: one wave per row, lane l holds columns 4l .. 4l+3.
__global__ __launch_bounds__(256) void l3_fwd_kernel(const float* prm, const float* h2, int rows, float* out) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  float s0 = 0.f, s1 = 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = 4 * lane + q;
    const float h = h2[(size_t)r * WIDTH + c];
    s0 += h * prm[OFF_W3 + 2 * c];
    s1 += h * prm[OFF_W3 + 2 * c + 1];
  }
  for (int m = 32; m > 0; m >>= 1) {
    s0 += __shfl_xor(s0, m);
    s1 += __shfl_xor(s1, m);
  }
  if (lane == 0) {
    out[2 * (size_t)r] = s0 + prm[OFF_B3];
    out[2 * (size_t)r + 1] = s1 + prm[OFF_B3 + 1];
  }
}

__global__ __launch_bounds__(256) void loss_partial_kernel(const float* out, const float* y, const float* ell_t,
                                                           const float* mask, const int* idx, int rows,
                                                           double* part) {
  __shared__ double sh[256];
  const int r = blockIdx.x * CHUNK + threadIdx.x;
  double bce = 0.0, ms = 0.0, sq = 0.0;
  if (r < rows) {
    const int src = idx ? idx[r] : r;
    const float s = out[2 * (size_t)r], l = out[2 * (size_t)r + 1];
    const float yv = y[src], lt = ell_t[src], mv = mask[src];
    bce = (double)(fmaxf(s, 0.f) - s * yv + log1pf(expf(-fabsf(s))));
    ms = mv;
    sq = (double)(mv * (l - lt) * (l - lt));
  }
  bce = block_sum(bce, sh);
  ms = block_sum(ms, sh);
  sq = block_sum(sq, sh);
  if (threadIdx.x == 0) {
    part[3 * (size_t)blockIdx.x] = bce;
    part[3 * (size_t)blockIdx.x + 1] = ms;
    part[3 * (size_t)blockIdx.x + 2] = sq;
  }
}

__global__ __launch_bounds__(256) void loss_final_kernel(const double* part, int nchunk, int rows, double* loss,
                                                         double* msum_out) {
  __shared__ double sh[256];
  double b = 0.0, m = 0.0, q = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += 256) {
    b += part[3 * (size_t)c];
    m += part[3 * (size_t)c + 1];
    q += part[3 * (size_t)c + 2];
  }
  b = block_sum(b, sh);
  m = block_sum(m, sh);
  q = block_sum(q, sh);
  if (threadIdx.x == 0) {
    const double ms = m > 1.0 ? m : 1.0;
    *msum_out = ms;
    if (loss) *loss = b / rows + q / ms;
  }
}

__global__ void loss_grad_kernel(const float* out, const float* y, const float* ell_t, const float* mask,
                                 const int* idx, int rows, const double* msum, float* dout) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  const int src = idx ? idx[r] : r;
  const float s = out[2 * (size_t)r], l = out[2 * (size_t)r + 1];
  const float inv_ms = (float)(1.0 / *msum);
  dout[2 * (size_t)r] = (sigm(s) - y[src]) / (float)rows;
  dout[2 * (size_t)r + 1] = 2.f * mask[src] * (l - ell_t[src]) * inv_ms;
}

// Partial sums over row chunks: part[chunk][t][c] = sum_r L[r][t] D[r][c]
// for t < T and sum_r D[r][c] for t = T (bias).  L rows may be gathered.
__global__ __launch_bounds__(256) void rowred_partial_kernel(const float* L, int ldl, const int* lidx, int T,
                                                             const float* D, int ldd, int C, int rows,
                                                             float* part) {
  const int chunk = blockIdx.x;
  const int r0 = chunk * CHUNK;
  const int r1 = r0 + CHUNK < rows ? r0 + CHUNK : rows;
  const int nout = (T + 1) * C;
  for (int o = threadIdx.x; o < nout; o += 256) {
    const int t = o / C, c = o % C;
    float acc = 0.f;
    for (int r = r0; r < r1; ++r) {
      const float lv = t < T ? L[(size_t)(lidx ? lidx[r] : r) * ldl + t] : 1.f;
      acc += lv * D[(size_t)r * ldd + c];
    }
    part[(size_t)chunk * nout + o] = acc;
  }
}
__global__ void rowred_final_kernel(const float* part, int nchunk, int T, int C, float* gW, float* gb) {
  const int nout = (T + 1) * C;
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= nout) return;
  float acc = 0.f;
  for (int c = 0; c < nchunk; ++c) acc += part[(size_t)c * nout + o];
  const int t = o / C;
  if (t < T) gW[o] = acc;
  else gb[o - T * C] = acc;
}

__global__ void da2_kernel(const float* prm, const float* dout, const float* a2, float* da2, size_t total) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const size_t r = e / WIDTH;
    const int c = (int)(e % WIDTH);
    const float g = dout[2 * r] * prm[OFF_W3 + 2 * c] + dout[2 * r + 1] * prm[OFF_W3 + 2 * c + 1];
    da2[e] = g * silu_grad(a2[e]);
  }
}

__global__ void act_bwd_kernel(float* dh, const float* a, size_t total) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256)
    dh[e] *= silu_grad(a[e]);
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                            float eps, float bc1, float bc2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * bc1) / (sqrtf(vi * bc2) + eps);
}

// ------------------------------------------------------------ network, BF16 inference
__global__ void pack_kernel(const float* prm, float* pk, __bf16* w2t) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < WIDTH * WIDTH) {
    const int n = e / WIDTH, k = e % WIDTH;
    w2t[e] = (__bf16)prm[OFF_W2 + k * WIDTH + n];
  }
  if (e < D_IN * WIDTH) pk[PK_W1 + e] = prm[OFF_W1 + e];
  if (e < WIDTH) {
    pk[PK_B1 + e] = prm[OFF_B1 + e];
    pk[PK_B2 + e] = prm[OFF_B2 + e];
  }
  if (e < WIDTH * D_OUT) pk[PK_W3 + e] = prm[OFF_W3 + e];
  if (e < D_OUT) pk[PK_B3 + e] = prm[OFF_B3 + e];
}

constexpr int IR = 64;         // rows per workgroup
constexpr int HLD = WIDTH + 8;  // LDS row stride (bf16), keeps 16-byte alignment

__global__ __launch_bounds__(256) void infer_bf16_kernel(const float* pk, const __bf16* w2t, const float* x,
                                                         int rows, float* out) {
  __shared__ float xs[IR][D_IN];
  __shared__ __attribute__((aligned(16))) __bf16 hs[IR * HLD];
  __shared__ float red[4][IR][D_OUT];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r0 = blockIdx.x * IR;
  for (int e = tid; e < IR * D_IN; e += 256) {
    const int r = e / D_IN, i = e % D_IN;
    xs[r][i] = r0 + r < rows ? x[(size_t)(r0 + r) * D_IN + i] : 0.f;
  }
  __syncthreads();
  {
    const int j = tid;
    float wj[D_IN];
#pragma unroll
    for (int i = 0; i < D_IN; ++i) wj[i] = pk[PK_W1 + i * WIDTH + j];
    const float bj = pk[PK_B1 + j];
    for (int r = 0; r < IR; ++r) {
      float a = bj;
#pragma unroll
      for (int i = 0; i < D_IN; ++i) a += xs[r][i] * wj[i];
      hs[r * HLD + j] = (__bf16)silu(a);
    }
  }
  __syncthreads();
  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int k0 = 0; k0 < WIDTH; k0 += 32) {
    const int koff = k0 + 8 * (lane >> 4);
    bf16x8_t a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = *(const bf16x8_t*)&hs[(16 * i + (lane & 15)) * HLD + koff];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = *(const bf16x8_t*)&w2t[(size_t)(64 * w + 16 * j + (lane & 15)) * WIDTH + koff];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
  // h2 = silu(acc + b2); partial out over this lane's columns, then over
  // the 16 lanes of a row group, then over the four waves.
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = 64 * w + 16 * j + (lane & 15);
        const float h = silu(acc[i][j][r] + pk[PK_B2 + col]);
        s0 += h * pk[PK_W3 + 2 * col];
        s1 += h * pk[PK_W3 + 2 * col + 1];
      }
      for (int m = 8; m > 0; m >>= 1) {
        s0 += __shfl_xor(s0, m);
        s1 += __shfl_xor(s1, m);
      }
      if ((lane & 15) == 0) {
        const int row = 16 * i + 4 * (lane >> 4) + r;
        red[w][row][0] = s0;
        red[w][row][1] = s1;
      }
    }
  __syncthreads();
  if (tid < IR * D_OUT) {
    const int row = tid / D_OUT, j = tid % D_OUT;
    if (r0 + row < rows)
      out[(size_t)(r0 + row) * D_OUT + j] =
          pk[PK_B3 + j] + ((red[0][row][j] + red[1][row][j]) + (red[2][row][j] + red[3][row][j]));
  }
}

// ------------------------------------------------------------ workspace layouts
struct FeatWs {
  double* S;
  double* raw;
};
FeatWs carve_feat(Carve& c, int R) { return {c.take<double>((size_t)R * R), c.take<double>((size_t)R * D_IN)}; }
size_t feat_bytes(int R) { return al(sizeof(double) * (size_t)R * R) + al(sizeof(double) * (size_t)R * D_IN); }

int enqueue_features(hipStream_t s, int n0, int R, const double* X0, const double* Z, float* feat, double* heur,
                     FeatWs w) {
  GemmF64 g{R, R, n0, X0, R, true, X0, nullptr, R, false, w.S, R, nullptr, 1.0, 0.0, nullptr};
  gemm_f64(s, g);
  hipLaunchKernelGGL(feat_rows_kernel, dim3(R), dim3(256), 0, s, Z, w.S, R, w.raw);
  hipLaunchKernelGGL(feat_cols_kernel, dim3((R + 255) / 256), dim3(256), 0, s, X0, n0, R, w.raw);
  hipLaunchKernelGGL(feat_standardise_kernel, dim3(D_IN), dim3(256), 0, s, w.raw, R, feat, heur);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

bool dims_ok(const int32_t n[4], int32_t r_thc, int32_t r_cp) {
  if (!n || r_thc <= 0 || r_cp <= 0 || r_cp > r_thc) return false;
  for (int m = 0; m < 4; ++m)
    if (n[m] <= 0) return false;
  return true;
}

size_t select_bytes(int R, int Rc) { return al(sizeof(int) * (size_t)Rc) + al(sizeof(double) * 4 * ((size_t)R + Rc)); }

int enqueue_select(hipStream_t s, const int32_t n[4], int R, int Rc, const double* const X[4], double* const F[4],
                   const int* perm, const float* ell, int stride, const double* const noise[4], double sigma,
                   double* norms) {
  ScatterArgs a;
  size_t most = 0;
  int nmax = 0;
  for (int m = 0; m < 4; ++m) {
    a.X[m] = X[m];
    a.noise[m] = (noise && sigma != 0.0) ? noise[m] : nullptr;
    a.F[m] = F[m];
    a.n[m] = n[m];
    most = (size_t)n[m] * Rc > most ? (size_t)n[m] * Rc : most;
    nmax = n[m] > nmax ? n[m] : nmax;
  }
  if (a.noise[0]) {
    const int cols = R > Rc ? R : Rc;
    hipLaunchKernelGGL(blend_norms_kernel, dim3((cols + 255) / 256, 4, 2), dim3(256), 0, s, a, R, Rc, norms);
  }
  hipLaunchKernelGGL(scatter_kernel, dim3(grid_of(most), 4), dim3(256), 0, s, a, R, Rc, perm, ell, stride, sigma,
                     norms);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

size_t mlp_ws_bytes(int rows) {
  const size_t act = al(sizeof(float) * (size_t)rows * WIDTH);
  const int nchunk = (rows + CHUNK - 1) / CHUNK;
  return 6 * act + al(sizeof(float) * (size_t)nchunk * (D_IN + 1) * WIDTH) + al(sizeof(double) * 3 * (size_t)nchunk) +
         al(sizeof(double));
}
struct MlpWs {
  float *a1, *h1, *a2, *h2, *d1, *d2, *part;
  double *lpart, *msum;
};
MlpWs carve_mlp(void* ws, int rows) {
  Carve c{(char*)ws};
  const size_t act = (size_t)rows * WIDTH;
  const int nchunk = (rows + CHUNK - 1) / CHUNK;
  MlpWs w;
  w.a1 = c.take<float>(act);
  w.h1 = c.take<float>(act);
  w.a2 = c.take<float>(act);
  w.h2 = c.take<float>(act);
  w.d1 = c.take<float>(act);
  w.d2 = c.take<float>(act);
  w.part = c.take<float>((size_t)nchunk * (D_IN + 1) * WIDTH);
  w.lpart = c.take<double>(3 * (size_t)nchunk);
  w.msum = c.take<double>(1);
  return w;
}

void rowred(hipStream_t s, const float* L, int ldl, const int* lidx, int T, const float* D, int ldd, int C,
            int rows, float* part, float* gW, float* gb) {
  const int nchunk = (rows + CHUNK - 1) / CHUNK;
  hipLaunchKernelGGL(rowred_partial_kernel, dim3(nchunk), dim3(256), 0, s, L, ldl, lidx, T, D, ldd, C, rows, part);
  const int nout = (T + 1) * C;
  hipLaunchKernelGGL(rowred_final_kernel, dim3((nout + 255) / 256), dim3(256), 0, s, part, nchunk, T, C, gW, gb);
}

// Scratch of the allocation-free feature entry point: S = X0^T X0
// (r_thc^2 doubles) and the raw features (r_thc x 8 doubles) for
// r_thc <= WS_NOALLOC_MAX_RTHC.  One copy per GPU, alive until the process
// ends; host code uses only the device address of this array looked up with
// hipGetSymbolAddress, once per device (the name itself is a host-side
// stand-in, not a device address).
constexpr int WS_NOALLOC_MAX_RTHC = 2048;
constexpr size_t al_c(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t WS_NOALLOC_BYTES =
    al_c(sizeof(double) * (size_t)WS_NOALLOC_MAX_RTHC * WS_NOALLOC_MAX_RTHC) +
    al_c(sizeof(double) * (size_t)WS_NOALLOC_MAX_RTHC * D_IN);
static __device__ __align__(256) char feat_scratch[WS_NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[MAX_DEVICES] = {};

// Device address of feat_scratch on the current device (looked up on the
// first call per device); nullptr if the lookup fails.
void* scratch_of_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(feat_scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

}  // namespace

extern "C" {

size_t cpd_ws_workspace_size(int32_t n0, int32_t r_thc, int32_t r_cp) {
  if (n0 <= 0 || r_thc <= 0 || r_cp <= 0 || r_cp > r_thc) return 0;
  const size_t R = r_thc, Rc = r_cp;
  return feat_bytes(r_thc) + al(sizeof(float) * R * D_IN) + al(sizeof(double) * R) + al(sizeof(float) * R * D_OUT) +
         select_bytes(r_thc, r_cp) + al(sizeof(int)) + al(sizeof(double) * Rc * R) + 2 * al(sizeof(double) * (Rc + R)) +
         4 * al(sizeof(int) * (Rc + R));
}

cpd_status cpd_ws_features(int32_t n0, int32_t r_thc, const double* X0, const double* Z, float* feat, double* heur,
                           void* workspace, size_t workspace_bytes, void* stream) {
  if (n0 <= 0 || r_thc <= 0 || !X0 || !Z || !feat || !workspace) return CPD_ERR_INVALID_ARG;
  if (workspace_bytes < feat_bytes(r_thc)) return CPD_ERR_WORKSPACE;
  Carve c{(char*)workspace};
  return enqueue_features((hipStream_t)stream, n0, r_thc, X0, Z, feat, heur, carve_feat(c, r_thc));
}

cpd_status cpd_ws_features_noalloc(int32_t n0, int32_t r_thc, const double* X0, const double* Z, float* feat,
                                   double* heur, void* stream) {
  if (n0 <= 0 || r_thc <= 0 || !X0 || !Z || !feat) return CPD_ERR_INVALID_ARG;
  if (r_thc > WS_NOALLOC_MAX_RTHC) return CPD_ERR_INVALID_ARG;
  void* ws = scratch_of_current_device();
  if (!ws) return CPD_ERR_HIP;
  Carve c{(char*)ws};
  return enqueue_features((hipStream_t)stream, n0, r_thc, X0, Z, feat, heur, carve_feat(c, r_thc));
}

cpd_status cpd_ws_select_init(const int32_t n[4], int32_t r_thc, int32_t r_cp, const double* const X[4],
                              const float* s, const float* ell, int32_t stride, const double* const noise[4],
                              double sigma, double* const init[4], void* workspace, size_t workspace_bytes,
                              void* stream) {
  if (!dims_ok(n, r_thc, r_cp) || !X || !s || !init || stride <= 0 || !workspace || !(sigma >= 0.0))
    return CPD_ERR_INVALID_ARG;
  for (int m = 0; m < 4; ++m)
    if (!X[m] || !init[m] || (noise && !noise[m])) return CPD_ERR_INVALID_ARG;
  if (workspace_bytes < select_bytes(r_thc, r_cp)) return CPD_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  Carve c{(char*)workspace};
  int* perm = c.take<int>(r_cp);
  double* norms = c.take<double>(4 * ((size_t)r_thc + r_cp));
  hipLaunchKernelGGL(rank_kernel<float>, dim3((r_thc + 255) / 256), dim3(256), 0, st, s, stride, r_thc, r_cp, perm);
  return enqueue_select(st, n, r_thc, r_cp, X, init, perm, ell, stride, noise, sigma, norms);
}

cpd_status cpd_ws_labels(const int32_t n[4], int32_t r_thc, int32_t r_cp, const double* const X[4],
                         const double* const F[4], const double* lam, float* y, float* ell, float* mask,
                         void* workspace, size_t workspace_bytes, void* stream) {
  if (!dims_ok(n, r_thc, r_cp) || !X || !F || !lam || !y || !ell || !mask || !workspace) return CPD_ERR_INVALID_ARG;
  for (int m = 0; m < 4; ++m)
    if (!X[m] || !F[m]) return CPD_ERR_INVALID_ARG;
  const size_t R = r_thc, Rc = r_cp;
  const size_t need = al(sizeof(double) * Rc * R) + 2 * al(sizeof(double) * (Rc + R)) + 4 * al(sizeof(int) * (Rc + R));
  if (workspace_bytes < need) return CPD_ERR_WORKSPACE;
  Carve c{(char*)workspace};
  double* C = c.take<double>(Rc * R);
  double* fn = c.take<double>(Rc + R);
  double* xn = fn + Rc;
  double* rowmax = c.take<double>(Rc + R);
  int* rowarg = c.take<int>(Rc + R);
  int* rowused = c.take<int>(Rc + R);
  int* colused = c.take<int>(Rc + R);
  int* match = c.take<int>(Rc + R);
  hipStream_t st = (hipStream_t)stream;
  GemmF64 g{r_cp, r_thc, n[0], F[0], r_cp, true, X[0], nullptr, r_thc, false, C, r_thc, nullptr, 1.0, 0.0, nullptr};
  gemm_f64(st, g);
  hipLaunchKernelGGL(col_norms_kernel, dim3((r_cp + 255) / 256), dim3(256), 0, st, F[0], n[0], r_cp, fn);
  hipLaunchKernelGGL(col_norms_kernel, dim3((r_thc + 255) / 256), dim3(256), 0, st, X[0], n[0], r_thc, xn);
  hipLaunchKernelGGL(abs_cos_kernel, dim3(grid_of(Rc * R)), dim3(256), 0, st, C, fn, xn, r_cp, r_thc);
  hipLaunchKernelGGL(row_argmax_kernel, dim3(r_cp), dim3(256), 0, st, C, r_thc, rowmax, rowarg);
  hipLaunchKernelGGL(greedy_kernel, dim3(1), dim3(1024), 0, st, C, r_cp, r_thc, rowmax, rowarg, rowused, colused,
                     match);
  for (float* a : {y, ell, mask}) hipLaunchKernelGGL(zero_f32, dim3(grid_of(R)), dim3(256), 0, st, a, R);
  LabelArgs la;
  for (int m = 0; m < 4; ++m) {
    la.X[m] = X[m];
    la.F[m] = F[m];
    la.n[m] = n[m];
  }
  hipLaunchKernelGGL(label_targets_kernel, dim3(r_cp), dim3(256), 0, st, la, lam, match, r_thc, r_cp, y, ell, mask);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

int32_t cpd_mlp_param_count(void) { return NPARAM; }
size_t cpd_mlp_workspace_size(int32_t rows) { return rows > 0 ? mlp_ws_bytes(rows) : 0; }
size_t cpd_mlp_packed_size(void) { return PK_BYTES; }

cpd_status cpd_mlp_forward(const float* params, const float* x, const int32_t* idx, int32_t rows, float* out,
                           void* workspace, size_t workspace_bytes, void* stream) {
  if (!params || !x || !out || rows <= 0 || !workspace) return CPD_ERR_INVALID_ARG;
  if (workspace_bytes < mlp_ws_bytes(rows)) return CPD_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  MlpWs w = carve_mlp(workspace, rows);
  const size_t act = (size_t)rows * WIDTH;
  hipLaunchKernelGGL(l1_fwd_kernel, dim3(rows), dim3(256), 0, s, params, x, idx, rows, w.a1, w.h1);
  GemmF32 g{rows, WIDTH, WIDTH, w.h1, WIDTH, false, params + OFF_W2, nullptr, WIDTH, false, w.a2, WIDTH, nullptr,
            1.f, 0.f, nullptr};
  gemm_f32(s, g);
  hipLaunchKernelGGL(bias_act_kernel, dim3(grid_of(act)), dim3(256), 0, s, w.a2, params + OFF_B2, w.h2, act);
  hipLaunchKernelGGL(l3_fwd_kernel, dim3((rows + 3) / 4), dim3(256), 0, s, params, w.h2, rows, out);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

cpd_status cpd_mlp_loss(const float* out, const float* y, const float* ell_t, const float* mask, const int32_t* idx,
                        int32_t rows, float* dout, double* loss_dev, void* workspace, size_t workspace_bytes,
                        void* stream) {
  if (!out || !y || !ell_t || !mask || !dout || rows <= 0 || !workspace) return CPD_ERR_INVALID_ARG;
  if (workspace_bytes < mlp_ws_bytes(rows)) return CPD_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  MlpWs w = carve_mlp(workspace, rows);
  const int nchunk = (rows + CHUNK - 1) / CHUNK;
  hipLaunchKernelGGL(loss_partial_kernel, dim3(nchunk), dim3(256), 0, s, out, y, ell_t, mask, idx, rows, w.lpart);
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, s, w.lpart, nchunk, rows, loss_dev, w.msum);
  hipLaunchKernelGGL(loss_grad_kernel, dim3((rows + 255) / 256), dim3(256), 0, s, out, y, ell_t, mask, idx, rows,
                     w.msum, dout);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

cpd_status cpd_mlp_backward(const float* params, const float* x, const int32_t* idx, const float* dout,
                            int32_t rows, float* grads, void* workspace, size_t workspace_bytes, void* stream) {
  if (!params || !x || !dout || !grads || rows <= 0 || !workspace) return CPD_ERR_INVALID_ARG;
  if (workspace_bytes < mlp_ws_bytes(rows)) return CPD_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  MlpWs w = carve_mlp(workspace, rows);
  const size_t act = (size_t)rows * WIDTH;
  // layer 3: dW3 = h2^T dout, db3 = sum dout
  rowred(s, w.h2, WIDTH, nullptr, WIDTH, dout, D_OUT, D_OUT, rows, w.part, grads + OFF_W3, grads + OFF_B3);
  // da2 = (dout W3^T) o silu'(a2)
  hipLaunchKernelGGL(da2_kernel, dim3(grid_of(act)), dim3(256), 0, s, params, dout, w.a2, w.d2, act);
  // layer 2: dW2 = h1^T da2, db2 = sum da2, dh1 = da2 W2^T
  GemmF32 gw{WIDTH, WIDTH, rows, w.h1, WIDTH, true, w.d2, nullptr, WIDTH, false, grads + OFF_W2, WIDTH, nullptr,
             1.f, 0.f, nullptr};
  gemm_f32(s, gw);
  rowred(s, nullptr, 0, nullptr, 0, w.d2, WIDTH, WIDTH, rows, w.part, nullptr, grads + OFF_B2);
  GemmF32 gd{rows, WIDTH, WIDTH, w.d2, WIDTH, false, params + OFF_W2, nullptr, WIDTH, true, w.d1, WIDTH, nullptr,
             1.f, 0.f, nullptr};
  gemm_f32(s, gd);
  // layer 1: da1 = dh1 o silu'(a1), dW1 = x^T da1, db1 = sum da1
  hipLaunchKernelGGL(act_bwd_kernel, dim3(grid_of(act)), dim3(256), 0, s, w.d1, w.a1, act);
  rowred(s, x, D_IN, idx, D_IN, w.d1, WIDTH, WIDTH, rows, w.part, grads + OFF_W1, grads + OFF_B1);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

cpd_status cpd_mlp_adam(float* params, const float* grads, float* m, float* v, int32_t step, float lr, float beta1,
                        float beta2, float eps, void* stream) {
  if (!params || !grads || !m || !v || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return CPD_ERR_INVALID_ARG;
  const double bc1 = 1.0 / (1.0 - pow((double)beta1, step));
  const double bc2 = 1.0 / (1.0 - pow((double)beta2, step));
  hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, grads, m, v,
                     NPARAM, lr, beta1, beta2, eps, (float)bc1, (float)bc2);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

cpd_status cpd_mlp_pack(const float* params, void* packed, void* stream) {
  if (!params || !packed) return CPD_ERR_INVALID_ARG;
  if ((uintptr_t)packed % 256) return CPD_ERR_INVALID_ARG;
  hipLaunchKernelGGL(pack_kernel, dim3((WIDTH * WIDTH + 255) / 256), dim3(256), 0, (hipStream_t)stream, params,
                     (float*)packed, (__bf16*)((char*)packed + PK_W2T_BYTES));
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

cpd_status cpd_mlp_infer_bf16(const void* packed, const float* x, int32_t rows, float* out, void* stream) {
  if (!packed || !x || !out || rows <= 0) return CPD_ERR_INVALID_ARG;
  if ((uintptr_t)packed % 256) return CPD_ERR_INVALID_ARG;
  hipLaunchKernelGGL(infer_bf16_kernel, dim3((rows + IR - 1) / IR), dim3(256), 0, (hipStream_t)stream,
                     (const float*)packed, (const __bf16*)((const char*)packed + PK_W2T_BYTES), x, rows, out);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

cpd_status cpd_ws_init(const int32_t n[4], int32_t r_thc, int32_t r_cp, const double* const X[4], const double* Z,
                       const void* packed, const double* const noise[4], double sigma, double* const init[4],
                       int32_t* source, void* workspace, size_t workspace_bytes, void* stream) {
  if (!dims_ok(n, r_thc, r_cp) || !X || !Z || !init || !workspace || !(sigma >= 0.0)) return CPD_ERR_INVALID_ARG;
  for (int m = 0; m < 4; ++m)
    if (!X[m] || !init[m] || (noise && !noise[m])) return CPD_ERR_INVALID_ARG;
  if (packed && (uintptr_t)packed % 256) return CPD_ERR_INVALID_ARG;
  if (workspace_bytes < cpd_ws_workspace_size(n[0], r_thc, r_cp)) return CPD_ERR_WORKSPACE;
  const int R = r_thc, Rc = r_cp;
  hipStream_t s = (hipStream_t)stream;
  Carve c{(char*)workspace};
  FeatWs fw = carve_feat(c, R);
  float* feat = c.take<float>((size_t)R * D_IN);
  double* heur = c.take<double>(R);
  float* out = c.take<float>((size_t)R * D_OUT);
  int* perm = c.take<int>(Rc);
  double* norms = c.take<double>(4 * ((size_t)R + Rc));
  int* bad = c.take<int>(1);
  int rc = enqueue_features(s, n[0], R, X[0], Z, feat, heur, fw);
  if (rc != CPD_OK) return rc;
  int src = 2;
  int hbad = 1;
  if (packed) {
    hipLaunchKernelGGL(infer_bf16_kernel, dim3((R + IR - 1) / IR), dim3(256), 0, s, (const float*)packed,
                       (const __bf16*)((const char*)packed + PK_W2T_BYTES), feat, R, out);
    WSCHK(hipMemsetAsync(bad, 0, sizeof(int), s));
    hipLaunchKernelGGL(finite_kernel<float>, dim3(grid_of((size_t)R * D_OUT)), dim3(256), 0, s, out,
                       (size_t)R * D_OUT, bad);
    WSCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    WSCHK(hipStreamSynchronize(s));
    if (!hbad) {
      hipLaunchKernelGGL(rank_kernel<float>, dim3((R + 255) / 256), dim3(256), 0, s, out, D_OUT, R, Rc, perm);
      rc = enqueue_select(s, n, R, Rc, X, init, perm, out + 1, D_OUT, noise, sigma, norms);
      src = 0;
    }
  }
  if (src == 2) {
    WSCHK(hipMemsetAsync(bad, 0, sizeof(int), s));
    hipLaunchKernelGGL(finite_kernel<double>, dim3(grid_of(R)), dim3(256), 0, s, heur, (size_t)R, bad);
    WSCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    WSCHK(hipStreamSynchronize(s));
    if (!hbad) {
      hipLaunchKernelGGL(rank_kernel<double>, dim3((R + 255) / 256), dim3(256), 0, s, heur, 1, R, Rc, perm);
      rc = enqueue_select(s, n, R, Rc, X, init, perm, nullptr, 1, noise, sigma, norms);
      src = 1;
    }
  }
  if (rc != CPD_OK) return rc;
  WSCHK(hipStreamSynchronize(s));
  if (source) *source = src;
  return CPD_OK;
}

}  // extern "C"
