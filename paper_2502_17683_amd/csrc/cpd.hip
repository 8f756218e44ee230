// C-ABI of libthccp.so: plan set-up, the matrix-free ALS sweep, fit,
// checkpointing and statistics.  See include/thccp.h for the contract.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/thccp.h"
#include "kernels.h"
#include "mixed.h"

namespace thccp {

static const int HIST_CAP = 4096;

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename T>
struct Bufs {
  const T* X[4];
  const T* Z;
  T* W[4];
  T* Y;
  T* Msol;
  T* Msave;
  T* F[4];
  T* Fsave[4];  // factors at the start of the sweep (fast-path checkpoint)
  T* G[4];
  T* V;
  T* linv;
  T* diagL;
  T* lam;
};

// Carves the workspace; with base == nullptr only computes the size.
struct Layout {
  size_t off = 0;
  char* base = nullptr;
  void* take(size_t bytes) {
    void* p = base ? (void*)(base + off) : nullptr;
    off = align_up(off + bytes);
    return p;
  }
};

}  // namespace thccp

using namespace thccp;

struct cpd_plan_s {
  cpd_desc d;
  hipStream_t stream;
  hipStream_t cap;
  // [fast][fit]: fast = checkpoint + factorisation fused with the forward
  // solve and no retry pass (a failed pivot is replayed by the host through
  // the safe graph); safe = damped retry pass inside the graph.
  hipGraph_t graph[2][2];
  hipGraphExec_t exec[2][2];
  bool have_graph;
  int fit_every;     // mixed precision: the fit (FP64) is evaluated every fit_every sweeps
  long launched;     // sweeps enqueued since init / set_factors
  int n[4], Rt, Rc, Tp, nblk, nmax;
  int prec;
  Bufs<double> b64;
  Bufs<float> b32;
  MixedBufs mx;
  DevState* st;
  DevState* st_save;
  double* fit_hist;
  double* inner_part;
  double* row_part;
  double* setup[3];
  double* partials;
  double* norm2;
  double* scratch64;  // n_max x Tp doubles (FP32 conversions)
  DevState* host_state;  // pinned
};

namespace {

int check_desc(const cpd_desc* d) {
  if (!d) return CPD_ERR_INVALID_ARG;
  for (int m = 0; m < 4; ++m) {
    if (d->n[m] <= 0 || !d->X[m] || !d->init[m]) return CPD_ERR_INVALID_ARG;
  }
  if (d->r_thc <= 0 || d->r_cp <= 0 || !d->Z) return CPD_ERR_INVALID_ARG;
  if (d->r_thc > (1 << 20) || d->r_cp > (1 << 16)) return CPD_ERR_INVALID_ARG;
  for (int m = 0; m < 4; ++m)
    if (d->n[m] > (1 << 24)) return CPD_ERR_INVALID_ARG;
  if (d->precision != CPD_FP64 && d->precision != CPD_FP32 && d->precision != CPD_MIXED_BF16)
    return CPD_ERR_INVALID_ARG;
  if (!(d->tol >= 0.0) || !(d->fit_floor >= 0.0)) return CPD_ERR_INVALID_ARG;
  return CPD_OK;
}

template <typename T>
void carve_typed(Layout& L, cpd_plan_s* p, Bufs<T>& b, bool own_inputs) {
  const int Rt = p->Rt, Tp = p->Tp;
  if (own_inputs) {
    for (int m = 0; m < 4; ++m) {
      int alias = -1;
      for (int q = 0; q < m; ++q)
        if (p->d.X[q] == p->d.X[m]) alias = q;
      b.X[m] = alias >= 0 ? b.X[alias] : (const T*)L.take(sizeof(T) * (size_t)p->n[m] * Rt);
    }
    b.Z = (const T*)L.take(sizeof(T) * (size_t)Rt * Rt);
  }
  for (int m = 0; m < 4; ++m) b.W[m] = (T*)L.take(sizeof(T) * (size_t)Rt * Tp);
  b.Y = (T*)L.take(sizeof(T) * (size_t)Rt * Tp);
  b.Msol = (T*)L.take(sizeof(T) * (size_t)p->nmax * Tp);
  b.Msave = (T*)L.take(sizeof(T) * (size_t)p->n[3] * Tp);
  for (int m = 0; m < 4; ++m) b.F[m] = (T*)L.take(sizeof(T) * (size_t)p->n[m] * Tp);
  for (int m = 0; m < 4; ++m) b.Fsave[m] = (T*)L.take(sizeof(T) * (size_t)p->n[m] * Tp);
  for (int m = 0; m < 4; ++m) b.G[m] = (T*)L.take(sizeof(T) * (size_t)Tp * Tp);
  b.V = (T*)L.take(sizeof(T) * (size_t)Tp * Tp);
  b.linv = (T*)L.take(sizeof(T) * (size_t)p->nblk * 64 * 64);
  b.diagL = (T*)L.take(sizeof(T) * (size_t)Tp);
  b.lam = (T*)L.take(sizeof(T) * (size_t)Tp);
}

size_t carve(cpd_plan_s* p, char* base) {
  Layout L;
  L.base = base;
  const int Rt = p->Rt, Tp = p->Tp;
  p->st = (DevState*)L.take(sizeof(DevState));
  p->st_save = (DevState*)L.take(sizeof(DevState));
  p->fit_hist = (double*)L.take(sizeof(double) * HIST_CAP);
  p->inner_part = (double*)L.take(sizeof(double) * Tp);
  p->row_part = (double*)L.take(sizeof(double) * Tp);
  p->norm2 = (double*)L.take(sizeof(double) * 8);
  const size_t nt = (size_t)((Rt + 63) / 64);
  p->partials = (double*)L.take(sizeof(double) * nt * nt);
  size_t setup_elems = (size_t)Rt * Rt;
  if ((size_t)p->nmax * Tp > setup_elems) setup_elems = (size_t)p->nmax * Tp;
  for (int i = 0; i < 3; ++i) p->setup[i] = (double*)L.take(sizeof(double) * setup_elems);
  p->scratch64 = (double*)L.take(sizeof(double) * (size_t)p->nmax * Tp);
  if (p->prec == CPD_FP64) {
    carve_typed<double>(L, p, p->b64, false);
    for (int m = 0; m < 4; ++m) p->b64.X[m] = p->d.X[m];
    p->b64.Z = p->d.Z;
  } else if (p->prec == CPD_FP32) {
    carve_typed<float>(L, p, p->b32, true);
  } else {
    // mixed: FP64 factors / Grams / solve, split-BF16 operand copies
    carve_typed<double>(L, p, p->b64, false);
    for (int m = 0; m < 4; ++m) p->b64.X[m] = p->d.X[m];
    p->b64.Z = p->d.Z;
    mixed_carve(L.base, &L.off, p->mx, p->n, Rt, p->Rc, p->d.X);
  }
  return L.off;
}

void fill_shape(cpd_plan_s* p, const cpd_desc* d) {
  p->d = *d;
  for (int m = 0; m < 4; ++m) p->n[m] = d->n[m];
  p->Rt = d->r_thc;
  p->Rc = d->r_cp;
  p->nblk = (d->r_cp + 63) / 64;
  p->Tp = p->nblk * 64;
  p->nmax = 0;
  for (int m = 0; m < 4; ++m)
    if (p->n[m] > p->nmax) p->nmax = p->n[m];
  p->prec = d->precision;
  p->fit_every = d->fit_every > 0 ? d->fit_every : 1;
  p->launched = 0;
}

#define HIPCHK(x)                                    \
  do {                                               \
    hipError_t e_ = (x);                             \
    if (e_ != hipSuccess) return CPD_ERR_HIP;        \
  } while (0)

// ------------------------------------------------------------------ set-up
int setup_norm2(cpd_plan_s* p, hipStream_t s) {
  const int Rt = p->Rt;
  double *A = p->setup[0], *B = p->setup[1], *C = p->setup[2];
  const double* const* X = p->d.X;
  auto syrk = [&](const double* x, int n, double* out) {
    GemmF64 g{Rt, Rt, n, x, Rt, true, x, nullptr, Rt, false, out, Rt, nullptr, 1.0, 0.0, nullptr};
    gemm_f64(s, g);
  };
  const size_t cnt = (size_t)Rt * Rt;
  syrk(X[0], p->n[0], A);
  if (X[1] == X[0]) hadamard_inplace_f64(s, A, A, cnt);
  else { syrk(X[1], p->n[1], B); hadamard_inplace_f64(s, A, B, cnt); }
  // P = Z^T (S0 o S1)
  { GemmF64 g{Rt, Rt, Rt, p->d.Z, Rt, true, A, nullptr, Rt, false, C, Rt, nullptr, 1.0, 0.0, nullptr}; gemm_f64(s, g); }
  if (!(X[2] == X[0] && X[3] == X[1])) {
    syrk(X[2], p->n[2], A);
    if (X[3] == X[2]) hadamard_inplace_f64(s, A, A, cnt);
    else { syrk(X[3], p->n[3], B); hadamard_inplace_f64(s, A, B, cnt); }
  }
  // Q = Z (S2 o S3)
  { GemmF64 g{Rt, Rt, Rt, p->d.Z, Rt, false, A, nullptr, Rt, false, B, Rt, nullptr, 1.0, 0.0, nullptr}; gemm_f64(s, g); }
  transposed_dot_f64(s, C, B, Rt, Rt, p->partials, p->norm2);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

template <typename T>
void gemm_t(hipStream_t s, int M, int N, int K, const T* A, int lda, bool at, const T* B1,
            const T* B2, int ldb, T* C, int ldc, T* C2, const int32_t* done);
template <>
void gemm_t<double>(hipStream_t s, int M, int N, int K, const double* A, int lda, bool at,
                    const double* B1, const double* B2, int ldb, double* C, int ldc, double* C2,
                    const int32_t* done) {
  GemmF64 g{M, N, K, A, lda, at, B1, B2, ldb, false, C, ldc, C2, 1.0, 0.0, done};
  gemm_f64(s, g);
}
template <>
void gemm_t<float>(hipStream_t s, int M, int N, int K, const float* A, int lda, bool at,
                   const float* B1, const float* B2, int ldb, float* C, int ldc, float* C2,
                   const int32_t* done) {
  GemmF32 g{M, N, K, A, lda, at, B1, B2, ldb, false, C, ldc, C2, 1.0f, 0.0f, done};
  gemm_f32(s, g);
}

// Projection W_m = X_m^T F_m and Gram F_m^T F_m of one mode.
template <typename T>
void refresh_mode(cpd_plan_s* p, Bufs<T>& b, int m, hipStream_t s, const int32_t* done) {
  const int Rt = p->Rt, Rc = p->Rc, Tp = p->Tp;
  gemm_t<T>(s, Rc, Rc, p->n[m], b.F[m], Tp, true, b.F[m], nullptr, Tp, b.G[m], Tp, nullptr, done);
  gemm_t<T>(s, Rt, Rc, p->n[m], b.X[m], Rt, true, b.F[m], nullptr, Tp, b.W[m], Tp, nullptr, done);
}

// Core product Y and back-projection M of mode n into `out` (ld Tp).
template <typename T>
void mttkrp_into(cpd_plan_s* p, Bufs<T>& b, int n, bool fresh_core, T* out, T* out2, hipStream_t s,
                 const int32_t* done) {
  const int Rt = p->Rt, Rc = p->Rc, Tp = p->Tp;
  if (fresh_core) {
    if (n < 2) gemm_t<T>(s, Rt, Rc, Rt, b.Z, Rt, false, b.W[2], b.W[3], Tp, b.Y, Tp, nullptr, done);
    else gemm_t<T>(s, Rt, Rc, Rt, b.Z, Rt, true, b.W[0], b.W[1], Tp, b.Y, Tp, nullptr, done);
  }
  static const int partner[4] = {1, 0, 3, 2};
  gemm_t<T>(s, p->n[n], Rc, Rt, b.X[n], Rt, false, b.W[partner[n]], b.Y, Tp, out, Tp, out2, done);
}

// Normal-equation solve of mode n, in place in Msol, then normalisation,
// Gram and projection of the new factor.
template <typename T>
void solve_mode(cpd_plan_s* p, Bufs<T>& b, int n, hipStream_t s, bool with_inner, bool fast) {
  const int Rc = p->Rc, Tp = p->Tp;
  DevState* st = p->st;
  const T* g[3];
  int q = 0;
  for (int m = 0; m < 4; ++m)
    if (m != n) g[q++] = b.G[m];
  form_normal_matrix<T>(s, b.V, Tp, Rc, g[0], g[1], g[2], st, 0);
  if (fast) {
    chol_factor_fwd<T>(s, b.V, p->nblk, b.linv, b.diagL, b.Msol, p->n[n], st);
    chol_solve_bwd<T>(s, b.V, p->nblk, b.linv, b.Msol, p->n[n], st);
  } else {
    chol_factor<T>(s, b.V, p->nblk, b.linv, b.diagL, st, 0);
    retry_prepare_launch<T>(s, st, p->d.chol_fallback, g[0], g[1], g[2], Rc, Tp);
    form_normal_matrix<T>(s, b.V, Tp, Rc, g[0], g[1], g[2], st, 1);
    chol_factor<T>(s, b.V, p->nblk, b.linv, b.diagL, st, 1);
    chol_solve_rows<T>(s, b.V, p->nblk, b.linv, b.Msol, p->n[n], st);
  }
  normalise_columns<T>(s, b.Msol, p->n[n], Rc, Tp, b.F[n], b.lam, with_inner ? b.Msave : nullptr,
                       with_inner ? p->inner_part : nullptr, st);
}

// Copies the factors and the device state to (dir = 0) or from (dir = 1)
// the sweep checkpoint.
struct CkptArgs {
  void* a[4];
  void* b[4];
  size_t bytes[4];
  DevState* st;
  DevState* st_save;
  int dir;
};
__global__ void checkpoint_kernel(CkptArgs c) {
  for (int m = 0; m < 4; ++m) {
    const uint32_t* src = (const uint32_t*)(c.dir ? c.b[m] : c.a[m]);
    uint32_t* dst = (uint32_t*)(c.dir ? c.a[m] : c.b[m]);
    const size_t words = c.bytes[m] / 4;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < words; e += (size_t)gridDim.x * 256)
      dst[e] = src[e];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (c.dir) *c.st = *c.st_save;
    else *c.st_save = *c.st;
  }
}

template <typename T>
void checkpoint(cpd_plan_s* p, Bufs<T>& b, hipStream_t s, int dir) {
  CkptArgs c;
  for (int m = 0; m < 4; ++m) {
    c.a[m] = b.F[m];
    c.b[m] = b.Fsave[m];
    c.bytes[m] = sizeof(T) * (size_t)p->n[m] * p->Tp;
  }
  c.st = p->st;
  c.st_save = p->st_save;
  c.dir = dir;
  hipLaunchKernelGGL(checkpoint_kernel, dim3(512), dim3(256), 0, s, c);
}

template <typename T>
void enqueue_sweep_typed(cpd_plan_s* p, Bufs<T>& b, hipStream_t s, bool fast) {
  const int32_t* done = &p->st->done;
  if (fast) checkpoint<T>(p, b, s, 0);
  for (int n = 0; n < 4; ++n) {
    mttkrp_into<T>(p, b, n, n == 0 || n == 2, b.Msol, n == 3 ? b.Msave : nullptr, s, done);
    solve_mode<T>(p, b, n, s, n == 3, fast);
    refresh_mode<T>(p, b, n, s, done);
  }
  const T* g[4] = {b.G[0], b.G[1], b.G[2], b.G[3]};
  fit_update<T>(s, g, b.lam, p->Rc, p->Tp, p->inner_part, p->row_part, p->fit_hist, HIST_CAP,
                p->d.tol, p->d.fit_floor, p->st);
}

__global__ void sweep_tick_kernel(DevState* st) {
  if (threadIdx.x == 0 && !st->done) st->sweeps += 1;
}

// Mixed precision: the three MTTKRP products in split BF16, everything
// else in FP64.  On fit sweeps the mode-3 MTTKRP is ALSO formed in FP64
// (from the FP64 factors) for <G, G~>: the residual is first-order
// sensitive to that inner product, which split BF16 cannot deliver.
void enqueue_sweep_mixed(cpd_plan_s* p, hipStream_t s, bool fit_sweep, bool fast) {
  Bufs<double>& b = p->b64;
  const int32_t* done = &p->st->done;
  const int Rt = p->Rt, Rc = p->Rc, Tp = p->Tp;
  if (fast) checkpoint<double>(p, b, s, 0);
  for (int n = 0; n < 4; ++n) {
    mixed_mttkrp(s, p->mx, n, n == 0 || n == 2, p->n, Rt, Rc, Tp, b.Msol, nullptr, done);
    if (n == 3 && fit_sweep) {
      for (int m = 0; m < 3; ++m)
        gemm_t<double>(s, Rt, Rc, p->n[m], b.X[m], Rt, true, b.F[m], nullptr, Tp, b.W[m], Tp, nullptr,
                       done);
      mttkrp_into<double>(p, b, 3, true, b.Msave, nullptr, s, done);
    }
    solve_mode<double>(p, b, n, s, n == 3 && fit_sweep, fast);
    gemm_t<double>(s, Rc, Rc, p->n[n], b.F[n], Tp, true, b.F[n], nullptr, Tp, b.G[n], Tp, nullptr,
                   done);
    mixed_refresh(s, p->mx, n, b.F[n], p->n, Rt, Rc, Tp, done);
  }
  if (fit_sweep) {
    const double* g[4] = {b.G[0], b.G[1], b.G[2], b.G[3]};
    fit_update<double>(s, g, b.lam, Rc, Tp, p->inner_part, p->row_part, p->fit_hist, HIST_CAP, p->d.tol,
                       p->d.fit_floor, p->st);
  } else {
    hipLaunchKernelGGL(sweep_tick_kernel, dim3(1), dim3(64), 0, s, p->st);
  }
}

void enqueue_sweep(cpd_plan_s* p, hipStream_t s, bool fit_sweep, bool fast) {
  if (p->prec == CPD_FP64) enqueue_sweep_typed<double>(p, p->b64, s, fast);
  else if (p->prec == CPD_FP32) enqueue_sweep_typed<float>(p, p->b32, s, fast);
  else enqueue_sweep_mixed(p, s, fit_sweep, fast);
}

bool is_fit_sweep(const cpd_plan_s* p, long index1) {
  return p->prec != CPD_MIXED_BF16 || p->fit_every <= 1 || index1 % p->fit_every == 0;
}

int capture(cpd_plan_s* p, bool fit_sweep, bool fast, hipGraph_t* g, hipGraphExec_t* e) {
  if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return CPD_ERR_HIP;
  enqueue_sweep(p, p->cap, fit_sweep, fast);
  if (hipStreamEndCapture(p->cap, g) != hipSuccess) return CPD_ERR_HIP;
  if (hipGraphInstantiate(e, *g, nullptr, nullptr, 0) != hipSuccess) return CPD_ERR_HIP;
  return CPD_OK;
}

__global__ void strided_to_dense_f32(const float* src, int rows, int cols, int ld, double* dst) {
  const size_t total = (size_t)rows * cols;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const size_t r = e / cols, c = e % cols;
    dst[e] = (double)src[r * ld + c];
  }
}
__global__ void dense_to_strided_f32(const double* src, int rows, int cols, int ld, float* dst) {
  const size_t total = (size_t)rows * cols;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const size_t r = e / cols, c = e % cols;
    dst[r * ld + c] = (float)src[e];
  }
}
__global__ void state_set_kernel(DevState* st, double prev_fit, int sweeps) {
  if (threadIdx.x == 0) {
    st->fit_prev = prev_fit;
    st->sweeps = sweeps;
    st->done = 0;
    st->flags = 0;
    st->chol_fail = 0;
    st->retry_active = 0;
  }
}

int grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

int copy_out(cpd_plan_s* p, const void* src_typed, int rows, int cols, double* dst, hipStream_t s) {
  if (p->prec == CPD_FP32) {
    hipLaunchKernelGGL(strided_to_dense_f32, dim3(grid_for((size_t)rows * cols)), dim3(256), 0, s,
                       (const float*)src_typed, rows, cols, p->Tp, dst);
    HIPCHK(hipGetLastError());
  } else {
    HIPCHK(hipMemcpy2DAsync(dst, sizeof(double) * cols, src_typed, sizeof(double) * p->Tp,
                            sizeof(double) * cols, rows, hipMemcpyDeviceToDevice, s));
  }
  return CPD_OK;
}

int copy_in(cpd_plan_s* p, const double* src, int rows, int cols, void* dst_typed, hipStream_t s) {
  if (p->prec == CPD_FP32) {
    hipLaunchKernelGGL(dense_to_strided_f32, dim3(grid_for((size_t)rows * cols)), dim3(256), 0, s,
                       src, rows, cols, p->Tp, (float*)dst_typed);
    HIPCHK(hipGetLastError());
  } else {
    HIPCHK(hipMemcpy2DAsync(dst_typed, sizeof(double) * p->Tp, src, sizeof(double) * cols,
                            sizeof(double) * cols, rows, hipMemcpyDeviceToDevice, s));
  }
  return CPD_OK;
}

int refresh_all(cpd_plan_s* p, hipStream_t s) {
  for (int m = 0; m < 4; ++m) {
    if (p->prec == CPD_FP64) refresh_mode<double>(p, p->b64, m, s, nullptr);
    else if (p->prec == CPD_FP32) refresh_mode<float>(p, p->b32, m, s, nullptr);
    else {
      gemm_t<double>(s, p->Rc, p->Rc, p->n[m], p->b64.F[m], p->Tp, true, p->b64.F[m], nullptr,
                     p->Tp, p->b64.G[m], p->Tp, nullptr, nullptr);
      mixed_refresh(s, p->mx, m, p->b64.F[m], p->n, p->Rt, p->Rc, p->Tp, nullptr);
    }
  }
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

int read_state(cpd_plan_s* p) {
  HIPCHK(hipMemcpyAsync(p->host_state, p->st, sizeof(DevState), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return CPD_OK;
}

int status_from_flags(int flags) {
  if (flags & FLAG_NOT_SPD) return CPD_ERR_NOT_SPD;
  if (flags & FLAG_NONFINITE) return CPD_ERR_NONFINITE;
  return CPD_OK;
}

int launch_sweep(cpd_plan_s* p, bool fit, bool fast) {
  if (p->have_graph) {
    HIPCHK(hipGraphLaunch(p->exec[fast ? 1 : 0][fit ? 1 : 0], p->stream));
  } else {
    enqueue_sweep(p, p->stream, fit, fast);
    HIPCHK(hipGetLastError());
  }
  return CPD_OK;
}

// Rewinds to the checkpoint taken at the start of the last fast sweep and
// recomputes the projections / Grams from the restored factors.
int rewind_sweep(cpd_plan_s* p) {
  if (p->prec == CPD_FP32) checkpoint<float>(p, p->b32, p->stream, 1);
  else checkpoint<double>(p, p->b64, p->stream, 1);
  HIPCHK(hipGetLastError());
  return refresh_all(p, p->stream);
}

}  // namespace

extern "C" {

size_t cpd_workspace_size(const cpd_desc* d) {
  if (check_desc(d) != CPD_OK) return 0;
  cpd_plan_s tmp;
  memset(&tmp, 0, sizeof(tmp));
  fill_shape(&tmp, d);
  return carve(&tmp, nullptr);
}

cpd_status cpd_init(const cpd_desc* d, cpd_plan* out) {
  if (!out) return CPD_ERR_INVALID_ARG;
  *out = nullptr;
  int rc = check_desc(d);
  if (rc != CPD_OK) return rc;
  cpd_plan_s* p = new (std::nothrow) cpd_plan_s;
  if (!p) return CPD_ERR_INVALID_ARG;
  memset(p, 0, sizeof(*p));
  fill_shape(p, d);
  const size_t need = carve(p, nullptr);
  if (!d->workspace || d->workspace_bytes < need) {
    delete p;
    return CPD_ERR_WORKSPACE;
  }
  carve(p, (char*)d->workspace);
  p->stream = (hipStream_t)d->stream;
  if (hipHostMalloc((void**)&p->host_state, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
    delete p;
    return CPD_ERR_HIP;
  }
  if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
    (void)hipHostFree(p->host_state);
    delete p;
    return CPD_ERR_HIP;
  }
  hipStream_t s = p->stream;
  fill_bytes(s, d->workspace, need);
  rc = setup_norm2(p, s);
  if (rc == CPD_OK) {
    if (p->prec == CPD_FP32) {
      for (int m = 0; m < 4; ++m) {
        bool first = true;
        for (int q = 0; q < m; ++q)
          if (d->X[q] == d->X[m]) first = false;
        if (first) cast_f64_to_f32(s, d->X[m], (float*)p->b32.X[m], (size_t)p->n[m] * p->Rt);
      }
      cast_f64_to_f32(s, d->Z, (float*)p->b32.Z, (size_t)p->Rt * p->Rt);
      for (int m = 0; m < 4; ++m) {
        copy_normalised_init(s, d->init[m], p->n[m], p->Rc, p->Tp, p->scratch64);
        cast_f64_to_f32(s, p->scratch64, p->b32.F[m], (size_t)p->n[m] * p->Tp);
      }
    } else {
      if (p->prec == CPD_MIXED_BF16) mixed_setup_inputs(s, p->mx, d->X, d->Z, p->n, p->Rt);
      for (int m = 0; m < 4; ++m)
        copy_normalised_init(s, d->init[m], p->n[m], p->Rc, p->Tp, p->b64.F[m]);
    }
    rc = refresh_all(p, s);
  }
  if (rc == CPD_OK) {
    state_reset(s, p->st, p->norm2);
    if (hipGetLastError() != hipSuccess) rc = CPD_ERR_HIP;
  }
  if (rc == CPD_OK && d->use_graph) {
    const bool nofit = p->prec == CPD_MIXED_BF16 && p->fit_every > 1;
    for (int fast = 0; fast < 2 && rc == CPD_OK; ++fast)
      for (int fit = nofit ? 0 : 1; fit < 2 && rc == CPD_OK; ++fit)
        rc = capture(p, fit == 1, fast == 1, &p->graph[fast][fit], &p->exec[fast][fit]);
    if (rc == CPD_OK) p->have_graph = true;
  }
  if (rc != CPD_OK) {
    cpd_destroy(p);
    return rc;
  }
  *out = p;
  return CPD_OK;
}


cpd_status cpd_sweep(cpd_plan p, int32_t nsweeps, double* fits_host, int32_t* n_run) {
  if (!p || nsweeps < 0) return CPD_ERR_INVALID_ARG;
  const bool sync = fits_host || n_run;
  int ran = 0;
  if (sync) {
    int rc = read_state(p);
    if (rc != CPD_OK) return rc;
    if (p->host_state->done) {
      if (n_run) *n_run = 0;
      return status_from_flags(p->host_state->flags);
    }
  }
  for (int i = 0; i < nsweeps; ++i) {
    const bool fit = is_fit_sweep(p, p->launched + 1);
    int rc;
    if (!sync) {
      // asynchronous: the damped retry must live inside the graph
      rc = launch_sweep(p, fit, false);
      if (rc != CPD_OK) return rc;
      p->launched += 1;
      ++ran;
      continue;
    }
    rc = launch_sweep(p, fit, true);
    if (rc == CPD_OK) rc = read_state(p);
    if (rc != CPD_OK) return rc;
    if (p->host_state->chol_fail) {
      // a pivot failed: replay this sweep with the damped-retry graph
      rc = rewind_sweep(p);
      if (rc == CPD_OK) rc = launch_sweep(p, fit, false);
      if (rc == CPD_OK) rc = read_state(p);
      if (rc != CPD_OK) return rc;
    }
    p->launched += 1;
    ++ran;
    if (fits_host) fits_host[ran - 1] = fit ? p->host_state->fit_prev : -1.0;
    if (p->host_state->done) break;
  }
  if (n_run) *n_run = ran;
  if (sync) return status_from_flags(p->host_state->flags);
  return CPD_OK;
}

cpd_status cpd_fit(cpd_plan p, double* fit_host) {
  if (!p || !fit_host) return CPD_ERR_INVALID_ARG;
  int rc = read_state(p);
  if (rc != CPD_OK) return rc;
  *fit_host = p->host_state->sweeps > 0 ? p->host_state->fit_prev : -1.0;
  return status_from_flags(p->host_state->flags);
}

cpd_status cpd_get_factors(cpd_plan p, double* const F_dev[4], double* lambda_dev) {
  if (!p) return CPD_ERR_INVALID_ARG;
  hipStream_t s = p->stream;
  for (int m = 0; m < 4; ++m) {
    if (!F_dev || !F_dev[m]) continue;
    const void* src = p->prec == CPD_FP32 ? (const void*)p->b32.F[m] : (const void*)p->b64.F[m];
    int rc = copy_out(p, src, p->n[m], p->Rc, F_dev[m], s);
    if (rc != CPD_OK) return rc;
  }
  if (lambda_dev) {
    const void* src = p->prec == CPD_FP32 ? (const void*)p->b32.lam : (const void*)p->b64.lam;
    int rc = copy_out(p, src, 1, p->Rc, lambda_dev, s);
    if (rc != CPD_OK) return rc;
  }
  return CPD_OK;
}

cpd_status cpd_set_factors(cpd_plan p, const double* const F_dev[4], const double* lambda_dev,
                           double prev_fit, int32_t sweeps) {
  if (!p || !F_dev || sweeps < 0) return CPD_ERR_INVALID_ARG;
  for (int m = 0; m < 4; ++m)
    if (!F_dev[m]) return CPD_ERR_INVALID_ARG;
  hipStream_t s = p->stream;
  for (int m = 0; m < 4; ++m) {
    void* dst = p->prec == CPD_FP32 ? (void*)p->b32.F[m] : (void*)p->b64.F[m];
    int rc = copy_in(p, F_dev[m], p->n[m], p->Rc, dst, s);
    if (rc != CPD_OK) return rc;
  }
  if (lambda_dev) {
    void* dst = p->prec == CPD_FP32 ? (void*)p->b32.lam : (void*)p->b64.lam;
    int rc = copy_in(p, lambda_dev, 1, p->Rc, dst, s);
    if (rc != CPD_OK) return rc;
  }
  int rc = refresh_all(p, s);
  if (rc != CPD_OK) return rc;
  hipLaunchKernelGGL(state_set_kernel, dim3(1), dim3(64), 0, s, p->st, prev_fit, (int)sweeps);
  HIPCHK(hipGetLastError());
  p->launched = sweeps;
  return CPD_OK;
}

cpd_status cpd_stats(cpd_plan p, cpd_stats_t* out) {
  if (!p || !out) return CPD_ERR_INVALID_ARG;
  int rc = read_state(p);
  if (rc != CPD_OK) return rc;
  const DevState& h = *p->host_state;
  out->sweeps = h.sweeps;
  out->converged = h.done;
  out->fallbacks = h.fallbacks;
  out->flags = h.flags;
  out->fit = h.sweeps > 0 ? h.fit_prev : -1.0;
  out->norm2 = h.norm2;
  out->inner = h.inner;
  out->model2 = h.model2;
  std::vector<double> dg(p->Rc);
  if (p->prec == CPD_FP32) {
    std::vector<float> df(p->Rc);
    HIPCHK(hipMemcpy(df.data(), p->b32.diagL, sizeof(float) * p->Rc, hipMemcpyDeviceToHost));
    for (int i = 0; i < p->Rc; ++i) dg[i] = df[i];
  } else {
    HIPCHK(hipMemcpy(dg.data(), p->b64.diagL, sizeof(double) * p->Rc, hipMemcpyDeviceToHost));
  }
  double lo = INFINITY, hi = 0.0;
  for (int i = 0; i < p->Rc; ++i) {
    const double v = fabs(dg[i]);
    if (v < lo) lo = v;
    if (v > hi) hi = v;
  }
  out->cond_est = (lo > 0.0 && h.sweeps > 0) ? (hi / lo) * (hi / lo) : -1.0;
  return CPD_OK;
}

cpd_status cpd_mttkrp(cpd_plan p, int32_t mode, double* M_dev) {
  if (!p || mode < 0 || mode > 3 || !M_dev) return CPD_ERR_INVALID_ARG;
  hipStream_t s = p->stream;
  if (p->prec == CPD_FP64) {
    mttkrp_into<double>(p, p->b64, mode, true, p->b64.Msol, nullptr, s, nullptr);
    return copy_out(p, p->b64.Msol, p->n[mode], p->Rc, M_dev, s);
  } else if (p->prec == CPD_FP32) {
    mttkrp_into<float>(p, p->b32, mode, true, p->b32.Msol, nullptr, s, nullptr);
    return copy_out(p, p->b32.Msol, p->n[mode], p->Rc, M_dev, s);
  }
  mixed_mttkrp(s, p->mx, mode, true, p->n, p->Rt, p->Rc, p->Tp, p->b64.Msol, nullptr, nullptr);
  return copy_out(p, p->b64.Msol, p->n[mode], p->Rc, M_dev, s);
}

cpd_status cpd_destroy(cpd_plan p) {
  if (!p) return CPD_ERR_INVALID_ARG;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      if (p->exec[a][b]) (void)hipGraphExecDestroy(p->exec[a][b]);
      if (p->graph[a][b]) (void)hipGraphDestroy(p->graph[a][b]);
    }
  if (p->cap) (void)hipStreamDestroy(p->cap);
  if (p->host_state) (void)hipHostFree(p->host_state);
  delete p;
  return CPD_OK;
}

cpd_status cpd_kernel_times(cpd_plan p, int32_t reps, double* ms_out) {
  if (!p || reps <= 0 || !ms_out) return CPD_ERR_INVALID_ARG;
  hipStream_t s = p->stream;
  hipLaunchKernelGGL(state_set_kernel, dim3(1), dim3(64), 0, s, p->st, -1.0, 0);
  HIPCHK(hipGetLastError());
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int Rt = p->Rt, Rc = p->Rc, Tp = p->Tp, n0 = p->n[0];
  const bool f32 = p->prec == CPD_FP32;
  for (int which = 0; which < 7; ++which) {
    auto body = [&]() {
      if (which == 4 || which == 5 || which == 6) {
        // normal-equation solve of mode 0: V, factorisation fused with the
        // forward solve, backward solve, normalisation
        if (f32) {
          Bufs<float>& b = p->b32;
          if (which != 6) form_normal_matrix<float>(s, b.V, Tp, Rc, b.G[1], b.G[2], b.G[3], p->st, 0);
          if (which != 6) chol_factor_fwd<float>(s, b.V, p->nblk, b.linv, b.diagL, b.Msol, n0, p->st);
          if (which != 5) chol_solve_bwd<float>(s, b.V, p->nblk, b.linv, b.Msol, n0, p->st);
          if (which == 4) normalise_columns<float>(s, b.Msol, n0, Rc, Tp, b.F[0], b.lam, nullptr, nullptr, p->st);
        } else {
          Bufs<double>& b = p->b64;
          if (which != 6) form_normal_matrix<double>(s, b.V, Tp, Rc, b.G[1], b.G[2], b.G[3], p->st, 0);
          if (which != 6) chol_factor_fwd<double>(s, b.V, p->nblk, b.linv, b.diagL, b.Msol, n0, p->st);
          if (which != 5) chol_solve_bwd<double>(s, b.V, p->nblk, b.linv, b.Msol, n0, p->st);
          if (which == 4) normalise_columns<double>(s, b.Msol, n0, Rc, Tp, b.F[0], b.lam, nullptr, nullptr, p->st);
        }
        return;
      }
      if (p->prec == CPD_MIXED_BF16) {
        Bufs<double>& b = p->b64;
        if (which == 0) mixed_refresh(s, p->mx, 0, b.F[0], p->n, Rt, Rc, Tp, nullptr);
        else if (which == 1 || which == 2) {
          // core product only (which == 1), or back-projection only (2)
          if (which == 1) mixed_mttkrp(s, p->mx, 0, true, p->n, Rt, Rc, Tp, b.Msol, nullptr, nullptr);
          else mixed_mttkrp(s, p->mx, 0, false, p->n, Rt, Rc, Tp, b.Msol, nullptr, nullptr);
        } else {
          gemm_t<double>(s, Rc, Rc, n0, b.F[0], Tp, true, b.F[0], nullptr, Tp, b.G[0], Tp, nullptr, nullptr);
        }
      } else if (p->prec == CPD_FP64) {
        Bufs<double>& b = p->b64;
        if (which == 0) gemm_t<double>(s, Rt, Rc, n0, b.X[0], Rt, true, b.F[0], nullptr, Tp, b.W[0], Tp, nullptr, nullptr);
        else if (which == 1) gemm_t<double>(s, Rt, Rc, Rt, b.Z, Rt, false, b.W[2], b.W[3], Tp, b.Y, Tp, nullptr, nullptr);
        else if (which == 2) gemm_t<double>(s, n0, Rc, Rt, b.X[0], Rt, false, b.W[1], b.Y, Tp, b.Msol, Tp, nullptr, nullptr);
        else gemm_t<double>(s, Rc, Rc, n0, b.F[0], Tp, true, b.F[0], nullptr, Tp, b.G[0], Tp, nullptr, nullptr);
      } else {
        Bufs<float>& b = p->b32;
        if (which == 0) gemm_t<float>(s, Rt, Rc, n0, b.X[0], Rt, true, b.F[0], nullptr, Tp, b.W[0], Tp, nullptr, nullptr);
        else if (which == 1) gemm_t<float>(s, Rt, Rc, Rt, b.Z, Rt, false, b.W[2], b.W[3], Tp, b.Y, Tp, nullptr, nullptr);
        else if (which == 2) gemm_t<float>(s, n0, Rc, Rt, b.X[0], Rt, false, b.W[1], b.Y, Tp, b.Msol, Tp, nullptr, nullptr);
        else gemm_t<float>(s, Rc, Rc, n0, b.F[0], Tp, true, b.F[0], nullptr, Tp, b.G[0], Tp, nullptr, nullptr);
      }
    };
    body();  // warm-up
    HIPCHK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) body();
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    ms_out[which] = (double)ms / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return CPD_OK;
}

const char* cpd_status_string(cpd_status s) {
  switch (s) {
    case CPD_OK: return "ok";
    case CPD_ERR_INVALID_ARG: return "invalid argument";
    case CPD_ERR_HIP: return "HIP runtime error";
    case CPD_ERR_NOT_SPD: return "normal matrix not positive definite";
    case CPD_ERR_NONFINITE: return "non-finite value in the fit";
    case CPD_ERR_WORKSPACE: return "workspace missing or too small";
    case CPD_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
  }
}

}  // extern "C"
