// Kernel-level entry points used by the unit tests: one GEMM, one
// normal-equation solve, one split-BF16 GEMM, each on caller memory.
#include <string.h>

#include "../../include/thccp.h"
#include "kernels.h"
#include "common.h"
#include "mixed.h"

using namespace thccp;

namespace {
size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename T>
__global__ void pad_square(const T* V, int R, int Tp, T* Vp) {
  const size_t total = (size_t)Tp * Tp;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const int i = (int)(e / Tp), j = (int)(e % Tp);
    Vp[e] = (i < R && j < R) ? V[(size_t)i * R + j] : (i == j ? T(1) : T(0));
  }
}
template <typename T>
__global__ void pad_rows(const T* M, int n, int R, int Tp, T* Mp) {
  const size_t total = (size_t)n * Tp;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const int i = (int)(e / Tp), j = (int)(e % Tp);
    Mp[e] = j < R ? M[(size_t)i * R + j] : T(0);
  }
}
template <typename T>
__global__ void unpad_rows(const T* Mp, int n, int R, int Tp, T* M) {
  const size_t total = (size_t)n * R;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const int i = (int)(e / R), j = (int)(e % R);
    M[e] = Mp[(size_t)i * Tp + j];
  }
}
__global__ void init_state(DevState* st) {
  if (threadIdx.x == 0) memset(st, 0, sizeof(DevState));
}
__global__ void to_f32_padded(const double* a, int rows, int cols, float* b, int ldb) {
  const size_t total = (size_t)rows * ldb;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const int i = (int)(e / ldb), j = (int)(e % ldb);
    b[e] = j < cols ? (float)a[(size_t)i * cols + j] : 0.f;
  }
}
int grid_of(size_t n) {
  size_t g = (n + 255) / 256;
  return (int)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

template <typename T>
size_t solve_ws(int R, int n) {
  const int nblk = (R + 63) / 64, Tp = nblk * 64;
  return al(sizeof(DevState)) + al(sizeof(T) * (size_t)Tp * Tp) + al(sizeof(T) * (size_t)nblk * 4096) +
         al(sizeof(T) * Tp) + al(sizeof(T) * (size_t)n * Tp) + al(sizeof(StepProb<T>)) + al(sizeof(int) * 3 * (nblk + 1)) +
         al(sizeof(GemmArgs<T>)) + al(sizeof(int32_t) * (size_t)((n + 63) / 64) * nblk) +
         al(sizeof(int32_t) * ((size_t)(nblk + 2) * nblk + CU_SLOTS)) + al(sizeof(T) * (size_t)nblk * 4096);
}

// One-problem run of the blocked factorisation, forward and backward solves
// (the schedules of a sweep with the damped retry left out).
template <typename T>
cpd_status solve_impl(int R, int n, const T* V, const T* M, T* F, void* ws, hipStream_t s, int32_t* failed,
                      int pw) {
  const int nblk = (R + 63) / 64, Tp = nblk * 64;
  char* b = (char*)ws;
  DevState* st = (DevState*)b; b += al(sizeof(DevState));
  T* Vp = (T*)b; b += al(sizeof(T) * (size_t)Tp * Tp);
  T* ldiag = (T*)b; b += al(sizeof(T) * (size_t)nblk * 4096);
  T* diagL = (T*)b; b += al(sizeof(T) * Tp);
  T* Mp = (T*)b; b += al(sizeof(T) * (size_t)n * Tp);
  StepProb<T>* prob = (StepProb<T>*)b; b += al(sizeof(StepProb<T>));
  int* offs = (int*)b; b += al(sizeof(int) * 3 * (nblk + 1));
  GemmArgs<T>* gtab = (GemmArgs<T>*)b; b += al(sizeof(GemmArgs<T>));
  int32_t* flow = (int32_t*)b; b += al(sizeof(int32_t) * (size_t)((n + 63) / 64) * nblk);
  int32_t* cflow = (int32_t*)b; b += al(sizeof(int32_t) * ((size_t)(nblk + 2) * nblk + CU_SLOTS));
  T* dpart = (T*)b;
  hipLaunchKernelGGL(init_state, dim3(1), dim3(64), 0, s, st);
  hipLaunchKernelGGL((pad_square<T>), dim3(grid_of((size_t)Tp * Tp)), dim3(256), 0, s, V, R, Tp, Vp);
  hipLaunchKernelGGL((pad_rows<T>), dim3(grid_of((size_t)n * Tp)), dim3(256), 0, s, M, n, R, Tp, Mp);
  StepProb<T> hp{Vp, ldiag, diagL, Mp, st, nblk, n, flow, cflow, dpart};
  if (hipMemcpyAsync(prob, &hp, sizeof(hp), hipMemcpyHostToDevice, s) != hipSuccess) return CPD_ERR_HIP;
  for (int sched : {SCHED_CHOL_FWD, SCHED_BWD}) {
    for (const SolveItem& it : solve_schedule(sched, nblk, pw)) {
      // tables are passed through a tiny per-launch upload (this hook is not
      // performance-critical)
      if (it.mode >= 0) {
        std::vector<int> tab = {0, step_tiles(it.mode, nblk, n, it.cfg)};
        int cnt = 1, total = tab[1];
        if (is_flow_mode(it.mode)) {
          tab = flow_segments(it.mode, {nblk}, {n});
          cnt = (int)tab.size() / 3 - 1;
          total = tab[3 * cnt];
        }
        if (hipMemcpyAsync(offs, tab.data(), sizeof(int) * tab.size(), hipMemcpyHostToDevice, s) != hipSuccess)
          return CPD_ERR_HIP;
        if (hipStreamSynchronize(s) != hipSuccess) return CPD_ERR_HIP;
        step_group<T>(s, it.mode, prob, offs, cnt, total, it.cfg, 0);
        continue;
      }
      for (int h = 0; h < 2; ++h) {
        GemmArgs<T> g;
        if (it.g_kind[h] < 0 || !panel_gemm<T>(it.g_kind[h], hp, pw, it.g_panel[h], g)) continue;
        int bm = gemm_default_tile(g.M, g.N);
        if (bm == 128 && !gemm_dma_ok(g, false)) bm = 64;
        int ho[2] = {0, gemm_tile_count(g.M, g.N, bm, g.lower)};
        if (hipMemcpyAsync(offs, ho, sizeof(ho), hipMemcpyHostToDevice, s) != hipSuccess) return CPD_ERR_HIP;
        if (hipMemcpyAsync(gtab, &g, sizeof(g), hipMemcpyHostToDevice, s) != hipSuccess) return CPD_ERR_HIP;
        if (hipStreamSynchronize(s) != hipSuccess) return CPD_ERR_HIP;
        gemm_group<T>(s, gtab, offs, 1, ho[1], false, it.g_kind[h] != PG_BWD, false, bm);
      }
    }
  }
  hipLaunchKernelGGL((unpad_rows<T>), dim3(grid_of((size_t)n * R)), dim3(256), 0, s, Mp, n, R, Tp, F);
  DevState h;
  if (hipMemcpyAsync(&h, st, sizeof(DevState), hipMemcpyDeviceToHost, s) != hipSuccess) return CPD_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return CPD_ERR_HIP;
  if (failed) *failed = h.chol_fail;
  if (h.flags & FLAG_SOLVE_STALL) return CPD_ERR_HIP;
  return h.chol_fail ? CPD_ERR_NOT_SPD : CPD_OK;
}
}  // namespace

extern "C" {

cpd_status cpd_test_gemm(int32_t fp32, int32_t M, int32_t N, int32_t K, const void* A, int32_t lda,
                         int32_t a_t, const void* B1, const void* B2, int32_t ldb, int32_t b_t, void* C,
                         int32_t ldc, void* stream) {
  if (M < 0 || N < 0 || K < 0 || !A || !B1 || !C) return CPD_ERR_INVALID_ARG;
  if (B2 && b_t) return CPD_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (fp32) {
    GemmF32 g{M, N, K, (const float*)A, lda, a_t != 0, (const float*)B1, (const float*)B2, ldb, b_t != 0,
              (float*)C, ldc, nullptr, 1.f, 0.f, nullptr};
    gemm_f32(s, g);
  } else {
    GemmF64 g{M, N, K, (const double*)A, lda, a_t != 0, (const double*)B1, (const double*)B2, ldb,
              b_t != 0, (double*)C, ldc, nullptr, 1.0, 0.0, nullptr};
    gemm_f64(s, g);
  }
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

size_t cpd_test_solve_workspace(int32_t fp32, int32_t R, int32_t n) {
  if (R <= 0 || n <= 0) return 0;
  return fp32 ? solve_ws<float>(R, n) : solve_ws<double>(R, n);
}

int32_t cpd_test_flow_spin_limit(int32_t polls) { return set_flow_spin_limit(polls); }
int32_t cpd_test_bwd_form(int32_t form) { return set_bwd_form(form); }

cpd_status cpd_test_solve(int32_t fp32, int32_t R, int32_t n, const void* V, const void* M, void* F,
                          void* workspace, size_t ws_bytes, void* stream, int32_t* failed, int32_t panel) {
  if (panel < 0) return CPD_ERR_INVALID_ARG;
  const int pw = panel > 0 ? panel : (R + 63) / 64;
  if (R <= 0 || n <= 0 || !V || !M || !F) return CPD_ERR_INVALID_ARG;
  if (!workspace || ws_bytes < cpd_test_solve_workspace(fp32, R, n)) return CPD_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (fp32) return solve_impl<float>(R, n, (const float*)V, (const float*)M, (float*)F, workspace, s, failed, pw);
  return solve_impl<double>(R, n, (const double*)V, (const double*)M, (double*)F, workspace, s, failed, pw);
}

size_t cpd_test_split_workspace(int32_t M, int32_t N, int32_t K) {
  if (M <= 0 || N <= 0 || K <= 0) return 0;
  const size_t Kp = (K + 31) / 32 * 32;
  // the hi / lo buffers hold the blocked layout's padded rows
  return 2 * al(2 * blk_elems(M, (int)Kp)) + 2 * al(2 * blk_elems(N, (int)Kp)) + 2 * al(4 * (size_t)M * Kp) +
         2 * al(4 * (size_t)N * Kp) + al(4 * (size_t)4 * M * N) + al(sizeof(SplitArgs)) + al(2 * sizeof(int));
}

// C (M x N, dense) = A B^T with A (M x K), B (N x K) dense FP64; when A2
// (B2) is non-null the A (B) operand is the FP32 element-wise product
// A o A2 (B o B2), split on the fly, as in the fused core product and
// back-projection.  bm/wide/kparts select the launch shape.
cpd_status cpd_test_gemm_split(int32_t M, int32_t N, int32_t K, const double* A, const double* A2,
                               const double* B, const double* B2, double* C, void* workspace, size_t ws_bytes,
                               void* stream, int32_t bm, int32_t wide, int32_t kparts) {
  if (M <= 0 || N <= 0 || K <= 0 || !A || !B || !C) return CPD_ERR_INVALID_ARG;
  if (wide == 2) {
    if (kparts < 1 || kparts > 4) return CPD_ERR_INVALID_ARG;
  } else if (wide) {
    if ((bm != 128 && bm != 256) || kparts < 1 || kparts > 4) return CPD_ERR_INVALID_ARG;
  } else {
    if (bm == 0) bm = split_default_bm(M, N);
    if ((bm != 64 && bm != 128) || kparts != 1) return CPD_ERR_INVALID_ARG;
  }
  if (!workspace || ws_bytes < cpd_test_split_workspace(M, N, K)) return CPD_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int Kp = (K + 31) / 32 * 32;
  char* b = (char*)workspace;
  __bf16* Ah = (__bf16*)b; b += al(2 * blk_elems(M, Kp));
  __bf16* Al = (__bf16*)b; b += al(2 * blk_elems(M, Kp));
  __bf16* Bh = (__bf16*)b; b += al(2 * blk_elems(N, Kp));
  __bf16* Bl = (__bf16*)b; b += al(2 * blk_elems(N, Kp));
  float* Ap = (float*)b; b += al(4 * (size_t)M * Kp);
  float* Aq = (float*)b; b += al(4 * (size_t)M * Kp);
  float* Bp = (float*)b; b += al(4 * (size_t)N * Kp);
  float* Bq = (float*)b; b += al(4 * (size_t)N * Kp);
  float* part = (float*)b; b += al(4 * (size_t)4 * M * N);
  SplitArgs* tab = (SplitArgs*)b; b += al(sizeof(SplitArgs));
  int* offs = (int*)b;
  auto operand = [&](const double* X, const double* X2, int rows, __bf16* h, __bf16* l, float* p, float* q) {
    if (X2) {
      hipLaunchKernelGGL(to_f32_padded, dim3(grid_of((size_t)rows * Kp)), dim3(256), 0, s, X, rows, K, p, Kp);
      hipLaunchKernelGGL(to_f32_padded, dim3(grid_of((size_t)rows * Kp)), dim3(256), 0, s, X2, rows, K, q, Kp);
      return SplitOperand{nullptr, nullptr, p, q, Kp};
    }
    split_rows_f64(s, X, rows, K, K, h, l, Kp, Kp);
    return SplitOperand{h, l, nullptr, nullptr, Kp};
  };
  SplitOperand opA = operand(A, A2, M, Ah, Al, Ap, Aq);
  SplitOperand opB = operand(B, B2, N, Bh, Bl, Bp, Bq);
  if (wide == 2) {
    // direct-load tiles take operands in the blocked split layout
    if (A2) {
      pair_split_blocked(s, Ap, Aq, Kp, M, Kp, Ah, Al, Kp);
    } else {
      split_blocked_f64(s, A, M, K, K, Ah, Al, Kp);
    }
    if (B2) {
      pair_split_blocked(s, Bp, Bq, Kp, N, Kp, Bh, Bl, Kp);
    } else {
      split_blocked_f64(s, B, N, K, K, Bh, Bl, Kp);
    }
    opA = SplitOperand{Ah, Al, nullptr, nullptr, Kp};
    opB = SplitOperand{Bh, Bl, nullptr, nullptr, Kp};
  }
  const SplitArgs ha{M, N, Kp, opA, opB, nullptr, C, nullptr, N, nullptr, nullptr, 0, part};
  const int tiles = wide == 2 ? split_dma_tile_count(M, N) * kparts
                    : wide ? split_wide_tile_count(M, N, bm) * kparts : split_tile_count(M, N, bm);
  const int ho[2] = {0, tiles};
  if (hipMemcpyAsync(tab, &ha, sizeof(ha), hipMemcpyHostToDevice, s) != hipSuccess) return CPD_ERR_HIP;
  if (hipMemcpyAsync(offs, ho, sizeof(ho), hipMemcpyHostToDevice, s) != hipSuccess) return CPD_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return CPD_ERR_HIP;  // host copies of ha/ho go out of scope
  if (wide == 2) {
    gemm_split_dma_group(s, tab, offs, 1, tiles, kparts);
    gemm_split_reduce_group(s, tab, 1, kparts, M, N);
  } else if (wide) {
    gemm_split_wide_group(s, tab, offs, 1, tiles, A2 != nullptr, B2 != nullptr, bm, kparts);
    gemm_split_reduce_group(s, tab, 1, kparts, M, N);
  } else {
    gemm_split_group(s, tab, offs, 1, tiles, A2 != nullptr, B2 != nullptr, bm);
  }
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

}  // extern "C"

// Lane-layout probe of the 16x16x4 FP64 / FP32 matrix instructions: probe
// p feeds a[p*64 + lane], b[p*64 + lane] to one wave with a zero
// accumulator and writes the 4 result registers to d[p*256 + lane*4 + r].
__global__ void mfma_probe_f64(const double* a, const double* b, double* d) {
  const int p = blockIdx.x, l = threadIdx.x;
  d4_t acc = {0, 0, 0, 0};
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p * 64 + l], b[p * 64 + l], acc, 0, 0, 0);
  for (int r = 0; r < 4; ++r) d[p * 256 + l * 4 + r] = acc[r];
}
__global__ void mfma_probe_f32(const float* a, const float* b, float* d) {
  const int p = blockIdx.x, l = threadIdx.x;
  f4_t acc = {0, 0, 0, 0};
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[p * 64 + l], b[p * 64 + l], acc, 0, 0, 0);
  for (int r = 0; r < 4; ++r) d[p * 256 + l * 4 + r] = acc[r];
}
extern "C" cpd_status cpd_test_mfma_probe(int32_t fp32, int32_t nprobe, const void* a, const void* b, void* d,
                                          void* stream) {
  if (nprobe <= 0 || !a || !b || !d) return CPD_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (fp32) hipLaunchKernelGGL(mfma_probe_f32, dim3(nprobe), dim3(64), 0, s, (const float*)a, (const float*)b, (float*)d);
  else hipLaunchKernelGGL(mfma_probe_f64, dim3(nprobe), dim3(64), 0, s, (const double*)a, (const double*)b, (double*)d);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}
