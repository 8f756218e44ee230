// Internal launchers shared by the translation units of libthccp.so.
// Not part of the public C-ABI (include/thccp.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace thccp {

// ---------------------------------------------------------------- GEMM (FP64)
// C[M x N] = alpha * op(A)[M x K] * op(B)[K x N] + beta * C, row-major C.
//   a_t = false: A[i*lda + k];  a_t = true: A[k*lda + i]   (A stored K x M)
//   b_t = false: B[k*ldb + j];  b_t = true: B[j*ldb + k]   (B stored N x K)
//   B2 != nullptr: every B element is B1[.] * B2[.] (Hadamard product fused
//   into the operand load; same layout and leading dimension).
//   C2 != nullptr: the result is also written to C2 (same ldc).
//   done != nullptr: the launch is a no-op once *done is set.
struct GemmF64 {
  int M, N, K;
  const double* A; int lda; bool a_t;
  const double* B1; const double* B2; int ldb; bool b_t;
  double* C; int ldc; double* C2;
  double alpha, beta;
  const int32_t* done;
};
void gemm_f64(hipStream_t s, const GemmF64& g);

// ---------------------------------------------------------------- GEMM (FP32)
struct GemmF32 {
  int M, N, K;
  const float* A; int lda; bool a_t;
  const float* B1; const float* B2; int ldb; bool b_t;
  float* C; int ldc; float* C2;
  float alpha, beta;
  const int32_t* done;
};
void gemm_f32(hipStream_t s, const GemmF32& g);

// ------------------------------------------------------ split-BF16 GEMM (mixed)
// Operands are pre-split pairs hi = bf16(x), lo = bf16(x - hi) stored in
// MFMA-ready k-packed layouts; see mixed.hip.
struct GemmSplit;
void gemm_split(hipStream_t s, const GemmSplit& g);

// -------------------------------------------------- Cholesky / triangular solve
// V: Tp x Tp row-major (Tp = 64 * nblk), lower triangle factorised in place
// (off-diagonal blocks); the diagonal blocks of L go to ldiag (nblk blocks
// of 64 x 64, row-major), the diagonal of L to diagL (Tp).
template <typename T>
void chol_factor(hipStream_t s, T* V, int nblk, T* ldiag, T* diagL, DevState* st, int retry_pass);
// Solve F V = M in place (M: n x Tp, ld Tp) given the factor above.
template <typename T>
void chol_solve_rows(hipStream_t s, const T* V, int nblk, const T* ldiag, T* M, int n, DevState* st);
// Backward half of the solve only (F L = G, in place).
template <typename T>
void chol_solve_bwd(hipStream_t s, const T* V, int nblk, const T* ldiag, T* M, int n, DevState* st);
// Factorisation fused with the forward half of the solve (G L^T = M, in
// place), no damped retry: a failed pivot leaves st->chol_fail set.
template <typename T>
void chol_factor_fwd(hipStream_t s, T* V, int nblk, T* ldiag, T* diagL, T* M, int n, DevState* st);

// ------------------------------------------------------------- element-wise
template <typename T>
void form_normal_matrix(hipStream_t s, T* V, int Tp, int R, const T* g0, const T* g1,
                        const T* g2, DevState* st, int retry_pass);
template <typename T>
void retry_prepare_launch(hipStream_t s, DevState* st, int allow_fallback, const T* g0, const T* g1,
                          const T* g2, int R, int Tp);
template <typename T>
void normalise_columns(hipStream_t s, const T* Msol, int n, int R, int ld, T* F, T* lam,
                       const T* Msave, double* inner_part, DevState* st);
template <typename T>
void fit_update(hipStream_t s, const T* const g[4], const T* lam, int R, int ld,
                const double* inner_part, double* scratch, double* fit_hist, int hist_cap,
                double tol, double fit_floor, DevState* st);
void hadamard_inplace_f64(hipStream_t s, double* A, const double* B, size_t count);
void transposed_dot_f64(hipStream_t s, const double* P, const double* Q, int R, int ld,
                        double* partials, double* out);
void fill_bytes(hipStream_t s, void* p, size_t bytes);
void state_reset(hipStream_t s, DevState* st, double* norm2_src);
void cast_f64_to_f32(hipStream_t s, const double* a, float* b, size_t count);
void cast_f32_to_f64(hipStream_t s, const float* a, double* b, size_t count);
void copy_normalised_init(hipStream_t s, const double* src, int n, int R, int ld, double* dst);

}  // namespace thccp
