// Split-BF16 operands and launchers of the mixed-precision MTTKRP.
//
// Every operand x of the three MTTKRP contractions is represented as
// x ~ hi + lo with hi = bf16(x) and lo = bf16(x - hi) (round to nearest
// even), and a product is formed as hi*hi + hi*lo + lo*hi on the BF16
// matrix cores with FP32 accumulation (the lo*lo term is dropped).  All
// operands are stored K-contiguous ("A: M x K, B: N x K") so that one lane
// fetches its 8-element fragment with a single 16-byte read.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace thccp {

struct MixedBufs {
  int Rtp;             // R_thc rounded up to 32 (contraction length of Z and X products)
  int npad[4];         // n_m rounded up to 32
  int npad_max;
  __bf16 *Xh[4], *Xl[4];    // n_m x Rtp
  __bf16 *XTh[4], *XTl[4];  // R_thc x npad_m
  __bf16 *Zh, *Zl;          // R_thc x Rtp   (Z)
  __bf16 *ZTh, *ZTl;        // R_thc x Rtp   (Z^T)
  float* WT[4];             // R_cp x Rtp    (W_m^T, FP32)
  float* YT;                // R_cp x Rtp    (Y^T, FP32)
  __bf16 *FTh, *FTl;        // R_cp x npad_max (current factor, transposed, split)
};

// Workspace carving (base == nullptr: sizing only).  `off` is advanced.
void mixed_carve(char* base, size_t* off, MixedBufs& mx, const int n[4], int Rt, int Rc,
                 const double* const X[4]);
// One-time split of X, X^T, Z, Z^T.
void mixed_setup_inputs(hipStream_t s, MixedBufs& mx, const double* const X[4], const double* Z,
                        const int n[4], int Rt);
// W_m^T = (split F_m)^T-product with X_m, from the FP64 factor F (n_m x Tp).
void mixed_refresh(hipStream_t s, MixedBufs& mx, int m, const double* F, const int n[4], int Rt, int Rc,
                   int Tp, const int32_t* done);
// Mode-n MTTKRP: (optionally) the core product, then the back-projection
// written in FP64 to out (n_n x Tp) and out2 (if non-null).
void mixed_mttkrp(hipStream_t s, MixedBufs& mx, int n, bool fresh_core, const int nd[4], int Rt, int Rc,
                  int Tp, double* out, double* out2, const int32_t* done);

// Raw launcher, exposed for the GEMM unit test entry point.
struct SplitOperand {
  const __bf16* hi;  // pre-split pair, or
  const __bf16* lo;
  const float* p;    // FP32 pair whose element-wise product is split on the fly
  const float* q;
  int ld;
};
void gemm_split_launch(hipStream_t s, int M, int N, int K, const SplitOperand& A, const SplitOperand& B,
                       float* C32, double* C64, double* C64b, int ldc, const int32_t* done);
void split_rows_f64(hipStream_t s, const double* src, int rows, int cols, int lds, __bf16* hi, __bf16* lo,
                    int ldd, int dcols);
void split_transpose_f64(hipStream_t s, const double* src, int rows, int cols, int lds, __bf16* hi,
                         __bf16* lo, int ldd, int dcols);

}  // namespace thccp
