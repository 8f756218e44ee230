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

// Split-BF16 operand buffers of one problem.
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
  // blocked split layout (direct-load products)
  __bf16 *XBh[4], *XBl[4];  // n_m rows x Rtp
  __bf16 *ZBh, *ZBl;        // Z,   R_thc rows x Rtp
  __bf16 *ZTBh, *ZTBl;      // Z^T, R_thc rows x Rtp
  __bf16 *PWh, *PWl;        // pair product of the current product, R_cp rows x Rtp
  __bf16 *XTBh[4], *XTBl[4];  // X_m^T, R_thc rows x npad_m
  __bf16 *FTBh, *FTBl;      // current factor transposed, R_cp rows x npad_m (blocked, per mode)
};

// One operand: a pre-split (hi, lo) pair, or a pair of FP32 matrices whose
// element-wise product is split on the fly.  K-contiguous, row stride ld.
struct SplitOperand {
  const __bf16* hi;
  const __bf16* lo;
  const float* p;
  const float* q;
  int ld;
};
// C[M x N] = A[M x K] B[N x K]^T (K a multiple of 32), output FP32 (C32)
// and/or FP64 (C64, C64b), row stride ldc.
struct SplitArgs {
  int M, N, K;
  SplitOperand A, B;
  float* C32;
  double* C64;
  double* C64b;
  int ldc;
  const int32_t* done;
  const int32_t* gate;  // skip unless *gate == want (per-problem precision path)
  int32_t want;
  float* part;          // split-K launches: kparts x M x ldc FP32 partial products
};
// Tiles of one product with row tile bm (128, or 64 for short M or when
// the 128-row tiles would leave most compute units idle: split_default_bm).
int split_tile_count(int M, int N, int bm);
int split_default_bm(int M, int N);
// Grouped launch: all problems share (A pair?, B pair?) and the row tile bm.
void gemm_split_group(hipStream_t s, const SplitArgs* tab, const int* offs, int nprob, int total_tiles,
                      bool apair, bool bpair, int bm);

// Wide tiles: bm x 256 per workgroup (bm = 128 or 256), each of the four
// waves holding a (bm/2) x 128 accumulator block, for products large
// enough to fill the compute units with them.  With kparts > 1 the K range
// is cut into kparts slices (split-K): each workgroup writes its partial
// product to SplitArgs::part and gemm_split_reduce_group sums the slices in
// order into C (deterministic).
int split_wide_tile_count(int M, int N, int bm);
void gemm_split_wide_group(hipStream_t s, const SplitArgs* tab, const int* offs, int nprob, int total_tiles,
                           bool apair, bool bpair, int bm, int kparts);
void gemm_split_reduce_group(hipStream_t s, const SplitArgs* tab, int nprob, int kparts, int max_m, int max_n);

// Blocked split layout of an operand half (hi or lo) with rows r and
// contraction index k (K padded to Kp, a multiple of 32; rows padded to
// blk_rows, a multiple of 256, with zeros): element (r, k) at
//   ((r / 16) * (Kp / 32) + k / 32) * 512 + ((k / 8) % 4) * 128 + (r % 16) * 8 + k % 8,
// so that a 16-row x 32-k block is one contiguous kilobyte in the lane
// order of a matrix-core fragment.
__host__ __device__ inline int blk_rows(int rows) { return (rows + 255) / 256 * 256; }
inline size_t blk_elems(int rows, int Kp) { return (size_t)blk_rows(rows) * Kp; }
// hi / lo (blocked) = split of an FP64 row-major matrix (rows x cols, row
// stride lds), zero beyond it; with trans, of its transpose (src is then
// cols x rows with row stride lds).
void split_blocked_f64(hipStream_t s, const double* src, int rows, int cols, int lds, __bf16* hi, __bf16* lo,
                       int Kp, bool trans = false);
// hi / lo (blocked) = split(p o q) of two FP32 row-major matrices (rows x
// cols, row stride ld), zero beyond them.
void pair_split_blocked(hipStream_t s, const float* p, const float* q, int ld, int rows, int cols, __bf16* hi,
                        __bf16* lo, int Kp);
// One pair split of a grouped launch: hi / lo (blocked, Kp) = split(p o q)
// for FP32 p, q (rows x cols, row stride ld a multiple of 4, 16-byte
// aligned), skipped when *done or when gate is set and *gate != want.
struct PairJob {
  const float* p;
  const float* q;
  int ld, rows, cols;
  __bf16* hi;
  __bf16* lo;
  int Kp;
  const int32_t* done;
  const int32_t* gate;
  int32_t want;
};
void pair_split_group(hipStream_t s, const PairJob* jobs, int njobs, size_t max_chunks);
// Direct-load tiles: 256 x 256 per workgroup from operands in the blocked
// split layout (SplitOperand hi, lo; ld = Kp; p, q unused; K = Kp), with
// split-K as above.
int split_dma_tile_count(int M, int N);
void gemm_split_dma_group(hipStream_t s, const SplitArgs* tab, const int* offs, int nprob, int total_tiles,
                          int kparts);

// dst (cols x ldd) = split(src^T): dst[c][r] for c < cols, r < dcols
// (r >= rows written as 0).
struct SplitTArgs {
  const double* src;
  __bf16* hi;
  __bf16* lo;
  const int32_t* done;
  const int32_t* gate;
  int rows, cols, lds, ldd, dcols;
};
void split_transpose_group(hipStream_t s, const SplitTArgs* tab, int nprob, int max_cols, int max_dcols);
// The same transposes into the blocked split layout (hi / lo: cols rows,
// Kp = dcols, a multiple of 32); max_chunks = the largest
// blk_rows(cols) * dcols / 8.
void split_transpose_blocked_group(hipStream_t s, const SplitTArgs* tab, int nprob, size_t max_chunks);
void split_rows_f64(hipStream_t s, const double* src, int rows, int cols, int lds, __bf16* hi, __bf16* lo,
                    int ldd, int dcols);
void split_transpose_f64(hipStream_t s, const double* src, int rows, int cols, int lds, __bf16* hi,
                         __bf16* lo, int ldd, int dcols);

}  // namespace thccp
