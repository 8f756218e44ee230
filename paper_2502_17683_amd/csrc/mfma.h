// MFMA wrappers and 64x64 tile helpers (gfx950, wave64).
//
// Register layouts of the 16x16x4 FP64 / FP32 matrix instructions on
// gfx950 (checked with the lane-layout probe hook):
//   A operand (16 x 4):  lane l holds A[l % 16][l / 16]
//   B operand (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16), FP32:   lane l, element r holds D[4 * (l / 16) + r][l % 16]
//   D (16 x 16), FP64:   lane l, element r holds D[l / 16 + 4 * r][l % 16]
#pragma once
#include "common.h"

namespace thccp {

template <typename T> struct Acc4;
template <> struct Acc4<double> { typedef d4_t type; };
template <> struct Acc4<float> { typedef f4_t type; };

__device__ __forceinline__ d4_t mfma4(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma4(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// 64x64 tiles held in LDS in "k-major" form: X[kk * LDT + idx].  The odd
// row stride puts the 16 / 32 lanes of a column-wise (transposed) store in
// distinct banks; row-wise fragment reads are consecutive either way.
constexpr int TB = 64;
constexpr int LDT = TB + 1;

// acc (wave w owns rows 16w..16w+15 and all 64 columns, 4 MFMA tiles)
//   += A(64 x 64) * B(64 x 64), A given as Ak[kk][row], B as Bk[kk][col].
template <typename T>
__device__ __forceinline__ void tile_mma64(typename Acc4<T>::type acc[4], const T* Ak,
                                           const T* Bk, int lane, int w) {
#pragma unroll 4
  for (int kk = 0; kk < TB; kk += 4) {
    const int k = kk + (lane >> 4);
    T a = Ak[k * LDT + 16 * w + (lane & 15)];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
      T b = Bk[k * LDT + 16 * tj + (lane & 15)];
      acc[tj] = mfma4(a, b, acc[tj]);
    }
  }
}

// Row, within a 16 x 16 result tile, of result element r of lane l.
template <typename T> __device__ __forceinline__ int dsub_row(int lane, int r);
template <> __device__ __forceinline__ int dsub_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }
template <> __device__ __forceinline__ int dsub_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }

// Row/column of element r of MFMA tile tj in the wave-w layout above.
template <typename T>
__device__ __forceinline__ int acc_row(int lane, int w, int r) { return 16 * w + dsub_row<T>(lane, r); }
__device__ __forceinline__ int acc_col(int lane, int tj) { return 16 * tj + (lane & 15); }

// Load a 64x64 row-major global block (rows beyond nrows read as 0) into
// LDS, either transposed (dst[c][r] = src[r][c]) or as is (dst[r][c]).
template <typename T, bool TRANSPOSE>
__device__ __forceinline__ void block_to_lds(T* dst, const T* src, size_t ld, int nrows, int tid) {
#pragma unroll 4
  for (int e = tid; e < TB * TB; e += 256) {
    const int r = e >> 6, c = e & 63;
    T v = (r < nrows) ? src[(size_t)r * ld + c] : T(0);
    if (TRANSPOSE) dst[c * LDT + r] = v;
    else dst[r * LDT + c] = v;
  }
}

}  // namespace thccp
