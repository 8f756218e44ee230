// Mixed-precision MTTKRP GEMMs on the BF16 matrix cores of gfx950
// (v_mfma_f32_16x16x32_bf16), with one split-precision correction pass:
//
//   x = hi + lo,  hi = bf16(x),  lo = bf16(x - hi)
//   A B ~ A_hi B_hi + A_hi B_lo + A_lo B_hi        (FP32 accumulation)
//
// C[M x N] = A[M x K] B[N x K]^T with both operands K-contiguous.  An
// operand is either a pre-split (hi, lo) pair or a pair of FP32 matrices
// whose element-wise product is formed and split while it is staged in
// LDS -- this is how the Hadamard products W_a o W_b and W_p o Y enter the
// core and back-projection products without ever being stored.
//
// Tiles: 128 x 128 per 256-thread workgroup (2 x 2 waves of 64 x 64),
// k-step 32, next k-tile prefetched into registers during the MFMAs.
#include "common.h"
#include "kernels.h"
#include "mixed.h"

namespace thccp {

namespace {
constexpr int SBM = 128, SBN = 128, SBK = 32, SLDK = SBK + 8;

__device__ __forceinline__ void split_f(float x, __bf16& h, __bf16& l) {
  h = (__bf16)x;
  l = (__bf16)(x - (float)h);
}
__device__ __forceinline__ void split_d(double x, __bf16& h, __bf16& l) {
  const float xf = (float)x;
  h = (__bf16)xf;
  l = (__bf16)(float)(x - (double)(float)h);
}

union Pack8 {
  uint4 u;
  __bf16 b[8];
};
}  // namespace


template <bool PAIR>
__device__ __forceinline__ void load_operand(const SplitOperand& op, int rows, int r0, int k0, int tid,
                                             uint4 h[2], uint4 l[2]) {
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int row = (tid + 256 * c) >> 2;
    const int kc = (tid & 3) * 8;
    const int gr = r0 + row;
    if (gr >= rows) {
      h[c] = make_uint4(0, 0, 0, 0);
      l[c] = make_uint4(0, 0, 0, 0);
      continue;
    }
    const size_t off = (size_t)gr * op.ld + k0 + kc;
    if (PAIR) {
      const float4 p0 = *(const float4*)(op.p + off);
      const float4 p1 = *(const float4*)(op.p + off + 4);
      const float4 q0 = *(const float4*)(op.q + off);
      const float4 q1 = *(const float4*)(op.q + off + 4);
      const float x[8] = {p0.x * q0.x, p0.y * q0.y, p0.z * q0.z, p0.w * q0.w,
                          p1.x * q1.x, p1.y * q1.y, p1.z * q1.z, p1.w * q1.w};
      Pack8 ph, pl;
#pragma unroll
      for (int j = 0; j < 8; ++j) split_f(x[j], ph.b[j], pl.b[j]);
      h[c] = ph.u;
      l[c] = pl.u;
    } else {
      h[c] = *(const uint4*)(op.hi + off);
      l[c] = *(const uint4*)(op.lo + off);
    }
  }
}

template <bool APAIR, bool BPAIR>
__global__ __launch_bounds__(256) void gemm_split_kernel(const SplitArgs* tab, const int* offs, int nprob) {
  __shared__ __attribute__((aligned(16))) __bf16 Ah[SBM * SLDK];
  __shared__ __attribute__((aligned(16))) __bf16 Al[SBM * SLDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[SBN * SLDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[SBN * SLDK];
  int pid = 0;
  while (pid + 1 < nprob && (int)blockIdx.x >= offs[pid + 1]) ++pid;
  const SplitArgs a = tab[pid];
  if (a.done && *a.done) return;
  if (a.gate && *a.gate != a.want) return;
  const int tiles_n = (a.N + SBN - 1) / SBN;
  const int bid = xcd_remap(blockIdx.x - offs[pid], offs[pid + 1] - offs[pid]);
  const int m0 = (bid / tiles_n) * SBM, n0 = (bid % tiles_n) * SBN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;

  uint4 rah[2], ral[2], rbh[2], rbl[2];
  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  auto store = [&]() {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int row = (tid + 256 * c) >> 2;
      const int kc = (tid & 3) * 8;
      *(uint4*)&Ah[row * SLDK + kc] = rah[c];
      *(uint4*)&Al[row * SLDK + kc] = ral[c];
      *(uint4*)&Bh[row * SLDK + kc] = rbh[c];
      *(uint4*)&Bl[row * SLDK + kc] = rbl[c];
    }
  };

  const int nk = a.K / SBK;
  load_operand<APAIR>(a.A, a.M, m0, 0, tid, rah, ral);
  load_operand<BPAIR>(a.B, a.N, n0, 0, tid, rbh, rbl);
  store();
  __syncthreads();
  const int koff = 8 * (lane >> 4);
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) {
      load_operand<APAIR>(a.A, a.M, m0, (kt + 1) * SBK, tid, rah, ral);
      load_operand<BPAIR>(a.B, a.N, n0, (kt + 1) * SBK, tid, rbh, rbl);
    }
    bf16x8_t ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = wm * 64 + i * 16 + (lane & 15);
      ah[i] = *(const bf16x8_t*)&Ah[row * SLDK + koff];
      al[i] = *(const bf16x8_t*)&Al[row * SLDK + koff];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = wn * 64 + j * 16 + (lane & 15);
      bh[j] = *(const bf16x8_t*)&Bh[col * SLDK + koff];
      bl[j] = *(const bf16x8_t*)&Bl[col * SLDK + koff];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
      }
    __syncthreads();
    if (kt + 1 < nk) {
      store();
      __syncthreads();
    }
  }

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn * 64 + j * 16 + (lane & 15);
        if (row < a.M && col < a.N) {
          const size_t off = (size_t)row * a.ldc + col;
          if (a.C32) a.C32[off] = acc[i][j][r];
          if (a.C64) a.C64[off] = (double)acc[i][j][r];
          if (a.C64b) a.C64b[off] = (double)acc[i][j][r];
        }
      }
}

int split_tile_count(int M, int N) { return ((M + SBM - 1) / SBM) * ((N + SBN - 1) / SBN); }

void gemm_split_group(hipStream_t s, const SplitArgs* tab, const int* offs, int nprob, int total_tiles,
                      bool apair, bool bpair) {
  if (total_tiles <= 0) return;
  dim3 grid(total_tiles), block(256);
  if (!apair && !bpair) hipLaunchKernelGGL((gemm_split_kernel<false, false>), grid, block, 0, s, tab, offs, nprob);
  else if (apair && !bpair) hipLaunchKernelGGL((gemm_split_kernel<true, false>), grid, block, 0, s, tab, offs, nprob);
  else if (!apair && bpair) hipLaunchKernelGGL((gemm_split_kernel<false, true>), grid, block, 0, s, tab, offs, nprob);
  else hipLaunchKernelGGL((gemm_split_kernel<true, true>), grid, block, 0, s, tab, offs, nprob);
}

// ------------------------------------------------------------- splitting
__global__ void split_rows_kernel(const double* src, int rows, int cols, int lds, __bf16* hi, __bf16* lo,
                                  int ldd, int dcols) {
  const size_t total = (size_t)rows * dcols;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const int r = (int)(e / dcols), c = (int)(e % dcols);
    const double x = c < cols ? src[(size_t)r * lds + c] : 0.0;
    __bf16 h, l;
    split_d(x, h, l);
    hi[(size_t)r * ldd + c] = h;
    lo[(size_t)r * ldd + c] = l;
  }
}

// dst[c][r] = split(src[r][c]); r < dcols (r >= rows written as 0), c < cols.
__device__ __forceinline__ void split_transpose_tile(const double* src, int rows, int cols, int lds, __bf16* hi,
                                                     __bf16* lo, int ldd, int dcols, int tr, int tc) {
  __shared__ double t[64][65];
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const int gr = tr + r, gc = tc + c;
    t[r][c] = (gr < rows && gc < cols) ? src[(size_t)gr * lds + gc] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int c = e >> 6, r = e & 63;  // consecutive threads -> consecutive r (dst columns)
    const int gr = tr + r, gc = tc + c;
    if (gc < cols && gr < dcols) {
      __bf16 h, l;
      split_d(t[r][c], h, l);
      hi[(size_t)gc * ldd + gr] = h;
      lo[(size_t)gc * ldd + gr] = l;
    }
  }
}
__global__ __launch_bounds__(256) void split_transpose_kernel(const double* src, int rows, int cols, int lds,
                                                              __bf16* hi, __bf16* lo, int ldd, int dcols) {
  split_transpose_tile(src, rows, cols, lds, hi, lo, ldd, dcols, blockIdx.y * 64, blockIdx.x * 64);
}
// Grouped: blockIdx.z selects the problem; tiles beyond a problem's extent exit.
__global__ __launch_bounds__(256) void split_transpose_group_kernel(const SplitTArgs* tab) {
  const SplitTArgs a = tab[blockIdx.z];
  if (a.done && *a.done) return;
  if (a.gate && *a.gate != 0) return;
  const int tr = blockIdx.y * 64, tc = blockIdx.x * 64;
  if (tr >= a.dcols || tc >= a.cols) return;
  split_transpose_tile(a.src, a.rows, a.cols, a.lds, a.hi, a.lo, a.ldd, a.dcols, tr, tc);
}
void split_transpose_group(hipStream_t s, const SplitTArgs* tab, int nprob, int max_cols, int max_dcols) {
  dim3 grid((max_cols + 63) / 64, (max_dcols + 63) / 64, nprob);
  hipLaunchKernelGGL(split_transpose_group_kernel, grid, dim3(256), 0, s, tab);
}

void split_rows_f64(hipStream_t s, const double* src, int rows, int cols, int lds, __bf16* hi, __bf16* lo,
                    int ldd, int dcols) {
  size_t total = (size_t)rows * dcols;
  int grid = (int)((total + 255) / 256);
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(split_rows_kernel, dim3(grid), dim3(256), 0, s, src, rows, cols, lds, hi, lo, ldd,
                     dcols);
}

void split_transpose_f64(hipStream_t s, const double* src, int rows, int cols, int lds, __bf16* hi,
                         __bf16* lo, int ldd, int dcols) {
  dim3 grid((cols + 63) / 64, (dcols + 63) / 64);
  hipLaunchKernelGGL(split_transpose_kernel, grid, dim3(256), 0, s, src, rows, cols, lds, hi, lo, ldd,
                     dcols);
}

}  // namespace thccp
