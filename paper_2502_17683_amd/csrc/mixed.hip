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

struct SplitArgs {
  int M, N, K;
  SplitOperand A, B;
  float* C32;
  double* C64;
  double* C64b;
  int ldc;
  const int32_t* done;
};

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
__global__ __launch_bounds__(256) void gemm_split_kernel(SplitArgs a) {
  __shared__ __attribute__((aligned(16))) __bf16 Ah[SBM * SLDK];
  __shared__ __attribute__((aligned(16))) __bf16 Al[SBM * SLDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[SBN * SLDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[SBN * SLDK];
  if (a.done && *a.done) return;
  const int tiles_n = (a.N + SBN - 1) / SBN;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
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

void gemm_split_launch(hipStream_t s, int M, int N, int K, const SplitOperand& A, const SplitOperand& B,
                       float* C32, double* C64, double* C64b, int ldc, const int32_t* done) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  SplitArgs a{M, N, K, A, B, C32, C64, C64b, ldc, done};
  const int tiles = ((M + SBM - 1) / SBM) * ((N + SBN - 1) / SBN);
  const bool ap = A.p != nullptr, bp = B.p != nullptr;
  if (!ap && !bp) hipLaunchKernelGGL((gemm_split_kernel<false, false>), dim3(tiles), dim3(256), 0, s, a);
  else if (ap && !bp) hipLaunchKernelGGL((gemm_split_kernel<true, false>), dim3(tiles), dim3(256), 0, s, a);
  else if (!ap && bp) hipLaunchKernelGGL((gemm_split_kernel<false, true>), dim3(tiles), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((gemm_split_kernel<true, true>), dim3(tiles), dim3(256), 0, s, a);
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
__global__ __launch_bounds__(256) void split_transpose_kernel(const double* src, int rows, int cols, int lds,
                                                              __bf16* hi, __bf16* lo, int ldd, int dcols) {
  __shared__ double t[64][65];
  const int tr = blockIdx.y * 64, tc = blockIdx.x * 64;  // tile origin in src (rows, cols)
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

// ------------------------------------------------------------ plan hooks
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

void mixed_carve(char* base, size_t* off, MixedBufs& mx, const int n[4], int Rt, int Rc,
                 const double* const X[4]) {
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? (void*)(base + *off) : nullptr;
    *off = al256(*off + bytes);
    return p;
  };
  mx.Rtp = (Rt + 31) / 32 * 32;
  mx.npad_max = 0;
  for (int m = 0; m < 4; ++m) {
    mx.npad[m] = (n[m] + 31) / 32 * 32;
    if (mx.npad[m] > mx.npad_max) mx.npad_max = mx.npad[m];
  }
  for (int m = 0; m < 4; ++m) {
    int alias = -1;
    for (int q = 0; q < m; ++q)
      if (X[q] == X[m]) alias = q;
    if (alias >= 0) {
      mx.Xh[m] = mx.Xh[alias]; mx.Xl[m] = mx.Xl[alias];
      mx.XTh[m] = mx.XTh[alias]; mx.XTl[m] = mx.XTl[alias];
      continue;
    }
    mx.Xh[m] = (__bf16*)take(2 * (size_t)n[m] * mx.Rtp);
    mx.Xl[m] = (__bf16*)take(2 * (size_t)n[m] * mx.Rtp);
    mx.XTh[m] = (__bf16*)take(2 * (size_t)Rt * mx.npad[m]);
    mx.XTl[m] = (__bf16*)take(2 * (size_t)Rt * mx.npad[m]);
  }
  mx.Zh = (__bf16*)take(2 * (size_t)Rt * mx.Rtp);
  mx.Zl = (__bf16*)take(2 * (size_t)Rt * mx.Rtp);
  mx.ZTh = (__bf16*)take(2 * (size_t)Rt * mx.Rtp);
  mx.ZTl = (__bf16*)take(2 * (size_t)Rt * mx.Rtp);
  for (int m = 0; m < 4; ++m) mx.WT[m] = (float*)take(4 * (size_t)Rc * mx.Rtp);
  mx.YT = (float*)take(4 * (size_t)Rc * mx.Rtp);
  mx.FTh = (__bf16*)take(2 * (size_t)Rc * mx.npad_max);
  mx.FTl = (__bf16*)take(2 * (size_t)Rc * mx.npad_max);
}

void mixed_setup_inputs(hipStream_t s, MixedBufs& mx, const double* const X[4], const double* Z,
                        const int n[4], int Rt) {
  for (int m = 0; m < 4; ++m) {
    bool first = true;
    for (int q = 0; q < m; ++q)
      if (X[q] == X[m]) first = false;
    if (!first) continue;
    split_rows_f64(s, X[m], n[m], Rt, Rt, mx.Xh[m], mx.Xl[m], mx.Rtp, mx.Rtp);
    split_transpose_f64(s, X[m], n[m], Rt, Rt, mx.XTh[m], mx.XTl[m], mx.npad[m], mx.npad[m]);
  }
  split_rows_f64(s, Z, Rt, Rt, Rt, mx.Zh, mx.Zl, mx.Rtp, mx.Rtp);
  split_transpose_f64(s, Z, Rt, Rt, Rt, mx.ZTh, mx.ZTl, mx.Rtp, mx.Rtp);
}

void mixed_refresh(hipStream_t s, MixedBufs& mx, int m, const double* F, const int n[4], int Rt, int Rc,
                   int Tp, const int32_t* done) {
  split_transpose_f64(s, F, n[m], Rc, Tp, mx.FTh, mx.FTl, mx.npad_max, mx.npad[m]);
  SplitOperand A{mx.FTh, mx.FTl, nullptr, nullptr, mx.npad_max};
  SplitOperand B{mx.XTh[m], mx.XTl[m], nullptr, nullptr, mx.npad[m]};
  gemm_split_launch(s, Rc, Rt, mx.npad[m], A, B, mx.WT[m], nullptr, nullptr, mx.Rtp, done);
}

void mixed_mttkrp(hipStream_t s, MixedBufs& mx, int n, bool fresh_core, const int nd[4], int Rt, int Rc,
                  int Tp, double* out, double* out2, const int32_t* done) {
  if (fresh_core) {
    const int a = n < 2 ? 2 : 0, b = n < 2 ? 3 : 1;
    SplitOperand A{nullptr, nullptr, mx.WT[a], mx.WT[b], mx.Rtp};
    SplitOperand B = n < 2 ? SplitOperand{mx.Zh, mx.Zl, nullptr, nullptr, mx.Rtp}
                           : SplitOperand{mx.ZTh, mx.ZTl, nullptr, nullptr, mx.Rtp};
    gemm_split_launch(s, Rc, Rt, mx.Rtp, A, B, mx.YT, nullptr, nullptr, mx.Rtp, done);
  }
  static const int partner[4] = {1, 0, 3, 2};
  SplitOperand A{mx.Xh[n], mx.Xl[n], nullptr, nullptr, mx.Rtp};
  SplitOperand B{nullptr, nullptr, mx.WT[partner[n]], mx.YT, mx.Rtp};
  gemm_split_launch(s, nd[n], Rc, mx.Rtp, A, B, nullptr, out, out2, Tp, done);
}

}  // namespace thccp
