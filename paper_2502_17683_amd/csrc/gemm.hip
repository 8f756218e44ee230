// Dense GEMM on the 16x16x4 FP64 / FP32 matrix cores, with the Hadamard
// product of two B operands fused into the operand load.
//
// This one kernel family carries every contraction of the matrix-free
// MTTKRP (projection X^T F, core product Z (W o W), back-projection
// X (W o Y)), the Gram matrices F^T F and the set-up products.
//
// Two forms, 256 threads = 2 x 2 waves each:
//   - register-staged (any shape, FP64 and FP32): block tile BM x BN (64 or
//     128), k-step 16 staged through LDS in k-major form, the next k-tile
//     prefetched into registers while the current one is multiplied;
//   - direct-load (FP64, qualifying shapes, gemm_dma_ok): 128 x 128 tiles
//     loaded from global memory straight into a two-stage LDS pipeline,
//     which keeps two workgroups per compute unit (below).
#include "kernels.h"
#include "mfma.h"

namespace thccp {

template <typename T, int BM, int BN, bool AT, bool BT, bool HAD>
__device__ __forceinline__ void gemm_body(const GemmArgs<T>& p, int bid_in, int nblocks) {
  constexpr int BK = 16;
  constexpr int WTM = BM / 2, WTN = BN / 2;
  constexpr int TI = WTM / 16, TJ = WTN / 16;
  constexpr int PAD = 1;  // odd row stride: the k-contiguous A stores hit distinct banks
  constexpr int AE = BM * BK / 256, BE = BN * BK / 256;
  typedef typename Acc4<T>::type acc_t;
  __shared__ T As[BK][BM + PAD];
  __shared__ T Bs[BK][BN + PAD];

  if (p.done && *p.done) return;
  if (p.gate && *p.gate != p.want) return;
  const int tiles_n = (p.N + BN - 1) / BN;
  const int bid = xcd_remap(bid_in, nblocks);
  int m0, n0;
  if (BM == BN && p.lower && p.M == p.N) {
    // only the lower tiles are launched, in row order (row r holds r + 1);
    // the XCD remap above then spreads them evenly
    int r = (int)((sqrtf(8.f * (float)bid + 1.f) - 1.f) * 0.5f);
    while ((r + 1) * (r + 2) / 2 <= bid) ++r;
    while (r * (r + 1) / 2 > bid) --r;
    m0 = r * BM;
    n0 = (bid - r * (r + 1) / 2) * BN;
  } else {
    int tm, tn;
    grouped_tile(bid, (p.M + BM - 1) / BM, tiles_n, 8, tm, tn);
    m0 = tm * BM;
    n0 = tn * BN;
    if (p.lower && n0 > m0 + BM - 1) return;  // tile strictly above the diagonal
  }
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const gptr<const T> gA = as_global(p.A), gB1 = as_global(p.B1), gB2 = as_global(p.B2);
  const gptr<T> gC = as_global(p.C), gC2 = as_global(p.C2);

  // Operand loads are unconditional: interior tiles (the whole k-tile in
  // range) load without checks; edge tiles read offset 0 for an
  // out-of-range element and zero it at the LDS store from the validity
  // bits.  The Hadamard product is also formed at the LDS store, so nothing
  // waits on the prefetch until the current k-tile's products are issued.
  T ra[AE], rb[BE], rb2[HAD ? BE : 1];
  uint32_t va = 0, vb = 0;
  const bool interior = m0 + BM <= p.M && n0 + BN <= p.N;
  auto load = [&](int k0) {
    if (interior && k0 + BK <= p.K) {
      va = vb = ~0u;
#pragma unroll
      for (int e = 0; e < AE; ++e) {
        const int idx = tid + e * 256;
        int i, k;
        if (AT) { i = idx % BM; k = idx / BM; } else { k = idx % BK; i = idx / BK; }
        ra[e] = AT ? gA[(size_t)(k0 + k) * p.lda + m0 + i] : gA[(size_t)(m0 + i) * p.lda + k0 + k];
      }
#pragma unroll
      for (int e = 0; e < BE; ++e) {
        const int idx = tid + e * 256;
        int j, k;
        if (BT) { k = idx % BK; j = idx / BK; } else { j = idx % BN; k = idx / BN; }
        const size_t off = BT ? (size_t)(n0 + j) * p.ldb + k0 + k : (size_t)(k0 + k) * p.ldb + n0 + j;
        rb[e] = gB1[off];
        if constexpr (HAD) rb2[e] = gB2[off];
      }
      return;
    }
    va = 0;
    vb = 0;
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const int idx = tid + e * 256;
      int i, k;
      if (AT) { i = idx % BM; k = idx / BM; } else { k = idx % BK; i = idx / BK; }
      const int gi = m0 + i, gk = k0 + k;
      const bool ok = gi < p.M && gk < p.K;
      const size_t off = ok ? (AT ? (size_t)gk * p.lda + gi : (size_t)gi * p.lda + gk) : 0;
      ra[e] = gA[off];
      va |= (uint32_t)ok << e;
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int idx = tid + e * 256;
      int j, k;
      if (BT) { k = idx % BK; j = idx / BK; } else { j = idx % BN; k = idx / BN; }
      const int gj = n0 + j, gk = k0 + k;
      const bool ok = gj < p.N && gk < p.K;
      const size_t off = ok ? (BT ? (size_t)gj * p.ldb + gk : (size_t)gk * p.ldb + gj) : 0;
      rb[e] = gB1[off];
      if constexpr (HAD) rb2[e] = gB2[off];
      vb |= (uint32_t)ok << e;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const int idx = tid + e * 256;
      int i, k;
      if (AT) { i = idx % BM; k = idx / BM; } else { k = idx % BK; i = idx / BK; }
      As[k][i] = (va >> e) & 1 ? ra[e] : T(0);
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int idx = tid + e * 256;
      int j, k;
      if (BT) { k = idx % BK; j = idx / BK; } else { j = idx % BN; k = idx / BN; }
      T v = rb[e];
      if constexpr (HAD) {
        // keeps the product (and the wait for both loads) here, after the
        // current k-tile's matrix-core products
        T w = rb2[e];
        asm volatile("" : "+v"(v), "+v"(w));
        v *= w;
      }
      Bs[k][j] = (vb >> e) & 1 ? v : T(0);
    }
  };

  acc_t acc[TI][TJ];
#pragma unroll
  for (int a = 0; a < TI; ++a)
#pragma unroll
    for (int b = 0; b < TJ; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  const int nk = (p.K + BK - 1) / BK;
  load(0);
  store();
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int k = kk + (lane >> 4);
      T af[TI], bf[TJ];
#pragma unroll
      for (int a = 0; a < TI; ++a) af[a] = As[k][wm * WTM + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < TJ; ++b) bf[b] = Bs[k][wn * WTN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TJ; ++b) acc[a][b] = mfma4(af[a], bf[b], acc[a][b]);
    }
    __syncthreads();
    if (kt + 1 < nk) {
      store();
      __syncthreads();
    }
  }

#pragma unroll
  for (int a = 0; a < TI; ++a)
#pragma unroll
    for (int b = 0; b < TJ; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WTM + a * 16 + dsub_row<T>(lane, r);
        const int col = n0 + wn * WTN + b * 16 + (lane & 15);
        if (row < p.M && col < p.N) {
          const size_t off = (size_t)row * p.ldc + col;
          T v = p.alpha * acc[a][b][r];
          if (p.beta != T(0)) v += p.beta * gC[off];
          gC[off] = v;
          if (p.C2) gC2[off] = v;
        }
      }
}

template <typename T, int BM, int BN, bool AT, bool BT, bool HAD>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs<T> p) {
  gemm_body<T, BM, BN, AT, BT, HAD>(p, blockIdx.x, gridDim.x);
}

// Grouped form: workgroup -> (problem, local tile) through the prefix sums.
// The FP64 64-tiles fit four workgroups per compute unit (<= 128
// registers, the accumulators in VGPRs; with a Hadamard operand a few
// values spill): the lower-triangle Gram at R = 4000 is then ~2 rounds of
// its 2016 tiles, and the back-projection's 819 tiles at n = 800 all
// resident at once.
template <typename T, int BM, int BN, bool AT, bool BT, bool HAD>
__global__ __launch_bounds__(256, (BM == 64 && sizeof(T) == 8) ? 4 : 1) void gemm_group_kernel(
    const GemmArgs<T>* tab, const int* offs, int nprob) {
  int pid = 0;
  while (pid + 1 < nprob && (int)blockIdx.x >= offs[pid + 1]) ++pid;
  const GemmArgs<T> p = tab[pid];
  gemm_body<T, BM, BN, AT, BT, HAD>(p, blockIdx.x - offs[pid], offs[pid + 1] - offs[pid]);
}

// ---------------------------------------------------------------------
// FP64 with 128 x 128 block tiles and direct global -> LDS loads
// (global_load_lds_dwordx4): no register staging, so the accumulators (64
// per lane, in AGPRs) and the fragments fit two workgroups per compute unit
// (~200 registers, 52-72 KB LDS with two stages), where the register-staged
// 128 x 128 form holds ~400 registers and one workgroup.  One barrier per
// k-step: the next k-tile is in flight while the current one is multiplied.
// LDS layouts (a wave instruction writes 64 consecutive 16-byte chunks):
//   - operand contiguous along its row index r (k-major, element (k, r) at
//     base[k ld + r]): row k of the tile, 128 doubles, at stage + k * 144
//     (the padding puts rows k and k + 1 in different banks);
//   - operand contiguous along k (element (r, k) at base[r ld + k]): k-pair
//     major, [k / 2][r][k % 2], so a fragment read of 16 consecutive r is
//     conflict-free.
// Rows or columns past the matrix edge read a clamped in-range address;
// they only feed result elements that are not stored.  Requirements (checked
// on the host, gemm_dma_ok): beta = 0, a full (not lower-triangle) result,
// K a multiple of the k-step (8 with a Hadamard operand pair, 16
// otherwise), even leading dimensions, 16-byte aligned operands.  (The
// lower-triangle Gram is faster on the 64-tiles: the 128-tiles on the
// diagonal would compute twice the needed elements.)
namespace {
constexpr int DM = 128, DROW = 144;
typedef __attribute__((address_space(3))) void* lds_vptr;
typedef const __attribute__((address_space(1))) void* glb_cvptr;
}  // namespace

template <bool KMAJOR, int BKD>
__device__ __forceinline__ void dma_operand(const double* base, int ld, int r0, int rows, int k0, double* stage,
                                            int w, int lane) {
#pragma unroll
  for (int i = 0; i < BKD / 4; ++i) {
    const int idx = w * (BKD / 4) + i;
    const double* g;
    double* dst;
    if (KMAJOR) {
      const int r = min(r0 + 2 * lane, (rows - 1) & ~1);
      g = base + (size_t)(k0 + idx) * ld + r;
      dst = stage + idx * DROW;
    } else {
      const int kp = idx >> 1, half = idx & 1;
      const int r = min(r0 + half * 64 + lane, rows - 1);
      g = base + (size_t)r * ld + k0 + 2 * kp;
      dst = stage + kp * (2 * DM) + half * 64 * 2;
    }
    __builtin_amdgcn_global_load_lds((glb_cvptr)g, (lds_vptr)dst, 16, 0, 0);
  }
}
template <bool KMAJOR>
__device__ __forceinline__ double dma_frag(const double* st, int r, int k) {
  return KMAJOR ? st[k * DROW + r] : st[(k >> 1) * (2 * DM) + r * 2 + (k & 1)];
}

template <bool AT, bool BT, bool HAD>
__device__ __forceinline__ void gemm_dma_body(const GemmArgs<double>& p, int bid_in, int nblocks) {
  constexpr int BKD = HAD ? 8 : 16;
  constexpr int OPK = BKD * DROW, OPM = (BKD / 2) * DM * 2;
  constexpr int SA = AT ? OPK : OPM, SB = BT ? OPM : OPK;
  constexpr int STAGE = SA + SB * (HAD ? 2 : 1);
  __shared__ __attribute__((aligned(16))) double lds[2 * STAGE];

  if (p.done && *p.done) return;
  if (p.gate && *p.gate != p.want) return;
  const int tiles_n = (p.N + DM - 1) / DM;
  const int bid = xcd_remap(bid_in, nblocks);
  int tm, tn;
  grouped_tile(bid, (p.M + DM - 1) / DM, tiles_n, 8, tm, tn);
  const int m0 = tm * DM, n0 = tn * DM;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  // C = (alpha A) B; beta must be 0 (gemm_dma_ok): any read of C here kept
  // the accumulators out of the AGPRs and cost the second workgroup per unit
  const gptr<double> gC = as_global(p.C), gC2 = as_global(p.C2);
  const double alpha = p.alpha;
  d4_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4_t{0, 0, 0, 0};
  auto issue = [&](int kt, int s) {
    double* st = lds + s * STAGE;
    dma_operand<AT, BKD>(p.A, p.lda, m0, p.M, kt * BKD, st, w, lane);
    dma_operand<!BT, BKD>(p.B1, p.ldb, n0, p.N, kt * BKD, st + SA, w, lane);
    if constexpr (HAD) dma_operand<!BT, BKD>(p.B2, p.ldb, n0, p.N, kt * BKD, st + SA + SB, w, lane);
  };
  const int nk = p.K / BKD;
  issue(0, 0);
  for (int kt = 0; kt < nk; ++kt) {
    // this wave's loads of k-tile kt have landed; the barrier makes every
    // wave's visible and ends all reads of the other stage
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (kt + 1 < nk) issue(kt + 1, (kt + 1) & 1);
    const double* st = lds + (kt & 1) * STAGE;
#pragma unroll
    for (int kk = 0; kk < BKD; kk += 4) {
      const int k = kk + (lane >> 4);
      double af[4], bf[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) af[a] = alpha * dma_frag<AT>(st, wm * 64 + a * 16 + (lane & 15), k);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int c = wn * 64 + b * 16 + (lane & 15);
        bf[b] = dma_frag<!BT>(st + SA, c, k);
        if constexpr (HAD) bf[b] *= dma_frag<!BT>(st + SA + SB, c, k);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma4(af[a], bf[b], acc[a][b]);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 64 + a * 16 + dsub_row<double>(lane, r);
        const int col = n0 + wn * 64 + b * 16 + (lane & 15);
        if (row < p.M && col < p.N) {
          const size_t off = (size_t)row * p.ldc + col;
          gC[off] = acc[a][b][r];
          if (p.C2) gC2[off] = acc[a][b][r];
        }
      }
}

template <bool AT, bool BT, bool HAD>
__global__ __launch_bounds__(256) void gemm_dma_kernel(GemmArgs<double> p) {
  gemm_dma_body<AT, BT, HAD>(p, blockIdx.x, gridDim.x);
}
template <bool AT, bool BT, bool HAD>
__global__ __launch_bounds__(256) void gemm_dma_group_kernel(const GemmArgs<double>* tab, const int* offs,
                                                              int nprob) {
  int pid = 0;
  while (pid + 1 < nprob && (int)blockIdx.x >= offs[pid + 1]) ++pid;
  const GemmArgs<double> p = tab[pid];
  gemm_dma_body<AT, BT, HAD>(p, blockIdx.x - offs[pid], offs[pid + 1] - offs[pid]);
}

template <typename T>
bool gemm_dma_ok(const GemmArgs<T>& g, bool had) {
  if (sizeof(T) != 8 || g.K <= 0 || g.M <= 0 || g.N <= 0) return false;
  auto al16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
  return g.beta == T(0) && !g.lower && g.K % (had ? 8 : 16) == 0 && g.lda % 2 == 0 && g.ldb % 2 == 0 &&
         al16(g.A) && al16(g.B1) && (!had || al16(g.B2));
}
template bool gemm_dma_ok<double>(const GemmArgs<double>&, bool);
template bool gemm_dma_ok<float>(const GemmArgs<float>&, bool);

static void launch_dma(hipStream_t s, const GemmArgs<double>& a, bool at, bool bt, bool had) {
  dim3 grid(gemm_tile_count(a.M, a.N, DM)), block(256);
#define THCCP_DMA_CASE(AT_, BT_, HAD_)                                                   \
  if (at == AT_ && bt == BT_ && had == HAD_) {                                           \
    hipLaunchKernelGGL((gemm_dma_kernel<AT_, BT_, HAD_>), grid, block, 0, s, a);         \
    return;                                                                              \
  }
  THCCP_DMA_CASE(false, false, false)
  THCCP_DMA_CASE(true, false, false)
  THCCP_DMA_CASE(false, false, true)
  THCCP_DMA_CASE(true, false, true)
  THCCP_DMA_CASE(false, true, false)
  THCCP_DMA_CASE(true, true, false)
#undef THCCP_DMA_CASE
}
static void launch_dma_group(hipStream_t s, const GemmArgs<double>* tab, const int* offs, int nprob, int tiles,
                             bool at, bool bt, bool had) {
  dim3 grid(tiles), block(256);
#define THCCP_DMA_GCASE(AT_, BT_, HAD_)                                                               \
  if (at == AT_ && bt == BT_ && had == HAD_) {                                                        \
    hipLaunchKernelGGL((gemm_dma_group_kernel<AT_, BT_, HAD_>), grid, block, 0, s, tab, offs, nprob); \
    return;                                                                                           \
  }
  THCCP_DMA_GCASE(false, false, false)
  THCCP_DMA_GCASE(true, false, false)
  THCCP_DMA_GCASE(false, false, true)
  THCCP_DMA_GCASE(true, false, true)
  THCCP_DMA_GCASE(false, true, false)
#undef THCCP_DMA_GCASE
}

template <typename T, int BM, int BN>
static void launch_tile(hipStream_t s, const GemmArgs<T>& a, bool at, bool bt, bool had) {
  const int tiles = BM == BN ? gemm_tile_count(a.M, a.N, BM, a.lower) : ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  dim3 grid(tiles), block(256);
#define THCCP_GEMM_CASE(AT_, BT_, HAD_)                                           \
  if (at == AT_ && bt == BT_ && had == HAD_) {                                    \
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, AT_, BT_, HAD_>), grid, block, 0, s, a); \
    return;                                                                       \
  }
  THCCP_GEMM_CASE(false, false, false)
  THCCP_GEMM_CASE(true, false, false)
  THCCP_GEMM_CASE(false, false, true)
  THCCP_GEMM_CASE(true, false, true)
  THCCP_GEMM_CASE(false, true, false)
  THCCP_GEMM_CASE(true, true, false)
#undef THCCP_GEMM_CASE
}

int gemm_default_tile(int M, int N) {
  // 64 x 64 tiles (three workgroups per compute unit) unless there are
  // thousands of 128 x 128 tiles
  const long t128 = (long)((M + 127) / 128) * ((N + 127) / 128);
  return t128 >= 4096 ? 128 : 64;
}

template <typename T>
static void gemm_dispatch(hipStream_t s, const GemmArgs<T>& a, bool at, bool bt, bool had) {
  if (a.M <= 0 || a.N <= 0) return;
  if constexpr (sizeof(T) == 8) {
    // the direct-load 128-tile path wherever its requirements hold
    if (!(had && bt) && gemm_dma_ok(a, had)) {
      launch_dma(s, a, at, bt, had);
      return;
    }
  }
  if (gemm_default_tile(a.M, a.N) == 128) launch_tile<T, 128, 128>(s, a, at, bt, had);
  else launch_tile<T, 64, 64>(s, a, at, bt, had);
}

template <typename T, int BM>
static void launch_group_tile(hipStream_t s, const GemmArgs<T>* tab, const int* offs, int nprob, int tiles,
                              bool at, bool bt, bool had) {
  dim3 grid(tiles), block(256);
#define THCCP_GEMM_GCASE(AT_, BT_, HAD_)                                                              \
  if (at == AT_ && bt == BT_ && had == HAD_) {                                                       \
    hipLaunchKernelGGL((gemm_group_kernel<T, BM, BM, AT_, BT_, HAD_>), grid, block, 0, s, tab, offs, nprob); \
    return;                                                                                          \
  }
  THCCP_GEMM_GCASE(false, false, false)
  THCCP_GEMM_GCASE(true, false, false)
  THCCP_GEMM_GCASE(false, false, true)
  THCCP_GEMM_GCASE(true, false, true)
  THCCP_GEMM_GCASE(false, true, false)
#undef THCCP_GEMM_GCASE
}

template <typename T>
void gemm_group(hipStream_t s, const GemmArgs<T>* tab, const int* offs, int nprob, int total_tiles, bool a_t,
                bool b_t, bool had, int bm) {
  if (total_tiles <= 0) return;
  if constexpr (sizeof(T) == 8) {
    // FP64: bm = 128 is the direct-load path (the caller checked gemm_dma_ok
    // for every entry)
    if (bm == 128) {
      launch_dma_group(s, (const GemmArgs<double>*)tab, offs, nprob, total_tiles, a_t, b_t, had);
      return;
    }
  }
  if (bm == 128) launch_group_tile<T, 128>(s, tab, offs, nprob, total_tiles, a_t, b_t, had);
  else launch_group_tile<T, 64>(s, tab, offs, nprob, total_tiles, a_t, b_t, had);
}
template void gemm_group<double>(hipStream_t, const GemmArgs<double>*, const int*, int, int, bool, bool, bool, int);
template void gemm_group<float>(hipStream_t, const GemmArgs<float>*, const int*, int, int, bool, bool, bool, int);

void gemm_f64(hipStream_t s, const GemmF64& g) {
  GemmArgs<double> a{g.M, g.N, g.K, g.A, g.lda, g.B1, g.B2, g.ldb, g.C, g.ldc, g.C2,
                     g.alpha, g.beta, g.done, nullptr, 0, 0};
  gemm_dispatch<double>(s, a, g.a_t, g.b_t, g.B2 != nullptr);
}

void gemm_f32(hipStream_t s, const GemmF32& g) {
  GemmArgs<float> a{g.M, g.N, g.K, g.A, g.lda, g.B1, g.B2, g.ldb, g.C, g.ldc, g.C2,
                    g.alpha, g.beta, g.done, nullptr, 0, 0};
  gemm_dispatch<float>(s, a, g.a_t, g.b_t, g.B2 != nullptr);
}

}  // namespace thccp
