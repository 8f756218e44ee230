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


typedef uint32_t u4_t __attribute__((ext_vector_type(4)));

// Register stage of one operand for one k-tile: two 8-element K-chunks per
// thread.  Loads are unconditional (a row past the end reads row r0 and is
// zeroed at the LDS store); a pair operand keeps the raw FP32 factors and
// forms the product and its split at the LDS store.  Every value is pinned
// there, so no wait on the prefetch moves ahead of the current k-tile's
// matrix-core products.
template <bool PAIR, int C>
struct Stage;

template <int C>
struct Stage<false, C> {
  u4_t h[C], l[C];
  uint32_t ok;
  __device__ __forceinline__ void load(const SplitOperand& op, int rows, int r0, int k0, int tid) {
    const gptr<const __bf16> hi = as_global(op.hi), lo = as_global(op.lo);
    ok = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int gr = r0 + ((tid + 256 * c) >> 2);
      const bool v = gr < rows;
      const size_t off = (size_t)(v ? gr : r0) * op.ld + k0 + (tid & 3) * 8;
      h[c] = *(const gptr<const u4_t>)(hi + off);
      l[c] = *(const gptr<const u4_t>)(lo + off);
      ok |= (uint32_t)v << c;
    }
  }
  // one chunk of a later k-tile into the same registers (the row, hence
  // its validity bit, does not depend on the k-tile)
  __device__ __forceinline__ void load_chunk(const SplitOperand& op, int rows, int r0, int k0, int tid, int c) {
    const gptr<const __bf16> hi = as_global(op.hi), lo = as_global(op.lo);
    const int gr = r0 + ((tid + 256 * c) >> 2);
    const size_t off = (size_t)(gr < rows ? gr : r0) * op.ld + k0 + (tid & 3) * 8;
    h[c] = *(const gptr<const u4_t>)(hi + off);
    l[c] = *(const gptr<const u4_t>)(lo + off);
  }
  __device__ __forceinline__ void get(int c, u4_t& H, u4_t& L) {
    u4_t x = h[c], y = l[c];
    asm volatile("" : "+v"(x), "+v"(y));
    const u4_t z = {0u, 0u, 0u, 0u};
    H = (ok >> c) & 1 ? x : z;
    L = (ok >> c) & 1 ? y : z;
  }
};

template <int C>
struct Stage<true, C> {
  f4_t p[C][2], q[C][2];
  uint32_t ok;
  __device__ __forceinline__ void load(const SplitOperand& op, int rows, int r0, int k0, int tid) {
    const gptr<const float> P = as_global(op.p), Q = as_global(op.q);
    ok = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int gr = r0 + ((tid + 256 * c) >> 2);
      const bool v = gr < rows;
      const size_t off = (size_t)(v ? gr : r0) * op.ld + k0 + (tid & 3) * 8;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        p[c][u] = *(const gptr<const f4_t>)(P + off + 4 * u);
        q[c][u] = *(const gptr<const f4_t>)(Q + off + 4 * u);
      }
      ok |= (uint32_t)v << c;
    }
  }
  __device__ __forceinline__ void load_chunk(const SplitOperand& op, int rows, int r0, int k0, int tid, int c) {
    const gptr<const float> P = as_global(op.p), Q = as_global(op.q);
    const int gr = r0 + ((tid + 256 * c) >> 2);
    const size_t off = (size_t)(gr < rows ? gr : r0) * op.ld + k0 + (tid & 3) * 8;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      p[c][u] = *(const gptr<const f4_t>)(P + off + 4 * u);
      q[c][u] = *(const gptr<const f4_t>)(Q + off + 4 * u);
    }
  }
  __device__ __forceinline__ void get(int c, u4_t& H, u4_t& L) {
    f4_t a0 = p[c][0], a1 = p[c][1], b0 = q[c][0], b1 = q[c][1];
    asm volatile("" : "+v"(a0), "+v"(a1), "+v"(b0), "+v"(b1));
    const f4_t x0 = a0 * b0, x1 = a1 * b1;
    Pack8 ph, pl;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      split_f(x0[j], ph.b[j], pl.b[j]);
      split_f(x1[j], ph.b[4 + j], pl.b[4 + j]);
    }
    const bool v = (ok >> c) & 1;
    H = v ? u4_t{ph.u.x, ph.u.y, ph.u.z, ph.u.w} : u4_t{0u, 0u, 0u, 0u};
    L = v ? u4_t{pl.u.x, pl.u.y, pl.u.z, pl.u.w} : u4_t{0u, 0u, 0u, 0u};
  }
};

// Block tile BM x 128 (BM = 128, or 64 for short M so that the launch
// still covers the compute units); 2 x 2 waves, each (BM / 2) x 64.
template <bool APAIR, bool BPAIR, int BM>
__global__ __launch_bounds__(256) void gemm_split_kernel(const SplitArgs* tab, const int* offs, int nprob) {
  constexpr int CA = BM / 64, TI = BM / 32;
  // two LDS stages: the next k-tile is stored into the other stage right
  // after the current products are issued, one barrier per k-tile
  constexpr int SA = BM * SLDK, SB = SBN * SLDK;
  __shared__ __attribute__((aligned(16))) __bf16 lds[2 * (2 * SA + 2 * SB)];
  int pid = 0;
  while (pid + 1 < nprob && (int)blockIdx.x >= offs[pid + 1]) ++pid;
  const SplitArgs a = tab[pid];
  if (a.done && *a.done) return;
  if (a.gate && *a.gate != a.want) return;
  const int tiles_n = (a.N + SBN - 1) / SBN, tiles_m = (a.M + BM - 1) / BM;
  const int bid = xcd_remap(blockIdx.x - offs[pid], offs[pid + 1] - offs[pid]);
  int tm, tn;
  grouped_tile(bid, tiles_m, tiles_n, 8, tm, tn);
  const int m0 = tm * BM, n0 = tn * SBN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;

  Stage<APAIR, CA> sa;
  Stage<BPAIR, 2> sb;
  f4_t acc[TI][4];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  auto store = [&](int s) {
    __bf16* Ah = lds + s * (2 * SA + 2 * SB);
    __bf16* Al = Ah + SA;
    __bf16* Bh = Al + SA;
    __bf16* Bl = Bh + SB;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int row = (tid + 256 * c) >> 2;
      const int kc = (tid & 3) * 8;
      u4_t h, l;
      if (c < CA) {
        sa.get(c, h, l);
        *(u4_t*)&Ah[row * SLDK + kc] = h;
        *(u4_t*)&Al[row * SLDK + kc] = l;
      }
      sb.get(c, h, l);
      *(u4_t*)&Bh[row * SLDK + kc] = h;
      *(u4_t*)&Bl[row * SLDK + kc] = l;
    }
  };

  const int nk = a.K / SBK;
  sa.load(a.A, a.M, m0, 0, tid);
  sb.load(a.B, a.N, n0, 0, tid);
  store(0);
  __syncthreads();
  const int koff = 8 * (lane >> 4);
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) {
      sa.load(a.A, a.M, m0, (kt + 1) * SBK, tid);
      sb.load(a.B, a.N, n0, (kt + 1) * SBK, tid);
    }
    const __bf16* Ah = lds + (kt & 1) * (2 * SA + 2 * SB);
    const __bf16* Al = Ah + SA;
    const __bf16* Bh = Al + SA;
    const __bf16* Bl = Bh + SB;
    bf16x8_t ah[TI], al[TI], bh[4], bl[4];
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      const int row = wm * (BM / 2) + i * 16 + (lane & 15);
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
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
      }
    // the other stage was last read in iteration kt - 1, which every wave
    // finished before the barrier that ended it
    if (kt + 1 < nk) store((kt + 1) & 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * (BM / 2) + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn * 64 + j * 16 + (lane & 15);
        if (row < a.M && col < a.N) {
          const size_t off = (size_t)row * a.ldc + col;
          if (a.C32) as_global(a.C32)[off] = acc[i][j][r];
          if (a.C64) as_global(a.C64)[off] = (double)acc[i][j][r];
          if (a.C64b) as_global(a.C64b)[off] = (double)acc[i][j][r];
        }
      }
}

int split_tile_count(int M, int N, int bm) { return ((M + bm - 1) / bm) * ((N + SBN - 1) / SBN); }
int split_default_bm(int M, int N) {
  const long r64 = (M + 63) / 64 * 64, r128 = (M + 127) / 128 * 128;
  return (4 * r128 >= 5 * r64 || split_tile_count(M, N, 128) < 128) ? 64 : 128;
}

void gemm_split_group(hipStream_t s, const SplitArgs* tab, const int* offs, int nprob, int total_tiles,
                      bool apair, bool bpair, int bm) {
  if (total_tiles <= 0) return;
  dim3 grid(total_tiles), block(256);
#define THCCP_SPLIT_CASE(AP, BP)                                                                      \
  if (apair == AP && bpair == BP) {                                                                  \
    if (bm == 64) hipLaunchKernelGGL((gemm_split_kernel<AP, BP, 64>), grid, block, 0, s, tab, offs, nprob); \
    else hipLaunchKernelGGL((gemm_split_kernel<AP, BP, 128>), grid, block, 0, s, tab, offs, nprob);        \
    return;                                                                                          \
  }
  THCCP_SPLIT_CASE(false, false)
  THCCP_SPLIT_CASE(true, false)
  THCCP_SPLIT_CASE(false, true)
  THCCP_SPLIT_CASE(true, true)
#undef THCCP_SPLIT_CASE
}

// ------------------------------------------------------------ wide tiles
// BM x 256 tiles, 2 x 2 waves of (BM / 2) x 128: each LDS fragment read
// feeds 3 * BM / 32 (A) or 24 (B) matrix-core products, against 3 x 4 in
// the 128 x 128 kernel above.  LDS rows are 32 bf16 (64 bytes) with no
// padding; the 16-byte chunk c of row r is stored at chunk
// c ^ (((r >> 1) ^ (r >> 3)) & 3), so the 16 lanes of a fragment read (rows
// r0..r0+15, one chunk) and the 16 lanes of a staging store (rows
// r0..r0+3, all chunks) touch distinct 16-byte bank groups, in every
// aligned group of 8 lanes as well.
namespace {
constexpr int WBN = 256;
__device__ __forceinline__ int swz(int row, int chunk) { return chunk ^ (((row >> 1) ^ (row >> 3)) & 3); }
}  // namespace

template <bool APAIR, bool BPAIR, int BM>
__global__ __launch_bounds__(256, 1) void gemm_split_wide_kernel(const SplitArgs* tab, const int* offs, int nprob,
                                                                  int kparts) {
  constexpr int CA = BM / 64, CB = WBN / 64;
  constexpr int TI = BM / 32;  // 16-row MFMA tiles per wave
  constexpr int TJ = 8;        // 16-column MFMA tiles per wave
  constexpr int SA = BM * SBK, SB = WBN * SBK;  // bf16 per half-operand per stage
  constexpr int STAGE = 2 * SA + 2 * SB;
  __shared__ __attribute__((aligned(16))) __bf16 lds[2 * STAGE];
  int pid = 0;
  while (pid + 1 < nprob && (int)blockIdx.x >= offs[pid + 1]) ++pid;
  const SplitArgs a = tab[pid];
  if (a.done && *a.done) return;
  if (a.gate && *a.gate != a.want) return;
  const int tiles_n = (a.N + WBN - 1) / WBN, tiles_m = (a.M + BM - 1) / BM;
  const int ntiles = tiles_m * tiles_n;
  const int local = blockIdx.x - offs[pid];
  const int kp = local / ntiles;
  const int bid = xcd_remap(local - kp * ntiles, ntiles);
  int tm, tn;
  grouped_tile(bid, tiles_m, tiles_n, 4, tm, tn);
  const int m0 = tm * BM, n0 = tn * WBN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int nk_all = a.K / SBK;
  const int kt0 = (int)((long)nk_all * kp / kparts), kt1 = (int)((long)nk_all * (kp + 1) / kparts);

  Stage<APAIR, CA> sa;
  Stage<BPAIR, CB> sb;
  f4_t acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  // staging store of chunk c: thread tid owns rows (tid + 256 c) >> 2, chunk
  // tid & 3, of both operands
  auto store_chunk = [&](int st, int c) {
    __bf16* Ah = lds + st * STAGE;
    __bf16* Al = Ah + SA;
    __bf16* Bh = Al + SA;
    __bf16* Bl = Bh + SB;
    const int row = (tid + 256 * c) >> 2;
    const int off = row * SBK + 8 * swz(row, tid & 3);
    u4_t h, l;
    if (c < CA) {
      sa.get(c, h, l);
      *(u4_t*)&Ah[off] = h;
      *(u4_t*)&Al[off] = l;
    }
    sb.get(c, h, l);
    *(u4_t*)&Bh[off] = h;
    *(u4_t*)&Bl[off] = l;
  };

  // The staging registers hold the k-tile after the one being stored: each
  // chunk of k-tile kt + 2 is loaded as soon as its registers have been
  // stored to LDS (for k-tile kt + 1, during the products of kt), so the
  // loads have about one and a half k-tiles of products to arrive in.
  if (kt0 < kt1) {
    sa.load(a.A, a.M, m0, kt0 * SBK, tid);
    sb.load(a.B, a.N, n0, kt0 * SBK, tid);
#pragma unroll
    for (int c = 0; c < CB; ++c) store_chunk(0, c);
    if (kt0 + 1 < kt1) {
      sa.load(a.A, a.M, m0, (kt0 + 1) * SBK, tid);
      sb.load(a.B, a.N, n0, (kt0 + 1) * SBK, tid);
    }
  }
  __syncthreads();
  const int fch = lane >> 4;  // fragment chunk: k offset 8 * fch
  for (int kt = kt0; kt < kt1; ++kt) {
    const int cur = (kt - kt0) & 1;
    const bool more = kt + 1 < kt1, more2 = kt + 2 < kt1;
    const __bf16* Ah = lds + cur * STAGE;
    const __bf16* Al = Ah + SA;
    const __bf16* Bh = Al + SA;
    const __bf16* Bl = Bh + SB;
    bf16x8_t ah[TI], al[TI];
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      const int row = wm * (BM / 2) + i * 16 + (lane & 15);
      const int off = row * SBK + 8 * swz(row, fch);
      ah[i] = *(const bf16x8_t*)&Ah[off];
      al[i] = *(const bf16x8_t*)&Al[off];
    }
    auto bfrag = [&](int j, bf16x8_t& h, bf16x8_t& l) {
      const int col = wn * 128 + j * 16 + (lane & 15);
      const int off = col * SBK + 8 * swz(col, fch);
      h = *(const bf16x8_t*)&Bh[off];
      l = *(const bf16x8_t*)&Bl[off];
    };
    bf16x8_t bh, bl;
    bfrag(0, bh, bl);
    // software pipeline over the 8 column tiles: the fragments of tile
    // j + 1 are read while tile j's products run; the staging stores of the
    // next k-tile are spread over the last column tiles
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      bf16x8_t nh, nl;
      if (j + 1 < TJ) bfrag(j + 1, nh, nl);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
      }
      // (the other stage was last read in the previous iteration, which
      // every wave finished before the barrier that ended it)
      if (more && j >= TJ - CB) {
        const int c = j - (TJ - CB);
        store_chunk(cur ^ 1, c);
        if (more2) {
          if (c < CA) sa.load_chunk(a.A, a.M, m0, (kt + 2) * SBK, tid, c);
          sb.load_chunk(a.B, a.N, n0, (kt + 2) * SBK, tid, c);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      if (j + 1 < TJ) {
        bh = nh;
        bl = nl;
      }
    }
    __syncthreads();
  }

  const bool partial = kparts > 1;
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * (BM / 2) + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn * 128 + j * 16 + (lane & 15);
        if (row < a.M && col < a.N) {
          const size_t off = (size_t)row * a.ldc + col;
          if (partial) {
            as_global(a.part)[(size_t)kp * a.M * a.ldc + off] = acc[i][j][r];
          } else {
            if (a.C32) as_global(a.C32)[off] = acc[i][j][r];
            if (a.C64) as_global(a.C64)[off] = (double)acc[i][j][r];
            if (a.C64b) as_global(a.C64b)[off] = (double)acc[i][j][r];
          }
        }
      }
}

// C = sum over the kparts slices, in slice order (FP32 sums, as the
// accumulation inside one slice).  blockIdx.y selects the problem.
__global__ __launch_bounds__(256) void split_reduce_kernel(const SplitArgs* tab, int kparts) {
  const SplitArgs a = tab[blockIdx.y];
  if (a.done && *a.done) return;
  if (a.gate && *a.gate != a.want) return;
  const size_t total = (size_t)a.M * a.N;
  const size_t slice = (size_t)a.M * a.ldc;
  const gptr<const float> P = as_global((const float*)a.part);
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const size_t r = e / a.N, c = e % a.N;
    const size_t off = r * a.ldc + c;
    float v = P[off];
    for (int k = 1; k < kparts; ++k) v += P[k * slice + off];
    if (a.C32) as_global(a.C32)[off] = v;
    if (a.C64) as_global(a.C64)[off] = (double)v;
    if (a.C64b) as_global(a.C64b)[off] = (double)v;
  }
}

int split_wide_tile_count(int M, int N, int bm) { return ((M + bm - 1) / bm) * ((N + WBN - 1) / WBN); }

void gemm_split_wide_group(hipStream_t s, const SplitArgs* tab, const int* offs, int nprob, int total_tiles,
                           bool apair, bool bpair, int bm, int kparts) {
  if (total_tiles <= 0) return;
  if (kparts < 1) kparts = 1;
  dim3 grid(total_tiles), block(256);
#define THCCP_WIDE_CASE(AP, BP)                                                                              \
  if (apair == AP && bpair == BP) {                                                                         \
    if (bm == 128)                                                                                          \
      hipLaunchKernelGGL((gemm_split_wide_kernel<AP, BP, 128>), grid, block, 0, s, tab, offs, nprob, kparts); \
    else                                                                                                    \
      hipLaunchKernelGGL((gemm_split_wide_kernel<AP, BP, 256>), grid, block, 0, s, tab, offs, nprob, kparts); \
    return;                                                                                                 \
  }
  THCCP_WIDE_CASE(false, false)
  THCCP_WIDE_CASE(true, false)
  THCCP_WIDE_CASE(false, true)
  THCCP_WIDE_CASE(true, true)
#undef THCCP_WIDE_CASE
}

void gemm_split_reduce_group(hipStream_t s, const SplitArgs* tab, int nprob, int kparts, int max_m, int max_n) {
  if (kparts <= 1 || nprob <= 0) return;
  size_t blocks = ((size_t)max_m * max_n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(split_reduce_kernel, dim3((unsigned)blocks, nprob), dim3(256), 0, s, tab, kparts);
}

// ------------------------------------------------- direct-to-LDS tiles
// 256 x 256 tiles of pre-split operands loaded straight into LDS
// (global_load_lds_dwordx4): no staging registers and no conversion in
// the loop, so the wave's instruction stream is the fragment reads and the
// matrix-core products.  The operands are stored in the blocked split
// layout (mixed.h): a 16-row x 32-k block is one contiguous kilobyte in
// fragment order (lane l of a fragment read: row l % 16, k chunk l / 16),
// so one direct-load instruction of a wave copies one block from memory to
// LDS unchanged and a fragment read is one contiguous kilobyte of LDS.
// The 160 KB of LDS hold five operand stages of 32 KB (hi and lo of 256
// rows x 32 k): two of the row operand and three of the column operand,
// so that two k-tiles are in flight while one is multiplied.  Rows are padded to the tile with zeros, so no row is
// clamped.
namespace {
typedef __attribute__((address_space(3))) void* lds_vptr_t;
typedef const __attribute__((address_space(1))) void* glb_cvptr_t;
constexpr int DT = 256;          // tile edge
constexpr int DHALF = DT * SBK;  // bf16 per operand half per k-tile
}  // namespace

__global__ __launch_bounds__(256, 1) void gemm_split_dma_kernel(const SplitArgs* tab, const int* offs, int nprob,
                                                                 int kparts) {
  __shared__ __attribute__((aligned(1024))) __bf16 lds[10 * DHALF];
  int pid = 0;
  while (pid + 1 < nprob && (int)blockIdx.x >= offs[pid + 1]) ++pid;
  const SplitArgs a = tab[pid];
  if (a.done && *a.done) return;
  if (a.gate && *a.gate != a.want) return;
  const int tiles_n = (a.N + DT - 1) / DT, tiles_m = (a.M + DT - 1) / DT;
  const int ntiles = tiles_m * tiles_n;
  const int local = blockIdx.x - offs[pid];
  const int kp = local / ntiles;
  const int bid = xcd_remap(local - kp * ntiles, ntiles);
  int tm, tn;
  grouped_tile(bid, tiles_m, tiles_n, 4, tm, tn);
  const int m0 = tm * DT, n0 = tn * DT;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int wm = wid >> 1, wn = wid & 1;
  const int KT = a.K / SBK;
  const int kt0 = (int)((long)KT * kp / kparts), kt1 = (int)((long)KT * (kp + 1) / kparts);

  f4_t acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  // Two k-tiles in flight: the row operand has two LDS stages, the column
  // operand three.  The column operand's k-tile t + 2 is loaded during the
  // first column tile of step t (its stage held k-tile t - 1); the row
  // operand's k-tile t + 2 during the second, after every wave has read its
  // fragments of k-tile t (they are all read during the first).  One load
  // instruction follows each row's products, so that no wave stalls on a
  // burst of loads.  Past the last k-tile the loads fetch the last k-tile
  // again into a stage that is not read any more: the loop body stays one
  // block and the wait counts are constants.
  const int n = kt1 - kt0;
  // load b of 8 (hi blocks, then lo blocks) of this wave's share of k-tile t
  auto dma_a = [&](int t, int b) {
    const int kt = kt0 + min(t, n - 1), rb = wid * 4 + (b & 3);
    const __bf16* g = (b < 4 ? a.A.hi : a.A.lo) + ((size_t)(m0 / 16 + rb) * KT + kt) * 512 + lane * 8;
    __bf16* d = lds + (t & 1) * 2 * DHALF + (b < 4 ? 0 : DHALF) + rb * 512;
    __builtin_amdgcn_global_load_lds((glb_cvptr_t)g, (lds_vptr_t)d, 16, 0, 0);
  };
  auto dma_b = [&](int t, int st, int b) {
    const int kt = kt0 + min(t, n - 1), rb = wid * 4 + (b & 3);
    const __bf16* g = (b < 4 ? a.B.hi : a.B.lo) + ((size_t)(n0 / 16 + rb) * KT + kt) * 512 + lane * 8;
    __bf16* d = lds + (4 + 2 * st) * DHALF + (b < 4 ? 0 : DHALF) + rb * 512;
    __builtin_amdgcn_global_load_lds((glb_cvptr_t)g, (lds_vptr_t)d, 16, 0, 0);
  };
  if (n > 0) {
#pragma unroll
    for (int b = 0; b < 8; ++b) dma_a(0, b);
#pragma unroll
    for (int b = 0; b < 8; ++b) dma_b(0, 0, b);
#pragma unroll
    for (int b = 0; b < 8; ++b) dma_a(1, b);
#pragma unroll
    for (int b = 0; b < 8; ++b) dma_b(1, 1, b);
  }
  int bs = 0;  // t % 3
  for (int t = 0; t < n; ++t) {
    // This wave's loads of k-tile t have landed (those of k-tile t + 1, 16
    // per wave, issued after them, may still be in flight); the barrier
    // makes every wave's visible and ends every read of step t - 1.  A
    // plain barrier: a fenced one would wait for all loads.
    __asm__ volatile("s_waitcnt vmcnt(16)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
    const int bs2 = bs == 0 ? 2 : bs - 1;  // (t + 2) % 3
    const __bf16* Ah = lds + (t & 1) * 2 * DHALF + (wm * 8) * 512 + lane * 8;
    const __bf16* Bh = lds + (4 + 2 * bs) * DHALF + (wn * 8) * 512 + lane * 8;
    // fragment reads: the first column tile's and the first four row
    // fragments, the other row fragments four products ahead of their use,
    // each later column tile's right after the first products of the tile
    // before
    bf16x8_t ah[8], al[8];
    bf16x8_t bh = *(const bf16x8_t*)Bh, bl = *(const bf16x8_t*)(Bh + DHALF);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ah[i] = *(const bf16x8_t*)(Ah + i * 512);
      al[i] = *(const bf16x8_t*)(Ah + DHALF + i * 512);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      bf16x8_t nh, nl;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if (j == 0 && i + 4 < 8) {
          ah[i + 4] = *(const bf16x8_t*)(Ah + (i + 4) * 512);
          al[i + 4] = *(const bf16x8_t*)(Ah + DHALF + (i + 4) * 512);
        }
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
        if (j == 0 || i == 0) __builtin_amdgcn_sched_barrier(0);
        if (j == 0) {
          dma_b(t + 2, bs2, i);
          __builtin_amdgcn_sched_barrier(0);
        } else if (j == 1) {
          dma_a(t + 2, i);
          __builtin_amdgcn_sched_barrier(0);
        }
        if (i == (j == 0 ? 4 : 0) && j + 1 < 8) {
          nh = *(const bf16x8_t*)(Bh + (j + 1) * 512);
          nl = *(const bf16x8_t*)(Bh + DHALF + (j + 1) * 512);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      if (j == 0) {
        // every wave's row fragments of k-tile t are in registers: its
        // stage takes k-tile t + 2 from here on
        __builtin_amdgcn_s_barrier();
        __asm__ volatile("" ::: "memory");
      }
      __builtin_amdgcn_sched_barrier(0);
      if (j + 1 < 8) {
        bh = nh;
        bl = nl;
      }
    }
    bs = bs == 2 ? 0 : bs + 1;
  }
  // no load into LDS may outlive the workgroup
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");

  const bool partial = kparts > 1;
  // the result's row and column bases are formed here, after the loop, so
  // that no address of the stores is held through it
  int row0 = m0 + wm * 128 + 4 * (lane >> 4), col0 = n0 + wn * 128 + (lane & 15);
  __asm__ volatile("" : "+v"(row0), "+v"(col0));
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + i * 16 + r;
        const int col = col0 + j * 16;
        if (row < a.M && col < a.N) {
          const size_t off = (size_t)row * a.ldc + col;
          if (partial) {
            as_global(a.part)[(size_t)kp * a.M * a.ldc + off] = acc[i][j][r];
          } else {
            if (a.C32) as_global(a.C32)[off] = acc[i][j][r];
            if (a.C64) as_global(a.C64)[off] = (double)acc[i][j][r];
            if (a.C64b) as_global(a.C64b)[off] = (double)acc[i][j][r];
          }
        }
      }
}

int split_dma_tile_count(int M, int N) { return ((M + DT - 1) / DT) * ((N + DT - 1) / DT); }

void gemm_split_dma_group(hipStream_t s, const SplitArgs* tab, const int* offs, int nprob, int total_tiles,
                          int kparts) {
  if (total_tiles <= 0) return;
  if (kparts < 1) kparts = 1;
  hipLaunchKernelGGL(gemm_split_dma_kernel, dim3(total_tiles), dim3(256), 0, s, tab, offs, nprob, kparts);
}

// ---------------------------------------------- blocked split layout
// One thread per 8-element chunk of the padded operand, taken in the
// blocked (output) order, so that a wave writes one contiguous kilobyte of
// hi and of lo; its lanes read 16 rows x 4 chunks, 128 contiguous bytes per
// row of each source.  Chunk e: block b = e / 64 (row block b / KT, k-tile
// b % KT), k chunk (e / 16) % 4 of the k-tile, row (e % 16) of the block.
__device__ __forceinline__ void blk_coords(size_t e, int KT, int& r, int& k) {
  const size_t b = e >> 6;
  const int w = (int)(e & 63);
  r = (int)(b / KT) * 16 + (w & 15);
  k = (int)(b % KT) * 32 + (w >> 4) * 8;
}
__global__ __launch_bounds__(256) void split_blocked_f64_kernel(const double* src, int rows, int cols, int lds,
                                                                __bf16* hi, __bf16* lo, int rows_p, int Kp,
                                                                bool trans) {
  const int KT = Kp / 32;
  const size_t total = (size_t)rows_p * (Kp / 8);
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    int r, k0;
    blk_coords(e, KT, r, k0);
    Pack8 ph, pl;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + j;
      const double x = (r < rows && k < cols) ? (trans ? src[(size_t)k * lds + r] : src[(size_t)r * lds + k]) : 0.0;
      split_d(x, ph.b[j], pl.b[j]);
    }
    as_global((u4_t*)hi)[e] = u4_t{ph.u.x, ph.u.y, ph.u.z, ph.u.w};
    as_global((u4_t*)lo)[e] = u4_t{pl.u.x, pl.u.y, pl.u.z, pl.u.w};
  }
}
__global__ __launch_bounds__(256) void pair_split_blocked_kernel(const float* p, const float* q, int ld, int rows,
                                                                 int cols, __bf16* hi, __bf16* lo, int rows_p,
                                                                 int Kp) {
  const int KT = Kp / 32;
  const size_t total = (size_t)rows_p * (Kp / 8);
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    int r, k0;
    blk_coords(e, KT, r, k0);
    Pack8 ph, pl;
    if (r < rows && k0 + 8 <= cols) {
      const gptr<const f4_t> P = as_global((const f4_t*)(p + (size_t)r * ld + k0));
      const gptr<const f4_t> Q = as_global((const f4_t*)(q + (size_t)r * ld + k0));
      const f4_t x0 = P[0] * Q[0], x1 = P[1] * Q[1];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        split_f(x0[j], ph.b[j], pl.b[j]);
        split_f(x1[j], ph.b[4 + j], pl.b[4 + j]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + j;
        const float x = (r < rows && k < cols) ? p[(size_t)r * ld + k] * q[(size_t)r * ld + k] : 0.f;
        split_f(x, ph.b[j], pl.b[j]);
      }
    }
    as_global((u4_t*)hi)[e] = u4_t{ph.u.x, ph.u.y, ph.u.z, ph.u.w};
    as_global((u4_t*)lo)[e] = u4_t{pl.u.x, pl.u.y, pl.u.z, pl.u.w};
  }
}
static int blk_grid(size_t n) {
  size_t g = (n + 255) / 256;
  return (int)(g > 16384 ? 16384 : (g < 1 ? 1 : g));
}
void split_blocked_f64(hipStream_t s, const double* src, int rows, int cols, int lds, __bf16* hi, __bf16* lo,
                       int Kp, bool trans) {
  const int rows_p = blk_rows(rows);
  hipLaunchKernelGGL(split_blocked_f64_kernel, dim3(blk_grid((size_t)rows_p * (Kp / 8))), dim3(256), 0, s, src, rows,
                     cols, lds, hi, lo, rows_p, Kp, trans);
}
// Grouped form: one job per blockIdx.y, skipped for a problem that is done
// or not on the path the job is for.
__global__ __launch_bounds__(256) void pair_split_group_kernel(const PairJob* jobs) {
  const PairJob jb = jobs[blockIdx.y];
  if (jb.done && *jb.done) return;
  if (jb.gate && *jb.gate != jb.want) return;
  const int KT = jb.Kp / 32;
  const size_t total = (size_t)blk_rows(jb.rows) * (jb.Kp / 8);
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    int r, k0;
    blk_coords(e, KT, r, k0);
    Pack8 ph, pl;
    if (r < jb.rows && k0 + 8 <= jb.cols) {
      const gptr<const f4_t> P = as_global((const f4_t*)(jb.p + (size_t)r * jb.ld + k0));
      const gptr<const f4_t> Q = as_global((const f4_t*)(jb.q + (size_t)r * jb.ld + k0));
      const f4_t x0 = P[0] * Q[0], x1 = P[1] * Q[1];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        split_f(x0[j], ph.b[j], pl.b[j]);
        split_f(x1[j], ph.b[4 + j], pl.b[4 + j]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + j;
        const float x = (r < jb.rows && k < jb.cols) ? jb.p[(size_t)r * jb.ld + k] * jb.q[(size_t)r * jb.ld + k] : 0.f;
        split_f(x, ph.b[j], pl.b[j]);
      }
    }
    as_global((u4_t*)jb.hi)[e] = u4_t{ph.u.x, ph.u.y, ph.u.z, ph.u.w};
    as_global((u4_t*)jb.lo)[e] = u4_t{pl.u.x, pl.u.y, pl.u.z, pl.u.w};
  }
}
void pair_split_group(hipStream_t s, const PairJob* jobs, int njobs, size_t max_chunks) {
  if (njobs <= 0) return;
  size_t g = (max_chunks + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(pair_split_group_kernel, dim3((unsigned)g, njobs), dim3(256), 0, s, jobs);
}

// Grouped blocked split of transposes: job blockIdx.y writes hi / lo
// (blocked, rows = its cols, Kp = its dcols) = split(src^T), zero for
// k >= rows (the padding); skipped as split_transpose_group_kernel.  In the
// blocked order the lanes of a wave read consecutive source columns.
__global__ __launch_bounds__(256) void split_transpose_blocked_group_kernel(const SplitTArgs* tab) {
  const SplitTArgs a = tab[blockIdx.y];
  if (a.done && *a.done) return;
  if (a.gate && *a.gate != 0) return;
  const int KT = a.dcols / 32;
  const size_t total = (size_t)blk_rows(a.cols) * (a.dcols / 8);
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    int r, k0;
    blk_coords(e, KT, r, k0);
    Pack8 ph, pl;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + j;
      const double x = (r < a.cols && k < a.rows) ? a.src[(size_t)k * a.lds + r] : 0.0;
      split_d(x, ph.b[j], pl.b[j]);
    }
    as_global((u4_t*)a.hi)[e] = u4_t{ph.u.x, ph.u.y, ph.u.z, ph.u.w};
    as_global((u4_t*)a.lo)[e] = u4_t{pl.u.x, pl.u.y, pl.u.z, pl.u.w};
  }
}
void split_transpose_blocked_group(hipStream_t s, const SplitTArgs* tab, int nprob, size_t max_chunks) {
  if (nprob <= 0) return;
  size_t g = (max_chunks + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(split_transpose_blocked_group_kernel, dim3((unsigned)g, nprob), dim3(256), 0, s, tab);
}

void pair_split_blocked(hipStream_t s, const float* p, const float* q, int ld, int rows, int cols, __bf16* hi,
                        __bf16* lo, int Kp) {
  const int rows_p = blk_rows(rows);
  hipLaunchKernelGGL(pair_split_blocked_kernel, dim3(blk_grid((size_t)rows_p * (Kp / 8))), dim3(256), 0, s, p, q, ld,
                     rows, cols, hi, lo, rows_p, Kp);
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
