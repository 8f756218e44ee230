// Internal launchers shared by the translation units of libthccp.so.
// Not part of the public C-ABI (include/thccp.h).
//
// Every kernel of the sweep is "grouped": one launch serves a table of
// independent problems (the CPDs of a batch; a single CPD is a group of
// one).  Argument tables live in device memory (the plan's workspace);
// `offs` tables hold the prefix sums of each problem's workgroup count.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "common.h"

namespace thccp {

// ---------------------------------------------------------------- GEMM
// C[M x N] = alpha * op(A)[M x K] * op(B)[K x N] + beta * C, row-major C.
//   a_t = false: A[i*lda + k];  a_t = true: A[k*lda + i]   (A stored K x M)
//   b_t = false: B[k*ldb + j];  b_t = true: B[j*ldb + k]   (B stored N x K)
//   B2 != nullptr: every B element is B1[.] * B2[.] (Hadamard product fused
//   into the operand load; same layout and leading dimension).
//   C2 != nullptr: the result is also written to C2 (same ldc).
//   done != nullptr: the problem is skipped once *done is set.
//   gate != nullptr: the problem is skipped unless *gate == want (per-problem
//   choice between the split-BF16 and the FP64 path).
//   lower != 0: tiles strictly above the diagonal are skipped (C is only
//   needed on and below it, as in a symmetric rank-k update); for square
//   C only the lower tiles are launched (see gemm_tile_count).
template <typename T>
struct GemmArgs {
  int M, N, K;
  const T* A; int lda;
  const T* B1; const T* B2; int ldb;
  T* C; int ldc; T* C2;
  T alpha, beta;
  const int32_t* done;
  const int32_t* gate = nullptr;
  int32_t want = 0;
  int32_t lower = 0;
};
struct GemmF64 {
  int M, N, K;
  const double* A; int lda; bool a_t;
  const double* B1; const double* B2; int ldb; bool b_t;
  double* C; int ldc; double* C2;
  double alpha, beta;
  const int32_t* done;
};
struct GemmF32 {
  int M, N, K;
  const float* A; int lda; bool a_t;
  const float* B1; const float* B2; int ldb; bool b_t;
  float* C; int ldc; float* C2;
  float alpha, beta;
  const int32_t* done;
};
void gemm_f64(hipStream_t s, const GemmF64& g);
void gemm_f32(hipStream_t s, const GemmF32& g);
// Tile edge the heuristic picks (64; 128 only for thousands of 128-tiles).
int gemm_default_tile(int M, int N);
// Tiles of one GEMM; a lower-triangle GEMM (lower != 0, square) launches
// only the T (T + 1) / 2 tiles on and below the diagonal.
inline int gemm_tile_count(int M, int N, int bm, int lower = 0) {
  const int tm = (M + bm - 1) / bm, tn = (N + bm - 1) / bm;
  return lower && M == N ? tm * (tm + 1) / 2 : tm * tn;
}
// Whether the FP64 direct-load 128-tile path can take this product: beta =
// 0, not lower-triangle, K a multiple of its k-step (8 with a Hadamard pair,
// 16 otherwise), even leading dimensions, 16-byte aligned operands (always
// false for FP32).
template <typename T>
bool gemm_dma_ok(const GemmArgs<T>& g, bool had);
// Grouped launch: tab[nprob] problems with identical (a_t, b_t, Hadamard)
// flags, tile edge bm (64 or 128; for FP64, 128 is the direct-load path and
// every entry must pass gemm_dma_ok), offs[nprob + 1] prefix sums of
// gemm_tile_count(M_p, N_p, bm).
template <typename T>
void gemm_group(hipStream_t s, const GemmArgs<T>* tab, const int* offs, int nprob, int total_tiles, bool a_t,
                bool b_t, bool had, int bm);

// -------------------------------------------------- Cholesky / triangular solve
// One problem of the blocked factorisation and row solves.  V: Tp x Tp
// row-major (Tp = 64 nblk); the diagonal blocks of L go to ldiag (nblk
// 64 x 64 blocks), the diagonal of L to diagL; M: n x Tp right-hand sides.
template <typename T>
struct StepProb {
  T* V;
  T* ldiag;
  T* diagL;
  T* M;
  DevState* st;
  int nblk;
  int n;
  int32_t* flow;   // ready flags of the dataflow solves, ceil(n / 64) x nblk
  int32_t* cflow;  // ready flags of the dataflow factorisation, nblk^2 + 2 nblk,
                   // then CU_SLOTS per-compute-unit counters
  T* dpart;        // diagonal blocks updated through column k - 2, nblk x 64 x 64
};
// Per-compute-unit counters of the dataflow factorisation (an XCC, shader
// engine, shader array and CU index from the hardware id registers).
constexpr int CU_SLOTS = 2048;
enum StepMode {
  STEP_CHOL = 0,
  STEP_FWD = 1,
  STEP_BWD = 2,
  STEP_CHOL_FWD = 3,
  STEP_FLOW_RESET = 4,     // clears the solve's ready flags (one workgroup per problem)
  STEP_BWD_FLOW = 5,       // the whole one-level backward solve as one dataflow launch
  STEP_CFLOW_RESET = 6,    // clears the factorisation's and the solve's ready flags
  STEP_CHOL_FWD_FLOW = 7,  // one-level factorisation + forward solve as one dataflow launch
  STEP_BWD_PREP = 8,       // per pair of block columns, the products of L the paired solve needs
  STEP_BWD_PAIR = 9        // the one-level backward solve as one dataflow launch, in block pairs
};

// Two-level blocking: the 64-wide block columns are grouped into panels of
// pw blocks.  Inside a panel the step kernel works one block column per
// launch (panel-local updates only); after a panel, one grouped GEMM applies
// its rank-(64 pw) update to everything right of it (factorisation, forward
// solve) or left of it (backward solve).  pw >= nblk is the one-level form:
// every step updates the whole trailing matrix.
// One step launch: factorisation step tc of panel pc and solve step tf of
// panel pf (a negative panel or step: none).  Factorisation step t of panel
// p updates the panel's remaining block columns with block column
// pw p - 1 + t (when inside the panel) and factors block column pw p + t;
// forward step t likewise for the right-hand sides; backward step t solves
// block column b1 - t of the panel (b1 its last block) after updating the
// panel's columns left of it.
struct StepCfg {
  int pw;
  int pc, tc;
  int pf, tf;
};
inline int panel_count(int nblk, int pw) { return (nblk + pw - 1) / pw; }
// Workgroups of problem (nblk, n) in a launch of `mode` with `cfg`.
int step_tiles(int mode, int nblk, int n, StepCfg cfg);
// Workgroup order of a grouped dataflow launch (STEP_CHOL_FWD_FLOW,
// STEP_BWD_FLOW, STEP_BWD_PAIR) over problems of nblk[p] blocks and n[p]
// rows: segments of one (problem, block column), block column by block
// column across the problems (ascending for the factorisation, from each
// problem's last column down for the backward solve), so every problem
// advances at the same pace and every wait is on a lower workgroup id.
// STEP_BWD_PAIR: segments of one (problem, pair of block columns), pairs
// from the last column down; per row tile the workgroup of the pair's upper
// block, then that of its lower block.  The one wait on a higher id is the
// upper block's wait for the lower block's first action (its right-hand
// side read), which waits on nothing.  Int triples (first workgroup,
// problem, column or pair), then (total workgroups, -1, -1).
std::vector<int> flow_segments(int mode, const std::vector<int>& nblk, const std::vector<int>& n);
inline bool is_flow_mode(int mode) {
  return mode == STEP_CHOL_FWD_FLOW || mode == STEP_BWD_FLOW || mode == STEP_BWD_PAIR;
}
// Polls a dataflow wait makes before it gives up (negative: the default);
// returns the previous value.  Applies to launches enqueued afterwards.
int set_flow_spin_limit(int polls);
// Form of the one-level backward solve for schedules built afterwards:
// 0 (default) two block columns per dependency hop (STEP_BWD_PREP +
// STEP_BWD_PAIR), 1 one block column per hop (STEP_BWD_FLOW); returns the
// previous value.
int set_bwd_form(int form);
// Launches one step of `mode`.  offs: nprob + 1 prefix sums of the
// problems' workgroups, or for a dataflow mode the segment table, with
// nprob its segment count.
template <typename T>
void step_group(hipStream_t s, int mode, const StepProb<T>* probs, const int* offs, int nprob, int total_tiles,
                StepCfg cfg, int retry_pass);
// The panel update GEMM of panel p for one problem (false: none needed):
//   PG_SYRK  V[c0:, c0:] -= L[c0:, panel] L[c0:, panel]^T (lower tiles),
//   PG_FWD   M[:, c0:]   -= G[:, panel] L[c0:, panel]^T,
//   PG_BWD   M[:, :b0]   -= X[:, panel] L[panel, :b0],
// with c0 the first column after the panel and b0 its first column.  SYRK
// and FWD take (a_t, b_t) = (false, true), BWD (false, false).
enum PanelGemm { PG_SYRK = 0, PG_FWD = 1, PG_BWD = 2 };
template <typename T>
bool panel_gemm(int kind, const StepProb<T>& q, int pw, int p, GemmArgs<T>& g);

// Launch order of a blocked solve with panel width pw for problems of up
// to max_nblk blocks: step launches (mode >= 0) and panel GEMM launches
// (mode < 0, up to two PanelGemm kinds in one grouped launch).
//   SCHED_CHOL      factorisation: per panel, its steps, then its SYRK.
//   SCHED_CHOL_FWD  factorisation fused with the forward solve.  With
//                   panels, the latter runs one panel behind: the launches
//                   of panel p also run the forward steps of panel p - 1, and
//                   one GEMM launch holds the SYRK of panel p and the
//                   forward update of panel p - 1.  One-level (pw >=
//                   max_nblk): one block column behind.
//   SCHED_FWD       forward solve alone;  SCHED_BWD  backward solve (panels
//                   from the last one down; one level: a flag reset, then
//                   STEP_BWD_PREP and the dataflow launch STEP_BWD_PAIR, or
//                   the dataflow launch STEP_BWD_FLOW; set_bwd_form).
enum SolveSched { SCHED_CHOL = 0, SCHED_CHOL_FWD = 1, SCHED_FWD = 2, SCHED_BWD = 3 };
struct SolveItem {
  int mode;
  StepCfg cfg;
  int g_kind[2];
  int g_panel[2];
};
std::vector<SolveItem> solve_schedule(int sched, int max_nblk, int pw);

// ------------------------------------------------------------- element-wise
template <typename T>
struct FormVArgs {
  T* V; const T* g0; const T* g1; const T* g2; DevState* st; int Tp; int R;
};
template <typename T>
void form_v_group(hipStream_t s, const FormVArgs<T>* tab, int nprob, int max_Tp, int retry_pass);
template <typename T>
void retry_prepare_group(hipStream_t s, const FormVArgs<T>* tab, int nprob, int allow_fallback);

template <typename T>
struct NormArgs {
  const T* Msol; T* F; T* lam; const T* Msave; double* inner_part; DevState* st; int n; int R; int ld;
};
template <typename T>
void normalise_group(hipStream_t s, const NormArgs<T>* tab, int nprob, int max_R);
// Tied model: <G, G~> partials lam[k] sum_s F3[s,k] M3[s,k] (F3 passed as
// Msol, M3 as Msave; F unused).
template <typename T>
void tied_inner_group(hipStream_t s, const NormArgs<T>* tab, int nprob, int max_R);

template <typename T>
struct FitArgs {
  const T* g[4]; const T* lam; const double* inner_part; double* row_part; double* fit_hist; DevState* st;
  int R; int ld;
};
template <typename T>
void fit_group(hipStream_t s, const FitArgs<T>* tab, int nprob, int max_R, int hist_cap, double tol,
               double fit_floor, int guard, double cond_limit, int rule_every);
// Non-fit sweep of a split-BF16 plan: sweep counter and precision guard.
void sweep_tick_group(hipStream_t s, DevState* const* st_tab, int nprob, int guard, double cond_limit);
// Precision guard bookkeeping (split-BF16 plans):
//   cond_track: st->cond_max = max(st->cond_max, (max diagL / min diagL)^2)
//   after each mode's factorisation; guard_begin: reset at sweep start.
template <typename T>
struct CondArgs {
  const T* diagL; DevState* st; int R;
};
template <typename T>
void cond_track_group(hipStream_t s, const CondArgs<T>* tab, int nprob);
void guard_begin_group(hipStream_t s, DevState* const* st_tab, int nprob);
// Sets path = 1 (FP64) and clears promote for the listed problems.
void set_path_group(hipStream_t s, DevState* const* st_tab, int nprob, const int32_t* flags_dev);

// Factor checkpoint: copies (dir = 0) F -> Fsave and st -> st_save, or back.
struct CkptArgs {
  void* a[4];
  void* b[4];
  size_t bytes[4];
  DevState* st;
  DevState* st_save;
  const int32_t* gate;  // non-NULL: copy only while *gate == want
  int32_t want;
};
// Copies a[m] -> b[m] (dir 0) or back (dir 1), bytes[m] each, and the
// device state with them; with st or st_save NULL only the regions (the
// tied model's factor copies, the right-hand-side backups of the solve).
void checkpoint_group(hipStream_t s, const CkptArgs* tab, int nprob, int dir);

void hadamard_inplace_f64(hipStream_t s, double* A, const double* B, size_t count);
void transposed_dot_f64(hipStream_t s, const double* P, const double* Q, int R, int ld, double* partials,
                        double* out);
void fill_bytes(hipStream_t s, void* p, size_t bytes);
void state_reset(hipStream_t s, DevState* st, double* norm2_src, double fit_target);
void cast_f64_to_f32(hipStream_t s, const double* a, float* b, size_t count);
void copy_normalised_init(hipStream_t s, const double* src, int n, int R, int ld, double* dst);
void lt_scale_rows(hipStream_t s, const double* X, const double* eps, int n, int r, double t, double sign,
                   double* out);

}  // namespace thccp
