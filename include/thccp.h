/*
 * thccp.h -- C-ABI of libthccp.so: matrix-free, THC-based CP-ALS of an
 * order-4 two-electron-integral tensor on one MI355X (gfx950).
 *
 * The tensor is never formed.  It is given in tensor-hypercontraction form
 * (Pierce & Morales, Section 2.1, eq. THC), in chemists' index order:
 *
 *   G[p,q,r,s] = sum_{P,Q} X0[p,P] X1[q,P] Z[P,Q] X2[r,Q] X3[s,Q]
 *
 * and fitted by a rank-R_cp canonical polyadic decomposition with column
 * weights (eq. cp4), G ~ sum_k lambda_k F0[:,k] o F1[:,k] o F2[:,k] o F3[:,k],
 * by alternating least squares on the THC-approximated loss (eq. lossF).
 * Each mode update needs only the projections W_m = X_m^T F_m, Hadamard
 * products, one core product Z (W o W) (reused by the partner mode) and a
 * back-projection X_n (W o Y) -- O(n R_thc R_cp + R_thc^2 R_cp) work and
 * O(R^2) storage -- followed by the FP64 normal-equation solve with the
 * Gram-Hadamard matrix V_n = o_{m != n} F_m^T F_m.  The fit is the paper's
 * ||T - T~|| / ||T|| (Computational Details), evaluated matrix-free.
 *
 * Conventions
 *   - All matrices are row-major, densely packed (leading dimension = number
 *     of columns), float64, in DEVICE memory unless stated otherwise.
 *   - Pointers passed in are borrowed: the library never frees them and
 *     they must stay valid for the life of the plan.
 *   - The library allocates no device memory: all state lives in the
 *     caller's workspace (size from cpd_workspace_size).  It creates one
 *     private HIP stream per plan for graph capture.
 *   - Work is enqueued on desc.stream; calls return without synchronising
 *     unless their comment says otherwise.
 *   - Errors are returned as negative cpd_status codes; nothing aborts and
 *     no C++ exception crosses the ABI.  Arguments are validated before any
 *     launch.  Device-side conditions (non-SPD normal matrix, non-finite
 *     fit) are latched in device flags and reported by the next call that
 *     synchronises (cpd_sweep with outputs, cpd_fit, cpd_stats).
 */
#ifndef THCCP_H
#define THCCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cpd_status;
enum {
  CPD_OK = 0,
  CPD_ERR_INVALID_ARG = -1, /* bad sizes, null pointers, unsupported option  */
  CPD_ERR_HIP = -2,         /* a HIP runtime call failed                      */
  CPD_ERR_NOT_SPD = -3,     /* normal matrix not positive definite (after the
                               damped retry, if enabled)                      */
  CPD_ERR_NONFINITE = -4,   /* NaN/Inf reached the fit or ||G||^2 <= 0        */
  CPD_ERR_WORKSPACE = -5,   /* workspace missing or smaller than required     */
  CPD_ERR_UNSUPPORTED = -6  /* option not available in this build             */
};

typedef enum {
  CPD_FP64 = 0,       /* every step in FP64 (matrix cores, 16x16x4 f64)        */
  CPD_FP32 = 1,       /* every step, including the Cholesky, in FP32;
                         scalar fit terms accumulate in FP64                  */
  CPD_MIXED_BF16 = 2  /* projection, core and back-projection products in
                         split BF16 (hi + lo, one correction pass) with FP32
                         accumulation; Gram, Cholesky, solve and fit in FP64.
                         A precision guard moves a problem to FP64 products
                         when its normal matrices become ill-conditioned;
                         synchronised sweeps that promote are replayed     */
} cpd_precision;

typedef struct cpd_plan_s* cpd_plan;

typedef struct {
  int32_t n[4];           /* mode sizes n_m (> 0)                                  */
  int32_t r_thc;          /* THC rank R_thc (> 0)                                  */
  int32_t r_cp;           /* CP rank R_cp (> 0)                                    */
  const double* X[4];     /* DEVICE n[m] x r_thc THC factors; may alias each other */
  const double* Z;        /* DEVICE r_thc x r_thc THC core (general; Z^T is used
                             for modes 2 and 3)                                   */
  const double* init[4];  /* DEVICE n[m] x r_cp initial factors (required); their
                             columns are normalised to unit 2-norm at init        */
  int32_t precision;      /* cpd_precision                                        */
  double tol;             /* stop when |f_k - f_{k-1}| <= tol f_{k-1}             */
  double fit_floor;       /* ... or when f_k <= fit_floor (0 disables)            */
  int32_t chol_fallback;  /* 1: one damped retry V + mu I, mu = 1e-12 tr(V)/R_cp,
                             on a non-positive pivot; 0: fail with NOT_SPD       */
  int32_t use_graph;      /* 1: replay each sweep as a captured hipGraph          */
  int32_t fit_every;      /* CPD_MIXED_BF16 only: evaluate the fit (in FP64, with
                             an FP64 mode-3 MTTKRP) and the stopping rule every
                             fit_every sweeps (<= 1: every sweep); other
                             precisions evaluate it every sweep               */
  int32_t autotune;       /* 1: time both GEMM tile shapes of every grouped
                             FP64/FP32 product at init and keep the faster
                             (cached per process by shape); 0: heuristic      */
  void* stream;           /* hipStream_t the work is ordered on (0 = null stream) */
  void* workspace;        /* DEVICE memory owned by the caller                    */
  size_t workspace_bytes;
} cpd_desc;

typedef struct {
  int32_t sweeps;         /* sweeps completed since init / set_factors            */
  int32_t converged;      /* the stopping rule fired                              */
  int32_t fallbacks;      /* damped Cholesky retries so far                       */
  int32_t flags;          /* device status bits (1 = not SPD, 2 = non-finite)     */
  double fit;             /* last fit (relative residual), -1 before any sweep    */
  double norm2;           /* ||G||^2                                              */
  double inner;           /* <G, G~> of the last sweep                            */
  double model2;          /* ||G~||^2 of the last sweep                           */
  double cond_est;        /* (max_i L_ii / min_i L_ii)^2 of the last factor       */
  int32_t fp64_path;      /* CPD_MIXED_BF16: 1 once the precision guard moved the
                             problem to the FP64 MTTKRP (cond estimate > 1e5, a
                             damped retry, or a rising fit)                   */
  int32_t reserved;
} cpd_stats_t;

/* Bytes of device workspace cpd_init needs for this descriptor (0 on
 * invalid arguments).  Host-only; launches nothing. */
size_t cpd_workspace_size(const cpd_desc* d);

/* Set-up (eq. lossF and the fit of Computational Details): validates d,
 * carves the workspace, computes S_m = X_m^T X_m and ||G||^2 =
 * <Z, (S0 o S1) Z (S2 o S3)>, copies and normalises the initial factors,
 * forms the projections W_m and the Gram matrices, and (use_graph) captures
 * one sweep as a hipGraph.  Asynchronous on d->stream.  *out receives a
 * host-side plan to be released with cpd_destroy. */
cpd_status cpd_init(const cpd_desc* d, cpd_plan* out);

/* Runs up to nsweeps ALS sweeps (modes 0,1,2,3 in order, then the fit and
 * the stopping rule).  Sweeps after convergence are no-ops on the device.
 * If fits_host or n_run is non-NULL the call synchronises after every sweep,
 * stops at convergence, writes the fit of each sweep run to fits_host
 * (length >= nsweeps) and the number of sweeps run to *n_run; otherwise it
 * only enqueues the work. */
cpd_status cpd_sweep(cpd_plan p, int32_t nsweeps, double* fits_host, int32_t* n_run);

/* Synchronises the plan's stream and returns the last fit (-1 if none). */
cpd_status cpd_fit(cpd_plan p, double* fit_host);

/* Copies the current factors (DEVICE n[m] x r_cp each, dense) and the
 * weights lambda (DEVICE r_cp) out; async.  Any pointer may be NULL. */
cpd_status cpd_get_factors(cpd_plan p, double* const F_dev[4], double* lambda_dev);

/* Restores factors and weights written by cpd_get_factors (checkpoint
 * resume): recomputes the projections and Grams from them and sets the
 * previous fit used by the stopping rule to prev_fit (< 0: none) and the
 * sweep counter to sweeps.  Async. */
cpd_status cpd_set_factors(cpd_plan p, const double* const F_dev[4], const double* lambda_dev,
                           double prev_fit, int32_t sweeps);

/* Synchronises and fills *out. */
cpd_status cpd_stats(cpd_plan p, cpd_stats_t* out);

/* Test hook: the matrix-free MTTKRP of `mode` from the current factors,
 * M = G_(mode) (Khatri-Rao of the other factors), into DEVICE
 * n[mode] x r_cp (dense).  Needs a plan that has not converged (the
 * grouped kernels skip converged problems).  Async. */
cpd_status cpd_mttkrp(cpd_plan p, int32_t mode, double* M_dev);

/* Measurement hook: average device time (ms, hipEvents on the plan's
 * stream, `reps` back-to-back repetitions after one warm-up) of each kernel
 * family of the sweep at the plan's shapes, for mode 0 (ms_out: 7 doubles):
 *   [0] projection X^T F,  [1] core product Z (W o W),
 *   [2] back-projection X (W o Y),  [3] Gram F^T F,
 *   [4] whole normal-equation solve (V, factorisation fused with the
 *       forward triangular solve, backward solve, normalisation),
 *   [5] V + factorisation/forward solve (nblk + 1 launches of the fused
 *       step kernel), [6] backward solve (nblk launches),
 *   with nblk = ceil(r_cp / 64).
 * Overwrites the plan's intermediate buffers and resets its stopping state:
 * re-initialise the plan before using it again.  Synchronises. */
cpd_status cpd_kernel_times(cpd_plan p, int32_t reps, double* ms_out);

/* ---- batched form (many independent CPDs of uneven size, e.g. one per
 * Laplace-transform point, Section 2.2: the LT-MP2 energy is a sum of
 * independent terms over the quadrature points) ----
 * All problems must use the same precision; tol, fit_floor, chol_fallback,
 * use_graph, fit_every, autotune and stream are taken from descs[0]; the
 * workspace is passed separately (descs[i].workspace is ignored).  Every
 * step of a sweep is one grouped launch over all problems, and a sweep is
 * one hipGraph launch.  Converged problems become no-ops while the others
 * continue. */
size_t cpd_batch_workspace_size(const cpd_desc* descs, int32_t count);
cpd_status cpd_batch_init(const cpd_desc* descs, int32_t count, void* workspace, size_t workspace_bytes,
                          cpd_plan* out);
/* Like cpd_sweep; fits_host (if non-NULL) is count x nsweeps, row-major by
 * problem (-1 where a fit was not evaluated or the problem had stopped);
 * stops early once every problem has converged. */
cpd_status cpd_batch_sweep(cpd_plan p, int32_t nsweeps, double* fits_host, int32_t* n_run);
/* Synchronises; per problem: last fit, converged flag, sweeps (any may be NULL). */
cpd_status cpd_batch_states(cpd_plan p, double* fits_host, int32_t* converged_host, int32_t* sweeps_host);
int32_t cpd_batch_count(cpd_plan p);
cpd_status cpd_batch_get_factors(cpd_plan p, int32_t idx, double* const F_dev[4], double* lambda_dev);
cpd_status cpd_batch_stats(cpd_plan p, int32_t idx, cpd_stats_t* out);
/* Autotuner decisions of the plan as "kind,M,N,K,...=tile" lines into buf
 * (NUL-terminated, truncated to len); returns the full length. */
int32_t cpd_autotune_log(cpd_plan p, char* buf, int32_t len);
/* Laplace-transform row scaling of THC factors (eq. mp1_t and the THC-LT
 * amplitude after it): out[p, :] = exp(sign * eps[p] * t) * X[p, :] for
 * X DEVICE n x r (row-major), eps DEVICE n; sign = +1 for occupied rows,
 * -1 for virtual rows.  Async on stream. */
cpd_status cpd_lt_scale_rows(const double* X, const double* eps, int32_t n, int32_t r, double t, double sign,
                             double* out, void* stream);

/* Releases the host plan and its private stream/graph (not the workspace). */
cpd_status cpd_destroy(cpd_plan p);

const char* cpd_status_string(cpd_status s);

/* ---- kernel-level test hooks (all pointers DEVICE, dense row-major) ----
 * cpd_test_gemm: C (M x N) = op(A) op(B1 [o B2]) on the FP64 (fp32 = 0) or
 *   FP32 (fp32 = 1) matrix cores.  a_t: A is stored K x M (lda); b_t: B is
 *   stored N x K (ldb); B2 (same layout as B1, b_t = 0 only) multiplies B1
 *   element-wise.  Async on stream. */
cpd_status cpd_test_gemm(int32_t fp32, int32_t M, int32_t N, int32_t K, const void* A, int32_t lda,
                         int32_t a_t, const void* B1, const void* B2, int32_t ldb, int32_t b_t, void* C,
                         int32_t ldc, void* stream);
/* cpd_test_solve: F (n x R) = M V^{-1} for SPD V (R x R) by the blocked
 *   Cholesky and triangular solves of the sweep (no damped retry).  Sync;
 *   returns CPD_ERR_NOT_SPD (and *failed = 1) on a non-positive pivot. */
size_t cpd_test_solve_workspace(int32_t fp32, int32_t R, int32_t n);
cpd_status cpd_test_solve(int32_t fp32, int32_t R, int32_t n, const void* V, const void* M, void* F,
                          void* workspace, size_t ws_bytes, void* stream, int32_t* failed);
/* cpd_test_gemm_split: C (M x N, FP64) = A B^T from FP64 A (M x K) and
 *   B (N x K) through the split-BF16 product (hi*hi + hi*lo + lo*hi, FP32
 *   accumulation).  With A2 != NULL the A operand is the FP32 product
 *   A o A2, split on the fly.  Uploads a one-entry argument table and
 *   synchronises before the launch. */
size_t cpd_test_split_workspace(int32_t M, int32_t N, int32_t K);
cpd_status cpd_test_gemm_split(int32_t M, int32_t N, int32_t K, const double* A, const double* A2,
                               const double* B, double* C, void* workspace, size_t ws_bytes, void* stream);
/* cpd_test_mfma_probe: lane-layout probe of the 16x16x4 FP64 (fp32 = 0) or
 *   FP32 matrix instruction.  Probe p (of nprobe) feeds a[64p + lane] and
 *   b[64p + lane] to one wave with a zero accumulator and writes the four
 *   result registers to d[256p + 4 lane + r].  Async on stream. */
cpd_status cpd_test_mfma_probe(int32_t fp32, int32_t nprobe, const void* a, const void* b, void* d,
                               void* stream);

#ifdef __cplusplus
}
#endif
#endif /* THCCP_H */
