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
  CPD_ERR_HIP = -2,         /* a HIP runtime call failed, or a wait of the
                               dataflow factorisation/solves gave up (the
                               device made no progress; the plan needs
                               cpd_init / cpd_batch_init again)              */
  CPD_ERR_NOT_SPD = -3,     /* normal matrix not positive definite (after the
                               damped retry, if enabled)                      */
  CPD_ERR_NONFINITE = -4,   /* NaN/Inf reached the fit or ||G||^2 <= 0        */
  CPD_ERR_WORKSPACE = -5,   /* workspace missing or smaller than required     */
  CPD_ERR_UNSUPPORTED = -6  /* option the library does not support           */
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
  double tol;             /* stop when |f_k - f_{k-fit_every}| <= tol f_{k-fit_every}
                             (Computational Details: relative change in fit) */
  double fit_floor;       /* ... or when f_k <= fit_floor (0 disables)            */
  int32_t chol_fallback;  /* 1: one damped retry V + mu I, mu = 1e-12 tr(V)/R_cp,
                             on a non-positive pivot; 0: fail with NOT_SPD       */
  int32_t use_graph;      /* 1: replay each sweep as a captured hipGraph          */
  int32_t fit_every;      /* cadence k of the stopping rule (<= 1: every sweep):
                             the rule is looked at after sweeps k, 2k, ... and
                             compares the fit with the fit k sweeps earlier, in
                             every precision.  CPD_MIXED_BF16 also evaluates
                             the fit itself (in FP64, with an FP64 mode-3
                             MTTKRP) only on those sweeps; FP64 and FP32
                             evaluate it every sweep                          */
  int32_t autotune;       /* 1: time the candidate launch shapes of every
                             grouped product at init and keep the fastest
                             (cached per process by shape): FP64/FP32 tile
                             edges 64/128; split BF16 128-column tiles of 64
                             or 128 rows, or 128/256 x 256 tiles, the
                             back-projection also with 2 or 4 K slices;
                             0: heuristic                                   */
  int32_t solve_panel;    /* blocked Cholesky and triangular solves: 0 = one
                             level (each 64-wide step updates the whole
                             trailing matrix); k >= 1 = panels of k 64-wide
                             blocks, the trailing matrix updated once per
                             panel by a rank-64k GEMM                       */
  void* stream;           /* hipStream_t the work is ordered on (0 = null stream) */
  void* workspace;        /* DEVICE memory owned by the caller                    */
  size_t workspace_bytes;
  int32_t tied;           /* 1: particle-tied model (eq. cp4: one factor for both
                             indices of a particle), F1 = F0 and F3 = F2, fitted by
                             symmetric ALS: each sweep updates modes 0 and 2 by
                             their normal equations with the tied copy held, then
                             copies them to modes 1 and 3.  Needs n[1] = n[0] and
                             n[3] = n[2]; init[1] and init[3] are not read.
                             FP64 and FP32 only (split BF16: UNSUPPORTED).  Every
                             problem of a batch must agree.  0: four factors  */
  const double* norm2;    /* optional DEVICE pointer to ||G||^2, read at init;
                             NULL: computed from X and Z, which costs
                             O(r_thc^3) and three r_thc^2 buffers (supply it
                             for the DF form, where r_thc = n^2)              */
  double fit_target;      /* stop the problem once an evaluated fit is at or
                             below fit_target (time to a given fit; per
                             problem in a batch); 0: off                     */
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

/* Runs up to nsweeps ALS sweeps (Section 2.1: alternating least squares on
 * eq. lossF; modes 0,1,2,3 in order, each mode update the projection, the
 * core product, the back-projection and the normal-equation solve with
 * V_n = o_{m != n} F_m^T F_m), then the fit and the stopping rule
 * (Computational Details: fit ||T - T~|| / ||T||, relative change in fit
 * below tol).  Sweeps after convergence are no-ops on the device.
 * If fits_host or n_run is non-NULL the call synchronises after every sweep,
 * stops at convergence, writes the fit of each sweep run to fits_host
 * (length >= nsweeps) and the number of sweeps run to *n_run; otherwise it
 * only enqueues the work. */
cpd_status cpd_sweep(cpd_plan p, int32_t nsweeps, double* fits_host, int32_t* n_run);

/* Synchronises the plan's stream and returns the last fit (-1 if none):
 * the paper's ||T - T~|| / ||T|| (Computational Details), computed
 * matrix-free from ||G||^2, <G, G~> and ||G~||^2 (eq. lossF). */
cpd_status cpd_fit(cpd_plan p, double* fit_host);

/* Copies the current factors (DEVICE n[m] x r_cp each, dense) and the
 * weights lambda (DEVICE r_cp) out -- the CPD of eq. cp4 with unit-norm
 * columns; async.  Any pointer may be NULL. */
cpd_status cpd_get_factors(cpd_plan p, double* const F_dev[4], double* lambda_dev);

/* Restores factors and weights written by cpd_get_factors (checkpoint
 * resume of the ALS iteration of Section 2.1, whose state between sweeps
 * is exactly the factors and weights of eq. cp4): recomputes the
 * projections and Grams from them and sets the
 * previous fit used by the stopping rule to prev_fit (< 0: none) and the
 * sweep counter to sweeps.  Async. */
cpd_status cpd_set_factors(cpd_plan p, const double* const F_dev[4], const double* lambda_dev,
                           double prev_fit, int32_t sweeps);

/* Synchronises and fills *out: sweep count, stopping state, the fit and
 * its terms ||G||^2, <G, G~>, ||G~||^2 (Computational Details; eq. lossF),
 * damped retries of the Cholesky of V_n and its condition estimate. */
cpd_status cpd_stats(cpd_plan p, cpd_stats_t* out);

/* Test hook: the matrix-free MTTKRP of `mode` from the current factors,
 * M = G_(mode) (Khatri-Rao of the other factors), into DEVICE
 * n[mode] x r_cp (dense).  Needs a plan that has not converged (the
 * grouped kernels skip converged problems).  Async. */
cpd_status cpd_mttkrp(cpd_plan p, int32_t mode, double* M_dev);

/* Measurement hook: average device time (ms, hipEvents on the plan's
 * stream, `reps` back-to-back repetitions after one warm-up) of each kernel
 * family of the sweep at the plan's shapes, for mode 0 (ms_out: 8 doubles):
 *   [0] projection X^T F,  [1] core product Z (W o W),
 *   [2] back-projection X (W o Y),  [3] Gram F^T F (lower triangle),
 *   [4] whole normal-equation solve (V, factorisation fused with the
 *       forward triangular solve, backward solve, normalisation),
 *   [5] V + factorisation/forward solve, [6] backward solve,
 *   [7] V alone (the Hadamard product of the Grams).
 *   For a one-level solve (r_cp up to the panel threshold) the
 *   factorisation/forward solve and the backward solve are one dataflow
 *   launch each, after a flag reset.
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
/* Autotuner decisions of the plan as "kind,M,N,K,...=shape" lines into buf
 * (NUL-terminated, truncated to len); returns the full length.  FP64/FP32
 * kinds: shape = tile edge; split-BF16 kinds (bf16core, bf16back, bf16proj):
 * shape = bm + 1000 (bm x 256 tiles) + 10000 kparts, or 100000 + 10000 kparts
 * for the 256 x 256 direct-load tiles of blocked operands. */
int32_t cpd_autotune_log(cpd_plan p, char* buf, int32_t len);
/* Laplace-transform row scaling of THC factors (eq. mp1_t and the THC-LT
 * amplitude after it): out[p, :] = exp(sign * eps[p] * t) * X[p, :] for
 * X DEVICE n x r (row-major), eps DEVICE n; sign = +1 for occupied rows,
 * -1 for virtual rows.  Async on stream. */
cpd_status cpd_lt_scale_rows(const double* X, const double* eps, int32_t n, int32_t r, double t, double sign,
                             double* out, void* stream);

/* ---- robust CPD+THC LT-MP2 exchange energy (Section 2.2) ----
 * One system, n_points Laplace points (t_k, w_k).  Tensors are in the
 * (i, a, j, b) mode order: the THC (ia|jb) = sum_PQ X_occ[i,P] X_virt[a,P]
 * Z[P,Q] X_occ[j,Q] X_virt[b,Q] (eq. THC) and its CPD
 * sum_r lam[r] F0[i,r] F1[a,r] F2[j,r] F3[b,r] (eq. cp4).  With the
 * exchange pairing K(T, S) = sum_{iajb} T[i,a,j,b] S[i,b,j,a] and the
 * Laplace factor exp(-(e_a + e_b - e_i - e_j) t_k) (eq. lt_D, eq. mp1_t):
 *   k_single[k] = K(THC scaled at t_k, CPD)         (eq. cpd_single_k)
 *   k_double[k] = K(CPD scaled at t_k, CPD)         (the double-CPD term)
 *   e_k[0]      = - sum_k w_k (2 k_single[k] - k_double[k])   (eq. rob_K)
 * The amplitude carries the whole factor w_k exp(-D t_k); the double-CPD
 * term pairs each occupied index with its own particle's factor (the
 * definition of g^{ba}_{ij}), so an exact CPD reproduces the exact
 * exchange energy.  By default the CPD of the scaled tensor is the
 * LT-scaled bare CPD (its rows scaled like the THC factors); then the
 * robust energy's error is second order in the CPD error.  With E_host,
 * separate CPDs of the scaled tensors (for instance the batched per-point
 * CPDs of cpd_batch_*) take that place in k_double.
 *   X_occ n_occ x r_thc, X_virt n_virt x r_thc, Z r_thc x r_thc (any Z; no
 *   symmetry is assumed), eps_occ n_occ, eps_virt n_virt, F0/F2
 *   n_occ x r_cp, F1/F3 n_virt x r_cp, lam r_cp (NULL: all ones): DEVICE,
 *   row-major, borrowed for the call.  t_host, w_host: HOST arrays of
 *   n_points finite values, read before the call returns.
 *   E_host: NULL, or a HOST array of 4 n_points DEVICE pointers, entry
 *   4k + m the mode-m factor (n_occ or n_virt x r_cp, modes i, a, j, b) of
 *   point k's CPD; lam_e_host: NULL (all ones) or a HOST array of n_points
 *   DEVICE pointers to their weights (an entry may be NULL: ones).
 *   k_single, k_double (n_points each) and e_k (1): DEVICE outputs.
 *   1 <= n_points <= CPD_LT_MAX_POINTS; n_points * r_cp must fit int32.
 *   workspace: DEVICE, at least cpd_lt_exchange_workspace(...,
 *   per_point_cpds = E_host != NULL) bytes, 256-byte aligned; holds the
 *   scaled factor stacks and the products of every point (about
 *   8 (2 n_occ + 2 n_virt + 5 r_thc + 3 r_cp) n_points r_cp bytes, plus
 *   8 (2 n_occ + 2 n_virt + r_cp + 1) n_points r_cp with per-point CPDs).
 * Errors: CPD_ERR_INVALID_ARG (sizes, NULL pointers, non-finite t or w),
 * CPD_ERR_WORKSPACE, CPD_ERR_HIP (launch failure).  Async on stream; the
 * result is bitwise reproducible (fixed-order reductions). */
#define CPD_LT_MAX_POINTS 64
size_t cpd_lt_exchange_workspace(int32_t n_occ, int32_t n_virt, int32_t r_thc, int32_t r_cp, int32_t n_points,
                                 int32_t per_point_cpds);
cpd_status cpd_lt_exchange(int32_t n_occ, int32_t n_virt, int32_t r_thc, int32_t r_cp, int32_t n_points,
                           const double* X_occ, const double* X_virt, const double* Z, const double* eps_occ,
                           const double* eps_virt, const double* t_host, const double* w_host, const double* F0,
                           const double* F1, const double* F2, const double* F3, const double* lam,
                           const double* const* E_host, const double* const* lam_e_host, double* k_single,
                           double* k_double, double* e_k, void* workspace, size_t workspace_bytes,
                           void* stream);

/* ---- THC LT-MP2 Coulomb and exchange terms and energy (Section 2.2) ----
 * Same tensors, mode order and Laplace factor as cpd_lt_exchange, with the
 * THC tensor on both sides:
 *   J[k] = sum_{iajb} exp(-D t_k) G[i,a,j,b] G[i,a,j,b]      (eq. thc_Ej)
 *   K[k] = sum_{iajb} exp(-D t_k) G[i,a,j,b] G[i,b,j,a]      (eq. thc_Ek)
 *   energies[0] = E_J = 2 sum_k w_k J[k]
 *   energies[1] = E_K = - sum_k w_k K[k]   (0 when thc_exchange = 0)
 *   energies[2] = E_J + E_K                                 (eq. LT-Emp2)
 * J costs O(n_points r_thc^3) through the grid overlaps and two (one with
 * z_symmetric = 1) wide products with Z.  K (thc_exchange = 1) forms the
 * (o v) x (o v) matrix (ia|jb) from the THC factors: O(o^2 v^2 r_thc) flops
 * and up to 16 (o v)^2 bytes of workspace, the cost the robust CPD+THC exchange
 * (cpd_lt_exchange) avoids.  The CPD+THC energy is E_J + cpd_lt_exchange's
 * e_k.
 *   X_occ, X_virt, Z, eps_occ, eps_virt: DEVICE, as for cpd_lt_exchange.
 *   z_symmetric = 1 asserts Z = Z^T (true of a THC core of the symmetric
 *   (ia|jb)); the Coulomb term then needs one product instead of two, and
 *   the exchange term forms only the blocks i >= j of (ia|jb) (about half
 *   the flops).  A non-symmetric Z with z_symmetric = 1 gives wrong
 *   results.
 *   t_host, w_host: HOST, n_points finite values.
 *   J, K (n_points each; K may be NULL when thc_exchange = 0), energies (3):
 *   DEVICE outputs.  1 <= n_points <= CPD_LT_MAX_POINTS; with thc_exchange,
 *   o v <= 46340 and o^2 v must fit int32.
 *   workspace: DEVICE, at least cpd_lt_mp2_workspace(...) bytes.
 * Errors: CPD_ERR_INVALID_ARG, CPD_ERR_WORKSPACE, CPD_ERR_HIP.  Async on
 * stream; fixed-order reductions (bitwise reproducible). */
size_t cpd_lt_mp2_workspace(int32_t n_occ, int32_t n_virt, int32_t r_thc, int32_t n_points, int32_t thc_exchange,
                            int32_t z_symmetric);
cpd_status cpd_lt_mp2(int32_t n_occ, int32_t n_virt, int32_t r_thc, int32_t n_points, const double* X_occ,
                      const double* X_virt, const double* Z, const double* eps_occ, const double* eps_virt,
                      const double* t_host, const double* w_host, int32_t thc_exchange, int32_t z_symmetric,
                      double* J, double* K, double* energies, void* workspace, size_t workspace_bytes,
                      void* stream);

/* ---- density-fitting tensors in THC form (eq. df_loss) ----
 * A DF tensor G[p,q,r,s] = sum_X B[(p,q),X] B[(r,s),X] is exactly the THC
 * tensor with the orbital pairs as grid, R_thc = n^2:
 *   X0[p, (p',q')] = [p = p'],  X1[q, (p',q')] = [q = q'],  Z = B B^T,
 * and ||G||^2 = ||B^T B||_F^2.  Passing X = {X0, X1, X0, X1}, Z and norm2
 * with r_thc = n^2 to cpd_init runs the CP-ALS of the DF loss matrix-free,
 * at O(n^4 R_cp) per sweep.
 *   B: DEVICE (n n) x n_aux, row (p, q) = p n + q; n_aux <= n^2.  X0, X1:
 *   DEVICE outputs, n x n^2 each; Z: DEVICE output, n^2 x n^2 (8 n^4
 *   bytes); norm2: DEVICE output, 1 value (may be NULL).  1 <= n <= 1024.
 * Errors: CPD_ERR_INVALID_ARG, CPD_ERR_HIP.  Async on stream. */
cpd_status cpd_df_to_thc(int32_t n, int32_t n_aux, const double* B, double* X0, double* X1, double* Z,
                         double* norm2, void* stream);

/* Releases the host plan and its private stream/graph (not the workspace). */
/* ---- learned warm start ----
 * An initial CP built from R_cp grid columns of the THC factors: with a
 * diagonal core the THC form (eq. THC) is an exact CPD whose columns are
 * X_m[:, P], so a scored selection of grid points, each column scaled, is
 * the starting guess (the paper reports that the sweep count depends
 * strongly on the initial guess, Results).  A network 8 -> 256 -> 256 -> 2
 * (SiLU) maps eight standardised features of each grid point to a
 * selection logit s and a log-scale ell.  Parameters: one FP32 vector of
 * cpd_mlp_param_count() values, W1 (8 x 256, row-major), b1, W2 (256 x 256),
 * b2, W3 (256 x 2), b3.  All pointers are DEVICE memory unless stated;
 * every call is asynchronous on `stream` (a hipStream_t) unless stated,
 * never allocates, and checks its arguments before any launch
 * (CPD_ERR_INVALID_ARG, CPD_ERR_WORKSPACE for a short workspace). */

/* Workspace bytes that cover cpd_ws_features, cpd_ws_labels and cpd_ws_init
 * for a problem with n[0] = n0 (0 on bad sizes; r_cp <= r_thc required). */
size_t cpd_ws_workspace_size(int32_t n0, int32_t r_thc, int32_t r_cp);

/* Features of the r_thc grid points from X0 (n0 x r_thc) and Z (r_thc x
 * r_thc), FP64 row-major, with S = X0^T X0:
 *   0 log Z_PP, 1 log sum_Q |Z_PQ|, 2 log S_PP, 3 log sum_Q S_PQ^2,
 *   4 log max_p |X0_pP|, 5 (sum_p X0_pP^2)^2 / (n0 sum_p X0_pP^4),
 *   6 log sum_Q S_PQ^2 |Z_PQ|, 7 log Z_PP S_PP^2
 * (log v = log max(v, 1e-300)), each standardised over P (population mean
 * and deviation; a feature with deviation <= 1e-9 max(1, |mean|) is 0).
 * feat: r_thc x 8 FP32 row-major.  heur (nullable): r_thc FP64, the raw
 * feature 7, the heuristic ranking score. */
cpd_status cpd_ws_features(int32_t n0, int32_t r_thc, const double* X0, const double* Z, float* feat,
                           double* heur, void* workspace, size_t workspace_bytes, void* stream);

/* cpd_ws_features without a workspace, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops).  Same
 * arguments, results and ordering as cpd_ws_features; its scratch (S and
 * the raw features, 8 r_thc^2 + 64 r_thc bytes) lives in a static device
 * array of the library, one per GPU, which the process holds from the first
 * call on that GPU to its end (33.7 MB).  Limit: r_thc <= 2048 (larger:
 * CPD_ERR_INVALID_ARG).  Calls on the same GPU share the array: calls whose
 * work overlaps on the device (different streams, or threads) race; calls
 * ordered on one stream do not.  The stream must belong to the current
 * device.  No device memory is allocated or freed.  Errors:
 * CPD_ERR_INVALID_ARG, CPD_ERR_HIP (the scratch address could not be
 * looked up, or a launch failed). */
cpd_status cpd_ws_features_noalloc(int32_t n0, int32_t r_thc, const double* X0, const double* Z, float* feat,
                                   double* heur, void* stream);

/* Initial factors from scores: grid points ranked by s (descending; ties:
 * smaller P first); for the top r_cp points P_k
 *   init[m][:, k] = exp(ell[P_k]) (X[m][:, P_k]
 *                   + sigma ||X[m][:, P_k]|| noise[m][:, k] / ||noise[m][:, k]||)
 * (ell NULL: scale 1; noise NULL or sigma = 0: the plain grid columns).
 * noise[m]: n[m] x r_cp FP64, the caller's random guess; it may alias
 * init[m].  The grid columns are positive and overlap strongly, so alone
 * they make a nearly degenerate start; the blend breaks that.  s and ell
 * are FP32 read with `stride` (2 for the network output) and must be
 * finite.  init[m]: n[m] x r_cp FP64.  Workspace: cpd_ws_workspace_size. */
cpd_status cpd_ws_select_init(const int32_t n[4], int32_t r_thc, int32_t r_cp, const double* const X[4],
                              const float* s, const float* ell, int32_t stride, const double* const noise[4],
                              double sigma, double* const init[4], void* workspace, size_t workspace_bytes,
                              void* stream);

/* Training targets from a converged CPD (F[m]: n[m] x r_cp with unit
 * columns, lam: r_cp weights): mode-0 columns matched one-to-one to grid
 * columns by |cosine| with X[0], largest first (ties: smaller k, then
 * smaller P).  For a matched P: y = 1 and ell = mean over m of
 * log |lam_k^(1/4) <F_m[:, k], X_m[:, P]> / ||X_m[:, P]||^2|, mask = 1;
 * all other grid points 0.  y, ell, mask: r_thc FP32. */
cpd_status cpd_ws_labels(const int32_t n[4], int32_t r_thc, int32_t r_cp, const double* const X[4],
                         const double* const F[4], const double* lam, float* y, float* ell, float* mask,
                         void* workspace, size_t workspace_bytes, void* stream);

/* Complete warm start, SYNCHRONOUS: features, then the network (packed
 * weights from cpd_mlp_pack, BF16 inference) and selection blended with
 * noise (as cpd_ws_select_init); if `packed` is NULL or its scores are not
 * finite, the heuristic score (feature 7, FP64) with scale 1; if that is
 * not finite either, init is left as it was (the caller's random guess).
 * *source (host, nullable): 0 network, 1 heuristic, 2 unchanged. */
cpd_status cpd_ws_init(const int32_t n[4], int32_t r_thc, int32_t r_cp, const double* const X[4], const double* Z,
                       const void* packed, const double* const noise[4], double sigma, double* const init[4],
                       int32_t* source, void* workspace, size_t workspace_bytes, void* stream);

int32_t cpd_mlp_param_count(void);
/* Workspace of the training calls for `rows` rows (activations kept from
 * cpd_mlp_forward for cpd_mlp_backward: pass the same workspace). */
size_t cpd_mlp_workspace_size(int32_t rows);

/* FP32 forward over rows x[idx[r]] (idx NULL: x[r]); x: 8 FP32 per row;
 * out: rows x 2 (s, ell). */
cpd_status cpd_mlp_forward(const float* params, const float* x, const int32_t* idx, int32_t rows, float* out,
                           void* workspace, size_t workspace_bytes, void* stream);

/* Loss over the rows of the last forward, targets gathered like x:
 *   L = (1/rows) sum BCE(s, y) + (1/max(1, sum mask)) sum mask (ell - ell_t)^2
 * with BCE(s, y) = max(s, 0) - s y + log(1 + exp(-|s|)).  dout: rows x 2,
 * dL/d(out).  loss_dev (nullable): one FP64. */
cpd_status cpd_mlp_loss(const float* out, const float* y, const float* ell_t, const float* mask,
                        const int32_t* idx, int32_t rows, float* dout, double* loss_dev, void* workspace,
                        size_t workspace_bytes, void* stream);

/* Gradients of the loss with respect to every parameter (same layout as
 * params), from dout and the activations of the last forward. */
cpd_status cpd_mlp_backward(const float* params, const float* x, const int32_t* idx, const float* dout,
                            int32_t rows, float* grads, void* workspace, size_t workspace_bytes, void* stream);

/* One Adam step (Kingma and Ba, bias-corrected; step counts from 1) on all
 * parameters; m and v: moment buffers of the same size, zero at step 1. */
cpd_status cpd_mlp_adam(float* params, const float* grads, float* m, float* v, int32_t step, float lr,
                        float beta1, float beta2, float eps, void* stream);

/* Inference weights: cpd_mlp_packed_size() bytes, 256-byte aligned (W2 in
 * BF16, the rest FP32). */
size_t cpd_mlp_packed_size(void);
cpd_status cpd_mlp_pack(const float* params, void* packed, void* stream);
/* BF16 inference: the 256 x 256 layer on BF16 matrix cores with FP32
 * accumulation, the other layers in FP32.  x: rows x 8, out: rows x 2. */
cpd_status cpd_mlp_infer_bf16(const void* packed, const float* x, int32_t rows, float* out, void* stream);

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
 *   Cholesky and triangular solves of the sweep (no damped retry), with
 *   panels of `panel` blocks (0: one level).  Sync; returns CPD_ERR_NOT_SPD
 *   (and *failed = 1) on a non-positive pivot. */
size_t cpd_test_solve_workspace(int32_t fp32, int32_t R, int32_t n);
/* cpd_test_flow_spin_limit: sets how many polls a wait of the dataflow
 *   factorisation and solves makes before it gives up (negative: restore
 *   the default, 2^20), for launches enqueued afterwards in this process;
 *   returns the previous value.  A wait that gives up makes the whole
 *   problem's launch end early and the call report CPD_ERR_HIP (the plan
 *   needs cpd_init again).  For failure-path tests only: the default never
 *   gives up on a working device.  Not thread-safe. */
int32_t cpd_test_flow_spin_limit(int32_t polls);
/* cpd_test_bwd_form: form of the one-level backward solve for plans and
 *   test solves created afterwards in this process: 0 (default) two block
 *   columns per dependency hop (a set-up launch forms the products of L it
 *   needs into the unused upper blocks of V), 1 one block column per hop.
 *   Any other value selects 0.  Returns the previous value.  For testing
 *   both forms against the same reference.  Not thread-safe. */
int32_t cpd_test_bwd_form(int32_t form);
/* cpd_test_split_force: forces the launch shape of every split-BF16
 *   product of plans created afterwards in this process to the given shape
 *   code (the encoding of cpd_autotune_log; 0 or negative: off, the
 *   heuristic and the autotuner decide again) wherever that shape is
 *   available for the product (direct-load tiles: core product,
 *   back-projection and projection; split-K: back-projection); returns the
 *   previous code.  For tests only.  Not thread-safe with plan creation. */
int32_t cpd_test_split_force(int32_t code);
cpd_status cpd_test_solve(int32_t fp32, int32_t R, int32_t n, const void* V, const void* M, void* F,
                          void* workspace, size_t ws_bytes, void* stream, int32_t* failed, int32_t panel);
/* cpd_test_gemm_split: C (M x N, FP64) = A B^T from FP64 A (M x K) and
 *   B (N x K) through the split-BF16 product (hi*hi + hi*lo + lo*hi, FP32
 *   accumulation).  With A2 != NULL (B2 != NULL) the A (B) operand is the
 *   FP32 product A o A2 (B o B2), split on the fly.  Launch shape: wide = 0:
 *   128-column tiles with bm = 64 or 128 rows (0: the heuristic the sweep
 *   uses), kparts = 1; wide = 1: bm x 256 tiles, bm = 128 or 256, with
 *   kparts = 1..4 K slices (split-K, summed in order by a second launch);
 *   wide = 2: 256 x 256 tiles loaded straight into LDS from pre-split
 *   operands (an operand pair is multiplied and split by a separate pass
 *   first), kparts = 1..4, bm ignored.
 *   Other values return CPD_ERR_INVALID_ARG.  Uploads a one-entry argument
 *   table and synchronises before the launch. */
size_t cpd_test_split_workspace(int32_t M, int32_t N, int32_t K);
cpd_status cpd_test_gemm_split(int32_t M, int32_t N, int32_t K, const double* A, const double* A2,
                               const double* B, const double* B2, double* C, void* workspace, size_t ws_bytes,
                               void* stream, int32_t bm, int32_t wide, int32_t kparts);
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
