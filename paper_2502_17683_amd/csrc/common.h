// Shared device-side definitions for the THC CP-ALS kernels (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

#define WAVE 64

// Pointers read from argument tables in memory are generic (flat) to the
// compiler, and flat loads and stores count against the LDS wait counter
// too, so a prefetch into registers would be waited on at the next LDS
// access.  Kernels convert such pointers once to the global address space.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)p;
}

// Device-side status flags written by kernels and read back by the host
// at synchronisation points.
enum {
  FLAG_NOT_SPD = 1,      // a Cholesky pivot was <= 0 or not finite
  FLAG_NONFINITE = 2,    // a non-finite value reached the fit
  FLAG_SOLVE_STALL = 4,  // a wait of the dataflow solve passed its spin limit
};

// Per-plan device state (lives in the caller's workspace).
struct DevState {
  double norm2;          // ||G||^2
  double fit_prev;       // fit of the previous sweep (-1 before the first)
  double inner;          // <G, G~> of the last sweep
  double model2;         // ||G~||^2 of the last sweep
  double mu;             // damping shift used by the retry (diagnostic)
  int32_t done;          // set once the stopping rule fired: sweeps become no-ops
  int32_t sweeps;        // sweeps completed
  int32_t flags;         // sticky FLAG_* bits
  int32_t chol_fail;     // current factorisation hit a bad pivot
  int32_t fallbacks;     // number of damped retries
  int32_t retry_active;  // retry pass armed for the current mode
  int32_t path;          // split-BF16 plans: 0 = split-BF16 MTTKRP, 1 = promoted to FP64
  int32_t promote;       // set by the precision guard in the sweep that promoted
  int32_t fallbacks_start;  // fallbacks at the start of the sweep
  double cond_max;       // largest (max L_ii / min L_ii)^2 seen in the sweep
  double fit_rule;       // fit at the last sweep the stopping rule looked at (-1: none)
  double fit_target;     // stop once a fit is at or below this (0: off)
};

// Tile (tm, tn) of linear index bid in groups of G tile rows: a group runs
// column by column over its G rows, so consecutive indices -- the tiles an
// XCD runs at the same time after xcd_remap -- form a roughly square block
// that shares its A and B panels in the XCD's L2.
__device__ __forceinline__ void grouped_tile(int bid, int tiles_m, int tiles_n, int G, int& tm, int& tn) {
  const int per_group = G * tiles_n;
  const int first = (bid / per_group) * G;
  const int gm = tiles_m - first < G ? tiles_m - first : G;
  const int in = bid - (bid / per_group) * per_group;
  tm = first + in % gm;
  tn = in / gm;
}

__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of tiles so neighbouring tiles share its L2.
  const int nx = 8;
  if (nblocks < 2 * nx) return bid;
  int per = nblocks / nx;
  int rem = nblocks - per * nx;
  int x = bid % nx;
  int j = bid / nx;
  if (j >= per) return per * nx + x;  // tail: blocks beyond the even split
  (void)rem;
  return x * per + j;
}
