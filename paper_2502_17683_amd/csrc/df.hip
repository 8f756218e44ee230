// Density-fitting (DF) tensors in THC form (eq. df_loss, eq. THC).
//
// A DF tensor G[p,q,r,s] = sum_X B[(p,q),X] B[(r,s),X] is exactly a THC
// tensor whose grid index runs over the orbital pairs P = (p', q'):
//   X0[p, P] = [p = p'],  X1[q, P] = [q = q'],  X2 = X0,  X3 = X1,
//   Z = B B^T  ((n n) x (n n)).
// and ||G||^2 = ||B^T B||_F^2 (which spares the CP-ALS set-up its
// O(R_thc^3) = O(n^6) products).
// With these inputs the matrix-free CP-ALS of the library is the CP-ALS on
// the DF loss; its products then cost O(n^4 R_cp) per sweep, the scaling
// the paper gives for the DF variant, where a THC rank proportional to n
// gives O(n^3 R_cp).
#include <stdint.h>

#include "../../include/thccp.h"
#include "common.h"
#include "kernels.h"

namespace thccp {
namespace {

// X0[p, P] = [P / n = p], X1[q, P] = [P % n = q]; blockIdx.y selects X0 / X1.
__global__ __launch_bounds__(256) void pair_selection_kernel(int n, double* X0, double* X1) {
  const size_t nn = (size_t)n * n, total = (size_t)n * nn;
  auto out = as_global(blockIdx.y ? X1 : X0);
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const size_t row = e / nn, P = e - row * nn;
    const size_t idx = blockIdx.y ? P % n : P / n;
    out[e] = idx == row ? 1.0 : 0.0;
  }
}

// out = sum of the squares of S (count values), one workgroup, fixed order.
__global__ __launch_bounds__(256) void sum_squares_kernel(const double* S, size_t count, double* out) {
  __shared__ double part[256];
  double acc = 0.0;
  for (size_t e = threadIdx.x; e < count; e += 256) {
    const double v = as_global(S)[e];
    acc += v * v;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) as_global(out)[0] = part[0];
}

}  // namespace
}  // namespace thccp

using namespace thccp;

extern "C" {

cpd_status cpd_df_to_thc(int32_t n, int32_t n_aux, const double* B, double* X0, double* X1, double* Z,
                         double* norm2, void* stream) {
  // the THC rank n^2 must stay within the CP-ALS limit (2^20)
  if (n <= 0 || n > 1024 || n_aux <= 0 || (int64_t)n_aux > (int64_t)n * n || !B || !X0 || !X1 || !Z)
    return CPD_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (norm2) {
    // ||G||^2 = ||B^T B||_F^2; B^T B (n_aux^2 <= n^4 values) is staged in Z
    // before Z itself is formed
    GemmF64 g{n_aux, n_aux, n * n, B, n_aux, true, B, nullptr, n_aux, false, Z, n_aux, nullptr, 1.0, 0.0,
              nullptr};
    gemm_f64(s, g);
    hipLaunchKernelGGL(sum_squares_kernel, dim3(1), dim3(256), 0, s, Z, (size_t)n_aux * n_aux, norm2);
  }
  const size_t total = (size_t)n * n * n;
  int grid = (int)((total + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(pair_selection_kernel, dim3(grid, 2), dim3(256), 0, s, n, X0, X1);
  const int nn = n * n;
  // Z = B B^T
  GemmF64 g{nn, nn, n_aux, B, n_aux, false, B, nullptr, n_aux, true, Z, nn, nullptr, 1.0, 0.0, nullptr};
  gemm_f64(s, g);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

}  // extern "C"
