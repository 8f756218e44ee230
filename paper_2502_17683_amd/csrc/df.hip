// Density-fitting (DF) tensors in THC form (eq. df_loss, eq. THC).
//
// A DF tensor G[p,q,r,s] = sum_X B[(p,q),X] B[(r,s),X] is exactly a THC
// tensor whose grid index runs over the orbital pairs P = (p', q'):
//   X0[p, P] = [p = p'],  X1[q, P] = [q = q'],  X2 = X0,  X3 = X1,
//   Z = B B^T  ((n n) x (n n)).
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

}  // namespace
}  // namespace thccp

using namespace thccp;

extern "C" {

cpd_status cpd_df_to_thc(int32_t n, int32_t n_aux, const double* B, double* X0, double* X1, double* Z,
                         void* stream) {
  // the THC rank n^2 must stay within the CP-ALS limit (2^20)
  if (n <= 0 || n > 1024 || n_aux <= 0 || !B || !X0 || !X1 || !Z) return CPD_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
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
