// Exact ridge leverage scores  tau_c = (K (K + lambda I)^-1)_cc = 1 - lambda [(K + lambda I)^-1]_cc
// (section 3, "Leverage score sampling"), from a dense FP64 factorization on
// the GPU: assemble K + lambda I column by column, Cholesky K_lambda = F F^T,
// invert F in place, and use [(K_lambda)^-1]_cc = |F^-1 e_c|^2 (column norms of
// F^-1).  Costs n^3/3 + n^3/3 flops and 8 n^2 bytes; meant for the training
// labels of the score network on moderate n.
#include "common.hpp"

namespace ffk {

__global__ void k_iota(int64_t* a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = i;
}

// tau_c = 1 - lambda sum_{r >= c} X[r + c n]^2   (one wave per column)
__global__ __launch_bounds__(256) void k_rls_from_inverse(const double* X, int64_t n, double lambda, double* tau) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  const double* col = X + c * n;
  double a = 0.0;
  for (int64_t r = c + lane; r < n; r += 64) a += col[r] * col[r];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  if (lane == 0) tau[c] = 1.0 - lambda * a;
}

void exact_rls(ffk_system* s, double lambda, double* tau, hipStream_t st) {
  const int64_t n = s->n;
  size_t freeb = 0, total = 0;
  HIPCHK(hipMemGetInfo(&freeb, &total));
  require((double)n * n * 8.0 < 0.9 * (double)freeb, "exact_rls: dense n x n matrix does not fit in device memory");
  DBuf A((size_t)n * n * 8), cols(n * 8);
  k_iota<<<cdiv(n, 256), 256, 0, st>>>(cols.as<int64_t>(), n);
  LAUNCHCHK();
  const int64_t chunk = 8192;
  for (int64_t c0 = 0; c0 < n; c0 += chunk) {
    const int64_t kc = std::min(chunk, n - c0);
    kernel_columns(s, cols.as<int64_t>() + c0, kc, A.as<double>() + c0 * n, n, lambda, st);
  }
  const int64_t bad = potrf_lower(A.as<double>(), n, n, st);
  if (bad >= 0) fail(FFK_ERR_NOT_SPD, "exact_rls: K + lambda I is not numerically positive definite");
  trtri_lower(A.as<double>(), n, n, st);
  k_rls_from_inverse<<<cdiv(n, 4), 256, 0, st>>>(A.as<double>(), n, lambda, tau);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));
}

}  // namespace ffk
