// Deterministic FP64 reductions: a fixed grid of at most kRedParts blocks
// writes one partial each, a single block combines them in a fixed order, so
// results are bitwise reproducible from run to run.
#include "common.hpp"

namespace ffk {

template <int OP>   // 0: dot, 1: max
__global__ __launch_bounds__(256) void k_red_part(const double* __restrict__ a, const double* __restrict__ b,
                                                  int64_t n, double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = OP == 0 ? 0.0 : -INFINITY;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    if (OP == 0) acc += a[e] * b[e];
    else acc = fmax(acc, a[e]);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = OP == 0 ? sh[threadIdx.x] + sh[threadIdx.x + o]
                                                  : fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

template <int OP>
__global__ __launch_bounds__(256) void k_red_final(const double* __restrict__ part, int np, double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = OP == 0 ? 0.0 : -INFINITY;
  for (int e = threadIdx.x; e < np; e += 256) acc = OP == 0 ? acc + part[e] : fmax(acc, part[e]);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = OP == 0 ? sh[threadIdx.x] + sh[threadIdx.x + o]
                                                  : fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

static int nparts(int64_t n) {
  int64_t b = (n + 2047) / 2048;
  if (b < 1) b = 1;
  if (b > kRedParts) b = kRedParts;
  return (int)b;
}

int dot64_parts(const double* a, const double* b, int64_t n, double* part, hipStream_t st) {
  const int np = nparts(n);
  k_red_part<0><<<np, 256, 0, st>>>(a, b, n, part);
  LAUNCHCHK();
  return np;
}

void dot64(const double* a, const double* b, int64_t n, double* part, double* out, hipStream_t st) {
  const int np = nparts(n);
  k_red_part<0><<<np, 256, 0, st>>>(a, b, n, part);
  LAUNCHCHK();
  k_red_final<0><<<1, 256, 0, st>>>(part, np, out);
  LAUNCHCHK();
}

int fused_parts(int64_t n) {
  int64_t b = (n + 511) / 512;
  if (b < 1) b = 1;
  if (b > kRedParts) b = kRedParts;
  return (int)b;
}

void sum_parts64(const double* part, int np, double* out, hipStream_t st) {
  k_red_final<0><<<1, 256, 0, st>>>(part, np, out);
  LAUNCHCHK();
}

void reduce_max64(const double* a, int64_t n, double* part, double* out, hipStream_t st) {
  const int np = nparts(n);
  k_red_part<1><<<np, 256, 0, st>>>(a, nullptr, n, part);
  LAUNCHCHK();
  k_red_final<1><<<1, 256, 0, st>>>(part, np, out);
  LAUNCHCHK();
}

}  // namespace ffk
