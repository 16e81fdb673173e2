// FP64 dense linear algebra on FP64 MFMA: strided GEMM, blocked Cholesky and
// triangular inversion (column-major, lower).  Used for the k x k Woodbury
// core of the preconditioner (Eq. 4), the panel updates of the incomplete
// Cholesky and the dense factorization behind the exact leverage scores.
#include "gemm.hpp"

namespace ffk {

template <int BN, bool AKC, bool BKC>
static void gemm64_t(int M, int N, int K, double alpha, View64 A, View64 B, double beta, double* C, int64_t scm,
                     int64_t scn, bool lower_only, bool a_lower, hipStream_t st) {
  ScalarArgs<double> g{};
  g.M = M;
  g.N = N;
  g.nseg = 1;
  g.seg[0] = SegS<double>{A.p, A.s0, A.s1, B.p, B.s0, B.s1, K};
  g.lower_only = lower_only;
  g.a_lower = a_lower;
  EpiAxpby<double> e{C, scm, scn, M, N, alpha, beta};
  dim3 grid(cdiv(N, BN), cdiv(M, 128));
  gemm_scalar_kernel<double, 128, BN, 16, AKC, BKC, EpiAxpby<double>><<<grid, 256, 0, st>>>(g, e);
  LAUNCHCHK();
}

static void gemm64_dispatch(int M, int N, int K, double alpha, View64 A, View64 B, double beta, double* C,
                            int64_t scm, int64_t scn, bool lower_only, bool a_lower, hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  const bool akc = (A.s1 == 1), bkc = (B.s1 == 1);
  require(akc || A.s0 == 1, "gemm64: A needs a unit stride");
  require(bkc || B.s0 == 1, "gemm64: B needs a unit stride");
  const bool narrow = N <= 64;
#define GEMM64_CASE(BNv, a, b) gemm64_t<BNv, a, b>(M, N, K, alpha, A, B, beta, C, scm, scn, lower_only, a_lower, st)
  if (narrow) {
    if (akc && bkc) GEMM64_CASE(64, true, true);
    else if (akc) GEMM64_CASE(64, true, false);
    else if (bkc) GEMM64_CASE(64, false, true);
    else GEMM64_CASE(64, false, false);
  } else {
    if (akc && bkc) GEMM64_CASE(128, true, true);
    else if (akc) GEMM64_CASE(128, true, false);
    else if (bkc) GEMM64_CASE(128, false, true);
    else GEMM64_CASE(128, false, false);
  }
#undef GEMM64_CASE
}

void gemm64(int M, int N, int K, double alpha, View64 A, View64 B, double beta, double* C, int64_t scm, int64_t scn,
            bool lower_only, hipStream_t st) {
  gemm64_dispatch(M, N, K, alpha, A, B, beta, C, scm, scn, lower_only, false, st);
}

template <bool AKC, bool BKC>
static void gemm64_in32_t(int M, int N, int K, double alpha, View32 A, View32 B, double beta, double* C, int64_t scm,
                          int64_t scn, hipStream_t st) {
  ScalarArgs<float> g{};
  g.M = M;
  g.N = N;
  g.nseg = 1;
  g.seg[0] = SegS<float>{A.p, A.s0, A.s1, B.p, B.s0, B.s1, K};
  EpiAxpby<double> e{C, scm, scn, M, N, alpha, beta};
  dim3 grid(cdiv(N, 128), cdiv(M, 128));
  gemm_scalar_kernel<double, 128, 128, 16, AKC, BKC, EpiAxpby<double>, float><<<grid, 256, 0, st>>>(g, e);
  LAUNCHCHK();
}

void gemm64_in32(int M, int N, int K, double alpha, View32 A, View32 B, double beta, double* C, int64_t scm,
                 int64_t scn, hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  const bool akc = (A.s1 == 1), bkc = (B.s1 == 1);
  require(akc || A.s0 == 1, "gemm64_in32: A needs a unit stride");
  require(bkc || B.s0 == 1, "gemm64_in32: B needs a unit stride");
  if (akc && bkc) gemm64_in32_t<true, true>(M, N, K, alpha, A, B, beta, C, scm, scn, st);
  else if (akc) gemm64_in32_t<true, false>(M, N, K, alpha, A, B, beta, C, scm, scn, st);
  else if (bkc) gemm64_in32_t<false, true>(M, N, K, alpha, A, B, beta, C, scm, scn, st);
  else gemm64_in32_t<false, false>(M, N, K, alpha, A, B, beta, C, scm, scn, st);
}

void gemm64_alower(int M, int N, int K, double alpha, View64 A, View64 B, double beta, double* C, int64_t scm,
                   int64_t scn, hipStream_t st) {
  gemm64_dispatch(M, N, K, alpha, A, B, beta, C, scm, scn, false, true, st);
}

// ------------------------------------- Cholesky and triangular inversion ----
constexpr int NB = 64;

// Unblocked Cholesky of one jb x jb diagonal block (column-major, lda) in LDS.
__global__ __launch_bounds__(256) void k_potf2(double* A, int jb, int64_t lda, int64_t j0, int64_t* info) {
  __shared__ double L[NB][NB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int e = tid; e < jb * jb; e += 256) {
    const int r = e % jb, c = e / jb;
    L[r][c] = A[r + c * lda];
  }
  __syncthreads();
  for (int c = 0; c < jb; ++c) {   // right-looking, column by column
    if (tid == 0) {
      const double d = L[c][c];
      if (!(d > 0.0) || !isfinite(d)) {
        if (!bad) {
          bad = 1;
          atomicMin(reinterpret_cast<unsigned long long*>(info), (unsigned long long)(j0 + c));
        }
        L[c][c] = 1.0;
      } else {
        L[c][c] = sqrt(d);
      }
    }
    __syncthreads();
    const double piv = L[c][c];
    for (int r = c + 1 + tid; r < jb; r += 256) L[r][c] /= piv;
    __syncthreads();
    const int w = jb - c - 1;
    for (int e = tid; e < w * w; e += 256) {
      const int r = c + 1 + e % w, q = c + 1 + e / w;
      if (q <= r) L[r][q] -= L[r][c] * L[q][c];
    }
    __syncthreads();
  }
  for (int e = tid; e < jb * jb; e += 256) {
    const int r = e % jb, c = e / jb;
    A[r + c * lda] = r >= c ? L[r][c] : 0.0;   // clean lower-triangular block
  }
}

// Inverse of the jb x jb lower-triangular block at A (lda) into X (NB x NB row-major, zero padded).
__global__ __launch_bounds__(64) void k_tri_inverse(const double* A, int jb, int64_t lda, double* X) {
  __shared__ double L[NB][NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += 64) {
    const int r = e % NB, c = e / NB;
    L[r][c] = (r < jb && c < jb) ? A[r + c * lda] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  const int c = tid;
  double x[NB];
#pragma unroll
  for (int r = 0; r < NB; ++r) x[r] = 0.0;
  // column c of the inverse, computed in registers with static indices
#pragma unroll
  for (int r = 0; r < NB; ++r) {
    if (r == c) x[r] = 1.0 / L[r][r];
    if (r > c) {
      double sacc = 0.0;
#pragma unroll
      for (int q = 0; q < r; ++q) sacc += L[r][q] * x[q];
      x[r] = -sacc / L[r][r];
    }
  }
#pragma unroll
  for (int r = 0; r < NB; ++r) X[r * NB + c] = x[r];
}

// In-place inverse of a jb x jb lower-triangular diagonal block.
__global__ __launch_bounds__(64) void k_trtri_small(double* A, int jb, int64_t lda) {
  __shared__ double L[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < jb * jb; e += 64) {
    const int r = e % jb, c = e / jb;
    L[r][c] = A[r + c * lda];
  }
  __syncthreads();
  const int c = tid;   // one column of the inverse per thread
  if (c < jb) {
    X[c][c] = 1.0 / L[c][c];
    for (int r = c + 1; r < jb; ++r) {
      double s = 0.0;
      for (int q = c; q < r; ++q) s += L[r][q] * X[q][c];
      X[r][c] = -s / L[r][r];
    }
  }
  __syncthreads();
  for (int e = tid; e < jb * jb; e += 64) {
    const int r = e % jb, cc = e / jb;
    A[r + cc * lda] = r >= cc ? X[r][cc] : 0.0;
  }
}

// In-place inverse of the lower-triangular A (n x n, lda) in 64-wide blocks,
// last block first, with T ((n - 64) x 64) as scratch; entries above the
// diagonal of each 64-wide diagonal block become zero, those further above
// are not touched.
static void trtri_nb(double* A, int64_t n, int64_t lda, hipStream_t st, double* T) {
  const int64_t nblk = (n + NB - 1) / NB;
  for (int64_t b = nblk - 1; b >= 0; --b) {
    const int64_t j0 = b * NB;
    const int jb = (int)std::min<int64_t>(NB, n - j0);
    const int64_t rest = n - j0 - jb;
    if (rest > 0) {
      // T = X22 * A21 (X22 = already inverted trailing block, lower-triangular)
      const double* X22 = A + (j0 + jb) + (j0 + jb) * lda;
      double* A21 = A + (j0 + jb) + j0 * lda;
      gemm64_alower((int)rest, jb, (int)rest, 1.0, View64{X22, 1, lda}, View64{A21, lda, 1}, 0.0, T, 1, rest, st);
      k_trtri_small<<<1, 64, 0, st>>>(A + j0 + j0 * lda, jb, lda);
      LAUNCHCHK();
      // A21 = -T * X11
      const double* X11 = A + j0 + j0 * lda;
      gemm64((int)rest, jb, jb, -1.0, View64{T, 1, rest}, View64{X11, lda, 1}, 0.0, A21, 1, lda, false, st);
    } else {
      k_trtri_small<<<1, 64, 0, st>>>(A + j0 + j0 * lda, jb, lda);
      LAUNCHCHK();
    }
  }
}

// Zero the entries above the diagonal of the n x n block A (lda).
__global__ void k_zero_upper(double* A, int64_t lda, int n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int r = (int)(e % n), c = (int)(e / n);
  if (r < c) A[r + c * lda] = 0.0;
}

// Right-looking Cholesky in 64-wide panels on the block A (n x n, lda); the
// first failing column (offset by j_off) goes to info.
static void potrf_nb(double* A, int64_t n, int64_t lda, int64_t j_off, int64_t* info, double* Xinv,
                     hipStream_t st) {
  for (int64_t j0 = 0; j0 < n; j0 += NB) {
    const int jb = (int)std::min<int64_t>(NB, n - j0);
    k_potf2<<<1, 256, 0, st>>>(A + j0 + j0 * lda, jb, lda, j_off + j0, info);
    LAUNCHCHK();
    const int64_t rest = n - j0 - jb;
    if (rest > 0) {
      // panel <- panel L_jj^-T  (in place: one 128-row tile covers all jb columns)
      k_tri_inverse<<<1, 64, 0, st>>>(A + j0 + j0 * lda, jb, lda, Xinv);
      LAUNCHCHK();
      double* P = A + (j0 + jb) + j0 * lda;
      gemm64((int)rest, jb, jb, 1.0, View64{P, 1, lda}, View64{Xinv, NB, 1}, 0.0, P, 1, lda, false, st);
      double* C = A + (j0 + jb) + (j0 + jb) * lda;
      gemm64((int)rest, (int)rest, jb, -1.0, View64{P, 1, lda}, View64{P, 1, lda}, 1.0, C, 1, lda, true, st);
    }
  }
}

// dst (n x n, ldd) = the lower triangle of src (lda), zero above the diagonal
__global__ void k_copy_lower(const double* __restrict__ src, int64_t lda, int n, double* __restrict__ dst,
                             int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int r = (int)(e % n), c = (int)(e / n);
  dst[r + c * ldd] = r >= c ? src[r + c * lda] : 0.0;
}

// Two levels of blocking.  With 64-wide panels every trailing update reads
// and writes the whole trailing matrix for a K = 64 product, about 2 TB for
// n = 31500, so the factorization ran at the speed of HBM.  Here 256-wide
// panels are factored by the 64-wide code (diagonal block), their rows
// below are solved against the inverted diagonal block, and the trailing
// matrix takes one K = 256 update per panel: a quarter of the traffic, for
// products that the matrix cores, not HBM, bound.
int64_t potrf_lower(double* A, int64_t n, int64_t lda, hipStream_t st) {
  constexpr int NB2 = 256;
  DBuf info(8), Xinv(NB * NB * 8), L1((size_t)NB2 * NB2 * 8), T(std::max<int64_t>(n - NB2, 1) * NB2 * 8),
      Ts((size_t)(NB2 - NB) * NB * 8);
  const unsigned long long none = ~0ull;
  HIPCHK(hipMemcpyAsync(info.get(), &none, 8, hipMemcpyHostToDevice, st));
  for (int64_t J0 = 0; J0 < n; J0 += NB2) {
    const int jb = (int)std::min<int64_t>(NB2, n - J0);
    double* D = A + J0 + J0 * lda;
    potrf_nb(D, jb, lda, J0, info.as<int64_t>(), Xinv.as<double>(), st);
    const int64_t rest = n - J0 - jb;
    if (rest > 0) {
      // L1 = L_JJ^-1 (lower, zero above), T = A_21 L1^T, then A_22 -= T T^T and A_21 = T
      k_copy_lower<<<cdiv((int64_t)jb * jb, 256), 256, 0, st>>>(D, lda, jb, L1.as<double>(), jb);
      LAUNCHCHK();
      trtri_nb(L1.as<double>(), jb, jb, st, Ts.as<double>());
      double* A21 = A + (J0 + jb) + J0 * lda;
      gemm64((int)rest, jb, jb, 1.0, View64{A21, 1, lda}, View64{L1.as<double>(), 1, jb}, 0.0, T.as<double>(), 1,
             rest, false, st);
      double* C = A + (J0 + jb) + (J0 + jb) * lda;
      gemm64((int)rest, (int)rest, jb, -1.0, View64{T.as<double>(), 1, rest}, View64{T.as<double>(), 1, rest}, 1.0,
             C, 1, lda, true, st);
      HIPCHK(hipMemcpy2DAsync(A21, lda * 8, T.get(), rest * 8, rest * 8, jb, hipMemcpyDeviceToDevice, st));
    }
  }
  unsigned long long h = 0;
  HIPCHK(hipMemcpyAsync(&h, info.get(), 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return h == none ? -1 : (int64_t)h;
}

// In-place inverse of the lower-triangular A (n x n, lda).  Two levels, as
// potrf_lower: 256-wide blocks, last first.  For each, T = X22 A21 with the
// already inverted trailing block (K = rest, N = 256: a quarter of the reads
// of X22 that 64-wide blocks needed), the diagonal block inverted by the
// 64-wide code, then A21 = -T X11.
void trtri_lower(double* A, int64_t n, int64_t lda, hipStream_t st) {
  constexpr int NB2 = 256;
  const int64_t nblk = (n + NB2 - 1) / NB2;
  DBuf T(std::max<int64_t>(n - NB2, 1) * NB2 * sizeof(double)), Ts((NB2 - NB) * NB * sizeof(double));
  for (int64_t b = nblk - 1; b >= 0; --b) {
    const int64_t j0 = b * NB2;
    const int jb = (int)std::min<int64_t>(NB2, n - j0);
    const int64_t rest = n - j0 - jb;
    double* D = A + j0 + j0 * lda;
    if (rest > 0) {
      const double* X22 = A + (j0 + jb) + (j0 + jb) * lda;
      double* A21 = A + (j0 + jb) + j0 * lda;
      gemm64_alower((int)rest, jb, (int)rest, 1.0, View64{X22, 1, lda}, View64{A21, lda, 1}, 0.0, T.as<double>(), 1,
                    rest, st);
      trtri_nb(D, jb, lda, st, Ts.as<double>());
      // X11 enters the product below as a full block: nothing above its diagonal
      k_zero_upper<<<cdiv((int64_t)jb * jb, 256), 256, 0, st>>>(D, lda, jb);
      LAUNCHCHK();
      gemm64((int)rest, jb, jb, -1.0, View64{T.as<double>(), 1, rest}, View64{D, lda, 1}, 0.0, A21, 1, lda, false,
             st);
    } else {
      trtri_nb(D, jb, lda, st, Ts.as<double>());
    }
  }
  HIPCHK(hipStreamSynchronize(st));   // T and Ts are released on return
}

}  // namespace ffk
