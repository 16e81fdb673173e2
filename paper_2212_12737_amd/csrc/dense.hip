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

// ------------------------------------------------------------- Cholesky ----
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

int64_t potrf_lower(double* A, int64_t n, int64_t lda, hipStream_t st) {
  DBuf info(8), Xinv(NB * NB * 8);
  const unsigned long long none = ~0ull;
  HIPCHK(hipMemcpyAsync(info.get(), &none, 8, hipMemcpyHostToDevice, st));
  for (int64_t j0 = 0; j0 < n; j0 += NB) {
    const int jb = (int)std::min<int64_t>(NB, n - j0);
    k_potf2<<<1, 256, 0, st>>>(A + j0 + j0 * lda, jb, lda, j0, info.as<int64_t>());
    LAUNCHCHK();
    const int64_t rest = n - j0 - jb;
    if (rest > 0) {
      // panel <- panel L_jj^-T  (in place: one 128-row tile covers all jb columns)
      k_tri_inverse<<<1, 64, 0, st>>>(A + j0 + j0 * lda, jb, lda, Xinv.as<double>());
      LAUNCHCHK();
      double* P = A + (j0 + jb) + j0 * lda;
      gemm64((int)rest, jb, jb, 1.0, View64{P, 1, lda}, View64{Xinv.as<double>(), NB, 1}, 0.0, P, 1, lda, false, st);
      double* C = A + (j0 + jb) + (j0 + jb) * lda;
      gemm64((int)rest, (int)rest, jb, -1.0, View64{P, 1, lda}, View64{P, 1, lda}, 1.0, C, 1, lda, true, st);
    }
  }
  unsigned long long h = 0;
  HIPCHK(hipMemcpyAsync(&h, info.get(), 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return h == none ? -1 : (int64_t)h;
}

// ------------------------------------------------ triangular inversion ----
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

void trtri_lower(double* A, int64_t n, int64_t lda, hipStream_t st) {
  const int64_t nblk = (n + NB - 1) / NB;
  DBuf T(std::max<int64_t>(n - NB, 1) * NB * sizeof(double));
  for (int64_t b = nblk - 1; b >= 0; --b) {
    const int64_t j0 = b * NB;
    const int jb = (int)std::min<int64_t>(NB, n - j0);
    const int64_t rest = n - j0 - jb;
    if (rest > 0) {
      // T = X22 * A21 (X22 = already inverted trailing block, lower-triangular)
      const double* X22 = A + (j0 + jb) + (j0 + jb) * lda;
      double* A21 = A + (j0 + jb) + j0 * lda;
      gemm64_alower((int)rest, jb, (int)rest, 1.0, View64{X22, 1, lda}, View64{A21, lda, 1}, 0.0, T.as<double>(),
                    1, rest, st);
      k_trtri_small<<<1, 64, 0, st>>>(A + j0 + j0 * lda, jb, lda);
      LAUNCHCHK();
      // A21 = -T * X11
      const double* X11 = A + j0 + j0 * lda;
      gemm64((int)rest, jb, jb, -1.0, View64{T.as<double>(), 1, rest}, View64{X11, lda, 1}, 0.0, A21, 1, lda,
             false, st);
    } else {
      k_trtri_small<<<1, 64, 0, st>>>(A + j0 + j0 * lda, jb, lda);
      LAUNCHCHK();
    }
  }
  HIPCHK(hipStreamSynchronize(st));   // T is released on return
}

}  // namespace ffk
