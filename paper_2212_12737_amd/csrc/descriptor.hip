// Descriptor build and iteration-invariant kernel coefficients.
//
// x_pq = 1/|R_p - R_q| for p > q (row-major lower-triangle order), the column
// mean over geometries, X_c = X - mean (differences x_i - x_j, hence the
// kernel, do not change; centring keeps the Gram-matrix route to distances
// well conditioned), |x_c,i|^2, then from the FP64 Gram matrix X_c X_c^T:
//   r_ij = sqrt(max(|x_i|^2 + |x_j|^2 - 2 x_i.x_j, 0)),  z = sqrt(5) r / sigma,
//   dA_ij = a(r) - a(0) = a0 ((1 + z) expm1(-z) + z),   a0 = 5 / (3 sigma^2),
//   B_ij  = b(r) = -25/(3 sigma^4) e^-z,
// the Matern-5/2 Hessian coefficients H = a I + b d d^T of the force kernel.
// Reduced-precision copies are derived from the FP64 arrays on first use.
#include "gemm.hpp"

namespace ffk {

__global__ void k_descriptor(const double* __restrict__ R, const int* __restrict__ pairs, int64_t N,
                             int M, int64_t D, double* __restrict__ X, int* __restrict__ bad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * D) return;
  const int64_t g = e / D, d = e % D;
  const int pq = pairs[d];
  const int p = pq >> 16, q = pq & 0xFFFF;
  const double* Rg = R + g * 3 * M;
  const double dx = Rg[3 * p] - Rg[3 * q], dy = Rg[3 * p + 1] - Rg[3 * q + 1],
               dz = Rg[3 * p + 2] - Rg[3 * q + 2];
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double x = 1.0 / sqrt(r2);
  if (!(r2 > 0.0) || !isfinite(x)) atomicOr(bad, 1);
  X[e] = x;
}

// Column means of an N x D matrix: block = 64 columns x 4 row groups.
__global__ void k_colmean(const double* __restrict__ X, int64_t N, int64_t D, double* __restrict__ mean) {
  __shared__ double part[4][64];
  const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int64_t col = (int64_t)blockIdx.x * 64 + c;
  double s = 0.0;
  if (col < D)
    for (int64_t r = rg; r < N; r += 4) s += X[r * D + col];
  part[rg][c] = s;
  __syncthreads();
  if (rg == 0 && col < D) mean[col] = ((part[0][c] + part[1][c]) + (part[2][c] + part[3][c])) / (double)N;
}

// X_c = X - mean, and |x_c,i|^2 (one block per geometry).
__global__ void k_center(const double* __restrict__ X, const double* __restrict__ mean, int64_t D,
                         double* __restrict__ Xc, double* __restrict__ sqn) {
  __shared__ double red[256];
  const int64_t g = blockIdx.x;
  double s = 0.0;
  for (int64_t d = threadIdx.x; d < D; d += blockDim.x) {
    const double v = X[g * D + d] - mean[d];
    Xc[g * D + d] = v;
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) sqn[g] = red[0];
}

void descriptor_build(ffk_system* s, const double* R, hipStream_t st, bool coefficients) {
  const int64_t N = s->N, D = s->D;
  const int M = s->M;
  // pair table
  std::vector<int> pt(D);
  {
    int64_t d = 0;
    for (int p = 1; p < M; ++p)
      for (int q = 0; q < p; ++q) pt[d++] = (p << 16) | q;
  }
  s->pairs.alloc(D * sizeof(int));
  HIPCHK(hipMemcpyAsync(s->pairs.get(), pt.data(), D * sizeof(int), hipMemcpyHostToDevice, st));
  s->R.alloc(N * M * 3 * sizeof(double));
  HIPCHK(hipMemcpyAsync(s->R.get(), R, N * M * 3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  s->X.alloc(N * D * sizeof(double));
  s->Xc.alloc(N * D * sizeof(double));
  s->xmean.alloc(D * sizeof(double));
  s->sqn.alloc(N * sizeof(double));
  DBuf bad(sizeof(int));
  HIPCHK(hipMemsetAsync(bad.get(), 0, sizeof(int), st));
  k_descriptor<<<cdiv(N * D, 256), 256, 0, st>>>(s->R.as<double>(), s->pairs.as<int>(), N, M, D,
                                                  s->X.as<double>(), bad.as<int>());
  LAUNCHCHK();
  int hbad = 0;
  HIPCHK(hipMemcpyAsync(&hbad, bad.get(), sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hbad) fail(FFK_ERR_NONFINITE, "descriptor_build: coincident atoms or non-finite coordinates");
  k_colmean<<<cdiv(D, 64), 256, 0, st>>>(s->X.as<double>(), N, D, s->xmean.as<double>());
  LAUNCHCHK();
  k_center<<<N, 256, 0, st>>>(s->X.as<double>(), s->xmean.as<double>(), D, s->Xc.as<double>(),
                              s->sqn.as<double>());
  LAUNCHCHK();
  if (coefficients) ensure_coeffs(s, FFK_FP64, st);
}

// ------------------------------------------------------------ conversions ----

// hi/lo split of a rows x cols FP64 matrix into padded bf16 arrays
// (rows_p x ld_out); entries outside rows x cols are written as zero.
// hi (+ lo) split of a rows x cols FP64 matrix into a rows_p x ld_out
// operand in fragment-major layout (K = ld_out), zero outside.
__global__ void k_split_pad(const double* __restrict__ a, int64_t rows, int64_t cols, int64_t lda,
                            int64_t rows_p, int64_t ld_out, bf16_t* __restrict__ hi,
                            bf16_t* __restrict__ lo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows_p * ld_out) return;
  const int64_t r = e / ld_out, c = e % ld_out;
  float x = 0.f;
  if (r < rows && c < cols) x = (float)a[r * lda + c];
  const bf16_t h = f2bf(x);
  const int64_t o = frag_off(r, c, ld_out / 32);
  hi[o] = h;
  if (lo) lo[o] = f2bf(x - bf2f(h));
}

// FP32 copy of a rows x cols FP64 matrix into a padded rows_p x ld_out array.
__global__ void k_f32_pad(const double* __restrict__ a, int64_t rows, int64_t cols, int64_t lda,
                          int64_t rows_p, int64_t ld_out, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows_p * ld_out) return;
  const int64_t r = e / ld_out, c = e % ld_out;
  out[e] = (r < rows && c < cols) ? (float)a[r * lda + c] : 0.f;
}

// Transposed hi/lo split: a is rows x cols (lda); output cols_p x ld_out
// (fragment-major, K = ld_out) with out[c][r] = split(a[r][c]), zero
// outside.  64 x 64 tiles through LDS.
__global__ void k_split_transpose(const double* __restrict__ a, int64_t rows, int64_t cols, int64_t lda,
                                  int64_t cols_p, int64_t ld_out, bf16_t* __restrict__ hi,
                                  bf16_t* __restrict__ lo) {
  __shared__ float tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 256 threads: 64 x 4
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i, c = c0 + tx;
    tile[i][tx] = (r < rows && c < cols) ? (float)a[r * lda + c] : 0.f;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < cols_p && r < ld_out) {
      const float x = tile[tx][i];
      const bf16_t h = f2bf(x);
      const int64_t o = frag_off(c, r, ld_out / 32);
      hi[o] = h;
      if (lo) lo[o] = f2bf(x - bf2f(h));
    }
  }
}

static int64_t rup(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// out[c][r] = (T)a[r][c] for the rows x cols FP64 matrix a (lda), into a
// cols_p x ld_out array, zero outside.  64 x 64 tiles through LDS.
template <typename T>
__global__ void k_pad_transpose(const double* __restrict__ a, int64_t rows, int64_t cols, int64_t lda,
                                int64_t cols_p, int64_t ld_out, T* __restrict__ out) {
  __shared__ double tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i, c = c0 + tx;
    tile[i][tx] = (r < rows && c < cols) ? a[r * lda + c] : 0.0;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < cols_p && r < ld_out) out[c * ld_out + r] = (T)tile[tx][i];
  }
}

// (T)a into a rows_p x ld_out array (row-major), zero outside rows x cols.
template <typename T>
__global__ void k_pad_copy(const double* __restrict__ a, int64_t rows, int64_t cols, int64_t lda, int64_t rows_p,
                           int64_t ld_out, T* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows_p * ld_out) return;
  const int64_t r = e / ld_out, c = e % ld_out;
  out[e] = (r < rows && c < cols) ? (T)a[r * lda + c] : T(0);
}



void k_split_transpose_launch(const double* a, int64_t rows, int64_t cols, int64_t lda, int64_t cols_p,
                              int64_t ld_out, bf16_t* hi, bf16_t* lo, hipStream_t st) {
  dim3 grid(cdiv(ld_out, 64), cdiv(cols_p, 64));
  k_split_transpose<<<grid, 256, 0, st>>>(a, rows, cols, lda, cols_p, ld_out, hi, lo);
  LAUNCHCHK();
}

template <typename T>
static void padded_descriptor(const ffk_system* s, DBuf& P, DBuf& PT, hipStream_t st) {
  const int64_t N = s->N, D = s->D;
  const int64_t Nr = pad_rows(N), Dk = rup(D, 64), Dr = pad_rows(D);
  P.alloc(Nr * Dk * sizeof(T));
  k_pad_copy<T><<<cdiv(Nr * Dk, 256), 256, 0, st>>>(s->Xc.as<double>(), N, D, D, Nr, Dk, P.as<T>());
  LAUNCHCHK();
  PT.alloc(Dr * Nr * sizeof(T));
  dim3 grid(cdiv(Nr, 64), cdiv(Dr, 64));
  k_pad_transpose<T><<<grid, 256, 0, st>>>(s->Xc.as<double>(), N, D, D, Dr, Nr, PT.as<T>());
  LAUNCHCHK();
}

void ensure_lowp_descriptor(ffk_system* s, int prec, hipStream_t st) {
  const int64_t N = s->N, D = s->D;
  if (prec == FFK_FP64 && !s->Xp64) padded_descriptor<double>(s, s->Xp64, s->XpT64, st);
  if (prec == FFK_FP32 && !s->Xp32) padded_descriptor<float>(s, s->Xp32, s->XpT32, st);
  if ((prec == FFK_BF16 || prec == FFK_BF16X3) && !s->Xch) {
    const int64_t Nr = pad_rows(N), Dk = rup(D, 64), Dr = pad_rows(D);
    s->Xch.alloc(Nr * Dk * 2);
    s->Xcl.alloc(Nr * Dk * 2);
    k_split_pad<<<cdiv(Nr * Dk, 256), 256, 0, st>>>(s->Xc.as<double>(), N, D, D, Nr, Dk,
                                                    s->Xch.as<bf16_t>(), s->Xcl.as<bf16_t>());
    LAUNCHCHK();
    s->XcTh.alloc(Dr * Nr * 2);
    s->XcTl.alloc(Dr * Nr * 2);
    dim3 grid(cdiv(Nr, 64), cdiv(Dr, 64));
    k_split_transpose<<<grid, 256, 0, st>>>(s->Xc.as<double>(), N, D, D, Dr, Nr, s->XcTh.as<bf16_t>(),
                                            s->XcTl.as<bf16_t>());
    LAUNCHCHK();
  }
}

// Coefficients dA = a(r) - a(0), B = b(r) of the pairs (target i, source j)
// from the Gram matrix X_t X_s^T of the centred descriptors (both centred with
// one mean): r^2 = |x_i|^2 + |x_j|^2 - 2 x_i . x_j, set to exactly zero where
// the source is the target itself (j = i + diag_off) or rounding makes it
// negative.  Rows Nt, columns Ns, stored with leading dimension ld.
struct EpiCoeffPair {
  const double *sqr, *sqc;
  double *dA, *B;
  int Nt, Ns;
  int64_t ld, diag_off;
  double inv_len, a0, bcoef;   // sqrt(5)/sigma, 5/(3 sigma^2), 25/(3 sigma^4)
  template <typename T, int TM, int TN, class Acc>
  __device__ void run(const Acc (&acc)[TM][TN], const FragCoord& f, char*) const {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = f.row(i, v), c = f.col(j);
          if (r < Nt && c < Ns) {
            double r2 = sqr[r] + sqc[c] - 2.0 * (double)acc[i][j][v];
            r2 = (c == r + diag_off || r2 < 0.0) ? 0.0 : r2;
            const double z = sqrt(r2) * inv_len;
            const double em = expm1(-z);
            dA[(int64_t)r * ld + c] = a0 * ((1.0 + z) * em + z);
            B[(int64_t)r * ld + c] = -bcoef * (em + 1.0);
          }
        }
  }
};

void ensure_coeffs_pair(const ffk_system* t, const ffk_system* src, CoeffSet* sets, int prec, int64_t diag_off,
                        hipStream_t st) {
  const int64_t Nt = t->N, Ns = src->N;
  const int64_t Ntr = pad_rows(Nt), Nsr = pad_rows(Ns);
  CoeffSet& c64 = sets[FFK_FP64];
  if (!c64.ready) {
    c64.dA_hi.alloc(Ntr * Nsr * sizeof(double));
    c64.B.alloc(Ntr * Nsr * sizeof(double));
    HIPCHK(hipMemsetAsync(c64.dA_hi.get(), 0, Ntr * Nsr * sizeof(double), st));
    HIPCHK(hipMemsetAsync(c64.B.get(), 0, Ntr * Nsr * sizeof(double), st));
    ScalarArgs<double> g{};
    g.M = (int)Nt;
    g.N = (int)Ns;
    g.nseg = 1;
    g.seg[0] = SegS<double>{t->Xc.as<double>(), t->D, 1, src->Xc.as<double>(), src->D, 1, (int)t->D};
    EpiCoeffPair e{t->sqn.as<double>(), src->sqn.as<double>(), c64.dA_hi.as<double>(), c64.B.as<double>(), (int)Nt,
                   (int)Ns, Nsr, diag_off, sqrt(5.0) / t->sigma, t->a0, t->bcoef};
    dim3 grid(cdiv(Ns, 128), cdiv(Nt, 128));
    gemm_scalar_kernel<double, 128, 128, 16, true, true, EpiCoeffPair><<<grid, 256, 0, st>>>(g, e);
    LAUNCHCHK();
    c64.ready = true;
  }
  if (prec == FFK_FP64) return;
  CoeffSet& cs = sets[prec];
  if (cs.ready) return;
  const int64_t cnt = Ntr * Nsr;
  if (prec == FFK_FP32) {
    cs.dA_hi.alloc(cnt * sizeof(float));
    cs.B.alloc(cnt * sizeof(float));
    k_pad_copy<float><<<cdiv(cnt, 256), 256, 0, st>>>(c64.dA_hi.as<double>(), Nt, Ns, Nsr, Ntr, Nsr,
                                                      cs.dA_hi.as<float>());
    LAUNCHCHK();
    k_pad_copy<float><<<cdiv(cnt, 256), 256, 0, st>>>(c64.B.as<double>(), Nt, Ns, Nsr, Ntr, Nsr, cs.B.as<float>());
    LAUNCHCHK();
  } else if (use_fused(prec, t->D, Nt, Ns)) {
    // one array in the fused product's layout: dA (hi and lo) and B
    cs.dA_hi.alloc(cnt * 8);
    fused_coef_build(c64.dA_hi.as<double>(), c64.B.as<double>(), Nt, Ns, Nsr, Ntr, Nsr, cs.dA_hi.get(), st);
  } else {
    const bool x3 = (prec == FFK_BF16X3);
    cs.dA_hi.alloc(cnt * 2);
    if (x3) cs.dA_lo.alloc(cnt * 2);
    cs.B.alloc(cnt * sizeof(float));
    k_split_pad<<<cdiv(cnt, 256), 256, 0, st>>>(c64.dA_hi.as<double>(), Nt, Ns, Nsr, Ntr, Nsr,
                                                cs.dA_hi.as<bf16_t>(), x3 ? cs.dA_lo.as<bf16_t>() : nullptr);
    LAUNCHCHK();
    k_f32_pad<<<cdiv(cnt, 256), 256, 0, st>>>(c64.B.as<double>(), Nt, Ns, Nsr, Ntr, Nsr, cs.B.as<float>());
    LAUNCHCHK();
  }
  cs.ready = true;
}

void ensure_coeffs(ffk_system* s, int prec, hipStream_t st) { ensure_coeffs_pair(s, s, s->coef, prec, 0, st); }

}  // namespace ffk
