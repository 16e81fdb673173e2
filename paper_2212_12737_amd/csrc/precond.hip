// Nystroem preconditioner P = L L^T + lambda I (Eq. 3-5) and its Woodbury
// inverse (Eq. 4).
//
// L is built as the incomplete Cholesky factor with pivots forced to the
// selected column order: for identical columns this equals the Nystroem
// factor K_nk K_kk^-1 K_nk^T (section 3).  The columns are processed in panels
// of 64: (1) evaluate the raw kernel columns, (2) subtract the contribution of
// all earlier panels with one FP64 MFMA GEMM, (3) factor the 64 x 64 pivot
// block (dropping columns whose remaining diagonal is <= 1e-12 max diag K) and
// invert it, (4) multiply the panel by that inverse (an in-place MFMA GEMM),
// (5) zero the rows of earlier pivots and set the exact pivot values, as
// Algorithm 1 leaves them.
// The core lambda I + L^T L is formed from the stored L (FP64 or FP32) in FP64,
// factored, and its triangular inverse Finv kept, so that
//   z = lambda^-1 (r - L Finv^T Finv L^T r).
// L and Finv are column-major with leading dimensions padded to 64 elements
// (zero padding), so the GEMVs of the apply use aligned 16-byte loads.
#include "gemm.hpp"

namespace ffk {

constexpr int PB = 64;   // panel width

inline int64_t pad64(int64_t a) { return (a + 63) / 64 * 64; }

// G[c][j] = L[idx[c] + j ld] for c < nb, j < m0  (row-major nb x m0)
__global__ void k_gather_rows(const double* L, int64_t ld, const int64_t* idx, int nb, int64_t m0, double* G) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nb * m0) return;
  const int c = (int)(e / m0);
  const int64_t j = e % m0;
  G[e] = L[idx[c] + j * ld];
}

// Factor the nb x nb pivot block T[c][c'] = panel[idx[c], c'] with drops and
// invert it.  Outputs: Lb (PB x PB row-major, lower; dropped columns zero),
// Linv (PB x PB row-major) = inverse of Lb with a unit diagonal put at dropped
// positions, drop flags.
__global__ __launch_bounds__(256) void k_panel_chol(const double* Lp, int64_t ld, const int64_t* idx, int nb,
                                                    double thr, double* Lb, double* Linv, unsigned char* dropped) {
  __shared__ double T[PB][PB + 1];
  __shared__ double X[PB][PB + 1];
  __shared__ unsigned char dr[PB];
  const int tid = threadIdx.x;
  for (int e = tid; e < PB * PB; e += 256) {
    const int r = e % PB, c = e / PB;
    T[r][c] = (r < nb && c < nb) ? Lp[idx[r] + (int64_t)c * ld] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    if (tid == 0) {
      const double d = T[c][c];
      if (!(d > thr)) {
        dr[c] = 1;
        T[c][c] = 0.0;
      } else {
        dr[c] = 0;
        T[c][c] = sqrt(d);
      }
    }
    __syncthreads();
    const bool drop = dr[c];
    const double piv = T[c][c];
    for (int r = c + 1 + tid; r < nb; r += 256) T[r][c] = drop ? 0.0 : T[r][c] / piv;
    __syncthreads();
    if (!drop) {
      const int w = nb - c - 1;
      for (int e = tid; e < w * w; e += 256) {
        const int r = c + 1 + e % w, q = c + 1 + e / w;
        if (q <= r) T[r][q] -= T[r][c] * T[q][c];
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < PB * PB; e += 256) {
    const int r = e / PB, c = e % PB;
    Lb[e] = (r < nb && c < nb && r >= c) ? T[r][c] : 0.0;
  }
  for (int c = tid; c < nb; c += 256) dropped[c] = dr[c];
  __syncthreads();
  // unit diagonal at dropped (and padding) positions: their columns are zero
  // below the diagonal, so the kept part of the solve is unaffected
  if (tid < PB && (tid >= nb || dr[tid])) T[tid][tid] = 1.0;
  __syncthreads();
  if (tid < PB) {   // column tid of the inverse by forward substitution
    const int c = tid;
    for (int r = 0; r < c; ++r) X[r][c] = 0.0;
    X[c][c] = 1.0 / T[c][c];
    for (int r = c + 1; r < PB; ++r) {
      double sacc = 0.0;
      for (int q = c; q < r; ++q) sacc += (q < nb && r < nb) ? T[r][q] * X[q][c] : 0.0;
      X[r][c] = -sacc / T[r][r];
    }
  }
  __syncthreads();
  for (int e = tid; e < PB * PB; e += 256) Linv[e] = X[e / PB][e % PB];
}

// Exact zeros at earlier pivot rows and the exact pivot value on the diagonal;
// dropped columns are cleared entirely.
__global__ void k_panel_fix(double* L, int64_t n, int64_t ld, const int64_t* idx, const unsigned char* kept,
                            int64_t m0, int nb, const double* Lb) {
  const int c = blockIdx.x;
  double* col = L + (m0 + c) * ld;
  if (!kept[m0 + c]) {
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) col[i] = 0.0;
    return;
  }
  for (int64_t j = threadIdx.x; j < m0 + c; j += blockDim.x)
    if (kept[j]) col[idx[j]] = 0.0;
  if (threadIdx.x == 0) col[idx[m0 + c]] = Lb[c * PB + c];
}

__global__ void k_set_kept(const unsigned char* dropped, int nb, unsigned char* kept) {
  const int c = threadIdx.x;
  if (c < nb) kept[c] = dropped[c] ? 0 : 1;
}

int64_t icd_forced(ffk_system* s, const int64_t* idx, int64_t k, double shift, double* L, int64_t ld,
                   std::vector<char>* kept_out, hipStream_t st) {
  const int64_t n = s->n;
  const double thr = 1e-12 * (max_diag(s, st) + shift);
  DBuf G((int64_t)PB * std::max<int64_t>(k, 1) * 8), Lb(PB * PB * 8), Linv(PB * PB * 8), dropped(PB),
      kept(std::max<int64_t>(k, 1));
  for (int64_t m0 = 0; m0 < k; m0 += PB) {
    const int nb = (int)std::min<int64_t>(PB, k - m0);
    double* Lp = L + m0 * ld;
    kernel_columns(s, idx + m0, nb, Lp, ld, shift, st);
    if (m0 > 0) {
      k_gather_rows<<<cdiv((int64_t)nb * m0, 256), 256, 0, st>>>(L, ld, idx + m0, nb, m0, G.as<double>());
      LAUNCHCHK();
      gemm64((int)n, nb, (int)m0, -1.0, View64{L, 1, ld}, View64{G.as<double>(), m0, 1}, 1.0, Lp, 1, ld, false, st);
    }
    k_panel_chol<<<1, 256, 0, st>>>(Lp, ld, idx + m0, nb, thr, Lb.as<double>(), Linv.as<double>(),
                                    dropped.as<unsigned char>());
    LAUNCHCHK();
    // panel <- panel Linv^T; in place is safe: one 128-row tile covers all nb columns
    gemm64((int)n, nb, nb, 1.0, View64{Lp, 1, ld}, View64{Linv.as<double>(), PB, 1}, 0.0, Lp, 1, ld, false, st);
    k_set_kept<<<1, PB, 0, st>>>(dropped.as<unsigned char>(), nb, kept.as<unsigned char>() + m0);
    LAUNCHCHK();
    k_panel_fix<<<nb, 256, 0, st>>>(L, n, ld, idx, kept.as<unsigned char>(), m0, nb, Lb.as<double>());
    LAUNCHCHK();
  }
  std::vector<char> hk(std::max<int64_t>(k, 1));
  HIPCHK(hipMemcpyAsync(hk.data(), kept.get(), k, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  int64_t keff = 0;
  for (int64_t j = 0; j < k; ++j) keff += hk[j] ? 1 : 0;
  if (kept_out) kept_out->assign(hk.begin(), hk.begin() + k);
  return keff;
}

// ----------------------------------------------------------------- build ----
__global__ void k_f64_to_f32(const double* a, float* b, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = (float)a[e];
}
__global__ void k_add_diag(double* C, int64_t k, int64_t ld, double lam) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) C[i + i * ld] += lam;
}

struct EpiStore64 {
  double* C; int64_t ldc; int M, N;
  template <typename T, int TM, int TN, class Acc>
  __device__ void run(const Acc (&acc)[TM][TN], const FragCoord& f, char*) const {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = f.row(i, v), c = f.col(j);
          if (r < M && c < N) C[r + (int64_t)c * ldc] = (double)acc[i][j][v];
        }
  }
};

// core = L^T L (k x k, column-major, ldc) from FP64 or FP32 storage, FP64 arithmetic.
template <typename TI>
static void gram_cols(const TI* L, int64_t n, int64_t ld, int64_t k, double* C, int64_t ldc, hipStream_t st) {
  ScalarArgs<TI> g{};
  g.M = (int)k;
  g.N = (int)k;
  g.nseg = 1;
  g.seg[0] = SegS<TI>{L, ld, 1, L, ld, 1, (int)n};
  EpiStore64 e{C, ldc, (int)k, (int)k};
  gemm_scalar_kernel<double, 128, 128, 16, true, true, EpiStore64, TI><<<dim3(cdiv(k, 128), cdiv(k, 128)), 256, 0, st>>>(g, e);
  LAUNCHCHK();
}

ffk_precond* precond_build(ffk_system* s, const int64_t* idx, int64_t k, double lambda, int store, bool* dropped_any,
                           hipStream_t st) {
  require(store == FFK_FP64 || store == FFK_FP32, "precond_build: store_L must be FFK_FP64 or FFK_FP32");
  const int64_t n = s->n;
  const int64_t ld = pad64(n);
  std::unique_ptr<ffk_precond> P(new ffk_precond());
  P->ctx = s->ctx;
  P->n = n;
  P->ld = ld;
  P->k = k;
  P->lambda = lambda;
  P->store = store;
  DBuf L64(ld * k * 8);
  HIPCHK(hipMemsetAsync(L64.get(), 0, ld * k * 8, st));
  std::vector<char> kept;
  const int64_t keff = icd_forced(s, idx, k, 0.0, L64.as<double>(), ld, &kept, st);
  *dropped_any = keff < k;
  // compact the kept columns to the front (in order; a column only moves left)
  {
    int64_t w = 0;
    for (int64_t j = 0; j < k; ++j) {
      if (!kept[j]) continue;
      if (w != j)
        HIPCHK(hipMemcpyAsync(L64.as<double>() + w * ld, L64.as<double>() + j * ld, ld * 8, hipMemcpyDeviceToDevice, st));
      ++w;
    }
  }
  P->k_eff = keff;
  const int64_t ke = std::max<int64_t>(keff, 1);
  const int64_t ldf = pad64(ke);
  P->ldf = ldf;
  DBuf core(ldf * ke * 8);
  HIPCHK(hipMemsetAsync(core.get(), 0, ldf * ke * 8, st));
  if (store == FFK_FP64) {
    if (keff > 0) gram_cols<double>(L64.as<double>(), n, ld, keff, core.as<double>(), ldf, st);
    P->L = std::move(L64);
  } else {
    P->L.alloc(ld * ke * 4);
    k_f64_to_f32<<<cdiv(ld * keff, 256), 256, 0, st>>>(L64.as<double>(), P->L.as<float>(), ld * keff);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(st));
    L64.release();
    if (keff > 0) gram_cols<float>(P->L.as<float>(), n, ld, keff, core.as<double>(), ldf, st);
  }
  if (keff > 0) {
    k_add_diag<<<cdiv(keff, 256), 256, 0, st>>>(core.as<double>(), keff, ldf, lambda);
    LAUNCHCHK();
    const int64_t bad = potrf_lower(core.as<double>(), keff, ldf, st);
    if (bad >= 0) fail(FFK_ERR_NOT_SPD, "precond_build: core lambda I + L^T L is not positive definite");
    trtri_lower(core.as<double>(), keff, ldf, st);
  }
  P->Finv = std::move(core);
  P->y.alloc(ldf * 8);
  P->t1.alloc(ldf * 8);
  P->t.alloc(ldf * 8);
  {
    const int64_t wt = (int64_t)cdiv(ld, 2048) * ke;           // transposed-product partials
    const int64_t wn = (int64_t)cdiv(ke, 64) * (ld + 1024);    // direct-product partials
    P->work.alloc(std::max(wt, wn) * 8);
  }
  P->bytes = (int64_t)(P->L.bytes() + P->Finv.bytes() + P->work.bytes() + 3 * ldf * 8);
  HIPCHK(hipStreamSynchronize(st));
  return P.release();
}

// ----------------------------------------------------------------- apply ----
// The four products of the apply are memory-bound GEMVs over column-major
// matrices whose leading dimension is a multiple of 64 with zero padding.
// Each lane streams 4 consecutive rows per 16-byte load (two loads for FP64),
// and the work is split over a 2-D grid so that enough loads are in flight to
// run at HBM rate; partial results are combined by a second small pass in a
// fixed order (deterministic).
template <typename TA> struct Row4;
template <> struct Row4<float> {
  __device__ static inline void load(const float* p, double (&v)[4]) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  }
};
template <> struct Row4<double> {
  __device__ static inline void load(const double* p, double (&v)[4]) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
};

constexpr int TR_ROWS = 2048;   // rows per block, transposed product (8 loads per lane per column)
constexpr int TR_COLS = 16;     // columns per block (4 per wave)
constexpr int DN_ROWS = 1024;   // rows per block, direct product (one 4-row load per lane per column)
constexpr int DN_COLS = 64;     // columns per block

// part[blockIdx.y][c] = sum_{i in block rows} A[i + c lda] x[i]   (i >= c only when tri)
template <typename TA>
__global__ __launch_bounds__(256) void k_gemvt_part(const TA* __restrict__ A, int64_t nrow, int64_t lda, int64_t ncol,
                                                    const double* __restrict__ x, double* __restrict__ part, int tri) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.y * TR_ROWS + 4 * lane;
  const int64_t c0 = (int64_t)blockIdx.x * TR_COLS + wave * 4;
  double xr[TR_ROWS / 256][4];
#pragma unroll
  for (int q = 0; q < TR_ROWS / 256; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = i0 + 256 * q + e;
      xr[q][e] = i < nrow ? x[i] : 0.0;
    }
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) {
    const int64_t c = c0 + cc;
    if (c >= ncol) break;
    const TA* col = A + c * lda;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int q = 0; q < TR_ROWS / 256; ++q) {
      const int64_t i = i0 + 256 * q;
      if (i < nrow) {
        double v[4];
        Row4<TA>::load(col + i, v);
        if (tri) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (i + e < c) v[e] = 0.0;
        }
        a0 += v[0] * xr[q][0] + v[1] * xr[q][1];
        a1 += v[2] * xr[q][2] + v[3] * xr[q][3];
      }
    }
    double a = a0 + a1;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if (lane == 0) part[(int64_t)blockIdx.y * ncol + c] = a;
  }
}

// y[c] = sum_b part[b][c]
__global__ void k_sum_rows(const double* __restrict__ part, int nb, int64_t ncol, double* __restrict__ y) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  double a0 = 0.0, a1 = 0.0;
  int b = 0;
  for (; b + 2 <= nb; b += 2) {
    a0 += part[(int64_t)b * ncol + c];
    a1 += part[(int64_t)(b + 1) * ncol + c];
  }
  if (b < nb) a0 += part[(int64_t)b * ncol + c];
  y[c] = a0 + a1;
}

// part[blockIdx.y][i] = sum_{c in block columns} A[i + c lda] t[c]   (c <= i only when tri)
template <typename TA>
__global__ __launch_bounds__(256) void k_gemvn_part(const TA* __restrict__ A, int64_t nrow, int64_t lda, int64_t ncol,
                                                    const double* __restrict__ t, double* __restrict__ part, int tri) {
  __shared__ double ts[DN_COLS];
  const int64_t c0 = (int64_t)blockIdx.y * DN_COLS;
  const int nc = (int)(ncol - c0 < DN_COLS ? ncol - c0 : DN_COLS);
  if (threadIdx.x < DN_COLS) ts[threadIdx.x] = threadIdx.x < nc ? t[c0 + threadIdx.x] : 0.0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * DN_ROWS + 4 * threadIdx.x;
  if (i >= nrow) return;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  const TA* base = A + c0 * lda + i;
  int cc = 0;
  for (; cc + 4 <= nc; cc += 4) {
    double v0[4], v1[4], v2[4], v3[4];
    Row4<TA>::load(base + (int64_t)cc * lda, v0);
    Row4<TA>::load(base + (int64_t)(cc + 1) * lda, v1);
    Row4<TA>::load(base + (int64_t)(cc + 2) * lda, v2);
    Row4<TA>::load(base + (int64_t)(cc + 3) * lda, v3);
    const double t0 = ts[cc], t1 = ts[cc + 1], t2 = ts[cc + 2], t3 = ts[cc + 3];
    const int64_t c = c0 + cc;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (!tri || c + 3 <= i + e) {
        a[e] += v0[e] * t0 + v1[e] * t1 + v2[e] * t2 + v3[e] * t3;
      } else {
        if (c <= i + e) a[e] += v0[e] * t0;
        if (c + 1 <= i + e) a[e] += v1[e] * t1;
        if (c + 2 <= i + e) a[e] += v2[e] * t2;
      }
    }
  }
  for (; cc < nc; ++cc) {
    double v[4];
    Row4<TA>::load(base + (int64_t)cc * lda, v);
    const double tc = ts[cc];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (!tri || c0 + cc <= i + e) a[e] += v[e] * tc;
  }
  double* out = part + (int64_t)blockIdx.y * ((int64_t)gridDim.x * DN_ROWS) + i;
#pragma unroll
  for (int e = 0; e < 4; ++e) out[e] = a[e];
}

// out_i = r ? alpha (r_i - s_i) : s_i with s_i = sum_b part[b][i]
__global__ void k_finish_n(const double* __restrict__ part, int nb, int64_t stride, int64_t nrow,
                           const double* __restrict__ r, double alpha, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrow) return;
  double a0 = 0.0, a1 = 0.0;
  int b = 0;
  for (; b + 2 <= nb; b += 2) {
    a0 += part[(int64_t)b * stride + i];
    a1 += part[(int64_t)(b + 1) * stride + i];
  }
  if (b < nb) a0 += part[(int64_t)b * stride + i];
  const double sm = a0 + a1;
  out[i] = r ? alpha * (r[i] - sm) : sm;
}

template <typename TA>
static void gemv_t(const TA* A, int64_t nrow, int64_t lda, int64_t ncol, const double* x, double* y, int tri,
                   double* part, hipStream_t st, int clk = -1) {
  const int nb = cdiv(nrow, TR_ROWS);
  if (clk >= 0) clk_begin(clk, st);
  k_gemvt_part<TA><<<dim3(cdiv(ncol, TR_COLS), nb), 256, 0, st>>>(A, nrow, lda, ncol, x, part, tri);
  LAUNCHCHK();
  if (clk >= 0) clk_end(clk, st);
  k_sum_rows<<<cdiv(ncol, 256), 256, 0, st>>>(part, nb, ncol, y);
  LAUNCHCHK();
}

template <typename TA>
static void gemv_n(const TA* A, int64_t nrow, int64_t lda, int64_t ncol, const double* t, const double* r,
                   double alpha, double* out, int tri, double* part, hipStream_t st, int clk = -1) {
  const int nb = cdiv(ncol, DN_COLS);
  const int gx = cdiv(nrow, DN_ROWS);
  if (clk >= 0) clk_begin(clk, st);
  k_gemvn_part<TA><<<dim3(gx, nb), 256, 0, st>>>(A, nrow, lda, ncol, t, part, tri);
  LAUNCHCHK();
  if (clk >= 0) clk_end(clk, st);
  k_finish_n<<<cdiv(nrow, 256), 256, 0, st>>>(part, nb, (int64_t)gx * DN_ROWS, nrow, r, alpha, out);
  LAUNCHCHK();
}

template <typename TA>
static void apply_t(const ffk_precond* P, const double* r, double* z, hipStream_t st) {
  const TA* L = P->L.as<TA>();
  const int64_t n = P->n, k = P->k_eff;
  const double* F = P->Finv.as<double>();
  double* part = P->work.as<double>();
  gemv_t<TA>(L, n, P->ld, k, r, P->y.as<double>(), 0, part, st, CLK_GEMV_T);
  clk_begin(CLK_CORE, st);
  gemv_n<double>(F, k, P->ldf, k, P->y.as<double>(), nullptr, 1.0, P->t1.as<double>(), 1, part, st);
  gemv_t<double>(F, k, P->ldf, k, P->t1.as<double>(), P->t.as<double>(), 1, part, st);
  clk_end(CLK_CORE, st);
  gemv_n<TA>(L, n, P->ld, k, P->t.as<double>(), r, 1.0 / P->lambda, z, 0, part, st, CLK_GEMV_N);
}

__global__ void k_scale(const double* r, double a, int64_t n, double* z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = a * r[i];
}

void precond_apply(const ffk_precond* P, const double* r, double* z, hipStream_t st) {
  if (P->k_eff == 0) {
    k_scale<<<cdiv(P->n, 256), 256, 0, st>>>(r, 1.0 / P->lambda, P->n, z);
    LAUNCHCHK();
    return;
  }
  if (P->store == FFK_FP64) apply_t<double>(P, r, z, st);
  else apply_t<float>(P, r, z, st);
}

// L (n x k_eff) as a dense column-major FP64 matrix with leading dimension n.
__global__ void k_export(const void* L, int store, int64_t n, int64_t ld, int64_t k, double* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int64_t c = e / n, i = e % n;
  out[e] = store == FFK_FP64 ? static_cast<const double*>(L)[i + c * ld] : (double)static_cast<const float*>(L)[i + c * ld];
}

void precond_export(const ffk_precond* P, double* L, hipStream_t st) {
  const int64_t cnt = P->n * P->k_eff;
  if (cnt == 0) return;
  k_export<<<cdiv(cnt, 256), 256, 0, st>>>(P->L.get(), P->store, P->n, P->ld, P->k_eff, L);
  LAUNCHCHK();
}

}  // namespace ffk
