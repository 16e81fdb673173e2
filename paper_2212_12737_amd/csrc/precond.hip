// Nystroem preconditioner P = L L^T + lambda I (Eq. 3-5) and its Woodbury
// inverse (Eq. 4).
//
// L is built as the incomplete Cholesky factor with pivots forced to the
// selected column order: for identical columns this equals the Nystroem
// factor K_nk K_kk^-1 K_nk^T (section 3).  The columns are processed in panels
// of 64: (1) evaluate the raw kernel columns, (2) subtract the contribution of
// all earlier panels with one FP64 MFMA GEMM, (3) factor the 64 x 64 pivot
// block (dropping columns whose remaining diagonal is <= 1e-12 max diag K),
// (4) solve the panel rows against it, (5) zero the rows of earlier pivots and
// set the exact pivot values, as Algorithm 1 leaves them.
// The core lambda I + L^T L is formed from the stored L (FP64 or FP32) in FP64,
// factored, and its triangular inverse Finv kept, so that
//   z = lambda^-1 (r - L Finv^T Finv L^T r).
#include "gemm.hpp"

namespace ffk {

constexpr int PB = 64;   // panel width

// G[c][j] = L[idx[c] + j n] for c < nb, j < m0  (row-major nb x m0)
__global__ void k_gather_rows(const double* L, int64_t n, const int64_t* idx, int nb, int64_t m0, double* G) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nb * m0) return;
  const int c = (int)(e / m0);
  const int64_t j = e % m0;
  G[e] = L[idx[c] + j * n];
}

// Factor the nb x nb pivot block T[c][c'] = panel[idx[c], c'] with drops.
// Writes Lb (row-major PB x PB, lower) and drop flags (1 = dropped).
__global__ __launch_bounds__(256) void k_panel_chol(const double* Lp, int64_t n, const int64_t* idx, int nb,
                                                    double thr, double* Lb, unsigned char* dropped) {
  __shared__ double T[PB][PB + 1];
  __shared__ unsigned char dr[PB];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int r = e % nb, c = e / nb;
    T[r][c] = Lp[idx[r] + (int64_t)c * n];
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
}

// panel row i: x Lb^T = a  (forward substitution, dropped columns -> 0)
__global__ __launch_bounds__(256) void k_panel_trsm(double* Lp, int64_t n, int nb, const double* Lb,
                                                    const unsigned char* dropped) {
  __shared__ double S[PB][PB + 1];
  __shared__ unsigned char dr[PB];
  const int tid = threadIdx.x;
  for (int e = tid; e < PB * PB; e += 256) S[e / PB][e % PB] = Lb[e];
  if (tid < PB) dr[tid] = tid < nb ? dropped[tid] : 1;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
  if (i >= n) return;
  double x[PB];
#pragma unroll
  for (int c = 0; c < PB; ++c) x[c] = c < nb ? Lp[i + (int64_t)c * n] : 0.0;
#pragma unroll
  for (int c = 0; c < PB; ++c) {
    double v = x[c];
#pragma unroll
    for (int q = 0; q < PB; ++q)
      if (q < c) v -= x[q] * S[c][q];
    x[c] = dr[c] ? 0.0 : v / S[c][c];
  }
#pragma unroll
  for (int c = 0; c < PB; ++c)
    if (c < nb) Lp[i + (int64_t)c * n] = x[c];
}

// Exact zeros at earlier pivot rows and the exact pivot value on the diagonal.
__global__ void k_panel_fix(double* L, int64_t n, const int64_t* idx, const unsigned char* kept, int64_t m0, int nb,
                            const double* Lb) {
  const int c = blockIdx.x;
  if (!kept[m0 + c]) return;
  double* col = L + (m0 + c) * n;
  for (int64_t j = threadIdx.x; j < m0 + c; j += blockDim.x)
    if (kept[j]) col[idx[j]] = 0.0;
  if (threadIdx.x == 0) col[idx[m0 + c]] = Lb[c * PB + c];
}

__global__ void k_set_kept(const unsigned char* dropped, int nb, unsigned char* kept) {
  const int c = threadIdx.x;
  if (c < nb) kept[c] = dropped[c] ? 0 : 1;
}

int64_t icd_forced(ffk_system* s, const int64_t* idx, int64_t k, double shift, double* L, std::vector<char>* kept_out,
                   hipStream_t st) {
  const int64_t n = s->n;
  const double thr = 1e-12 * (max_diag(s, st) + shift);
  DBuf G((int64_t)PB * std::max<int64_t>(k, 1) * 8), Lb(PB * PB * 8), dropped(PB), kept(std::max<int64_t>(k, 1));
  for (int64_t m0 = 0; m0 < k; m0 += PB) {
    const int nb = (int)std::min<int64_t>(PB, k - m0);
    double* Lp = L + m0 * n;
    kernel_columns(s, idx + m0, nb, Lp, n, shift, st);
    if (m0 > 0) {
      k_gather_rows<<<cdiv((int64_t)nb * m0, 256), 256, 0, st>>>(L, n, idx + m0, nb, m0, G.as<double>());
      LAUNCHCHK();
      gemm64((int)n, nb, (int)m0, -1.0, View64{L, 1, n}, View64{G.as<double>(), m0, 1}, 1.0, Lp, 1, n, false, st);
    }
    k_panel_chol<<<1, 256, 0, st>>>(Lp, n, idx + m0, nb, thr, Lb.as<double>(), dropped.as<unsigned char>());
    LAUNCHCHK();
    k_panel_trsm<<<cdiv(n, 256), 256, 0, st>>>(Lp, n, nb, Lb.as<double>(), dropped.as<unsigned char>());
    LAUNCHCHK();
    k_set_kept<<<1, PB, 0, st>>>(dropped.as<unsigned char>(), nb, kept.as<unsigned char>() + m0);
    LAUNCHCHK();
    k_panel_fix<<<nb, 256, 0, st>>>(L, n, idx, kept.as<unsigned char>(), m0, nb, Lb.as<double>());
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
__global__ void k_add_diag(double* C, int64_t k, double lam) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) C[i + i * k] += lam;
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

// core = L^T L (k x k, column-major) from FP64 or FP32 storage, FP64 arithmetic.
template <typename TI>
static void gram_cols(const TI* L, int64_t n, int64_t k, double* C, hipStream_t st) {
  ScalarArgs<TI> g{};
  g.M = (int)k;
  g.N = (int)k;
  g.nseg = 1;
  g.seg[0] = SegS<TI>{L, n, 1, L, n, 1, (int)n};
  EpiStore64 e{C, k, (int)k, (int)k};
  gemm_scalar_kernel<double, 128, 128, 16, true, true, EpiStore64, TI><<<dim3(cdiv(k, 128), cdiv(k, 128)), 256, 0, st>>>(g, e);
  LAUNCHCHK();
}

ffk_precond* precond_build(ffk_system* s, const int64_t* idx, int64_t k, double lambda, int store, bool* dropped_any,
                           hipStream_t st) {
  require(store == FFK_FP64 || store == FFK_FP32, "precond_build: store_L must be FFK_FP64 or FFK_FP32");
  const int64_t n = s->n;
  std::unique_ptr<ffk_precond> P(new ffk_precond());
  P->ctx = s->ctx;
  P->n = n;
  P->k = k;
  P->lambda = lambda;
  P->store = store;
  DBuf L64(n * k * 8);
  std::vector<char> kept;
  const int64_t keff = icd_forced(s, idx, k, 0.0, L64.as<double>(), &kept, st);
  *dropped_any = keff < k;
  // compact the kept columns to the front (in order; a column only moves left)
  {
    int64_t w = 0;
    for (int64_t j = 0; j < k; ++j) {
      if (!kept[j]) continue;
      if (w != j)
        HIPCHK(hipMemcpyAsync(L64.as<double>() + w * n, L64.as<double>() + j * n, n * 8, hipMemcpyDeviceToDevice, st));
      ++w;
    }
  }
  P->k_eff = keff;
  const int64_t ke = std::max<int64_t>(keff, 1);
  DBuf core(ke * ke * 8);
  if (store == FFK_FP64) {
    if (keff > 0) gram_cols<double>(L64.as<double>(), n, keff, core.as<double>(), st);
    P->L = std::move(L64);
  } else {
    P->L.alloc(n * ke * 4);
    k_f64_to_f32<<<cdiv(n * keff, 256), 256, 0, st>>>(L64.as<double>(), P->L.as<float>(), n * keff);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(st));
    L64.release();
    if (keff > 0) gram_cols<float>(P->L.as<float>(), n, keff, core.as<double>(), st);
  }
  if (keff > 0) {
    k_add_diag<<<cdiv(keff, 256), 256, 0, st>>>(core.as<double>(), keff, lambda);
    LAUNCHCHK();
    const int64_t bad = potrf_lower(core.as<double>(), keff, keff, st);
    if (bad >= 0) fail(FFK_ERR_NOT_SPD, "precond_build: core lambda I + L^T L is not positive definite");
    trtri_lower(core.as<double>(), keff, keff, st);
  }
  P->Finv = std::move(core);
  P->y.alloc(ke * 8);
  P->t1.alloc(ke * 8);
  P->t.alloc(ke * 8);
  P->bytes = (int64_t)(P->L.bytes() + P->Finv.bytes() + 3 * ke * 8);
  HIPCHK(hipStreamSynchronize(st));
  return P.release();
}

// ----------------------------------------------------------------- apply ----
// y_c = sum_i A[i + c lda] x_i  for c < ncol (one wave per column; optional
// triangular start row c when tri, i.e. only rows i >= c).
template <typename TA>
__global__ __launch_bounds__(256) void k_gemv_t(const TA* A, int64_t nrow, int64_t lda, int64_t ncol,
                                                const double* x, double* y, bool tri) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= ncol) return;
  const TA* col = A + c * lda;
  double a0 = 0.0, a1 = 0.0;
  int64_t i = (tri ? c : 0) + lane;
  for (; i + 64 < nrow; i += 128) {
    a0 += (double)col[i] * x[i];
    a1 += (double)col[i + 64] * x[i + 64];
  }
  if (i < nrow) a0 += (double)col[i] * x[i];
  double v = a0 + a1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) y[c] = v;
}

// out_i = alpha * (r_i - sum_c A[i + c lda] t_c)  (or, with r == null,
// out_i = sum_c A[i + c lda] t_c restricted to c <= i when tri).  Thread per row.
template <typename TA>
__global__ __launch_bounds__(256) void k_gemv_n(const TA* A, int64_t nrow, int64_t lda, int64_t ncol,
                                                const double* t, const double* r, double alpha, double* out,
                                                bool tri) {
  constexpr int CH = 2048;
  __shared__ double st_[CH];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int64_t c0 = 0; c0 < ncol; c0 += CH) {
    const int64_t cn = ncol - c0 < CH ? ncol - c0 : CH;
    __syncthreads();
    for (int64_t c = threadIdx.x; c < cn; c += 256) st_[c] = t[c0 + c];
    __syncthreads();
    if (i < nrow) {
      int64_t cend = cn;
      if (tri) {
        const int64_t lim = i - c0 + 1;   // columns c <= i
        cend = lim < 0 ? 0 : (lim < cn ? lim : cn);
      }
      const TA* Ai = A + i + c0 * lda;
      int64_t c = 0;
      for (; c + 4 <= cend; c += 4) {
        a0 += (double)Ai[c * lda] * st_[c];
        a1 += (double)Ai[(c + 1) * lda] * st_[c + 1];
        a2 += (double)Ai[(c + 2) * lda] * st_[c + 2];
        a3 += (double)Ai[(c + 3) * lda] * st_[c + 3];
      }
      for (; c < cend; ++c) a0 += (double)Ai[c * lda] * st_[c];
    }
  }
  if (i < nrow) {
    const double s = (a0 + a1) + (a2 + a3);
    out[i] = r ? alpha * (r[i] - s) : s;
  }
}

template <typename TA>
static void apply_t(const ffk_precond* P, const double* r, double* z, hipStream_t st) {
  const TA* L = P->L.as<TA>();
  const int64_t n = P->n, k = P->k_eff;
  const double* F = P->Finv.as<double>();
  k_gemv_t<TA><<<cdiv(k, 4), 256, 0, st>>>(L, n, n, k, r, P->y.as<double>(), false);
  LAUNCHCHK();
  k_gemv_n<double><<<cdiv(k, 256), 256, 0, st>>>(F, k, k, k, P->y.as<double>(), nullptr, 1.0, P->t1.as<double>(), true);
  LAUNCHCHK();
  k_gemv_t<double><<<cdiv(k, 4), 256, 0, st>>>(F, k, k, k, P->t1.as<double>(), P->t.as<double>(), true);
  LAUNCHCHK();
  k_gemv_n<TA><<<cdiv(n, 256), 256, 0, st>>>(L, n, n, k, P->t.as<double>(), r, 1.0 / P->lambda, z, false);
  LAUNCHCHK();
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

__global__ void k_f32_to_f64(const float* a, double* b, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = (double)a[e];
}

void precond_export(const ffk_precond* P, double* L, hipStream_t st) {
  const int64_t cnt = P->n * P->k_eff;
  if (cnt == 0) return;
  if (P->store == FFK_FP64) {
    HIPCHK(hipMemcpyAsync(L, P->L.get(), cnt * 8, hipMemcpyDeviceToDevice, st));
  } else {
    k_f32_to_f64<<<cdiv(cnt, 256), 256, 0, st>>>(P->L.as<float>(), L, cnt);
    LAUNCHCHK();
  }
}

}  // namespace ffk
