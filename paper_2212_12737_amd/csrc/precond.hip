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
// The core C = lambda I + L^T L is formed from the stored L (FP64, FP32 or BF16)
// in FP64 and factored, C = F F^T, and the triangular inverse F^-1 is kept:
// z = lambda^-1 (r - L F^-T F^-1 L^T r), two passes over L and two over the
// triangle of F^-1.  (Multiplying out F^-T F^-1 into one dense inverse would
// save a pass but applies far less accurately at small lambda: the solve
// then needs half again as many iterations.)
// L and F^-1 are column-major with leading dimensions padded to 64 elements
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

// The same from FP32 storage.
__global__ void k_gather_rows32(const float* L, int64_t ld, const int64_t* idx, int nb, int64_t m0, float* G) {
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
// (The panel's column c is at L + (m0 - col0 + c) ld: col0 = 0 when L is the
// whole factor, col0 = m0 when L is a panel buffer of its own.)
__global__ void k_panel_fix(double* L, int64_t n, int64_t ld, const int64_t* idx, const unsigned char* kept,
                            int64_t m0, int nb, const double* Lb, int64_t col0) {
  const int c = blockIdx.x;
  double* col = L + (m0 - col0 + c) * ld;
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
    k_panel_fix<<<nb, 256, 0, st>>>(L, n, ld, idx, kept.as<unsigned char>(), m0, nb, Lb.as<double>(), 0);
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

__global__ void k_cols_to_f32(const double* P, int64_t ld, int64_t n, int nb, float* L32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ld * nb) return;
  L32[e] = (float)P[e];
}

// icd_forced with the factor kept in FP32: each panel is computed in FP64
// (raw columns, update by the earlier FP32 columns with FP64 accumulation,
// pivot-block factorization and drops) and then stored in FP32.  Needs
// n k 4 + n 64 8 bytes instead of n k 8.
static int64_t icd_forced_f32(ffk_system* s, const int64_t* idx, int64_t k, float* L32, int64_t ld,
                              std::vector<char>* kept_out, hipStream_t st) {
  const int64_t n = s->n;
  const double thr = 1e-12 * max_diag(s, st);
  DBuf P64(ld * PB * 8), G((int64_t)PB * std::max<int64_t>(k, 1) * 4), Lb(PB * PB * 8), Linv(PB * PB * 8),
      dropped(PB), kept(std::max<int64_t>(k, 1));
  double* Lp = P64.as<double>();
  for (int64_t m0 = 0; m0 < k; m0 += PB) {
    const int nb = (int)std::min<int64_t>(PB, k - m0);
    HIPCHK(hipMemsetAsync(Lp, 0, ld * PB * 8, st));
    kernel_columns(s, idx + m0, nb, Lp, ld, 0.0, st);
    if (m0 > 0) {
      k_gather_rows32<<<cdiv((int64_t)nb * m0, 256), 256, 0, st>>>(L32, ld, idx + m0, nb, m0, G.as<float>());
      LAUNCHCHK();
      gemm64_in32((int)n, nb, (int)m0, -1.0, View32{L32, 1, ld}, View32{G.as<float>(), m0, 1}, 1.0, Lp, 1, ld, st);
    }
    k_panel_chol<<<1, 256, 0, st>>>(Lp, ld, idx + m0, nb, thr, Lb.as<double>(), Linv.as<double>(),
                                    dropped.as<unsigned char>());
    LAUNCHCHK();
    gemm64((int)n, nb, nb, 1.0, View64{Lp, 1, ld}, View64{Linv.as<double>(), PB, 1}, 0.0, Lp, 1, ld, false, st);
    k_set_kept<<<1, PB, 0, st>>>(dropped.as<unsigned char>(), nb, kept.as<unsigned char>() + m0);
    LAUNCHCHK();
    k_panel_fix<<<nb, 256, 0, st>>>(Lp, n, ld, idx, kept.as<unsigned char>(), m0, nb, Lb.as<double>(), m0);
    LAUNCHCHK();
    k_cols_to_f32<<<cdiv(ld * nb, 256), 256, 0, st>>>(Lp, ld, n, nb, L32 + m0 * ld);
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
// The stored factor, and in L64 an FP64 copy of exactly the stored values,
// so that the core can be formed from L64 on the FP64 MFMA engine.
__global__ void k_round_f32(double* L64, float* L32, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float f = (float)L64[e];
  L32[e] = f;
  L64[e] = (double)f;
}
__global__ void k_round_bf16(double* L64, bf16_t* Lb, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const bf16_t h = f2bf((float)L64[e]);
  Lb[e] = h;
  L64[e] = (double)bf2f(h);
}
// zero the strict upper triangle of a column-major k x k matrix (ld rows)
__global__ void k_zero_upper(double* A, int64_t k, int64_t ld) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ld * k) return;
  const int64_t r = e % ld, c = e / ld;
  if (r < c) A[e] = 0.0;
}
// B = A^T for column-major k x k matrices with leading dimension ld (the
// padding rows of B are left as they are)
__global__ void k_transpose_sq(const double* __restrict__ A, int64_t k, int64_t ld, double* __restrict__ B) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
  for (int q = ty; q < 32; q += 8)
    if (r0 + tx < k && c0 + q < k) tile[q][tx] = A[(r0 + tx) + (c0 + q) * ld];
  __syncthreads();
  for (int q = ty; q < 32; q += 8)
    if (c0 + tx < k && r0 + q < k) B[(c0 + tx) + (r0 + q) * ld] = tile[tx][q];
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

// core[r + c ldc] = sum_z part[z][r][c] for r >= c (the lower triangle),
// from the split-K partials of gram_dma (plane = k ldp doubles per split)
__global__ void k_gram_reduce(const double* __restrict__ part, int splits, int64_t k, int64_t ldp, int64_t plane,
                              double* __restrict__ C, int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * k) return;
  const int64_t r = e / k, c = e % k;
  if (r < c) return;
  double a = 0.0;
  for (int z = 0; z < splits; ++z) a += part[(int64_t)z * plane + r * ldp + c];
  C[r + c * ldc] = a;
}

// Rows of the Gram operand are padded to this (the tile of gram_dma).
constexpr int64_t kGramTile = 128;

// Lower triangle of core = L^T L from the FP64 factor on the pipelined FP64
// MFMA engine.  The columns of the column-major L are the K-contiguous
// operand rows (K = ld, zero padding rows), for A and B alike; L holds kp
// columns (a multiple of the tile) so that every tile row is allocated.  Only
// tiles on or below the diagonal run, split over K for enough workgroups,
// and a fixed-order pass sums the splits.
static void gram_dma(const double* L, int64_t ld, int64_t k, int64_t kp, double* C, int64_t ldc, hipStream_t st) {
  typedef DmaTile<kGramTile, kGramTile, 2, 2, 4> TG;
  require(kp % kGramTile == 0 && kp >= k && ld % 8 == 0, "gram_dma: operand padding");
  const int64_t nt = kp / kGramTile;
  const int64_t lower = nt * (nt + 1) / 2;
  int splits = 1;
  while (lower * splits < 512 && splits < 16 && ld / 8 >= (int64_t)splits * 2 * 64) splits *= 2;
  DBuf part((size_t)splits * k * kp * 8);
  DmaArgs g{};
  g.nseg = 1;
  g.lower_only = 1;
  g.seg[0] = SegD{L, nullptr, L, nullptr, ld, ld, (int)ld};
  EpiPart<double> e{part.as<double>(), kp, (int)k, (int)k};
  gemm_dma_kernel<double, TG, false, EpiPart<double>><<<dim3((unsigned)nt, (unsigned)nt, splits), TG::NT, 0, st>>>(g, e);
  LAUNCHCHK();
  k_gram_reduce<<<cdiv(k * k, 256), 256, 0, st>>>(part.as<double>(), splits, k, kp, k * kp, C, ldc);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));   // before the partials are freed
}

int64_t precond_work_doubles(int64_t n, int64_t ld, int64_t keff, int store);

// compact the kept columns to the front (in order; a column only moves left)
static void compact_columns(char* L, int64_t ld, int64_t esize, const std::vector<char>& kept, hipStream_t st) {
  int64_t w = 0;
  for (size_t j = 0; j < kept.size(); ++j) {
    if (!kept[j]) continue;
    if (w != (int64_t)j)
      HIPCHK(hipMemcpyAsync(L + w * ld * esize, L + (int64_t)j * ld * esize, ld * esize, hipMemcpyDeviceToDevice, st));
    ++w;
  }
}

// Rows sel of the factor L (ld) as a k x k column-major matrix (ldf): the
// factor's rows at its own pivots, lower triangular by construction.
__global__ void k_rows_at(const double* __restrict__ L, int64_t ld, const int64_t* __restrict__ sel, int64_t k,
                          int64_t ldf, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * k) return;
  const int64_t m = e / k, j = e % k;   // column m, row j
  out[m * ldf + j] = L[m * ld + sel[j]];
}

static void make_matrix_free(ffk_precond* P, ffk_system* s, const int64_t* idx, const std::vector<char>& kept,
                             hipStream_t st);

ffk_precond* precond_build(ffk_system* s, const int64_t* idx, int64_t k, double lambda, int store, bool lowmem,
                           bool* dropped_any, hipStream_t st, bool matrix_free) {
  require(store == FFK_FP64 || store == FFK_FP32 || store == FFK_BF16,
          "precond_build: store_L must be FFK_FP64, FFK_FP32 or FFK_BF16");
  require(!matrix_free || (store == FFK_FP64 && !lowmem),
          "precond_build: the matrix-free form is built from an FP64 factor");
  const int64_t n = s->n;
  const int64_t ld = pad64(n);
  std::unique_ptr<ffk_precond> P(new ffk_precond());
  P->ctx = s->ctx;
  P->n = n;
  P->ld = ld;
  P->k = k;
  P->lambda = lambda;
  P->store = store;
  if (store == FFK_FP32 && !lowmem) {
    size_t freeb = 0, total = 0;
    HIPCHK(hipMemGetInfo(&freeb, &total));
    lowmem = (double)ld * k * 12.0 > 0.9 * (double)freeb;   // FP64 factor + its FP32 copy
  }
  std::vector<char> kept;
  DBuf L64;
  int64_t keff;
  if (lowmem) {
    require(store == FFK_FP32, "precond_build: the low-memory build stores L in FP32");
    P->L.alloc(ld * k * 4);
    keff = icd_forced_f32(s, idx, k, P->L.as<float>(), ld, &kept, st);
    compact_columns(P->L.as<char>(), ld, 4, kept, st);
  } else {
    // columns padded to the Gram tile; the extra ones stay zero
    const int64_t kp = (k + kGramTile - 1) / kGramTile * kGramTile;
    L64.alloc(ld * kp * 8);
    HIPCHK(hipMemsetAsync(L64.get(), 0, ld * kp * 8, st));
    keff = icd_forced(s, idx, k, 0.0, L64.as<double>(), ld, &kept, st);
    compact_columns(L64.as<char>(), ld, 8, kept, st);
  }
  *dropped_any = keff < k;
  P->k_eff = keff;
  const int64_t ke = std::max<int64_t>(keff, 1);
  const int64_t ldf = pad64(ke);
  P->ldf = ldf;
  DBuf core(ldf * ke * 8);
  HIPCHK(hipMemsetAsync(core.get(), 0, ldf * ke * 8, st));
  if (lowmem) {
    if (keff > 0) gram_cols<float>(P->L.as<float>(), n, ld, keff, core.as<double>(), ldf, st);
  } else {
    // the core is formed from the stored factor: FP64 as is, FP32 and BF16
    // after rounding L64 to exactly the stored values
    const int64_t kp = (k + kGramTile - 1) / kGramTile * kGramTile;
    if (store == FFK_FP32) {
      P->L.alloc(ld * ke * 4);
      if (keff > 0) k_round_f32<<<cdiv(ld * keff, 256), 256, 0, st>>>(L64.as<double>(), P->L.as<float>(), ld * keff);
      LAUNCHCHK();
    } else if (store == FFK_BF16) {
      P->L.alloc(ld * ke * 2);
      if (keff > 0) k_round_bf16<<<cdiv(ld * keff, 256), 256, 0, st>>>(L64.as<double>(), P->L.as<bf16_t>(), ld * keff);
      LAUNCHCHK();
    }
    if (keff > 0) gram_dma(L64.as<double>(), ld, keff, kp, core.as<double>(), ldf, st);
    if (store == FFK_FP64) P->L = std::move(L64);
    else L64.release();
  }
  if (keff > 0) {
    k_add_diag<<<cdiv(keff, 256), 256, 0, st>>>(core.as<double>(), keff, ldf, lambda);
    LAUNCHCHK();
    const int64_t bad = potrf_lower(core.as<double>(), keff, ldf, st);
    if (bad >= 0) fail(FFK_ERR_NOT_SPD, "precond_build: core lambda I + L^T L is not positive definite");
    trtri_lower(core.as<double>(), keff, ldf, st);
    // keep F^-1 strictly lower-triangular: the apply skips the zero triangle
    k_zero_upper<<<cdiv(ldf * keff, 256), 256, 0, st>>>(core.as<double>(), keff, ldf);
    LAUNCHCHK();
  }
  P->FinvT.alloc(ldf * ke * 8);
  HIPCHK(hipMemsetAsync(P->FinvT.get(), 0, ldf * ke * 8, st));
  if (keff > 0) {
    k_transpose_sq<<<dim3(cdiv(keff, 32), cdiv(keff, 32)), 256, 0, st>>>(core.as<double>(), keff, ldf,
                                                                          P->FinvT.as<double>());
    LAUNCHCHK();
  }
  P->Finv = std::move(core);
  P->y.alloc(ldf * 8);
  P->t1.alloc(ldf * 8);
  P->t.alloc(ldf * 8);
  if (matrix_free && keff > 0) {
    make_matrix_free(P.get(), s, idx, kept, st);
    P->bytes = (int64_t)(P->Finv.bytes() + P->FinvT.bytes() + P->Tinv.bytes() + P->TinvT.bytes() + P->q.bytes() +
                         P->u.bytes() + P->sel.bytes() + 3 * ldf * 8);
  } else {
    P->work.alloc(precond_work_doubles(n, ld, ke, store) * 8);
    P->bytes = (int64_t)(P->L.bytes() + P->Finv.bytes() + P->FinvT.bytes() + P->work.bytes() + 3 * ldf * 8);
  }
  HIPCHK(hipStreamSynchronize(st));
  return P.release();
}

// The matrix-free form of a built FP64 preconditioner.  The forced-order
// incomplete Cholesky interpolates K on its pivots: (L L^T)[:, S] = K[:, S],
// i.e. K[:, S] = L L_SS^T with L_SS = L[S, :] lower triangular (a pivot's row
// is zero in every later column).  Hence L = K[:, S] T^T with T = L_SS^-1,
// and the apply needs only T, the core and two kernel products:
//   L^T r = T (K r)_S,   L t = K (scatter_S T^T t).
// The core lambda I + L^T L was formed from the same FP64 factor.
static void make_matrix_free(ffk_precond* P, ffk_system* s, const int64_t* idx, const std::vector<char>& kept,
                             hipStream_t st) {
  const int64_t n = P->n, k = P->k_eff, ldf = P->ldf;
  std::vector<int64_t> h_idx(kept.size()), h_sel;
  HIPCHK(hipMemcpyAsync(h_idx.data(), idx, kept.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (size_t j = 0; j < kept.size(); ++j)
    if (kept[j]) h_sel.push_back(h_idx[j]);
  require((int64_t)h_sel.size() == k, "precond_build: kept pivots do not match the factor");
  P->sel.alloc(k * 8);
  HIPCHK(hipMemcpyAsync(P->sel.get(), h_sel.data(), k * 8, hipMemcpyHostToDevice, st));
  P->Tinv.alloc(ldf * k * 8);
  HIPCHK(hipMemsetAsync(P->Tinv.get(), 0, ldf * k * 8, st));
  k_rows_at<<<cdiv(k * k, 256), 256, 0, st>>>(P->L.as<double>(), P->ld, P->sel.as<int64_t>(), k, ldf,
                                               P->Tinv.as<double>());
  LAUNCHCHK();
  trtri_lower(P->Tinv.as<double>(), k, ldf, st);
  k_zero_upper<<<cdiv(ldf * k, 256), 256, 0, st>>>(P->Tinv.as<double>(), k, ldf);
  LAUNCHCHK();
  P->TinvT.alloc(ldf * k * 8);
  HIPCHK(hipMemsetAsync(P->TinvT.get(), 0, ldf * k * 8, st));
  k_transpose_sq<<<dim3(cdiv(k, 32), cdiv(k, 32)), 256, 0, st>>>(P->Tinv.as<double>(), k, ldf,
                                                                  P->TinvT.as<double>());
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));
  P->L.release();
  P->q.alloc(n * 8);
  P->u.alloc(n * 8);
  P->sys = s;
  P->matrix_free = true;
}

// ----------------------------------------------------------------- apply ----
// The two products of the apply with L are memory-bound GEMVs over a
// column-major matrix whose leading dimension is a multiple of 64 with zero
// padding.
// Every lane issues 16-byte loads (2 doubles, 4 floats or 8 bfloat16 of one
// column), all of a lane's loads for a tile of columns back to back, and
// accumulates in FP64.  Partial results of the 2-D grid are combined by a
// second small pass in a fixed order (deterministic).
// 16 bytes of one column: V consecutive elements, loaded raw and expanded to
// FP64 only when consumed (keeps the loads in flight cheap in registers).
template <typename TA> struct Vec16;
template <> struct Vec16<double> {
  static constexpr int V = 2;
  __device__ static inline void expand(const uint4& a, double (&v)[2]) {
    v[0] = __hiloint2double((int)a.y, (int)a.x);
    v[1] = __hiloint2double((int)a.w, (int)a.z);
  }
};
template <> struct Vec16<float> {
  static constexpr int V = 4;
  __device__ static inline void expand(const uint4& a, double (&v)[4]) {
    v[0] = __uint_as_float(a.x); v[1] = __uint_as_float(a.y);
    v[2] = __uint_as_float(a.z); v[3] = __uint_as_float(a.w);
  }
};
template <> struct Vec16<bf16_t> {
  static constexpr int V = 8;
  __device__ static inline void expand(const uint4& a, double (&v)[8]) {
    const unsigned w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[2 * e] = (double)__uint_as_float(w[e] << 16);
      v[2 * e + 1] = (double)__uint_as_float(w[e] & 0xFFFF0000u);
    }
  }
};
// The matrices of the apply are streamed once per pass (L does not fit in
// the last-level cache): non-temporal loads keep them from evicting the
// vectors and run closer to the HBM rate.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
template <typename TA> __device__ inline uint4 load16(const TA* p) {
  const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

constexpr int LT_COLS = 16;    // columns per block of the transposed product
constexpr int LN_UNROLL = 16;  // loads in flight per lane in the direct product
// columns per block of the direct product: wide, so few partial sums remain
// (on n = 126000, k = 2000: 1024 measured 2% faster than 512, 512 5% faster
// than 256)
constexpr int LN_COLS = 1024;
static_assert(LN_COLS % LN_UNROLL == 0, "direct-product column tile");

// Sum of v[0..C) over the 64 lanes of a wave, one column per lane group:
// recursive halving (each exchange step hands half of the values to the
// partner lane) followed by plain butterflies.  On return lane l holds, in
// v[0], the wave total of column lt_col<C>(l).
template <int C>
__device__ inline void wave_reduce_cols(double (&v)[C], int lane) {
  int h = C / 2;
#pragma unroll
  for (int off = 32; off >= 64 / C; off >>= 1) {
    const bool upper = (lane & off) != 0;
#pragma unroll
    for (int j = 0; j < C / 2; ++j) {
      if (j < h) {
        const double send = upper ? v[j] : v[j + h];
        const double keep = upper ? v[j + h] : v[j];
        v[j] = keep + __shfl_xor(send, off);
      }
    }
    h >>= 1;
  }
#pragma unroll
  for (int off = 32 / C; off >= 1; off >>= 1) v[0] += __shfl_xor(v[0], off);
}
template <int C> __device__ inline int lt_col(int lane) {
  int c = 0;
#pragma unroll
  for (int off = 32, bit = C / 2; off >= 64 / C; off >>= 1, bit >>= 1)
    if (lane & off) c += bit;
  return c;
}

// part[blockIdx.y][c] = sum over the block's rows i of A[i + c lda] x[i].
// Block: 256 lanes, C columns, rows [blockIdx.y rpb, +rpb) walked in chunks of
// 256 V rows.  Loads are software-pipelined: the next chunk's C loads per
// lane are in flight while the current chunk is multiplied, and the lanes
// combine their sums once, at the end.
template <typename TA, int C>
__global__ __launch_bounds__(256) void k_lt_part(const TA* __restrict__ A, int64_t nrow, int64_t lda, int64_t ncol,
                                                 const double* __restrict__ x, double* __restrict__ part,
                                                 int64_t rpb) {
  constexpr int V = Vec16<TA>::V;
  constexpr int64_t CH = 256 * V;
  __shared__ double red[4][C];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * C;
  const int64_t r0 = (int64_t)blockIdx.y * rpb;
  const int64_t r1 = r0 + rpb < nrow ? r0 + rpb : nrow;
  double acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0;
  uint4 a0[C], a1[C];
  double x0[V], x1[V];
  // i + V <= lda whenever i < nrow: i is a multiple of V and lda of 64
  auto load = [&](int64_t base, uint4 (&a)[C], double (&xr)[V]) {
    const int64_t i = base + (int64_t)threadIdx.x * V;
#pragma unroll
    for (int e = 0; e < V; ++e) xr[e] = (i + e < r1) ? x[i + e] : 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c)
      a[c] = (i < r1 && c0 + c < ncol) ? load16(A + (c0 + c) * lda + i) : make_uint4(0, 0, 0, 0);
  };
  auto mul = [&](const uint4 (&a)[C], const double (&xr)[V]) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      double v[V];
      Vec16<TA>::expand(a[c], v);
#pragma unroll
      for (int e = 0; e < V; ++e) acc[c] += v[e] * xr[e];
    }
  };
  int64_t b0 = r0;
  if (b0 < r1) load(b0, a0, x0);
  while (b0 < r1) {
    const int64_t b1 = b0 + CH;
    if (b1 < r1) load(b1, a1, x1);
    mul(a0, x0);
    if (b1 >= r1) break;
    const int64_t b2 = b1 + CH;
    if (b2 < r1) load(b2, a0, x0);
    mul(a1, x1);
    b0 = b2;
  }
  wave_reduce_cols<C>(acc, lane);
  if ((lane & (64 / C - 1)) == 0) red[wave][lt_col<C>(lane)] = acc[0];
  __syncthreads();
  if (threadIdx.x < C && c0 + threadIdx.x < ncol)
    part[(int64_t)blockIdx.y * ncol + c0 + threadIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// y[c] = sum_b part[b][c]: 16 columns per block of 256 lanes; the 16 lanes of
// column c take row blocks q, q + 16, ... and combine by a fixed butterfly
__global__ __launch_bounds__(256) void k_sum_rows(const double* __restrict__ part, int nb, int64_t ncol,
                                                  double* __restrict__ y) {
  const int64_t c = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  const int q = threadIdx.x & 15;
  double s = 0.0;
  if (c < ncol)
    for (int b = q; b < nb; b += 16) s += part[(int64_t)b * ncol + c];
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (q == 0 && c < ncol) y[c] = s;
}

// part[blockIdx.y][i] = sum over the block's columns c of A[i + c lda] t[c].
// Block: 256 lanes x V rows, LN_COLS columns.
template <typename TA>
__global__ __launch_bounds__(256) void k_ln_part(const TA* __restrict__ A, int64_t nrow, int64_t lda, int64_t ncol,
                                                 const double* __restrict__ t, double* __restrict__ part,
                                                 int64_t stride) {
  constexpr int V = Vec16<TA>::V;
  constexpr int CB = LN_COLS;
  __shared__ double ts[CB];
  const int64_t c0 = (int64_t)blockIdx.y * CB;
  const int nc = (int)(ncol - c0 < CB ? ncol - c0 : CB);
  for (int c = threadIdx.x; c < CB; c += 256) ts[c] = c < nc ? t[c0 + c] : 0.0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * (256 * V) + (int64_t)threadIdx.x * V;
  if (i >= nrow) return;
  const int cend = nc;
  double acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = 0.0;
  const TA* base = A + c0 * lda + i;
  // software-pipelined: the next LN_UNROLL loads are in flight while the
  // current ones are used
  uint4 a0[LN_UNROLL], a1[LN_UNROLL];
  auto load = [&](int cc, uint4 (&a)[LN_UNROLL]) {
#pragma unroll
    for (int u = 0; u < LN_UNROLL; ++u)
      a[u] = (cc + u < cend) ? load16(base + (int64_t)(cc + u) * lda) : make_uint4(0, 0, 0, 0);
  };
  auto mul = [&](int cc, const uint4 (&a)[LN_UNROLL]) {
#pragma unroll
    for (int u = 0; u < LN_UNROLL; ++u) {
      const double tc = ts[cc + u];   // cc + u < CB: cc < nc <= CB, a multiple of LN_UNROLL
      double v[V];
      Vec16<TA>::expand(a[u], v);
#pragma unroll
      for (int e = 0; e < V; ++e) acc[e] += v[e] * tc;
    }
  };
  int cc = 0;
  load(0, a0);
  while (cc < cend) {
    if (cc + LN_UNROLL < cend) load(cc + LN_UNROLL, a1);
    mul(cc, a0);
    if (cc + LN_UNROLL >= cend) break;
    if (cc + 2 * LN_UNROLL < cend) load(cc + 2 * LN_UNROLL, a0);
    mul(cc + LN_UNROLL, a1);
    cc += 2 * LN_UNROLL;
  }
  double* out = part + (int64_t)blockIdx.y * stride + i;
#pragma unroll
  for (int e = 0; e < V; ++e)
    if (i + e < nrow) out[e] = acc[e];
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

// z_i = alpha (r_i - sum_b part[b][i]) and the block partials of r^T z
// (fused_parts grid)
__global__ __launch_bounds__(256) void k_finish_n_dot(const double* __restrict__ part, int nb, int64_t stride,
                                                      int64_t nrow, const double* __restrict__ r, double alpha,
                                                      double* __restrict__ z, double* __restrict__ rz_part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nrow; i += (int64_t)gridDim.x * 256) {
    double a0 = 0.0, a1 = 0.0;
    int b = 0;
    for (; b + 2 <= nb; b += 2) {
      a0 += part[(int64_t)b * stride + i];
      a1 += part[(int64_t)(b + 1) * stride + i];
    }
    if (b < nb) a0 += part[(int64_t)b * stride + i];
    const double zi = alpha * (r[i] - (a0 + a1));
    z[i] = zi;
    acc += r[i] * zi;
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) rz_part[blockIdx.x] = s;
}
__global__ __launch_bounds__(256) void k_scale_dot(const double* __restrict__ r, double a, int64_t n,
                                                   double* __restrict__ z, double* __restrict__ rz_part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double zi = a * r[i];
    z[i] = zi;
    acc += r[i] * zi;
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) rz_part[blockIdx.x] = s;
}

template <typename TA>
static int64_t ln_rows() { return 256 * Vec16<TA>::V; }           // rows per block, direct product
// Row ranges of the transposed product: about 512 blocks in all (two per CU
// at its register use; 500 measured faster than 250, 1000 or 2000 on
// n = 126000, k = 2000), each a whole number of 256 V-row chunks.  Returns
// the block count along the rows; *rpb gets the rows per block.
static int64_t lt_target(int64_t ncol) {
  const int64_t cb = cdiv(ncol, LT_COLS);
  return std::max<int64_t>(1, (512 + cb / 2) / cb);
}
template <typename TA>
static int lt_row_blocks(int64_t nrow, int64_t ncol, int64_t* rpb) {
  const int64_t ch = 256 * Vec16<TA>::V;
  const int64_t nch = cdiv(nrow, ch);
  const int64_t y = std::max<int64_t>(1, std::min(lt_target(ncol), nch));
  *rpb = cdiv(nch, y) * ch;
  return (int)cdiv(nrow, *rpb);   // <= y: cdiv(a, cdiv(a, y)) <= y
}

// workspace (doubles) needed by gemv_t / gemv_n for any operand of at most
// nrow rows and ncol columns (the row-block count of the transposed product
// is at most min(lt_target, chunks of nrow), whatever the row count)
template <typename TA>
static int64_t gemv_work(int64_t nrow, int64_t ncol) {
  const int64_t wt = std::min<int64_t>(lt_target(ncol), cdiv(nrow, 256 * Vec16<TA>::V)) * ncol;
  const int64_t wn = cdiv(ncol, LN_COLS) * (cdiv(nrow, ln_rows<TA>()) * ln_rows<TA>());
  return std::max(wt, wn);
}

template <typename TA>
static void gemv_t(const TA* A, int64_t nrow, int64_t lda, int64_t ncol, const double* x, double* y, double* part,
                   hipStream_t st, int clk = -1) {
  int64_t rpb;
  const int nb = lt_row_blocks<TA>(nrow, ncol, &rpb);
  if (clk >= 0) clk_begin(clk, st);
  k_lt_part<TA, LT_COLS><<<dim3(cdiv(ncol, LT_COLS), nb), 256, 0, st>>>(A, nrow, lda, ncol, x, part, rpb);
  LAUNCHCHK();
  if (clk >= 0) clk_end(clk, st);
  k_sum_rows<<<cdiv(ncol, 16), 256, 0, st>>>(part, nb, ncol, y);
  LAUNCHCHK();
}

template <typename TA>
static void gemv_n(const TA* A, int64_t nrow, int64_t lda, int64_t ncol, const double* t, const double* r,
                   double alpha, double* out, double* part, hipStream_t st, int clk = -1) {
  const int nb = cdiv(ncol, LN_COLS);
  const int gx = cdiv(nrow, ln_rows<TA>());
  const int64_t stride = (int64_t)gx * ln_rows<TA>();
  if (clk >= 0) clk_begin(clk, st);
  k_ln_part<TA><<<dim3(gx, nb), 256, 0, st>>>(A, nrow, lda, ncol, t, part, stride);
  LAUNCHCHK();
  if (clk >= 0) clk_end(clk, st);
  k_finish_n<<<cdiv(nrow, 256), 256, 0, st>>>(part, nb, stride, nrow, r, alpha, out);
  LAUNCHCHK();
}

// The Woodbury core t = F^-T F^-1 y as two kernels of column dot products,
// one block per output and no partial sums: s_j = (column j of F^-T) . y over
// rows 0..j, then t_j = (column j of F^-1) . s over rows j..k-1.  Both
// triangles are stored with zeros in the other half, so the 16-byte loads
// start at an even row and the extra entries add zero; rows at or beyond k
// are never read.  Ordinary (cached) loads: the 2 x 8 k^2 bytes can stay in
// the last-level cache between iterations.
template <bool FROM_DIAG>
__global__ __launch_bounds__(256) void k_tri_dots(const double* __restrict__ A, int64_t lda, int64_t k,
                                                  const double* __restrict__ x, double* __restrict__ out) {
  __shared__ double red[4];
  const int64_t j = blockIdx.x;
  const int64_t lo = FROM_DIAG ? (j & ~(int64_t)1) : 0;
  const int64_t hi = FROM_DIAG ? k : j + 1;
  const double* col = A + j * lda;
  double a0 = 0.0, a1 = 0.0;
  // i is even, so i + 1 < k when k is even and i + 1 <= k < lda when k is
  // odd: the second element of a load is inside the column
  for (int64_t i = lo + 2 * (int64_t)threadIdx.x; i < hi; i += 512) {
    const double2 v = *reinterpret_cast<const double2*>(col + i);
    a0 += v.x * x[i];
    if (i + 1 < hi) a1 += v.y * x[i + 1];
  }
  double acc = a0 + a1;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[j] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename TA>
static void apply_t(const ffk_precond* P, const double* r, double* z, hipStream_t st, double* rz_part = nullptr) {
  const TA* L = P->L.as<TA>();
  const int64_t n = P->n, k = P->k_eff;
  const double* F = P->Finv.as<double>();
  double* part = P->work.as<double>();
  gemv_t<TA>(L, n, P->ld, k, r, P->y.as<double>(), part, st, CLK_GEMV_T);
  clk_begin(CLK_CORE, st);
  k_tri_dots<false><<<k, 256, 0, st>>>(P->FinvT.as<double>(), P->ldf, k, P->y.as<double>(),
                                                 P->t1.as<double>());
  LAUNCHCHK();
  k_tri_dots<true><<<k, 256, 0, st>>>(F, P->ldf, k, P->t1.as<double>(), P->t.as<double>());
  LAUNCHCHK();
  clk_end(CLK_CORE, st);
  if (!rz_part) {
    gemv_n<TA>(L, n, P->ld, k, P->t.as<double>(), r, 1.0 / P->lambda, z, part, st, CLK_GEMV_N);
    return;
  }
  // the same L t pass, finished together with the partials of r^T z
  const int nb = cdiv(k, LN_COLS);
  const int gx = cdiv(n, ln_rows<TA>());
  const int64_t stride = (int64_t)gx * ln_rows<TA>();
  clk_begin(CLK_GEMV_N, st);
  k_ln_part<TA><<<dim3(gx, nb), 256, 0, st>>>(L, n, P->ld, k, P->t.as<double>(), part, stride);
  LAUNCHCHK();
  clk_end(CLK_GEMV_N, st);
  const int np = fused_parts(n);
  k_finish_n_dot<<<np, 256, 0, st>>>(part, nb, stride, n, r, 1.0 / P->lambda, z, rz_part);
  LAUNCHCHK();
}

__global__ void k_gather_at(const double* __restrict__ v, const int64_t* __restrict__ sel, int64_t k,
                            double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k) out[j] = v[sel[j]];
}
__global__ void k_zero64(double* __restrict__ v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = 0.0;
}
__global__ void k_scatter_at(const double* __restrict__ w, const int64_t* __restrict__ sel, int64_t k,
                             double* __restrict__ v) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k) v[sel[j]] = w[j];
}

// z = lambda^-1 (r - L C^-1 L^T r) with L = K[:, S] T^T: two FP64 kernel
// products, the two triangular products with T and the core in between
static void apply_matrix_free(const ffk_precond* P, const double* r, double* z, hipStream_t st,
                              double* rz_part = nullptr) {
  const int64_t n = P->n, k = P->k_eff, ldf = P->ldf;
  double* q = P->q.as<double>();
  double* u = P->u.as<double>();
  const int64_t* sel = P->sel.as<int64_t>();
  kernel_mvm(P->sys, r, q, 0.0, FFK_FP64, st);                                   // K r
  k_gather_at<<<cdiv(k, 256), 256, 0, st>>>(q, sel, k, P->t1.as<double>());      // (K r)_S
  LAUNCHCHK();
  k_tri_dots<false><<<k, 256, 0, st>>>(P->TinvT.as<double>(), ldf, k, P->t1.as<double>(), P->y.as<double>());
  LAUNCHCHK();                                                                      // y = L^T r = T (K r)_S
  clk_begin(CLK_CORE, st);
  k_tri_dots<false><<<k, 256, 0, st>>>(P->FinvT.as<double>(), ldf, k, P->y.as<double>(), P->t1.as<double>());
  LAUNCHCHK();
  k_tri_dots<true><<<k, 256, 0, st>>>(P->Finv.as<double>(), ldf, k, P->t1.as<double>(), P->t.as<double>());
  LAUNCHCHK();
  clk_end(CLK_CORE, st);
  k_tri_dots<true><<<k, 256, 0, st>>>(P->Tinv.as<double>(), ldf, k, P->t.as<double>(), P->t1.as<double>());
  LAUNCHCHK();                                                                      // T^T t
  k_zero64<<<cdiv(n, 256), 256, 0, st>>>(u, n);
  LAUNCHCHK();
  k_scatter_at<<<cdiv(k, 256), 256, 0, st>>>(P->t1.as<double>(), sel, k, u);
  LAUNCHCHK();
  kernel_mvm(P->sys, u, q, 0.0, FFK_FP64, st);                                   // L t = K (scatter T^T t)
  if (!rz_part) {
    k_finish_n<<<cdiv(n, 256), 256, 0, st>>>(q, 1, n, n, r, 1.0 / P->lambda, z);
  } else {
    k_finish_n_dot<<<fused_parts(n), 256, 0, st>>>(q, 1, n, n, r, 1.0 / P->lambda, z, rz_part);
  }
  LAUNCHCHK();
}

int64_t precond_work_doubles(int64_t n, int64_t ld, int64_t keff, int store) {
  (void)n;
  if (store == FFK_FP64) return gemv_work<double>(ld, keff);
  if (store == FFK_FP32) return gemv_work<float>(ld, keff);
  return gemv_work<bf16_t>(ld, keff);
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
  if (P->matrix_free) apply_matrix_free(P, r, z, st);
  else if (P->store == FFK_FP64) apply_t<double>(P, r, z, st);
  else if (P->store == FFK_FP32) apply_t<float>(P, r, z, st);
  else apply_t<bf16_t>(P, r, z, st);
}

int precond_apply_parts(const ffk_precond* P, const double* r, double* z, double* part, hipStream_t st) {
  const int np = fused_parts(P->n);
  if (P->k_eff == 0) {
    k_scale_dot<<<np, 256, 0, st>>>(r, 1.0 / P->lambda, P->n, z, part);
    LAUNCHCHK();
  } else if (P->matrix_free) {
    apply_matrix_free(P, r, z, st, part);
  } else if (P->store == FFK_FP64) {
    apply_t<double>(P, r, z, st, part);
  } else if (P->store == FFK_FP32) {
    apply_t<float>(P, r, z, st, part);
  } else {
    apply_t<bf16_t>(P, r, z, st, part);
  }
  return np;
}

// L (n x k_eff) as a dense column-major FP64 matrix with leading dimension n.
__global__ void k_export(const void* L, int store, int64_t n, int64_t ld, int64_t k, double* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int64_t c = e / n, i = e % n;
  const int64_t a = i + c * ld;
  out[e] = store == FFK_FP64   ? static_cast<const double*>(L)[a]
           : store == FFK_FP32 ? (double)static_cast<const float*>(L)[a]
                               : (double)bf2f(static_cast<const bf16_t*>(L)[a]);
}

void precond_export(const ffk_precond* P, double* L, hipStream_t st) {
  const int64_t cnt = P->n * P->k_eff;
  if (cnt == 0) return;
  if (P->matrix_free) {
    // L = K[:, S] T^T, formed from the kernel's columns
    const int64_t n = P->n, k = P->k_eff;
    DBuf C(n * k * 8);
    kernel_columns(P->sys, P->sel.as<int64_t>(), k, C.as<double>(), n, 0.0, st);
    gemm64((int)n, (int)k, (int)k, 1.0, View64{C.as<double>(), 1, n}, View64{P->Tinv.as<double>(), 1, P->ldf}, 0.0,
           L, 1, n, false, st);
    HIPCHK(hipStreamSynchronize(st));
    return;
  }
  k_export<<<cdiv(cnt, 256), 256, 0, st>>>(P->L.get(), P->store, P->n, P->ld, P->k_eff, L);
  LAUNCHCHK();
}

}  // namespace ffk
