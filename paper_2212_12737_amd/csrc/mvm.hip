// Matrix-free kernel matrix-vector product  y = K v + shift v.
//
// With u_j = J_j v_j (the descriptor Jacobian applied per geometry), the block
// sum  g_i = sum_j (a_ij u_j + b_ij d_ij (d_ij . u_j)),  d_ij = x_i - x_j,  is
// rewritten as dense products over the N x N geometry pairs:
//   P  = X_c U^T                      (GEMM 1, K = D)
//   W  = B o (P - 1 diag(P)^T)        (fused in the GEMM 1 epilogue, with row sums w)
//   G  = dA U - W X_c + diag(w) X_c + a(0) 1 (1^T U)      (GEMM 2, K = 2N)
//   y_i = J_i^T g_i + shift v_i
// because sum_j W_ij d_ij = w_i x_i - (W X)_i and a_ij = a(0) + dA_ij.  The
// constant a(0) part and the row sums are kept in FP64; only the two products
// run in the requested precision.
#include "gemm.hpp"

namespace ffk {

static int64_t rup(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// u_j = J_j v_j for one geometry per block; also pd_j = x_c,j . u_j and
// optional reduced-precision copies of U.
template <bool W32, bool WBF>
__global__ void k_jv(const double* __restrict__ R, const int* __restrict__ pairs,
                     const double* __restrict__ v, const double* __restrict__ Xc, int M, int64_t D,
                     double* __restrict__ U64, double* __restrict__ pd, float* __restrict__ U32,
                     bf16_t* __restrict__ Uh, bf16_t* __restrict__ Ul, int64_t ldu) {
  extern __shared__ double sm[];
  double* sR = sm;
  double* sv = sm + 3 * M;
  __shared__ double red[256];
  const int64_t g = blockIdx.x;
  for (int i = threadIdx.x; i < 3 * M; i += blockDim.x) {
    sR[i] = R[g * 3 * M + i];
    sv[i] = v[g * 3 * M + i];
  }
  __syncthreads();
  double acc = 0.0;
  for (int64_t d = threadIdx.x; d < D; d += blockDim.x) {
    const int pq = pairs[d];
    const int p = 3 * (pq >> 16), q = 3 * (pq & 0xFFFF);
    const double dx = sR[p] - sR[q], dy = sR[p + 1] - sR[q + 1], dz = sR[p + 2] - sR[q + 2];
    const double ir = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    const double ir3 = ir * ir * ir;
    const double u = -(dx * (sv[p] - sv[q]) + dy * (sv[p + 1] - sv[q + 1]) + dz * (sv[p + 2] - sv[q + 2])) * ir3;
    U64[g * D + d] = u;
    acc += u * Xc[g * D + d];
    if (W32) U32[g * D + d] = (float)u;
    if (WBF) {
      const float uf = (float)u;
      const bf16_t h = f2bf(uf);
      Uh[g * ldu + d] = h;
      Ul[g * ldu + d] = f2bf(uf - bf2f(h));
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) pd[g] = red[0];
}

// Column sums of an N x D matrix in two deterministic stages.
__global__ void k_colsum_part(const double* __restrict__ U, int64_t N, int64_t D, double* __restrict__ part) {
  __shared__ double sh[4][64];
  const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int64_t col = (int64_t)blockIdx.x * 64 + c;
  const int64_t r0 = (int64_t)blockIdx.y * 256;
  double s = 0.0;
  if (col < D)
    for (int r = rg; r < 256 && r0 + r < N; r += 4) s += U[(r0 + r) * D + col];
  sh[rg][c] = s;
  __syncthreads();
  if (rg == 0 && col < D) part[(int64_t)blockIdx.y * D + col] = (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]);
}
__global__ void k_colsum_final(const double* __restrict__ part, int nchunk, int64_t D, double scale,
                               double* __restrict__ s) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= D) return;
  double a = 0.0;
  for (int i = 0; i < nchunk; ++i) a += part[(int64_t)i * D + col];
  s[col] = a * scale;
}

void colsum(const double* U, int64_t N, int64_t D, double* part, double* s, double scale, hipStream_t st) {
  const int nchunk = cdiv(N, 256);
  k_colsum_part<<<dim3(cdiv(D, 64), nchunk), 256, 0, st>>>(U, N, D, part);
  LAUNCHCHK();
  k_colsum_final<<<cdiv(D, 256), 256, 0, st>>>(part, nchunk, D, scale, s);
  LAUNCHCHK();
}

// y_g = J_g^T G_g + shift v_g, one geometry per block (thread per atom).
__global__ void k_jtg(const double* __restrict__ R, const double* __restrict__ G,
                      const double* __restrict__ v, double shift, int M, int64_t D,
                      double* __restrict__ y) {
  extern __shared__ double sm[];
  double* sR = sm;
  double* sG = sm + 3 * M;
  const int64_t g = blockIdx.x;
  for (int i = threadIdx.x; i < 3 * M; i += blockDim.x) sR[i] = R[g * 3 * M + i];
  for (int64_t i = threadIdx.x; i < D; i += blockDim.x) sG[i] = G[g * D + i];
  __syncthreads();
  for (int a = threadIdx.x; a < M; a += blockDim.x) {
    double ax = 0.0, ay = 0.0, az = 0.0;
    const double xa = sR[3 * a], ya = sR[3 * a + 1], za = sR[3 * a + 2];
    for (int b = 0; b < M; ++b) {
      if (b == a) continue;
      const int idx = a > b ? a * (a - 1) / 2 + b : b * (b - 1) / 2 + a;
      const double dx = xa - sR[3 * b], dy = ya - sR[3 * b + 1], dz = za - sR[3 * b + 2];
      const double ir = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
      const double c = sG[idx] * ir * ir * ir;
      ax -= c * dx;
      ay -= c * dy;
      az -= c * dz;
    }
    const int64_t o = g * 3 * M + 3 * a;
    if (v) {
      ax += shift * v[o];
      ay += shift * v[o + 1];
      az += shift * v[o + 2];
    }
    y[o] = ax;
    y[o + 1] = ay;
    y[o + 2] = az;
  }
}

// ------------------------------------------------------------- epilogues ----
// GEMM 1: W = B o (P - pd 1^T)^T ..., stores -W and the row-sum partials of W.
template <typename CT, int BM>
struct EpiW {
  const CT* Bc; int64_t ldb;
  const double* pd;
  CT* Wn; int64_t ldw;
  double* wpart; int ntn;
  int Nr, Nc;   // valid rows / cols
  template <typename T, int TM, int TN, class Acc>
  __device__ void run(const Acc (&acc)[TM][TN], const FragCoord& f, char* smem) const {
    double* red = reinterpret_cast<double*>(smem);   // [2][BM]
    const int wn = (f.wn0 - f.n0) != 0;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = f.row(i, v);
        double rs = 0.0;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int c = f.col(j);
          if (r < Nr && c < Nc) {
            const double w = (double)Bc[(int64_t)r * ldb + c] * ((double)acc[i][j][v] - pd[c]);
            Wn[(int64_t)r * ldw + c] = (CT)(-w);
            rs += w;
          }
        }
        rs += __shfl_xor(rs, 1);
        rs += __shfl_xor(rs, 2);
        rs += __shfl_xor(rs, 4);
        rs += __shfl_xor(rs, 8);
        if ((f.lane & 15) == 0) red[wn * BM + (r - f.m0)] = rs;
      }
    __syncthreads();
    for (int t = threadIdx.x; t < BM; t += blockDim.x) {
      const int r = f.m0 + t;
      if (r < Nr) wpart[(int64_t)r * ntn + blockIdx.x] = red[t] + red[BM + t];
    }
  }
};

// BF16 variant: coefficient in FP32, -W stored as bf16 hi (+lo), all padded
// entries written (they are zero because B is zero there).
template <int BM, bool X3>
struct EpiWbf {
  const float* Bc; int64_t ld;   // B and Wn share the padded leading dimension
  const double* pd;
  bf16_t* Wh; bf16_t* Wl;
  double* wpart; int ntn;
  int N;
  template <typename T, int TM, int TN, class Acc>
  __device__ void run(const Acc (&acc)[TM][TN], const FragCoord& f, char* smem) const {
    double* red = reinterpret_cast<double*>(smem);
    const int wn = (f.wn0 - f.n0) != 0;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = f.row(i, v);
        double rs = 0.0;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int c = f.col(j);
          const float pdc = c < N ? (float)pd[c] : 0.f;
          const float w = Bc[(int64_t)r * ld + c] * (acc[i][j][v] - pdc);
          const bf16_t h = f2bf(-w);
          Wh[(int64_t)r * ld + c] = h;
          if (X3) Wl[(int64_t)r * ld + c] = f2bf(-w - bf2f(h));
          rs += (double)w;
        }
        rs += __shfl_xor(rs, 1);
        rs += __shfl_xor(rs, 2);
        rs += __shfl_xor(rs, 4);
        rs += __shfl_xor(rs, 8);
        if ((f.lane & 15) == 0) red[wn * BM + (r - f.m0)] = rs;
      }
    __syncthreads();
    for (int t = threadIdx.x; t < BM; t += blockDim.x) {
      const int r = f.m0 + t;
      if (r < N) wpart[(int64_t)r * ntn + blockIdx.x] = red[t] + red[BM + t];
    }
  }
};

// GEMM 2: G = acc + a0 s_c + w_r Xt_r,c   (w_r = sum of the row-sum partials).
template <int BM>
struct EpiG {
  const double* s;
  const double* Xt; int64_t ldx;   // target descriptor (centred), rows r
  const double* wpart; int ntn;
  double a0;
  double* G; int64_t ldg;
  int Nr, Nc;
  template <typename T, int TM, int TN, class Acc>
  __device__ void run(const Acc (&acc)[TM][TN], const FragCoord& f, char* smem) const {
    double* wsh = reinterpret_cast<double*>(smem);
    for (int t = threadIdx.x; t < BM; t += blockDim.x) {
      const int r = f.m0 + t;
      double w = 0.0;
      if (r < Nr)
        for (int q = 0; q < ntn; ++q) w += wpart[(int64_t)r * ntn + q];
      wsh[t] = w;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = f.row(i, v), c = f.col(j);
          if (r < Nr && c < Nc)
            G[(int64_t)r * ldg + c] = (double)acc[i][j][v] + a0 * s[c] + wsh[r - f.m0] * Xt[(int64_t)r * ldx + c];
        }
  }
};

// Gram epilogue for a rectangular (target x source) pair -> dA, B (FP64).
struct EpiCoeffRect {
  const double *sqr, *sqc;
  double *dA, *B;
  int Nr, Nc;
  double inv_len, a0, bcoef;
  template <typename T, int TM, int TN, class Acc>
  __device__ void run(const Acc (&acc)[TM][TN], const FragCoord& f, char*) const {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = f.row(i, v), c = f.col(j);
          if (r < Nr && c < Nc) {
            double r2 = sqr[r] + sqc[c] - 2.0 * (double)acc[i][j][v];
            r2 = r2 < 0.0 ? 0.0 : r2;
            const double z = sqrt(r2) * inv_len;
            const double em = expm1(-z);
            dA[(int64_t)r * Nc + c] = a0 * ((1.0 + z) * em + z);
            B[(int64_t)r * Nc + c] = -bcoef * (em + 1.0);
          }
        }
  }
};

// ---------------------------------------------------------------- driver ----
static inline void mark(hipEvent_t* ev, int i, hipStream_t st) {
  if (ev) HIPCHK(hipEventRecord(ev[i], st));
}

template <typename T>
static void mvm_scalar(ffk_system* s, int prec, const double* pd, const double* sv, hipStream_t st,
                       hipEvent_t* ev) {
  const int N = (int)s->N;
  const int64_t D = s->D;
  MvmWork& w = s->work;
  CoeffSet& cs = s->coef[prec];
  const T* Xc = prec == FFK_FP64 ? (const T*)s->Xc.get() : (const T*)s->Xc32.get();
  const T* U = prec == FFK_FP64 ? (const T*)w.U64.get() : (const T*)w.U32.get();
  T* Wn = prec == FFK_FP64 ? (T*)w.Wn64.get() : (T*)w.Wn32.get();
  const int ntn = cdiv(N, 128);
  {
    ScalarArgs<T> g{};
    g.M = N;
    g.N = N;
    g.nseg = 1;
    g.seg[0] = SegS<T>{Xc, D, 1, U, D, 1, (int)D};
    EpiW<T, 128> e{(const T*)cs.B.get(), N, pd, Wn, N, w.wpart.as<double>(), ntn, N, N};
    gemm_scalar_kernel<T, 128, 128, 16, true, true, EpiW<T, 128>><<<dim3(ntn, ntn), 256, 0, st>>>(g, e);
    LAUNCHCHK();
  }
  mark(ev, 3, st);
  {
    ScalarArgs<T> g{};
    g.M = N;
    g.N = (int)D;
    g.nseg = 2;
    g.seg[0] = SegS<T>{(const T*)cs.dA_hi.get(), N, 1, U, 1, D, N};
    g.seg[1] = SegS<T>{Wn, N, 1, Xc, 1, D, N};
    EpiG<128> e{sv, s->Xc.as<double>(), D, w.wpart.as<double>(), ntn, s->a0, w.G.as<double>(), D, N, (int)D};
    gemm_scalar_kernel<T, 128, 128, 16, true, false, EpiG<128>><<<dim3(cdiv(D, 128), ntn), 256, 0, st>>>(g, e);
    LAUNCHCHK();
  }
}

template <bool X3>
static void mvm_bf16(ffk_system* s, int prec, const double* pd, const double* sv, hipStream_t st, hipEvent_t* ev) {
  const int64_t N = s->N, D = s->D;
  const int64_t Nr = rup(N, 128), Dk = rup(D, 64), Dr = rup(D, 128);
  MvmWork& w = s->work;
  CoeffSet& cs = s->coef[prec];
  const int ntn = (int)(Nr / 128);
  {
    Bf16Args g{};
    g.nseg = 1;
    g.seg[0] = SegB{s->Xch.as<bf16_t>(), s->Xcl.as<bf16_t>(), w.Uh.as<bf16_t>(), w.Ul.as<bf16_t>(), Dk, Dk, (int)Dk};
    EpiWbf<128, X3> e{cs.B.as<float>(), Nr, pd, w.Wnh.as<bf16_t>(), w.Wnl.as<bf16_t>(), w.wpart.as<double>(), ntn, (int)N};
    gemm_bf16_kernel<128, 128, 64, X3, EpiWbf<128, X3>><<<dim3(ntn, ntn), 256, 0, st>>>(g, e);
    LAUNCHCHK();
  }
  mark(ev, 3, st);
  {
    Bf16Args g{};
    g.nseg = 2;
    g.seg[0] = SegB{cs.dA_hi.as<bf16_t>(), cs.dA_lo.as<bf16_t>(), w.UTh.as<bf16_t>(), w.UTl.as<bf16_t>(), Nr, Nr, (int)Nr};
    g.seg[1] = SegB{w.Wnh.as<bf16_t>(), w.Wnl.as<bf16_t>(), s->XcTh.as<bf16_t>(), s->XcTl.as<bf16_t>(), Nr, Nr, (int)Nr};
    EpiG<128> e{sv, s->Xc.as<double>(), D, w.wpart.as<double>(), ntn, s->a0, w.G.as<double>(), D, (int)N, (int)D};
    gemm_bf16_kernel<128, 128, 64, X3, EpiG<128>><<<dim3(Dr / 128, ntn), 256, 0, st>>>(g, e);
    LAUNCHCHK();
  }
}

void k_split_transpose_launch(const double* a, int64_t rows, int64_t cols, int64_t lda, int64_t cols_p,
                              int64_t ld_out, bf16_t* hi, bf16_t* lo, hipStream_t st);

static void ensure_work(ffk_system* s, int prec, hipStream_t st) {
  const int64_t N = s->N, D = s->D;
  MvmWork& w = s->work;
  if (!w.U64) {
    w.U64.alloc(N * D * 8);
    w.pd.alloc(N * 8);
    w.s.alloc(D * 8);
    w.spart.alloc((int64_t)cdiv(N, 256) * D * 8);
    w.G.alloc(N * D * 8);
    w.wpart.alloc(N * (rup(N, 128) / 128) * 8);
  }
  if (prec == FFK_FP64 && !w.Wn64) w.Wn64.alloc(N * N * 8);
  if (prec == FFK_FP32 && !w.U32) {
    w.U32.alloc(N * D * 4);
    w.Wn32.alloc(N * N * 4);
  }
  if ((prec == FFK_BF16 || prec == FFK_BF16X3) && !w.Uh) {
    const int64_t Nr = rup(N, 128), Dk = rup(D, 64), Dr = rup(D, 128);
    w.Uh.alloc(Nr * Dk * 2);
    w.Ul.alloc(Nr * Dk * 2);
    HIPCHK(hipMemsetAsync(w.Uh.get(), 0, Nr * Dk * 2, st));
    HIPCHK(hipMemsetAsync(w.Ul.get(), 0, Nr * Dk * 2, st));
    w.UTh.alloc(Dr * Nr * 2);
    w.UTl.alloc(Dr * Nr * 2);
    w.Wnh.alloc(Nr * Nr * 2);
    w.Wnl.alloc(Nr * Nr * 2);
  }
}

void kernel_mvm_ev(ffk_system* s, const double* v, double* y, double shift, int prec, hipStream_t st,
                   hipEvent_t* ev) {
  require(prec >= FFK_FP64 && prec <= FFK_BF16X3, "kernel_mvm: unknown precision");
  ensure_coeffs(s, prec, st);
  ensure_lowp_descriptor(s, prec, st);
  ensure_work(s, prec, st);
  mark(ev, 0, st);
  const int64_t N = s->N, D = s->D;
  const int M = s->M;
  MvmWork& w = s->work;
  const bool bf = (prec == FFK_BF16 || prec == FFK_BF16X3);
  const int64_t ldu = rup(D, 64);
  const size_t shm = 6 * M * sizeof(double);
  if (prec == FFK_FP32)
    k_jv<true, false><<<N, 256, shm, st>>>(s->R.as<double>(), s->pairs.as<int>(), v, s->Xc.as<double>(), M, D,
                                           w.U64.as<double>(), w.pd.as<double>(), w.U32.as<float>(), nullptr,
                                           nullptr, 0);
  else if (bf)
    k_jv<false, true><<<N, 256, shm, st>>>(s->R.as<double>(), s->pairs.as<int>(), v, s->Xc.as<double>(), M, D,
                                           w.U64.as<double>(), w.pd.as<double>(), nullptr, w.Uh.as<bf16_t>(),
                                           w.Ul.as<bf16_t>(), ldu);
  else
    k_jv<false, false><<<N, 256, shm, st>>>(s->R.as<double>(), s->pairs.as<int>(), v, s->Xc.as<double>(), M, D,
                                            w.U64.as<double>(), w.pd.as<double>(), nullptr, nullptr, nullptr, 0);
  LAUNCHCHK();
  mark(ev, 1, st);
  colsum(w.U64.as<double>(), N, D, w.spart.as<double>(), w.s.as<double>(), 1.0, st);
  const double* pd = w.pd.as<double>();
  const double* sv = w.s.as<double>();
  if (prec == FFK_FP64) {
    mark(ev, 2, st);
    mvm_scalar<double>(s, prec, pd, sv, st, ev);
  } else if (prec == FFK_FP32) {
    mark(ev, 2, st);
    mvm_scalar<float>(s, prec, pd, sv, st, ev);
  } else {
    const int64_t Nr = rup(N, 128), Dr = rup(D, 128);
    k_split_transpose_launch(w.U64.as<double>(), N, D, D, Dr, Nr, w.UTh.as<bf16_t>(), w.UTl.as<bf16_t>(), st);
    mark(ev, 2, st);
    if (prec == FFK_BF16X3)
      mvm_bf16<true>(s, prec, pd, sv, st, ev);
    else
      mvm_bf16<false>(s, prec, pd, sv, st, ev);
  }
  mark(ev, 4, st);
  const int tb = M <= 64 ? 64 : 128;
  k_jtg<<<N, tb, (3 * M + D) * sizeof(double), st>>>(s->R.as<double>(), w.G.as<double>(), v, shift, M, D, y);
  LAUNCHCHK();
  mark(ev, 5, st);
}

void kernel_mvm(ffk_system* s, const double* v, double* y, double shift, int prec, hipStream_t st) {
  kernel_mvm_ev(s, v, y, shift, prec, st, nullptr);
}

// Average time of each phase over `iters` products: [J v, column sums (+ bf16
// transposes), GEMM 1 + W epilogue, GEMM 2 + G epilogue, J^T G].
void kernel_mvm_phases(ffk_system* s, const double* v, double* y, double shift, int prec, int iters, double* ms,
                       hipStream_t st) {
  hipEvent_t ev[6];
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  for (int p = 0; p < 5; ++p) ms[p] = 0.0;
  for (int it = 0; it < iters; ++it) {
    kernel_mvm_ev(s, v, y, shift, prec, st, ev);
    HIPCHK(hipEventSynchronize(ev[5]));
    for (int p = 0; p < 5; ++p) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, ev[p], ev[p + 1]));
      ms[p] += t / iters;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
}

// ----------------------------------------------------------- prediction ----
__global__ void k_center_with(const double* __restrict__ X, const double* __restrict__ mean, int64_t D,
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

void kernel_predict(const ffk_system* tr, const ffk_system* te, const double* alpha, double* F, hipStream_t st) {
  require(tr->M == te->M, "kernel_predict: train and test molecules differ in size");
  require(tr->sigma == te->sigma, "kernel_predict: sigma differs");
  const int64_t Ns = tr->N, Nt = te->N, D = tr->D;
  const int M = tr->M;
  DBuf U(Ns * D * 8), pd(Ns * 8), sv(D * 8), spart((int64_t)cdiv(Ns, 256) * D * 8);
  DBuf Xt(Nt * D * 8), sqt(Nt * 8), dA(Nt * Ns * 8), B(Nt * Ns * 8), Wn(Nt * Ns * 8);
  const int ntn = cdiv(Ns, 128);
  DBuf wpart(Nt * ntn * 8), G(Nt * D * 8);
  k_jv<false, false><<<Ns, 256, 6 * M * sizeof(double), st>>>(tr->R.as<double>(), tr->pairs.as<int>(), alpha,
                                                              tr->Xc.as<double>(), M, D, U.as<double>(),
                                                              pd.as<double>(), nullptr, nullptr, nullptr, 0);
  LAUNCHCHK();
  colsum(U.as<double>(), Ns, D, spart.as<double>(), sv.as<double>(), 1.0, st);
  k_center_with<<<Nt, 256, 0, st>>>(te->X.as<double>(), tr->xmean.as<double>(), D, Xt.as<double>(),
                                    sqt.as<double>());
  LAUNCHCHK();
  {
    ScalarArgs<double> g{};
    g.M = (int)Nt;
    g.N = (int)Ns;
    g.nseg = 1;
    g.seg[0] = SegS<double>{Xt.as<double>(), D, 1, tr->Xc.as<double>(), D, 1, (int)D};
    EpiCoeffRect e{sqt.as<double>(), tr->sqn.as<double>(), dA.as<double>(), B.as<double>(), (int)Nt, (int)Ns,
                   sqrt(5.0) / tr->sigma, tr->a0, tr->bcoef};
    gemm_scalar_kernel<double, 128, 128, 16, true, true, EpiCoeffRect><<<dim3(ntn, cdiv(Nt, 128)), 256, 0, st>>>(g, e);
    LAUNCHCHK();
  }
  {
    ScalarArgs<double> g{};
    g.M = (int)Nt;
    g.N = (int)Ns;
    g.nseg = 1;
    g.seg[0] = SegS<double>{Xt.as<double>(), D, 1, U.as<double>(), D, 1, (int)D};
    EpiW<double, 128> e{B.as<double>(), Ns, pd.as<double>(), Wn.as<double>(), Ns, wpart.as<double>(), ntn,
                        (int)Nt, (int)Ns};
    gemm_scalar_kernel<double, 128, 128, 16, true, true, EpiW<double, 128>><<<dim3(ntn, cdiv(Nt, 128)), 256, 0, st>>>(g, e);
    LAUNCHCHK();
  }
  {
    ScalarArgs<double> g{};
    g.M = (int)Nt;
    g.N = (int)D;
    g.nseg = 2;
    g.seg[0] = SegS<double>{dA.as<double>(), Ns, 1, U.as<double>(), 1, D, (int)Ns};
    g.seg[1] = SegS<double>{Wn.as<double>(), Ns, 1, tr->Xc.as<double>(), 1, D, (int)Ns};
    EpiG<128> e{sv.as<double>(), Xt.as<double>(), D, wpart.as<double>(), ntn, tr->a0, G.as<double>(), D, (int)Nt, (int)D};
    gemm_scalar_kernel<double, 128, 128, 16, true, false, EpiG<128>><<<dim3(cdiv(D, 128), cdiv(Nt, 128)), 256, 0, st>>>(g, e);
    LAUNCHCHK();
  }
  const int tb = M <= 64 ? 64 : 128;
  k_jtg<<<Nt, tb, (3 * M + D) * sizeof(double), st>>>(te->R.as<double>(), G.as<double>(), nullptr, 0.0, M, D, F);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));   // temporaries are freed on return
}

}  // namespace ffk
