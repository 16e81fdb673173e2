// Score network for learned inducing-column selection: D -> H -> H -> 1 with
// exact-erf GELU, trained in FP32 on FP32 MFMA (forward, backward and Adam are
// the kernels below), inferred either in FP32 or in BF16 on MFMA with FP32
// accumulation.  The network maps a standardised descriptor to a predicted
// log block leverage score; sampling weights are exp(prediction) (the
// Efraimidis-Spirakis keys are invariant to a common scale).
//
// Parameter layout (floats): W1 (H x D row-major), b1 (H), W2 (H x H), b2 (H),
// w3 (H), b3 (1); after the parameters: input mean (D) and inverse std (D).
#include "gemm.hpp"

namespace ffk {

__device__ inline float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

struct Offs {
  int64_t W1, b1, W2, b2, w3, b3, mean, istd, end;
};
static Offs offs(int D, int H) {
  Offs o;
  o.W1 = 0;
  o.b1 = o.W1 + (int64_t)H * D;
  o.W2 = o.b1 + H;
  o.b2 = o.W2 + (int64_t)H * H;
  o.w3 = o.b2 + H;
  o.b3 = o.w3 + H;
  o.mean = o.b3 + 1;
  o.istd = o.mean + D;
  o.end = o.istd + D;
  return o;
}

// --------------------------------------------------------------- epilogues ----
// Z = acc + bias[c]; H = gelu(Z) (row-major, ld), Z stored when requested.
struct EpiBiasGelu {
  const float* bias;
  float* Z;
  float* Hout;
  bf16_t* Hbf;   // optional bf16 copy of H (ldb)
  int64_t ld, ldb;
  int M, N;
  template <typename T, int TM, int TN, class Acc>
  __device__ void run(const Acc (&acc)[TM][TN], const FragCoord& f, char*) const {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = f.row(i, v), c = f.col(j);
          if (r < M && c < N) {
            const float z = (float)acc[i][j][v] + bias[c];
            const float h = gelu_f(z);
            if (Z) Z[(int64_t)r * ld + c] = z;
            if (Hout) Hout[(int64_t)r * ld + c] = h;
            if (Hbf) Hbf[(int64_t)r * ldb + c] = f2bf(h);
          }
        }
  }
};

// C = acc (row-major, ldc), optionally times gelu'(Zg) elementwise.
struct EpiStoreF {
  float* C;
  int64_t ldc;
  const float* Zg;   // optional
  int M, N;
  template <typename T, int TM, int TN, class Acc>
  __device__ void run(const Acc (&acc)[TM][TN], const FragCoord& f, char*) const {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = f.row(i, v), c = f.col(j);
          if (r < M && c < N) {
            float x = (float)acc[i][j][v];
            if (Zg) x *= gelu_grad_f(Zg[(int64_t)r * ldc + c]);
            C[(int64_t)r * ldc + c] = x;
          }
        }
  }
};

template <bool AKC, bool BKC, class Epi>
static void gemm_f32(int M, int N, int K, const float* A, int64_t sa0, int64_t sa1, const float* B, int64_t sb0,
                     int64_t sb1, const Epi& e, hipStream_t st) {
  ScalarArgs<float> g{};
  g.M = M;
  g.N = N;
  g.nseg = 1;
  g.seg[0] = SegS<float>{A, sa0, sa1, B, sb0, sb1, K};
  if (N <= 64)
    gemm_scalar_kernel<float, 128, 64, 16, AKC, BKC, Epi><<<dim3(cdiv(N, 64), cdiv(M, 128)), 256, 0, st>>>(g, e);
  else
    gemm_scalar_kernel<float, 128, 128, 16, AKC, BKC, Epi><<<dim3(cdiv(N, 128), cdiv(M, 128)), 256, 0, st>>>(g, e);
  LAUNCHCHK();
}

// ----------------------------------------------------------- small kernels ----
// out[b] = H2[b] . w3 + b3 (one wave per row)
__global__ __launch_bounds__(256) void k_rowdot(const float* H2, int64_t B, int H, const float* w3, const float* b3,
                                                float* out) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= B) return;
  float a = 0.f;
  for (int h = lane; h < H; h += 64) a += H2[b * H + h] * w3[h];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  if (lane == 0) out[b] = a + b3[0];
}

// dout = 2 (out - y) / B and loss partials (single block, deterministic)
__global__ __launch_bounds__(256) void k_loss(const float* out, const float* y, int64_t B, float* dout, float* loss) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int64_t b = threadIdx.x; b < B; b += 256) {
    const float d = out[b] - y[b];
    dout[b] = 2.0f * d / (float)B;
    a += (double)d * d;
  }
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(sh[0] / (double)B);
}

// colsum[h] = sum_b A[b][h] * (w ? w[b] : 1)  (thread per column, fixed order)
__global__ void k_colsum_w(const float* A, int64_t B, int H, const float* w, float* colsum) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= H) return;
  float a0 = 0.f, a1 = 0.f;
  int64_t b = 0;
  for (; b + 2 <= B; b += 2) {
    a0 += A[b * H + h] * (w ? w[b] : 1.f);
    a1 += A[(b + 1) * H + h] * (w ? w[b + 1] : 1.f);
  }
  if (b < B) a0 += A[b * H + h] * (w ? w[b] : 1.f);
  colsum[h] = a0 + a1;
}

// dZ2[b][h] = dout[b] * w3[h] * gelu'(Z2[b][h])
__global__ void k_dz2(const float* dout, const float* w3, const float* Z2, int64_t B, int H, float* dZ2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * H) return;
  const int64_t b = e / H;
  const int h = (int)(e % H);
  dZ2[e] = dout[b] * w3[h] * gelu_grad_f(Z2[e]);
}

__global__ void k_sum1(const float* a, int64_t n, float* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += a[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)sh[0];
}

__global__ void k_adam(float* theta, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 copy of a rows x cols FP32 matrix into a zero-padded rows_p x ld array
__global__ void k_f32_to_bf16_pad(const float* a, int64_t rows, int64_t cols, int64_t lda, int64_t rows_p, int64_t ld,
                                  bf16_t* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows_p * ld) return;
  const int64_t r = e / ld, c = e % ld;
  out[e] = (r < rows && c < cols) ? f2bf(a[r * lda + c]) : (bf16_t)0;
}

// standardised descriptor rows of a system as bf16 (rows_p x ld, zero padded)
__global__ void k_standardize_bf16(const double* X, int64_t N, int64_t D, const float* mean, const float* istd,
                                   int64_t rows_p, int64_t ld, bf16_t* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows_p * ld) return;
  const int64_t r = e / ld, c = e % ld;
  out[e] = (r < N && c < D) ? f2bf((float)((X[r * D + c] - mean[c]) * istd[c])) : (bf16_t)0;
}

__global__ void k_exp_scores(const float* out, int64_t N, double* scores) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) scores[i] = exp((double)out[i]);
}

// ------------------------------------------------------------------ driver ----
static int64_t rup(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

ffk_mlp* mlp_create(int32_t D, int32_t H, uint64_t seed) {
  std::unique_ptr<ffk_mlp> m(new ffk_mlp());
  m->D = D;
  m->H = H;
  const Offs o = offs(D, H);
  m->nparam = o.mean;
  m->theta.alloc(o.end * 4);
  m->m.alloc(m->nparam * 4);
  m->v.alloc(m->nparam * 4);
  // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases; identity standardisation
  std::vector<float> h(o.end, 0.f);
  uint64_t ctr = 0;
  auto fill = [&](int64_t off, int64_t cnt, int fan_in) {
    const double a = 1.0 / sqrt((double)fan_in);
    for (int64_t i = 0; i < cnt; ++i) h[off + i] = (float)((2.0 * uniform01_at(seed, 4, ctr++) - 1.0) * a);
  };
  fill(o.W1, (int64_t)H * D, D);
  fill(o.W2, (int64_t)H * H, H);
  fill(o.w3, H, H);
  for (int64_t i = 0; i < D; ++i) h[o.istd + i] = 1.f;
  HIPCHK(hipMemcpy(m->theta.get(), h.data(), o.end * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(m->m.get(), 0, m->nparam * 4));
  HIPCHK(hipMemset(m->v.get(), 0, m->nparam * 4));
  return m.release();
}

// Activations of a batch: Z1, H1, Z2, H2 (B x H each), out, dout (B), dZ2, dZ1 (B x H)
static float* act(const ffk_mlp* net, int64_t B) {
  const int64_t need = (6 * B * net->H + 2 * B) * 4;
  ffk_mlp* m = const_cast<ffk_mlp*>(net);
  m->work.ensure(need);
  return m->work.as<float>();
}

static void forward_f32(const ffk_mlp* net, const float* X, int64_t B, float* out, float* Z1, float* H1, float* Z2,
                        float* H2, hipStream_t st) {
  const int D = net->D, H = net->H;
  const Offs o = offs(D, H);
  const float* th = net->theta.as<float>();
  gemm_f32<true, true>((int)B, H, D, X, D, 1, th + o.W1, D, 1, EpiBiasGelu{th + o.b1, Z1, H1, nullptr, H, 0, (int)B, H}, st);
  gemm_f32<true, true>((int)B, H, H, H1, H, 1, th + o.W2, H, 1, EpiBiasGelu{th + o.b2, Z2, H2, nullptr, H, 0, (int)B, H}, st);
  k_rowdot<<<cdiv(B, 4), 256, 0, st>>>(H2, B, H, th + o.w3, th + o.b3, out);
  LAUNCHCHK();
}

static void forward_bf16(const ffk_mlp* net, const bf16_t* Xb, int64_t B, int64_t ldx, float* out, hipStream_t st) {
  const int D = net->D, H = net->H;
  const Offs o = offs(D, H);
  ffk_mlp* m = const_cast<ffk_mlp*>(net);
  const int64_t Dk = rup(D, 64), Hr = rup(H, 128), Br = rup(B, 128);
  require(ldx == Dk, "mlp: bf16 input leading dimension mismatch");
  const float* th = net->theta.as<float>();
  if (!m->wbf_valid) {
    m->wbf.ensure((Hr * Dk + Hr * rup(H, 64)) * 2);
    bf16_t* w1 = m->wbf.as<bf16_t>();
    bf16_t* w2 = w1 + Hr * Dk;
    k_f32_to_bf16_pad<<<cdiv(Hr * Dk, 256), 256, 0, st>>>(th + o.W1, H, D, D, Hr, Dk, w1);
    LAUNCHCHK();
    k_f32_to_bf16_pad<<<cdiv(Hr * rup(H, 64), 256), 256, 0, st>>>(th + o.W2, H, H, H, Hr, rup(H, 64), w2);
    LAUNCHCHK();
    m->wbf_valid = true;
  }
  const bf16_t* w1 = m->wbf.as<bf16_t>();
  const bf16_t* w2 = w1 + Hr * Dk;
  const int64_t Hk = rup(H, 64);
  DBuf h1b(Br * Hk * 2), h2(Br * H * 4);
  HIPCHK(hipMemsetAsync(h1b.get(), 0, Br * Hk * 2, st));
  {
    Bf16Args g{};
    g.nseg = 1;
    g.seg[0] = SegB{Xb, nullptr, w1, nullptr, Dk, Dk, (int)Dk};
    EpiBiasGelu e{th + o.b1, nullptr, nullptr, h1b.as<bf16_t>(), 0, Hk, (int)B, H};
    gemm_bf16_kernel<128, 128, 64, false, EpiBiasGelu><<<dim3(Hr / 128, Br / 128), 256, 0, st>>>(g, e);
    LAUNCHCHK();
  }
  {
    Bf16Args g{};
    g.nseg = 1;
    g.seg[0] = SegB{h1b.as<bf16_t>(), nullptr, w2, nullptr, Hk, Hk, (int)Hk};
    EpiBiasGelu e{th + o.b2, nullptr, h2.as<float>(), nullptr, H, 0, (int)B, H};
    gemm_bf16_kernel<128, 128, 64, false, EpiBiasGelu><<<dim3(Hr / 128, Br / 128), 256, 0, st>>>(g, e);
    LAUNCHCHK();
  }
  k_rowdot<<<cdiv(B, 4), 256, 0, st>>>(h2.as<float>(), B, H, th + o.w3, th + o.b3, out);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));   // temporaries are freed on return
}

void mlp_forward(const ffk_mlp* net, const float* X, int64_t B, float* out, int prec, hipStream_t st) {
  if (prec == FFK_FP32) {
    float* w = act(net, B);
    const int64_t bh = B * net->H;
    forward_f32(net, X, B, out, w, w + bh, w + 2 * bh, w + 3 * bh, st);
    return;
  }
  const int64_t Dk = rup(net->D, 64), Br = rup(B, 128);
  DBuf xb(Br * Dk * 2);
  k_f32_to_bf16_pad<<<cdiv(Br * Dk, 256), 256, 0, st>>>(X, B, net->D, net->D, Br, Dk, xb.as<bf16_t>());
  LAUNCHCHK();
  forward_bf16(net, xb.as<bf16_t>(), B, Dk, out, st);
}

void mlp_grad(ffk_mlp* net, const float* X, const float* y, int64_t B, float* loss, float* grad, hipStream_t st) {
  const int D = net->D, H = net->H;
  const Offs o = offs(D, H);
  const float* th = net->theta.as<float>();
  float* w = act(net, B);
  const int64_t bh = B * H;
  float *Z1 = w, *H1 = w + bh, *Z2 = w + 2 * bh, *H2 = w + 3 * bh, *dZ2 = w + 4 * bh, *dZ1 = w + 5 * bh;
  float* out = w + 6 * bh;
  float* dout = out + B;
  forward_f32(net, X, B, out, Z1, H1, Z2, H2, st);
  k_loss<<<1, 256, 0, st>>>(out, y, B, dout, loss);
  LAUNCHCHK();
  // output layer
  k_colsum_w<<<cdiv(H, 256), 256, 0, st>>>(H2, B, H, dout, grad + o.w3);
  LAUNCHCHK();
  k_sum1<<<1, 256, 0, st>>>(dout, B, grad + o.b3);
  LAUNCHCHK();
  // second hidden layer
  k_dz2<<<cdiv(bh, 256), 256, 0, st>>>(dout, th + o.w3, Z2, B, H, dZ2);
  LAUNCHCHK();
  // g_W2[i][j] = sum_b dZ2[b][i] H1[b][j]
  gemm_f32<false, false>(H, H, (int)B, dZ2, 1, H, H1, 1, H, EpiStoreF{grad + o.W2, H, nullptr, H, H}, st);
  k_colsum_w<<<cdiv(H, 256), 256, 0, st>>>(dZ2, B, H, nullptr, grad + o.b2);
  LAUNCHCHK();
  // dZ1 = (dZ2 W2) o gelu'(Z1)
  gemm_f32<true, false>((int)B, H, H, dZ2, H, 1, th + o.W2, 1, H, EpiStoreF{dZ1, H, Z1, (int)B, H}, st);
  // g_W1[i][d] = sum_b dZ1[b][i] X[b][d]
  gemm_f32<false, false>(H, D, (int)B, dZ1, 1, H, X, 1, D, EpiStoreF{grad + o.W1, D, nullptr, H, D}, st);
  k_colsum_w<<<cdiv(H, 256), 256, 0, st>>>(dZ1, B, H, nullptr, grad + o.b1);
  LAUNCHCHK();
}

void mlp_adam(ffk_mlp* net, const float* grad, float lr, hipStream_t st) {
  net->t += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = (float)(1.0 - pow((double)b1, (double)net->t));
  const float c2 = (float)(1.0 - pow((double)b2, (double)net->t));
  k_adam<<<cdiv(net->nparam, 256), 256, 0, st>>>(net->theta.as<float>(), grad, net->m.as<float>(), net->v.as<float>(),
                                                  net->nparam, lr, b1, b2, eps, c1, c2);
  LAUNCHCHK();
  net->wbf_valid = false;
}

void mlp_scores(const ffk_mlp* net, const ffk_system* s, double* scores, hipStream_t st) {
  const int D = net->D;
  const Offs o = offs(D, net->H);
  const int64_t N = s->N, Dk = rup(D, 64), Br = rup(N, 128);
  const float* th = net->theta.as<float>();
  DBuf xb(Br * Dk * 2), out(N * 4);
  k_standardize_bf16<<<cdiv(Br * Dk, 256), 256, 0, st>>>(s->X.as<double>(), N, D, th + o.mean, th + o.istd, Br, Dk,
                                                          xb.as<bf16_t>());
  LAUNCHCHK();
  forward_bf16(net, xb.as<bf16_t>(), N, Dk, out.as<float>(), st);
  k_exp_scores<<<cdiv(N, 256), 256, 0, st>>>(out.as<float>(), N, scores);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));
}

// ---------------------------------------------------- training-data helpers ----
// X_out (N x D float) = descriptor rows of a system, standardised with the
// network's mean / inverse std when `standardize`.
__global__ void k_prepare(const double* X, int64_t N, int64_t D, const float* mean, const float* istd, int standardize,
                          float* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * D) return;
  const int64_t c = e % D;
  out[e] = standardize ? (float)((X[e] - mean[c]) * istd[c]) : (float)X[e];
}

void mlp_prepare_inputs(const ffk_mlp* net, const ffk_system* s, float* out, int standardize, hipStream_t st) {
  const Offs o = offs(net->D, net->H);
  const float* th = net->theta.as<float>();
  k_prepare<<<cdiv(s->N * s->D, 256), 256, 0, st>>>(s->X.as<double>(), s->N, s->D, th + o.mean, th + o.istd,
                                                    standardize, out);
  LAUNCHCHK();
}

// mean and inverse standard deviation of the B rows of X (B x D), per column
__global__ void k_fit_norm(const float* X, int64_t B, int D, float* mean, float* istd) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= D) return;
  double s = 0.0, s2 = 0.0;
  for (int64_t b = 0; b < B; ++b) {
    const double x = X[b * D + c];
    s += x;
    s2 += x * x;
  }
  const double m = s / (double)B;
  const double var = s2 / (double)B - m * m;
  mean[c] = (float)m;
  istd[c] = (float)(1.0 / sqrt(var > 1e-30 ? var : 1e-30));
}

void mlp_fit_norm(ffk_mlp* net, const float* X, int64_t B, hipStream_t st) {
  const Offs o = offs(net->D, net->H);
  float* th = net->theta.as<float>();
  k_fit_norm<<<cdiv(net->D, 128), 128, 0, st>>>(X, B, net->D, th + o.mean, th + o.istd);
  LAUNCHCHK();
}

// y_g = log(sum of the 3M column scores of geometry g) - mean over g
__global__ __launch_bounds__(256) void k_block_log(const double* tau, int64_t N, int m3, float* y) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t g = threadIdx.x; g < N; g += 256) {
    double s = 0.0;
    for (int c = 0; c < m3; ++c) s += tau[g * m3 + c];
    const double l = log(s > 1e-300 ? s : 1e-300);
    y[g] = (float)l;
    acc += l;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const float mu = (float)(sh[0] / (double)N);
  for (int64_t g = threadIdx.x; g < N; g += 256) y[g] -= mu;
}

void block_log_scores(const double* tau, int64_t N, int M, float* y, hipStream_t st) {
  k_block_log<<<1, 256, 0, st>>>(tau, N, 3 * M, y);
  LAUNCHCHK();
}

}  // namespace ffk
