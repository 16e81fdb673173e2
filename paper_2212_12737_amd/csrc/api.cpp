// C ABI of libffkrr: argument checks, handle management and error mapping.
// No C++ exception crosses this boundary.
#include <cmath>

#include "common.hpp"

using namespace ffk;

namespace {

ffk_status set_err(ffk_ctx* ctx, ffk_status s, const char* msg) {
  if (ctx) ctx->last_error = msg;
  return s;
}

template <class F>
ffk_status guarded(ffk_ctx* ctx, F&& f) {
  try {
    if (ctx) {
      ctx->last_error.clear();
      HIPCHK(hipSetDevice(ctx->device));
    }
    return f();
  } catch (const Error& e) {
    return set_err(ctx, e.status, e.what());
  } catch (const std::bad_alloc&) {
    return set_err(ctx, FFK_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_err(ctx, FFK_ERR_HIP, e.what());
  }
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

void check_indices(const int64_t* idx_dev, int64_t k, int64_t n, hipStream_t st, const char* who) {
  std::vector<int64_t> h(k);
  HIPCHK(hipMemcpyAsync(h.data(), idx_dev, k * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int64_t i = 0; i < k; ++i)
    if (h[i] < 0 || h[i] >= n) fail(FFK_ERR_ARG, std::string(who) + ": column index out of range");
}

}  // namespace

namespace ffk {
void select_uniform_n(int64_t n, int64_t k, uint64_t seed, int stream, int64_t* out, hipStream_t st);
void expand_scores(const double* geom, int64_t N, int M, double* w, hipStream_t st);
void precond_export(const ffk_precond* P, double* L, hipStream_t st);
}  // namespace ffk

extern "C" {

const char* ffk_version(void) { return "ffkrr 1.0 gfx950"; }

ffk_status ffk_create(ffk_ctx** out, int device) {
  if (!out) return FFK_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FFK_ERR_ARG;
  // the device address of the scratch array for this device, taken with the
  // device current (the caller's current device is restored)
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return FFK_ERR_HIP;
  if (hipSetDevice(device) != hipSuccess) return FFK_ERR_HIP;
  ffk_status st = guarded(nullptr, [&]() {
    scratch_init(device);
    return FFK_OK;
  });
  (void)hipSetDevice(prev);
  if (st != FFK_OK) return st;
  ffk_ctx* c = new (std::nothrow) ffk_ctx();
  if (!c) return FFK_ERR_OOM;
  c->device = device;
  *out = c;
  return FFK_OK;
}

void ffk_destroy(ffk_ctx* ctx) { delete ctx; }

const char* ffk_last_error(const ffk_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

ffk_status ffk_descriptor_build(ffk_ctx* ctx, const double* R_dev, int64_t N, int32_t M, double sigma,
                                ffk_system** out, void* stream) {
  if (!ctx || !out) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(R_dev != nullptr, "descriptor_build: R is null");
    require(N >= 1 && M >= 3 && M < 2048, "descriptor_build: need N >= 1 and 3 <= M < 2048");
    require(sigma > 0.0 && std::isfinite(sigma), "descriptor_build: sigma must be positive");
    std::unique_ptr<ffk_system> s(new ffk_system());
    s->ctx = ctx;
    s->N = N;
    s->M = M;
    s->D = (int64_t)M * (M - 1) / 2;
    s->n = 3 * (int64_t)M * N;
    s->sigma = sigma;
    s->a0 = 5.0 / (3.0 * sigma * sigma);
    s->bcoef = 25.0 / (3.0 * sigma * sigma * sigma * sigma);
    descriptor_build(s.get(), R_dev, S(stream));
    HIPCHK(hipStreamSynchronize(S(stream)));
    *out = s.release();
    return FFK_OK;
  });
}

void ffk_system_free(ffk_system* sys) { delete sys; }

ffk_status ffk_system_info(const ffk_system* s, int64_t* N, int32_t* M, int64_t* D, int64_t* n) {
  if (!s) return FFK_ERR_ARG;
  if (N) *N = s->N;
  if (M) *M = s->M;
  if (D) *D = s->D;
  if (n) *n = s->n;
  return FFK_OK;
}

ffk_status ffk_system_set_symmetries(ffk_ctx* ctx, ffk_system* s, const int32_t* perms, int32_t nperm,
                                     void* stream) {
  if (!ctx || !s) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    set_symmetries(s, perms, nperm, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_descriptor_export(ffk_ctx* ctx, const ffk_system* s, double* X_dev, void* stream) {
  if (!ctx || !s || !X_dev) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    HIPCHK(hipMemcpyAsync(X_dev, s->X.get(), s->N * s->D * 8, hipMemcpyDeviceToDevice, S(stream)));
    return FFK_OK;
  });
}

ffk_status ffk_kernel_mvm(ffk_ctx* ctx, ffk_system* s, const double* v, double* y, double shift,
                          ffk_precision prec, void* stream) {
  if (!ctx || !s) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(v && y && v != y, "kernel_mvm: v and y must be distinct device buffers");
    require(std::isfinite(shift), "kernel_mvm: shift must be finite");
    kernel_mvm(s, v, y, shift, (int)prec, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_kernel_mvm_noalloc(ffk_ctx* ctx, ffk_system* s, const double* v, double* y, double shift,
                                  ffk_precision prec, void* stream) {
  if (!ctx || !s) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(v && y && v != y, "kernel_mvm_noalloc: v and y must be distinct device buffers");
    require(std::isfinite(shift), "kernel_mvm_noalloc: shift must be finite");
    void* base = scratch_ptr(ctx->device);
    if (!base) fail(FFK_ERR_HIP, "kernel_mvm_noalloc: the scratch array of this device has no address");
    kernel_mvm_scratch(s, v, y, shift, (int)prec, S(stream), base, kScratchBytes);
    return FFK_OK;
  });
}

ffk_status ffk_kernel_mvm_phases(ffk_ctx* ctx, ffk_system* s, const double* v, double* y, double shift,
                                 ffk_precision prec, int32_t iters, double* ms, void* stream) {
  if (!ctx || !s || !ms) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(v && y && v != y, "kernel_mvm_phases: v and y must be distinct device buffers");
    require(iters >= 1, "kernel_mvm_phases: iters must be >= 1");
    kernel_mvm_phases(s, v, y, shift, (int)prec, iters, ms, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_clock_enable(ffk_ctx* ctx, int32_t stride) {
  if (!ctx) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(stride >= 0, "clock_enable: stride must be >= 0");
    clock_enable(stride);
    return FFK_OK;
  });
}

ffk_status ffk_clock_read(ffk_ctx* ctx, int32_t id, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(id >= 0 && id < FFK_CLK_COUNT, "clock_read: unknown clock id");
    clock_read(id, total_ms, launches);
    return FFK_OK;
  });
}

ffk_status ffk_kernel_predict(ffk_ctx* ctx, const ffk_system* train, const ffk_system* test, const double* alpha,
                              double* F, void* stream) {
  if (!ctx || !train || !test) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(alpha && F, "kernel_predict: null buffer");
    kernel_predict(train, test, alpha, F, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_kernel_columns(ffk_ctx* ctx, const ffk_system* s, const int64_t* cols, int64_t k, double* out,
                              void* stream) {
  if (!ctx || !s) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(k >= 0 && (k == 0 || (cols && out)), "kernel_columns: bad arguments");
    if (k == 0) return FFK_OK;
    check_indices(cols, k, s->n, S(stream), "kernel_columns");
    kernel_columns(s, cols, k, out, s->n, 0.0, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_kernel_diag(ffk_ctx* ctx, const ffk_system* s, double* d, void* stream) {
  if (!ctx || !s || !d) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    kernel_diag(s, d, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_nystrom_select(ffk_ctx* ctx, ffk_system* s, ffk_select strategy, int64_t k, double lambda,
                              uint64_t seed, int64_t pilot, const double* weights, int64_t* idx,
                              int64_t* k_eff, double* tau_dev, void* stream) {
  if (!ctx || !s) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    hipStream_t st = S(stream);
    require(idx && k_eff, "nystrom_select: null output");
    require(k >= 1 && k <= s->n, "nystrom_select: need 1 <= k <= n");
    *k_eff = 0;
    switch (strategy) {
      case FFK_SEL_UNIFORM:
        select_uniform(s, k, seed, idx, st);
        *k_eff = k;
        break;
      case FFK_SEL_LEVERAGE: {
        require(lambda > 0.0, "nystrom_select: lambda must be > 0 for leverage scores");
        const int64_t ns = pilot > 0 ? std::min(pilot, s->n) : k;
        DBuf pil(ns * 8), tauown;
        double* tau = tau_dev;
        if (!tau) {
          tauown.alloc(s->n * 8);
          tau = tauown.as<double>();
        }
        select_uniform_n(s->n, ns, seed, 1, pil.as<int64_t>(), st);
        leverage_estimate(s, pil.as<int64_t>(), ns, lambda, tau, st);
        select_weighted(s->n, tau, k, seed, 2, idx, st);
        *k_eff = k;
        break;
      }
      case FFK_SEL_PIVCHOL:
        *k_eff = select_pivchol(s, k, idx, st);
        break;
      case FFK_SEL_SCORES: {
        require(weights != nullptr, "nystrom_select: SCORES needs per-geometry weights");
        DBuf w(s->n * 8);
        expand_scores(weights, s->N, s->M, w.as<double>(), st);
        select_weighted(s->n, w.as<double>(), k, seed, 3, idx, st);
        *k_eff = k;
        break;
      }
      default:
        fail(FFK_ERR_ARG, "nystrom_select: unknown strategy");
    }
    HIPCHK(hipStreamSynchronize(st));
    return FFK_OK;
  });
}

ffk_status ffk_precond_build_ex(ffk_ctx* ctx, ffk_system* s, const int64_t* idx, int64_t k, double lambda,
                                ffk_precision store_L, int32_t flags, ffk_precond** out, void* stream) {
  if (!ctx || !s || !out) return FFK_ERR_ARG;
  *out = nullptr;
  return guarded(ctx, [&]() {
    require(idx != nullptr, "precond_build: idx is null");
    require(k >= 1 && k <= s->n, "precond_build: need 1 <= k <= n");
    require(lambda > 0.0 && std::isfinite(lambda), "precond_build: lambda must be > 0");
    require((flags & ~(FFK_BUILD_LOWMEM | FFK_BUILD_MATRIX_FREE)) == 0, "precond_build: unknown flags");
    require(!(flags & FFK_BUILD_LOWMEM) || store_L == FFK_FP32, "precond_build: the low-memory build stores FP32");
    require(!(flags & FFK_BUILD_MATRIX_FREE) || (store_L == FFK_FP64 && !(flags & FFK_BUILD_LOWMEM)),
            "precond_build: the matrix-free form is built from an FP64 factor (store_L = FFK_FP64, no LOWMEM)");
    check_indices(idx, k, s->n, S(stream), "precond_build");
    bool dropped = false;
    *out = precond_build(s, idx, k, lambda, (int)store_L, (flags & FFK_BUILD_LOWMEM) != 0, &dropped, S(stream),
                         (flags & FFK_BUILD_MATRIX_FREE) != 0);
    return dropped ? FFK_WARN_RANK_DROPPED : FFK_OK;
  });
}

ffk_status ffk_precond_build(ffk_ctx* ctx, ffk_system* s, const int64_t* idx, int64_t k, double lambda,
                             ffk_precision store_L, ffk_precond** out, void* stream) {
  return ffk_precond_build_ex(ctx, s, idx, k, lambda, store_L, 0, out, stream);
}

void ffk_precond_free(ffk_precond* P) { delete P; }

ffk_status ffk_precond_info(const ffk_precond* P, int64_t* k, int64_t* k_eff, int64_t* bytes) {
  if (!P) return FFK_ERR_ARG;
  if (k) *k = P->k;
  if (k_eff) *k_eff = P->k_eff;
  if (bytes) *bytes = P->bytes;
  return FFK_OK;
}

ffk_status ffk_precond_apply(ffk_ctx* ctx, const ffk_precond* P, const double* r, double* z, void* stream) {
  if (!ctx || !P) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(r && z && r != z, "precond_apply: r and z must be distinct device buffers");
    precond_apply(P, r, z, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_precond_export(ffk_ctx* ctx, const ffk_precond* P, double* L_dev, void* stream) {
  if (!ctx || !P || !L_dev) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    precond_export(P, L_dev, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_pcg_solve(ffk_ctx* ctx, ffk_system* s, const ffk_precond* P, const double* F, double* alpha,
                         const ffk_pcg_opts* opts, ffk_pcg_report* rep, void* stream) {
  if (!ctx || !s || !opts) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(F && alpha && F != alpha, "pcg_solve: F and alpha must be distinct device buffers");
    require(opts->resume == 0 || opts->resume == 1, "pcg_solve: resume must be 0 or 1");
    require(!opts->direction_dev || (opts->direction_dev != F && opts->direction_dev != alpha),
            "pcg_solve: the direction buffer may not alias F or alpha");
    return pcg_solve(s, P, F, alpha, opts, rep, S(stream));
  });
}

ffk_status ffk_exact_rls(ffk_ctx* ctx, ffk_system* s, double lambda, double* tau, void* stream) {
  if (!ctx || !s || !tau) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(lambda > 0.0, "exact_rls: lambda must be > 0");
    exact_rls(s, lambda, tau, S(stream));
    return FFK_OK;
  });
}

int64_t ffk_mlp_num_params(int32_t D, int32_t H) {
  return (int64_t)H * D + H + (int64_t)H * H + H + H + 1;
}

ffk_status ffk_mlp_create(ffk_ctx* ctx, int32_t D, int32_t H, uint64_t seed, ffk_mlp** out) {
  if (!ctx || !out) return FFK_ERR_ARG;
  *out = nullptr;
  return guarded(ctx, [&]() {
    require(D >= 1 && H >= 1 && H % 64 == 0, "mlp_create: need D >= 1 and H a multiple of 64");
    ffk_mlp* m = mlp_create(D, H, seed);
    m->ctx = ctx;
    *out = m;
    return FFK_OK;
  });
}

void ffk_mlp_free(ffk_mlp* net) { delete net; }

ffk_status ffk_mlp_set_params(ffk_ctx* ctx, ffk_mlp* net, const float* theta, void* stream) {
  if (!ctx || !net || !theta) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    HIPCHK(hipMemcpyAsync(net->theta.get(), theta, net->nparam * 4, hipMemcpyDeviceToDevice, S(stream)));
    net->wbf_valid = false;
    return FFK_OK;
  });
}

ffk_status ffk_mlp_get_params(ffk_ctx* ctx, const ffk_mlp* net, float* theta, void* stream) {
  if (!ctx || !net || !theta) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    HIPCHK(hipMemcpyAsync(theta, net->theta.get(), net->nparam * 4, hipMemcpyDeviceToDevice, S(stream)));
    return FFK_OK;
  });
}

ffk_status ffk_mlp_set_norm(ffk_ctx* ctx, ffk_mlp* net, const float* mean, const float* inv_std, void* stream) {
  if (!ctx || !net || !mean || !inv_std) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    float* base = net->theta.as<float>() + net->nparam;
    HIPCHK(hipMemcpyAsync(base, mean, net->D * 4, hipMemcpyDeviceToDevice, S(stream)));
    HIPCHK(hipMemcpyAsync(base + net->D, inv_std, net->D * 4, hipMemcpyDeviceToDevice, S(stream)));
    return FFK_OK;
  });
}

ffk_status ffk_mlp_forward(ffk_ctx* ctx, const ffk_mlp* net, const float* X, int64_t B, float* out,
                           ffk_precision prec, void* stream) {
  if (!ctx || !net) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(X && out && B >= 1, "mlp_forward: bad arguments");
    require(prec == FFK_FP32 || prec == FFK_BF16, "mlp_forward: precision must be FFK_FP32 or FFK_BF16");
    mlp_forward(net, X, B, out, (int)prec, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_mlp_grad(ffk_ctx* ctx, ffk_mlp* net, const float* X, const float* y, int64_t B, float* loss,
                        float* grad, void* stream) {
  if (!ctx || !net) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(X && y && loss && grad && B >= 1, "mlp_grad: bad arguments");
    mlp_grad(net, X, y, B, loss, grad, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_mlp_adam_step(ffk_ctx* ctx, ffk_mlp* net, const float* grad, float lr, void* stream) {
  if (!ctx || !net || !grad) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    mlp_adam(net, grad, lr, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_mlp_scores(ffk_ctx* ctx, const ffk_mlp* net, const ffk_system* s, double* scores, void* stream) {
  if (!ctx || !net || !s || !scores) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(net->D == s->D, "mlp_scores: network input size differs from the descriptor size");
    mlp_scores(net, s, scores, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_block_log_scores(ffk_ctx* ctx, const double* tau, int64_t N, int32_t M, float* y, void* stream) {
  if (!ctx || !tau || !y) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(N >= 1 && M >= 3, "block_log_scores: need N >= 1 and M >= 3");
    block_log_scores(tau, N, M, y, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_mlp_prepare_inputs(ffk_ctx* ctx, const ffk_mlp* net, const ffk_system* s, float* X, int32_t standardize,
                                  void* stream) {
  if (!ctx || !net || !s || !X) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(net->D == s->D, "mlp_prepare_inputs: network input size differs from the descriptor size");
    mlp_prepare_inputs(net, s, X, standardize, S(stream));
    return FFK_OK;
  });
}

ffk_status ffk_mlp_fit_norm(ffk_ctx* ctx, ffk_mlp* net, const float* X, int64_t B, void* stream) {
  if (!ctx || !net || !X) return FFK_ERR_ARG;
  return guarded(ctx, [&]() {
    require(B >= 2, "mlp_fit_norm: need at least two rows");
    mlp_fit_norm(net, X, B, S(stream));
    return FFK_OK;
  });
}

int64_t ffk_rule_of_thumb(int64_t n, double k_min, double m) {
  if (n < 1 || !(k_min > 0) || !(m > 0)) return -1;
  const double k = std::pow(std::pow(k_min, m) * m * (double)n * (double)n / 2.0, 1.0 / (2.0 + m));
  int64_t r = (int64_t)std::llround(k);
  if (r < 1) r = 1;
  if (r > n) r = n;
  return r;
}

int64_t ffk_rule_of_thumb_calibrated(int64_t n, double k_min, double m, double a, double b, double c) {
  if (n < 1 || !(k_min > 0) || !(m > 0) || !(a >= 0) || !(b >= 0) || !(c >= 0) || !(a + b > 0)) return -1;
  auto f = [&](int64_t k) {
    const double x = (double)k;
    return (double)n * std::pow(k_min / x, m) * (a + b * x) + c * x * x;
  };
  int64_t lo = 1, hi = n;
  while (hi - lo > 2) {
    const int64_t m1 = lo + (hi - lo) / 3, m2 = hi - (hi - lo) / 3;
    if (f(m1) < f(m2)) hi = m2 - 1;
    else if (f(m1) > f(m2)) lo = m1 + 1;
    else { lo = m1; hi = m2; }   // equal values of a unimodal f bracket its minimum
  }
  int64_t best = lo;
  for (int64_t k = lo + 1; k <= hi; ++k)
    if (f(k) < f(best)) best = k;
  return best;
}

ffk_status ffk_rot_fit(const int64_t* k, const int64_t* iters, int32_t count, int64_t n, double* k_min,
                       double* m) {
  if (!k || !iters || !k_min || !m || count < 2 || n < 1) return FFK_ERR_ARG;
  double sx = 0.0, sy = 0.0;
  for (int32_t i = 0; i < count; ++i) {
    if (k[i] < 1 || iters[i] < 1) return FFK_ERR_ARG;
    sx += std::log((double)k[i]);
    sy += std::log((double)iters[i] / (double)n);
  }
  const double mx = sx / count, my = sy / count;
  double sxx = 0.0, sxy = 0.0;
  for (int32_t i = 0; i < count; ++i) {
    const double dx = std::log((double)k[i]) - mx;
    sxx += dx * dx;
    sxy += dx * (std::log((double)iters[i] / (double)n) - my);
  }
  if (!(sxx > 0.0)) return FFK_ERR_ARG;
  const double slope = sxy / sxx;   // = -m
  if (!(slope < 0.0)) return FFK_ERR_ARG;
  const double mm = -slope;
  *m = mm;
  *k_min = std::exp((my + mm * mx) / mm);
  return FFK_OK;
}

}  // extern "C"
