// Preconditioned conjugate gradients for (K + lambda I) alpha = F (Eq. 1-2).
//
// Standard PCG (Hestenes-Stiefel recurrences) with alpha_0 = 0.  All vectors
// and CG scalars are FP64 on the device; scalars never leave it except the two
// needed for the stopping test and breakdown check (|r|^2 and p^T A p), read
// back once per iteration while the GPU already works on the next direction.
// The kernel product inside the iteration can run in
// a reduced precision; then the true residual r = F - K_lambda alpha is
// recomputed with the FP64 product every `refresh_every` iterations and
// replaces the recursively updated one (residual replacement; p is kept), and
// convergence is only declared on an FP64 true residual.  With `escalate`,
// a refresh moves the product one rung up the ladder
// BF16 -> BF16X3 -> FP32 -> FP64 when the true residual has drifted from the
// recursive one by more than half of its norm (the products' rounding now
// shows; CG then restarts from the true residual, p = z) or has not improved
// for 3000 iterations (the direction is kept).  A
// refresh that shows divergence (10x the best true residual) also moves up a
// rung, and restarts from the best iterate.
// `flexible` switches beta to Polak-Ribiere, -gamma z^T q / rho.
// `switch_below` > 0 runs the first iterations with more accurate products
// (`switch_from`: FP64 or FP32) and moves to the reduced precision once the
// residual has fallen below switch_below |F| (accurate products while the
// residual is large, cheap ones afterwards).
// A breakdown (p^T q <= 0) under a reduced-precision product escalates like a
// diverging refresh (restart from the best iterate) when `escalate` is set.
// An escalation before the switch escalates the products of the first phase
// (FP32 -> FP64) and ends that phase.
#include <chrono>
#include <cstdio>

#include "common.hpp"

namespace ffk {

enum { S_RHO0 = 0, S_RHO1 = 1, S_PAP = 2, S_RR = 3, S_ZQ = 4, S_FF = 5, S_TMP = 6, NSC = 8 };

// Escalation tests at a refresh (reduced-precision products only).  A true
// residual whose distance from the recursive one, |r_true - r|, exceeds
// kGapEscalate |r_true| (or the caller's threshold) means the products' rounding now shows in the
// residual; no new best
// true residual for kStallIterations iterations means no progress at all.  Both
// move one rung up and keep the direction.  CG's residual norm is not
// monotone, so a plateau above an earlier best alone is not taken as a sign.
constexpr int64_t kVyMaxGeometries = 4096;
constexpr double kGapEscalate = 0.5;
constexpr int64_t kStallIterations = 3000;

// x += g p, r -= g q with g = rho / p^T q, and the block partials of |r|^2 of
// the updated r (fused_parts grid) in rr_part[0 .. gridDim.x).  Every block
// forms p^T q itself from the np_pq partials of dot64_parts (same fixed order
// in every block); block 0 stores it in sc and after the partials, in
// rr_part[gridDim.x], so that the host reads both with one copy.
__global__ __launch_bounds__(256) void k_axpy2_rr(double* __restrict__ x, double* __restrict__ r,
                                                  const double* __restrict__ p, const double* __restrict__ q,
                                                  double* __restrict__ sc, int rho, int64_t n,
                                                  const double* __restrict__ pq_part, int np_pq,
                                                  double* __restrict__ rr_part) {
  __shared__ double sh[256], sh_pq[256];
  const double pq = sum_parts_block(pq_part, np_pq, sh_pq);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[S_PAP] = pq;
    rr_part[gridDim.x] = pq;
  }
  const double g = sc[rho] / pq;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    x[i] += g * p[i];
    const double ri = r[i] - g * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) rr_part[blockIdx.x] = s;
}

// pn = z + beta p (out of place, so that a speculative update can be redone).
// With rz_part, every block forms rho_new = r^T z from the np_rz partials of
// the preconditioner apply (fixed order) and block 0 stores it in sc.
__global__ __launch_bounds__(256) void k_update_p(double* __restrict__ pn, const double* __restrict__ p,
                                                  const double* __restrict__ z, double* __restrict__ sc, int rho_old,
                                                  int rho_new, int flexible, int64_t n,
                                                  const double* __restrict__ rz_part, int np_rz) {
  __shared__ double sh[256];
  double rn;
  if (rz_part) {
    rn = sum_parts_block(rz_part, np_rz, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) sc[rho_new] = rn;
  } else {
    rn = sc[rho_new];
  }
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double beta;
  if (flexible) {
    const double g = sc[rho_old] / sc[S_PAP];
    beta = -g * sc[S_ZQ] / sc[rho_old];
  } else {
    beta = rn / sc[rho_old];
  }
  pn[i] = z[i] + beta * p[i];
}

__global__ void k_sub(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ c, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = a[i] - b[i];
}
// b = a - b
__global__ void k_rsub(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i] - b[i];
}

static int next_rung(int prec) {
  switch (prec) {
    case FFK_BF16: return FFK_BF16X3;
    case FFK_BF16X3: return FFK_FP32;
    default: return FFK_FP64;
  }
}

struct Timer {
  bool on;
  hipStream_t st;
  hipEvent_t a, b;
  double* acc;
  Timer(bool on_, hipStream_t s, double* acc_) : on(on_), st(s), acc(acc_) {
    if (on) {
      HIPCHK(hipEventCreate(&a));
      HIPCHK(hipEventCreate(&b));
      HIPCHK(hipEventRecord(a, st));
    }
  }
  ~Timer() {
    if (on) {
      (void)hipEventRecord(b, st);
      (void)hipEventSynchronize(b);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, a, b);
      *acc += ms;
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  }
};

ffk_status pcg_solve(ffk_system* s, const ffk_precond* P, const double* F, double* alpha, const ffk_pcg_opts* o,
                     ffk_pcg_report* rep, hipStream_t st) {
  const auto t_start = std::chrono::steady_clock::now();
  const int64_t n = s->n;
  const double lam = o->lambda;
  require(lam > 0.0, "pcg_solve: lambda must be > 0");
  require(o->tol > 0.0, "pcg_solve: tol must be > 0");
  require(o->prec >= FFK_FP64 && o->prec <= FFK_BF16X3, "pcg_solve: unknown precision");
  require(o->switch_from == FFK_FP64 || o->switch_from == FFK_FP32,
          "pcg_solve: the products before the switch must be FP64 or FP32");
  if (P) require(P->n == n, "pcg_solve: preconditioner size does not match the system");
  const int64_t max_iter = o->max_iter > 0 ? o->max_iter : n;
  const bool timing = o->timing != 0;
  const double gap_thr = o->gap_escalate > 0.0 ? o->gap_escalate : kGapEscalate;
  double t_mvm = 0, t_prec = 0, t_vec = 0, t_ref = 0;

  DBuf r(n * 8), z(n * 8), p(n * 8), p2(n * 8), q(n * 8), tmp(n * 8), best(n * 8), sc(NSC * 8),
      part((2 * kRedParts + 1) * 8);
  double* R = r.as<double>();
  double* Z = z.as<double>();
  double* Pv = p.as<double>();
  double* Pn = p2.as<double>();
  double* Q = q.as<double>();
  double* SC = sc.as<double>();
  double* PART = part.as<double>();              // partials of one reduction
  double* PART2 = PART + kRedParts;                // a second set: |r|^2 partials, then p^T q
  // p^T q from the product's per-geometry partials when they are few enough
  // for every block of the update to sum them; otherwise a dot-product pass
  DBuf vy(s->N <= kVyMaxGeometries ? s->N * 8 : 0);
  double* VY = s->N <= kVyMaxGeometries ? vy.as<double>() : nullptr;
  const int nb = cdiv(n, 256);
  const int np_fused = fused_parts(n);
  s->ctx->host_scratch.ensure((kRedParts + 8) * 8);
  double* hs = s->ctx->host_scratch.as<double>();
  struct Ev {
    hipEvent_t e = nullptr;
    ~Ev() { if (e) (void)hipEventDestroy(e); }
  } done;
  HIPCHK(hipEventCreateWithFlags(&done.e, hipEventDisableTiming));

  auto apply_prec = [&](const double* in, double* out) {
    Timer tm(timing, st, &t_prec);
    if (P) precond_apply(P, in, out, st);
    else HIPCHK(hipMemcpyAsync(out, in, n * 8, hipMemcpyDeviceToDevice, st));
  };
  // r = F - K_lambda alpha (FP64); returns |r|^2
  auto true_residual = [&]() -> double {
    Timer tm(timing, st, &t_ref);
    kernel_mvm(s, alpha, tmp.as<double>(), lam, FFK_FP64, st);
    k_sub<<<nb, 256, 0, st>>>(F, tmp.as<double>(), R, n);
    LAUNCHCHK();
    dot64(R, R, n, PART, SC + S_RR, st);
    HIPCHK(hipMemcpyAsync(hs, SC + S_RR, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return hs[0];
  };
  // At a refresh: r_true = F - K_lambda alpha (FP64) replaces the recursive r.
  // Returns |r_true|^2, and |r_true - r|^2 in *gap2.  Z holds the difference:
  // every refresh recomputes the next direction, and Z with it.
  auto refresh_residual = [&](double* gap2) -> double {
    Timer tm(timing, st, &t_ref);
    double* T = tmp.as<double>();
    kernel_mvm(s, alpha, T, lam, FFK_FP64, st);
    k_rsub<<<nb, 256, 0, st>>>(F, T, n);
    k_sub<<<nb, 256, 0, st>>>(T, R, Z, n);
    LAUNCHCHK();
    dot64(T, T, n, PART, SC + S_RR, st);
    dot64(Z, Z, n, PART, SC + S_TMP, st);
    HIPCHK(hipMemcpyAsync(R, T, n * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(hs, SC + S_RR, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hs + 2, SC + S_TMP, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *gap2 = hs[2];
    return hs[0];
  };

  dot64(F, F, n, PART, SC + S_FF, st);
  HIPCHK(hipMemcpyAsync(hs, SC + S_FF, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double fnorm = sqrt(hs[0]);
  if (!std::isfinite(fnorm)) fail(FFK_ERR_NONFINITE, "pcg_solve: F contains NaN or Inf");

  double best_true = fnorm * fnorm;   // alpha = 0
  double rel_upd = 1.0, rel_true = 1.0;
  int64_t n_ref = 0;
  const bool resume = o->resume && fnorm > 0.0;   // F = 0: the solution is alpha = 0 either way
  if (resume) {
    // continue from the caller's alpha: the true residual replaces r, as at a refresh
    best_true = true_residual();
    ++n_ref;
    rel_true = rel_upd = sqrt(best_true) / fnorm;
  } else {
    HIPCHK(hipMemsetAsync(alpha, 0, n * 8, st));
    HIPCHK(hipMemcpyAsync(R, F, n * 8, hipMemcpyDeviceToDevice, st));
  }
  HIPCHK(hipMemcpyAsync(best.get(), alpha, n * 8, hipMemcpyDeviceToDevice, st));
  int prec = o->prec;
  const int first = o->switch_from;
  bool hi_phase = o->switch_below > 0.0 && prec != FFK_FP64 && prec != first;
  int64_t switch_iter = hi_phase ? -1 : 0;
  int64_t esc_iter[3] = {-1, -1, -1};
  int rho = S_RHO0;
  auto restart_direction = [&]() {
    apply_prec(R, Z);
    dot64(R, Z, n, PART, SC + rho, st);
    HIPCHK(hipMemcpyAsync(Pv, Z, n * 8, hipMemcpyDeviceToDevice, st));
  };
  if (resume && o->direction_dev) {
    // the caller's direction, with rho = r^T P^-1 r of the true residual
    apply_prec(R, Z);
    dot64(R, Z, n, PART, SC + rho, st);
    HIPCHK(hipMemcpyAsync(Pv, o->direction_dev, n * 8, hipMemcpyDeviceToDevice, st));
  } else {
    restart_direction();
  }

  ffk_status status = FFK_NOT_CONVERGED;
  int64_t best_it = 0;   // iteration of the best true residual so far
  int64_t it = 0, n_esc = 0;
  if (fnorm == 0.0 || (resume && rel_true <= o->tol)) {
    status = FFK_OK;
    if (fnorm == 0.0) rel_upd = rel_true = 0.0;
  }
  int64_t hist_len = 0;
  const int refresh = o->refresh_every;
  // Move the products one rung up from the precision now in use.  Before the
  // switch that is `first`: the first phase ends there, one rung above it
  // (FP32 -> FP64), whatever the reduced precision would have been.
  auto rung_up = [&]() {
    if (n_esc < 3) esc_iter[n_esc] = it;
    if (hi_phase) {
      hi_phase = false;
      switch_iter = it;
      prec = next_rung(first);
    } else {
      prec = next_rung(prec);
    }
    ++n_esc;
  };
  // One rung up without a restart: the residual has just been replaced by the
  // true one, and the direction is kept (a residual replacement).
  auto step_up = [&]() {
    rung_up();
    best_it = it;
  };
  auto escalate_now = [&]() {
    rung_up();
    HIPCHK(hipMemcpyAsync(alpha, best.get(), n * 8, hipMemcpyDeviceToDevice, st));
    true_residual();
    ++n_ref;
    best_it = it;
    restart_direction();
  };
  // Next direction from the current r: z = M^-1 r, rho_new = r^T z, pn = z + beta p.
  auto next_direction = [&](int rho_new) {
    int np_rz = 0;   // > 0: r^T z is still in PART as partials, summed by k_update_p
    if (P) {
      Timer tm(timing, st, &t_prec);
      np_rz = precond_apply_parts(P, R, Z, PART, st);
    } else {
      apply_prec(R, Z);
      dot64(R, Z, n, PART, SC + rho_new, st);
    }
    Timer tm(timing, st, &t_vec);
    if (o->flexible) {
      if (np_rz) sum_parts64(PART, np_rz, SC + rho_new, st);
      np_rz = 0;
      dot64(Z, Q, n, PART, SC + S_ZQ, st);
    }
    k_update_p<<<nb, 256, 0, st>>>(Pn, Pv, Z, SC, rho, rho_new, o->flexible, n, np_rz ? PART : nullptr, np_rz);
    LAUNCHCHK();
  };
  // The host reads |r|^2 and p^T q once per iteration.  Except on refresh
  // iterations, the next direction is enqueued before that read, so the GPU
  // keeps working while the host waits; if the read then calls for a
  // breakdown restart or a residual replacement, the speculative direction is
  // discarded (p is only replaced after the decision).
  while (status == FFK_NOT_CONVERGED && it < max_iter) {
    const int cur = hi_phase ? first : prec;
    int np_pq = 0;   // > 0: the product left p^T q as partials in VY
    {
      Timer tm(timing, st, &t_mvm);
      np_pq = VY ? kernel_mvm_vy(s, Pv, Q, lam, cur, st, VY) : (kernel_mvm(s, Pv, Q, lam, cur, st), 0);
    }
    {
      Timer tm(timing, st, &t_vec);
      const double* pq_part = VY;
      if (np_pq == 0) {
        np_pq = dot64_parts(Pv, Q, n, PART, st);
        pq_part = PART;
      }
      k_axpy2_rr<<<np_fused, 256, 0, st>>>(alpha, R, Pv, Q, SC, rho, n, pq_part, np_pq, PART2);
      LAUNCHCHK();
      // the |r|^2 partials and p^T q go to the host, which sums the partials
      HIPCHK(hipMemcpyAsync(hs, PART2, (np_fused + 1) * 8, hipMemcpyDeviceToHost, st));
      HIPCHK(hipEventRecord(done.e, st));
    }
    ++it;
    const int rho_new = rho ^ 1;
    const bool periodic = refresh > 0 && (it % refresh) == 0 && cur != FFK_FP64;
    bool have_next = false;
    if (!periodic) {
      next_direction(rho_new);
      have_next = true;
    }
    HIPCHK(hipEventSynchronize(done.e));
    double rr = 0.0;
    for (int b = 0; b < np_fused; ++b) rr += hs[b];
    const double pap = hs[np_fused];
    if (!(pap > 0.0) || !std::isfinite(pap) || !std::isfinite(rr)) {
      if (o->escalate && cur != FFK_FP64) {
        escalate_now();
        continue;
      }
      status = FFK_ERR_BREAKDOWN;
      break;
    }
    rel_upd = sqrt(rr) / fnorm;
    if (hi_phase && rel_upd <= o->switch_below) {
      hi_phase = false;
      switch_iter = it;
    }
    if (rep && rep->hist_host && hist_len < rep->hist_cap) rep->hist_host[hist_len++] = rel_upd;
    if (o->progress_every > 0 && it % o->progress_every == 0) {
      static const char* names[4] = {"fp64", "fp32", "bf16", "bf16x3"};
      fprintf(stderr, "pcg it %lld  updated residual %.3e  last true residual %.3e  products %s\n", (long long)it,
              rel_upd, rel_true, names[cur]);
      fflush(stderr);
    }
    const bool candidate = rel_upd <= o->tol;
    if (candidate || periodic) {
      const double upd = rel_upd;   // the recursive residual the true one replaces
      double gap2 = 0.0;
      const double tr = refresh_residual(&gap2);
      ++n_ref;
      rel_true = sqrt(tr) / fnorm;
      rel_upd = rel_true;
      const double gap = tr > 0.0 ? sqrt(gap2 / tr) : 0.0;   // |r_true - r| / |r_true|
      if (o->progress_every > 0) {
        fprintf(stderr, "pcg refresh at %lld  true %.4e  recursive %.4e  gap %.4f\n", (long long)it, rel_true, upd,
                gap);
        fflush(stderr);
      }
      if (rel_true <= o->tol) {
        status = FFK_OK;
        break;
      }
      if (tr < best_true) {
        best_true = tr;
        best_it = it;
        HIPCHK(hipMemcpyAsync(best.get(), alpha, n * 8, hipMemcpyDeviceToDevice, st));
      }
      if (o->escalate && cur != FFK_FP64) {
        if (tr > 100.0 * best_true) {   // diverging: back to the best iterate
          escalate_now();
          continue;
        }
        if (gap > gap_thr) {
          // the recursive residual had drifted away from the true one, so
          // the last direction was built from a wrong residual: one rung up,
          // and CG restarts from the true residual (p = z)
          step_up();
          restart_direction();
          continue;
        }
        if (it - best_it >= kStallIterations) step_up();
      }
      have_next = false;   // r was replaced: the direction must come from it
    }
    if (!have_next) next_direction(rho_new);
    std::swap(Pv, Pn);
    rho = rho_new;
  }
  if (status == FFK_NOT_CONVERGED && it > 0) {
    rel_true = sqrt(true_residual()) / fnorm;
    ++n_ref;
    if (rel_true <= o->tol) status = FFK_OK;
  }
  if (o->direction_dev) HIPCHK(hipMemcpyAsync(o->direction_dev, Pv, n * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  const double total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  if (rep) {
    rep->iters = it;
    rep->n_refresh = n_ref;
    rep->n_escalations = n_esc;
    rep->rel_res_true = rel_true;
    rep->rel_res_updated = rel_upd;
    rep->final_prec = hi_phase ? first : prec;
    rep->status = status;
    rep->switch_iter = switch_iter;
    for (int e = 0; e < 3; ++e) rep->esc_iter[e] = esc_iter[e];
    rep->t_mvm_ms = t_mvm;
    rep->t_prec_ms = t_prec;
    rep->t_vec_ms = t_vec;
    rep->t_refresh_ms = t_ref;
    rep->t_total_ms = total;
    rep->hist_len = hist_len;
  }
  return status;
}

}  // namespace ffk
