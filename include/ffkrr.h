/*
 * ffkrr.h -- C ABI of the MI355X (gfx950) library for the preconditioned
 * conjugate-gradient solve of the force-field kernel ridge system
 *
 *     (K + lambda I) alpha = F                                  (paper, Eq. 1)
 *
 * K (n x n, n = 3 M N) is the force-field kernel of N geometries of M atoms
 * (section 2.1): block (i,j) is J_i^T H(x_i, x_j) J_j, with x the inverse-
 * distance descriptor (D = M(M-1)/2 entries, pairs p > q in row-major lower-
 * triangle order), J its Jacobian and H = a(r) I + b(r) d d^T the Hessian of the
 * Matern-5/2 kernel of length scale sigma (d = x_i - x_j, r = |d|,
 * a = 5/(3 sigma^2)(1+z)e^-z, b = -25/(3 sigma^4) e^-z, z = sqrt(5) r/sigma).
 * K is never formed.  Index order of n-vectors: 3 M g + 3 p + c for geometry g,
 * atom p, coordinate c (the paper's (n_train, d, 3) reshape, appendix A.1).
 *
 * Conventions for every entry point:
 *  - Return value: FFK_OK (0), an error (< 0) or a warning (> 0).  The message
 *    of the last failure on a context is returned by ffk_last_error().  No C++
 *    exception crosses the ABI.
 *  - Pointers named *_dev are device pointers on the context's GPU; the caller
 *    owns them and the library never frees them.  Arrays are densely packed in
 *    the layout stated per argument.  Host pointers are named *_host.
 *  - Opaque handles (ffk_system, ffk_precond, ffk_mlp) are created and owned by
 *    the library, hold their own device workspaces, and are released by the
 *    matching *_free call.  Handles are not thread-safe; concurrent calls on the
 *    same handle race.
 *  - `stream` is a hipStream_t (NULL = the null stream).  All device work is
 *    enqueued on it.  Calls that return host values synchronize the stream.
 *  - Argument checks (sizes, lambda > 0, k <= n, M >= 3) are done before any
 *    work is enqueued; a failed check returns FFK_ERR_ARG and changes nothing.
 */
#ifndef FFKRR_H
#define FFKRR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FFK_OK = 0,
  FFK_ERR_ARG = -1,        /* invalid argument */
  FFK_ERR_OOM = -2,        /* device allocation failed */
  FFK_ERR_HIP = -3,        /* a HIP runtime call failed */
  FFK_ERR_NOT_SPD = -4,    /* a Cholesky factorization met a non-positive pivot */
  FFK_ERR_BREAKDOWN = -5,  /* p^T A p <= 0 or non-finite inside CG */
  FFK_ERR_NONFINITE = -6,  /* NaN/Inf in an input */
  FFK_NOT_CONVERGED = 1,   /* PCG stopped at max_iter above the tolerance */
  FFK_WARN_RANK_DROPPED = 2 /* some inducing columns were dropped as dependent */
} ffk_status;

/* Arithmetic of the kernel matrix-vector product.  FFK_FP64/FFK_FP32 run the
 * contractions on FP64/FP32 MFMA.  FFK_BF16 runs them on BF16 MFMA with FP32
 * accumulation; FFK_BF16X3 splits each operand into a BF16 high and low part
 * and sums hi*hi + hi*lo + lo*hi (three BF16 MFMAs, FP32 accumulation). */
typedef enum { FFK_FP64 = 0, FFK_FP32 = 1, FFK_BF16 = 2, FFK_BF16X3 = 3 } ffk_precision;

/* Inducing-column selection strategies (section 3, "Column selection
 * strategies"; SCORES = sampling by externally supplied per-geometry scores,
 * e.g. from ffk_mlp_scores). */
typedef enum { FFK_SEL_UNIFORM = 0, FFK_SEL_LEVERAGE = 1, FFK_SEL_PIVCHOL = 2,
               FFK_SEL_SCORES = 3 } ffk_select;

typedef struct ffk_ctx ffk_ctx;
typedef struct ffk_system ffk_system;
typedef struct ffk_precond ffk_precond;
typedef struct ffk_mlp ffk_mlp;

/* ---- context ------------------------------------------------------------ */

/* Create a context bound to GPU `device`.  *out receives the handle. */
ffk_status ffk_create(ffk_ctx** out, int device);
void ffk_destroy(ffk_ctx* ctx);
/* Message of the last failure on ctx (empty string if none).  Valid until the
 * next call on ctx. */
const char* ffk_last_error(const ffk_ctx* ctx);
/* Library version string, e.g. "ffkrr 1.0 gfx950". */
const char* ffk_version(void);

/* ---- descriptor and kernel (section 2.1) -------------------------------- */

/* Build the per-system state from the geometries R_dev (N x M x 3 float64,
 * Angstrom): the descriptor X (N x D), its column mean, the centred X_c and the
 * iteration-invariant kernel coefficients a(r_ij) - a(0) and b(r_ij) for all
 * geometry pairs, computed from the Gram matrix X_c X_c^T.  Coefficients for a
 * reduced precision are derived lazily on first use.  M >= 3, N >= 1,
 * sigma > 0.  Returns FFK_ERR_NONFINITE if R has coincident atoms or NaN. */
ffk_status ffk_descriptor_build(ffk_ctx* ctx, const double* R_dev, int64_t N, int32_t M,
                                double sigma, ffk_system** out, void* stream);
void ffk_system_free(ffk_system* sys);
/* Sizes of a system: N, M, D = M(M-1)/2, n = 3 M N (any pointer may be NULL). */
ffk_status ffk_system_info(const ffk_system* sys, int64_t* N, int32_t* M, int64_t* D, int64_t* n);
/* Copy the (uncentred) descriptor X (N x D row-major float64) to X_dev. */
ffk_status ffk_descriptor_export(ffk_ctx* ctx, const ffk_system* sys, double* X_dev, void* stream);

/* Symmetrize the kernel of `sys` over a group of S atom permutations, the
 * sGDML form of the paper's kernels (section 2.1):
 *   k_S(R, R') = sum_q k(x(R), x(P_q R')),   (P_q R)_a = R_{p_q(a)},
 * so the force-kernel block is sum_q J(R_i)^T H(x_i, x(P_q R_j)) J(P_q R_j)
 * Pi_q (Pi_q permutes the atoms of a coordinate vector the same way).
 * perms_host: S x M int32 in host memory, row q = p_q.  The rows must form a
 * group: permutations of 0 .. M-1, no repeats, the identity included, closed
 * under composition; otherwise FFK_ERR_ARG and nothing changes.  The group of
 * the identity alone restores the plain kernel.  Afterwards every call on
 * `sys` uses K_S: ffk_kernel_mvm (every precision), ffk_kernel_columns,
 * ffk_kernel_diag, selection, the preconditioner, PCG, the exact leverage
 * scores, and ffk_kernel_predict with `sys` as the training system.  The
 * product runs as one product against the N S stacked permuted geometries
 * (N x N S coefficient sets, built per precision on first use and kept);
 * ffk_kernel_mvm_noalloc refuses a symmetrized system.
 * Finding the permutations (sGDML matches the molecular graph) is left to
 * the caller. */
ffk_status ffk_system_set_symmetries(ffk_ctx* ctx, ffk_system* sys, const int32_t* perms_host, int32_t S,
                                     void* stream);

/* y = K v + shift * v for the training system (v, y: n float64), with the
 * contractions in precision `prec`.  Matrix free: U = J v (N x D),
 * P = X_c U^T, W = B o (P - 1 diag(P)^T), G = a(0) 1 1^T U + dA U - W X_c +
 * diag(W 1) X_c, y = J^T G (per geometry).  v and y may not alias. */
ffk_status ffk_kernel_mvm(ffk_ctx* ctx, ffk_system* sys, const double* v_dev, double* y_dev,
                          double shift, ffk_precision prec, void* stream);

/* ffk_kernel_mvm for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, result and numerics as ffk_kernel_mvm; the product's
 * workspace (J v in the GEMM operand layouts, -W, the row-sum and split-K
 * partials, G) lives in a fixed scratch array of 128 MiB that the library
 * holds on every device it runs on until the process ends, and the call makes
 * no allocation of any kind.  Conditions:
 *  - the system's coefficients and descriptor copies for `prec` must exist:
 *    one earlier ffk_kernel_mvm (or a solve) in that precision on `sys` builds
 *    them; otherwise FFK_ERR_ARG;
 *  - the workspace must fit: about N^2 (8 B FP64, 4 B FP32 and BF16 x2 arrays;
 *    none for the BF16 products that run fused, at short D) plus 3 N D
 *    doubles; N <= 3500 or so in FP64, about 5000 in split BF16 at D = 210.
 *    Larger systems return FFK_ERR_ARG and change nothing;
 *  - a symmetrized system returns FFK_ERR_ARG.
 * Every call on a GPU shares that GPU's scratch, which keeps the last call's
 * contents (each call clears what it needs zeroed itself): two calls that
 * overlap on one GPU (different streams or threads) race and give wrong
 * results.  The library's kernel clocks do not time this variant. */
ffk_status ffk_kernel_mvm_noalloc(ffk_ctx* ctx, ffk_system* sys, const double* v_dev, double* y_dev,
                                  double shift, ffk_precision prec, void* stream);

/* Profiling variant of ffk_kernel_mvm: runs the product `iters` times and
 * returns in phase_ms_host[0..4] the average milliseconds of its phases, timed
 * with HIP events on `stream`: [0] U = J v, [1] column sums of U (and the BF16
 * transposes), [2] GEMM 1 with the W epilogue, [3] GEMM 2 with the G
 * epilogue, [4] y = J^T G.  Synchronizes the stream. */
ffk_status ffk_kernel_mvm_phases(ffk_ctx* ctx, ffk_system* sys, const double* v_dev, double* y_dev,
                                 double shift, ffk_precision prec, int32_t iters,
                                 double* phase_ms_host, void* stream);

/* Kernel clocks.  While enabled, the library records a HIP event pair on the
 * launching stream around every `stride`-th launch of each kernel named
 * below and adds the elapsed time to that kernel's clock; recording never
 * waits for the GPU.  ffk_clock_enable synchronizes the device and zeroes
 * every clock (stride = 0 stops recording, stride < 0 is FFK_ERR_ARG).
 * ffk_clock_read synchronizes the device and returns the total milliseconds
 * and the number of timed launches of clock `id`.  Process-wide, for the
 * device that was current when enabled; not thread-safe. */
typedef enum {
  FFK_CLK_JV = 0,          /* U = J v (+ low-precision copies, column partials) */
  FFK_CLK_COLSUM = 1,      /* column sums 1^T U */
  FFK_CLK_GEMM1 = 2,       /* P = X_c U^T with the fused W / row-sum epilogue */
  FFK_CLK_GEMM2 = 3,       /* [dA | -W] [U ; X_c] (split-K partials or G epilogue) */
  FFK_CLK_GEMM2_REDUCE = 4,/* split-K reduction with the G epilogue */
  FFK_CLK_JTG = 5,         /* y = J^T G + shift v */
  FFK_CLK_GEMV_T = 6,      /* preconditioner apply: L^T r partials (one pass over L) */
  FFK_CLK_GEMV_N = 7,      /* preconditioner apply: L t partials (one pass over L) */
  FFK_CLK_CORE = 8,        /* preconditioner apply: the two k x k triangular products */
  FFK_CLK_FUSED = 9,       /* BF16 products at short D (<= 96; <= 128 up to N^2 = 4096^2): both GEMMs in one kernel */
  FFK_CLK_COUNT = 10
} ffk_clock;
ffk_status ffk_clock_enable(ffk_ctx* ctx, int32_t stride);
ffk_status ffk_clock_read(ffk_ctx* ctx, int32_t id, double* total_ms_host, int64_t* launches_host);

/* Force prediction F_test = K(test, train) alpha (section 2.1: predictions
 * cost linear in n_train).  test and train must have the same M and sigma.
 * alpha: 3 M N_train float64; F_test: 3 M N_test float64.  FP64. */
ffk_status ffk_kernel_predict(ffk_ctx* ctx, const ffk_system* train, const ffk_system* test,
                              const double* alpha_dev, double* F_dev, void* stream);

/* Columns K[:, cols] for k column indices cols_dev (int64, device), written to
 * out_dev column-major (n x k, leading dimension n).  0 <= cols < n. */
ffk_status ffk_kernel_columns(ffk_ctx* ctx, const ffk_system* sys, const int64_t* cols_dev,
                              int64_t k, double* out_dev, void* stream);
/* diag(K) (n float64): a(0) |J_g e_c|^2 since H(x, x) = a(0) I. */
ffk_status ffk_kernel_diag(ffk_ctx* ctx, const ffk_system* sys, double* d_dev, void* stream);

/* ---- Nystroem preconditioner (section 3, Eq. 3-5, Algorithm 1) ---------- */

/* Select k inducing columns; idx_dev (int64, device, capacity k) receives them
 * in selection order and *k_eff_host how many are valid.
 *  UNIFORM : k columns with the largest SplitMix64 draws u_i (stream 0);
 *  LEVERAGE: ridge leverage estimates from a uniform pilot set of size
 *            `pilot` (<= 0 means k) drawn on stream 1,
 *            tau_i = (K_ii - K_iS (K_SS + lambda I)^-1 K_Si)/lambda clipped to
 *            [1e-12, 1] (pilot columns get 1), then k columns without
 *            replacement by Efraimidis-Spirakis keys log(u_i)/tau_i (stream 2);
 *  PIVCHOL : Algorithm 1, greedy pivot on the largest remaining diagonal of
 *            the Schur complement (ties to the lower index), stopping early
 *            (k_eff < k) once it falls to 1e-12 max(diag K);
 *  SCORES  : weights_dev holds N positive per-geometry scores; every column
 *            of geometry g gets weight max(score_g, 1e-12) and k columns are
 *            drawn by Efraimidis-Spirakis keys (stream 3).
 * weights_dev is ignored except for SCORES.  tau_dev (n float64, may be NULL)
 * receives the leverage estimates for LEVERAGE. */
ffk_status ffk_nystrom_select(ffk_ctx* ctx, ffk_system* sys, ffk_select strategy, int64_t k,
                              double lambda, uint64_t seed, int64_t pilot,
                              const double* weights_dev, int64_t* idx_dev, int64_t* k_eff_host,
                              double* tau_dev, void* stream);

/* Build P = L L^T + lambda I (Eq. 3) from the k columns idx_dev (in the given
 * order): L is the incomplete Cholesky factor of K with pivots forced to that
 * order (equal to the Nystroem factor K_nk K_kk^-1 K_nk^T, Eq. 5), computed in
 * FP64 by column panels; a column whose remaining diagonal falls to
 * 1e-12 max(diag K) is dropped (returns FFK_WARN_RANK_DROPPED).  Then the k x k
 * core lambda I + L^T L is factored in FP64 and its triangular inverse kept.
 * store_L = FFK_FP64, FFK_FP32 or FFK_BF16 selects the storage of L (rounded
 * to nearest; the core is always built in FP64 from the stored L, so P stays
 * symmetric positive definite and the apply is exact for the stored L).
 * FFK_BF16X3 is FFK_ERR_ARG. */
ffk_status ffk_precond_build(ffk_ctx* ctx, ffk_system* sys, const int64_t* idx_dev, int64_t k,
                             double lambda, ffk_precision store_L, ffk_precond** out, void* stream);
/* ffk_precond_build with flags.  FFK_BUILD_LOWMEM (store_L must be FFK_FP32)
 * computes each 64-column panel of L in FP64 from the earlier columns as
 * stored in FP32 and keeps only the FP32 factor: n k 4 bytes instead of the
 * n k 12 of an FP64 factor plus its FP32 copy.  The factor then differs from
 * the rounded FP64 one by FP32 rounding in the panel updates (the
 * preconditioner stays exactly SPD, its core built from the stored L).
 * ffk_precond_build picks this build by itself for FFK_FP32 storage when the
 * FP64 factor and its copy would not fit in the device's free memory. */
/* FFK_BUILD_MATRIX_FREE (store_L must be FFK_FP64) keeps no n x k factor: the
 * forced-order factor interpolates K on its kept pivots S, K[:, S] = L L_SS^T
 * with L_SS = L[S, :] lower triangular, so L = K[:, S] L_SS^-T (section 3,
 * Eq. 5) and the apply of Eq. 4 runs as
 *   L^T r = L_SS^-1 (K r)_S,  L t = K (L_SS^-T t scattered onto S),
 * two FP64 kernel products on `sys` plus k x k triangular products, in place
 * of the two passes over L.  The build still forms the FP64 factor once (to
 * form the core lambda I + L^T L) and then frees it; the preconditioner then
 * holds O(k^2) memory and refers to `sys`, which must stay alive and
 * unchanged while the preconditioner is used.  ffk_precond_export forms L
 * from the kernel's columns. */
enum { FFK_BUILD_LOWMEM = 1, FFK_BUILD_MATRIX_FREE = 2 };
ffk_status ffk_precond_build_ex(ffk_ctx* ctx, ffk_system* sys, const int64_t* idx_dev, int64_t k,
                                double lambda, ffk_precision store_L, int32_t flags, ffk_precond** out,
                                void* stream);
void ffk_precond_free(ffk_precond* P);
/* k requested, k_eff kept, bytes of device memory held. */
ffk_status ffk_precond_info(const ffk_precond* P, int64_t* k, int64_t* k_eff, int64_t* bytes);
/* z = P^-1 r = lambda^-1 (r - L (lambda I + L^T L)^-1 L^T r)  (Eq. 4).
 * r, z: n float64; may not alias. */
ffk_status ffk_precond_apply(ffk_ctx* ctx, const ffk_precond* P, const double* r_dev,
                             double* z_dev, void* stream);
/* Copy L (n x k_eff, column-major float64) to L_dev. */
ffk_status ffk_precond_export(ffk_ctx* ctx, const ffk_precond* P, double* L_dev, void* stream);

/* ---- PCG (section 2.1-2.2, Eq. 1-2) ------------------------------------- */

typedef struct {
  double lambda;          /* ridge, > 0 */
  double tol;             /* stop when |F - K_lambda alpha|_2 <= tol |F|_2 (FP64 true residual) */
  int64_t max_iter;       /* <= 0: n */
  int32_t prec;           /* ffk_precision of the MVM inside the iteration */
  int32_t refresh_every;  /* recompute r = F - K_lambda alpha in FP64 every so many
                             iterations (<= 0: never, except at convergence) */
  int32_t escalate;       /* 1: move to a more accurate MVM precision (BF16 -> BF16X3 ->
                             FP32 -> FP64) when a refresh finds |r_true - r| > |r_true| / 2
                             (r the recursive residual), no new best true residual for
                             3000 iterations, or divergence (10x the best; then
                             the solve restarts from the best iterate) */
  int32_t flexible;       /* 1: Polak-Ribiere beta (robust to inexact operators) */
  int32_t timing;         /* 1: time MVM / preconditioner / vector phases with events */
  double switch_below;    /* > 0: `switch_from` products while the updated residual is
                             above switch_below |F|, then `prec` (0: `prec` from the start) */
  int32_t progress_every; /* > 0: print one line to stderr every so many iterations
                             (iteration, updated and true residual, precision) */
  int32_t switch_from;    /* precision of the products before the switch: FFK_FP64 (0,
                             the default) or FFK_FP32; anything else is FFK_ERR_ARG.  An
                             escalation before the switch ends the first phase and moves
                             its products one rung up (FP32 -> FP64) */
  double gap_escalate;    /* threshold of the escalation test |r_true - r| > gap_escalate
                             |r_true| at a refresh (<= 0: 0.5) */
  int32_t resume;         /* 1: start from the alpha in alpha_dev (instead of alpha_0 = 0):
                             r = F - K_lambda alpha in FP64, as at a refresh */
  double* direction_dev;  /* optional, n float64.  With resume, on entry: the search
                             direction to continue along (NULL: restart, p = P^-1 r).  On
                             return (any status): the direction the next iteration would
                             take.  Saving alpha and this direction lets a solve stop and
                             continue later (another process, another device) the way the
                             periodic refresh continues: true residual, direction kept */
} ffk_pcg_opts;

typedef struct {
  int64_t iters;          /* iterations taken */
  int64_t n_refresh;      /* FP64 true-residual recomputations */
  int64_t n_escalations;  /* precision escalations */
  double rel_res_true;    /* final FP64 |F - K_lambda alpha| / |F| */
  double rel_res_updated; /* final recursively updated residual / |F| */
  int32_t final_prec;     /* precision in use at the end */
  int32_t status;         /* same as the return value */
  int64_t switch_iter;    /* iteration at which the products left `switch_from` (-1: never) */
  int64_t esc_iter[3];    /* iterations at which escalations happened (-1: none) */
  double t_mvm_ms, t_prec_ms, t_vec_ms, t_refresh_ms, t_total_ms;
  double* hist_host;      /* optional caller buffer: updated residual norm / |F| per iteration */
  int64_t hist_cap;       /* capacity of hist_host */
  int64_t hist_len;       /* entries written */
} ffk_pcg_report;

/* Solve (K + lambda I) alpha = F by preconditioned CG with P (NULL = plain CG),
 * alpha_0 = 0 (or alpha_dev's content with opts->resume).  CG scalars and dot
 * products are FP64 on the device (deterministic two-stage reductions).
 * F, alpha: n float64; direction_dev may not alias either. */
ffk_status ffk_pcg_solve(ffk_ctx* ctx, ffk_system* sys, const ffk_precond* P,
                         const double* F_dev, double* alpha_dev, const ffk_pcg_opts* opts,
                         ffk_pcg_report* report, void* stream);

/* ---- learned column selection (additions to the paper's method) --------- */

/* Exact ridge leverage scores tau_c = (K (K + lambda I)^-1)_cc = 1 -
 * lambda [(K + lambda I)^-1]_cc (section 3) from a dense FP64 Cholesky
 * factorization on the GPU (needs 8 n^2 bytes of device memory). tau: n float64. */
ffk_status ffk_exact_rls(ffk_ctx* ctx, ffk_system* sys, double lambda, double* tau_dev,
                         void* stream);

/* Score network D -> H -> H -> 1, exact-erf GELU, FP32 weights.  Flat
 * parameter layout: W1 (H x D row-major), b1 (H), W2 (H x H), b2 (H), w3 (H),
 * b3 (1); then the input standardisation mean (D) and inverse std (D), and the
 * output offset/scale (2) applied by ffk_mlp_scores. */
ffk_status ffk_mlp_create(ffk_ctx* ctx, int32_t D, int32_t H, uint64_t seed, ffk_mlp** out);
void ffk_mlp_free(ffk_mlp* net);
int64_t ffk_mlp_num_params(int32_t D, int32_t H);
ffk_status ffk_mlp_set_params(ffk_ctx* ctx, ffk_mlp* net, const float* theta_dev, void* stream);
ffk_status ffk_mlp_get_params(ffk_ctx* ctx, const ffk_mlp* net, float* theta_dev, void* stream);
/* Set the input standardisation (mean_dev, inv_std_dev: D floats). */
ffk_status ffk_mlp_set_norm(ffk_ctx* ctx, ffk_mlp* net, const float* mean_dev,
                            const float* inv_std_dev, void* stream);
/* out = net(X) for B rows of X (B x D row-major float32, already standardised).
 * prec = FFK_FP32 (FP32 MFMA) or FFK_BF16 (BF16 MFMA, FP32 accumulation). */
ffk_status ffk_mlp_forward(ffk_ctx* ctx, const ffk_mlp* net, const float* X_dev, int64_t B,
                           float* out_dev, ffk_precision prec, void* stream);
/* Mean squared error of net(X) against y (B floats) and its gradient (flat,
 * n_params floats) in FP32; loss_dev: 1 float. */
ffk_status ffk_mlp_grad(ffk_ctx* ctx, ffk_mlp* net, const float* X_dev, const float* y_dev,
                        int64_t B, float* loss_dev, float* grad_dev, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the gradient grad_dev. */
ffk_status ffk_mlp_adam_step(ffk_ctx* ctx, ffk_mlp* net, const float* grad_dev, float lr,
                             void* stream);
/* Per-geometry sampling weights for a system: exp(net(standardised X_g)) for
 * every geometry g (N floats64, > 0), with BF16 MFMA inference. */
ffk_status ffk_mlp_scores(ffk_ctx* ctx, const ffk_mlp* net, const ffk_system* sys,
                          double* scores_dev, void* stream);

/* Training-data helpers for the score network.
 * ffk_block_log_scores: per-geometry targets from column scores tau_dev
 *   (n = 3 M N float64): y_g = log(sum_{c in geometry g} tau_c) minus the mean
 *   over the N geometries, written to y_dev (N floats).
 * ffk_mlp_prepare_inputs: the system's descriptor rows as floats (N x D
 *   row-major) in X_dev, standardised with the network's mean / inverse std
 *   when `standardize` is 1, raw otherwise.
 * ffk_mlp_fit_norm: set the network's standardisation to the column mean and
 *   inverse standard deviation of the B raw rows X_dev (B x D floats). */
ffk_status ffk_block_log_scores(ffk_ctx* ctx, const double* tau_dev, int64_t N, int32_t M, float* y_dev,
                                void* stream);
ffk_status ffk_mlp_prepare_inputs(ffk_ctx* ctx, const ffk_mlp* net, const ffk_system* sys, float* X_dev,
                                  int32_t standardize, void* stream);
ffk_status ffk_mlp_fit_norm(ffk_ctx* ctx, ffk_mlp* net, const float* X_dev, int64_t B, void* stream);

/* ---- rule of thumb (section 4.3, Eq. 8) ---------------------------------- */

/* k_RoT = (k_min^m m n^2 / 2)^(1/(2+m)), rounded to the nearest integer in [1, n]. */
int64_t ffk_rule_of_thumb(int64_t n, double k_min, double m);

/* The rule of thumb with measured costs: the integer k in [1, n] that
 * minimises runtime(k) = n (k_min/k)^m (a + b k) + c k^2, i.e. the power-law
 * iteration count times a per-iteration cost a + b k (b prices the two passes
 * of the preconditioner apply over the n x k factor) plus a build cost c k^2.
 * Eq. 7 is the case a = n^2, b = 0, c = n, which returns k_RoT.  The model is
 * unimodal in k for m > 0; it is minimised by an integer ternary search.
 * Returns -1 for n < 1, k_min <= 0, m <= 0, a negative cost or a + b = 0. */
int64_t ffk_rule_of_thumb_calibrated(int64_t n, double k_min, double m, double a, double b, double c);

/* Fit of the power law #/n = (k_min / k)^m between the preconditioner size k
 * and the PCG iteration count # at kernel size n (section 4.3, the trade-off
 * behind Eq. 7): least squares of log(#/n) = m log k_min - m log k over
 * `count` measured pairs (k_host[i], iters_host[i]) in host memory.  Host
 * computation only (no device work, no context).  Returns FFK_ERR_ARG when
 * count < 2, n < 1, a k or an iteration count is < 1, all k are equal, or the
 * fitted m is not positive (iterations that do not fall with k); the outputs
 * are then left unchanged. */
ffk_status ffk_rot_fit(const int64_t* k_host, const int64_t* iters_host, int32_t count, int64_t n,
                       double* k_min_host, double* m_host);

#ifdef __cplusplus
}
#endif
#endif /* FFKRR_H */
