// Internal declarations shared by the translation units of libffkrr.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ffkrr.h"

namespace ffk {

// ---------------------------------------------------------------- errors ----
struct Error : std::runtime_error {
  ffk_status status;
  Error(ffk_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] inline void fail(ffk_status s, const std::string& msg) { throw Error(s, msg); }

inline void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e != hipSuccess) {
    char buf[512];
    snprintf(buf, sizeof(buf), "%s failed at %s:%d: %s", what, file, line, hipGetErrorString(e));
    fail(e == hipErrorOutOfMemory ? FFK_ERR_OOM : FFK_ERR_HIP, buf);
  }
}
#define HIPCHK(x) ::ffk::hip_check((x), #x, __FILE__, __LINE__)
#define LAUNCHCHK() ::ffk::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

inline void require(bool ok, const std::string& msg) {
  if (!ok) fail(FFK_ERR_ARG, msg);
}

// ------------------------------------------------------- device buffers ----
// Owning device allocation; released on destruction.
class DBuf {
 public:
  DBuf() = default;
  explicit DBuf(size_t bytes) { alloc(bytes); }
  ~DBuf() { release(); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p_ = o.p_; n_ = o.n_; o.p_ = nullptr; o.n_ = 0; }
    return *this;
  }
  void alloc(size_t bytes) {
    release();
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      char buf[160];
      snprintf(buf, sizeof(buf), "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
      fail(FFK_ERR_OOM, buf);
    }
    p_ = p;
    n_ = bytes;
  }
  // Grow to at least `bytes` (contents are not preserved).
  void ensure(size_t bytes) { if (n_ < bytes) alloc(bytes); }
  void release() {
    if (p_) (void)hipFree(p_);
    p_ = nullptr;
    n_ = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(p_); }
  void* get() const { return p_; }
  size_t bytes() const { return n_; }
  explicit operator bool() const { return p_ != nullptr; }

 private:
  void* p_ = nullptr;
  size_t n_ = 0;
};

// Pinned host staging buffer for small readbacks.
class HBuf {
 public:
  HBuf() = default;
  ~HBuf() { if (p_) (void)hipHostFree(p_); }
  HBuf(const HBuf&) = delete;
  HBuf& operator=(const HBuf&) = delete;
  void ensure(size_t bytes) {
    if (n_ >= bytes) return;
    if (p_) (void)hipHostFree(p_);
    p_ = nullptr;
    HIPCHK(hipHostMalloc(&p_, bytes, hipHostMallocDefault));
    n_ = bytes;
  }
  template <class T> T* as() const { return static_cast<T*>(p_); }

 private:
  void* p_ = nullptr;
  size_t n_ = 0;
};

inline int cdiv(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// ----------------------------------------------------------- bf16 helpers ----
typedef uint16_t bf16_t;   // raw storage of a bfloat16

__host__ __device__ inline bf16_t f2bf(float x) {
  // round to nearest even (inputs are finite here)
  uint32_t u;
  memcpy(&u, &x, 4);
  uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<bf16_t>(r >> 16);
}
__host__ __device__ inline float bf2f(bf16_t h) {
  uint32_t u = static_cast<uint32_t>(h) << 16;
  float x;
  memcpy(&x, &u, 4);
  return x;
}

// ------------------------------------------------------------- handles ----
}  // namespace ffk

struct ffk_ctx {
  int device = 0;
  std::string last_error;
  ffk::HBuf host_scratch;          // pinned readback area
};

namespace ffk {

// Coefficients of the kernel for one storage precision: dA = a(r) - a(0),
// B = b(r), as Nr x Nr row-major matrices (Nr = N rounded up to 128, zero
// padding).
struct CoeffSet {
  DBuf dA_hi, dA_lo;   // FP64: dA_hi holds double; FP32: float; BF16: hi (+lo for BF16X3)
  DBuf B;              // FP64: double, otherwise float
  bool ready = false;
};

// Per-precision MVM workspaces.
struct MvmWork {
  DBuf U64, UT64;      // J v as FP64: Nr x Dk and transposed Dr x Nr (zero padding)
  DBuf pd;             // N double      (x_c,j . u_j)
  DBuf s;              // D double      (column sums of U)
  DBuf spart;          // partials of s
  DBuf U32, UT32;      // the same in FP32
  DBuf Uh, Ul;         // Nr x Dk bf16 hi / lo
  DBuf UTh, UTl;       // Dr x Nr bf16 hi / lo
  DBuf Wn64;           // Nr x Nr double  (-W, zero padding)
  DBuf Wn32;           // Nr x Nr float
  DBuf Wnh, Wnl;       // Nr x Nr bf16
  DBuf wpart;          // N x tilesN double (row-sum partials of W)
  DBuf G;              // N x D double
  DBuf part;           // split-K partials of GEMM 2
};

}  // namespace ffk

namespace ffk {
// Fixed coefficients and workspaces of a rectangular product K(tgt, src)
// whose geometries do not change (a permuted copy of a symmetrized system,
// as the source, against the system itself); valid while tgt is the target.
struct RectCache {
  const ffk_system* tgt = nullptr;
  DBuf Xt, sqt, dA, B, Wn, U, pd, sv, cpart, wpart, G, part;
};
}  // namespace ffk

struct ffk_system {
  ffk_ctx* ctx = nullptr;
  int64_t N = 0;
  int32_t M = 0;
  int64_t D = 0;
  int64_t n = 0;
  double sigma = 10.0;
  double a0 = 0.0;          // a(0) = 5/(3 sigma^2)
  double bcoef = 0.0;       // 25/(3 sigma^4)
  ffk::DBuf R;              // N x M x 3 double
  ffk::DBuf pairs;          // D int32: (p << 16) | q
  ffk::DBuf X;              // N x D double (uncentred)
  ffk::DBuf xmean;          // D double
  ffk::DBuf Xc;             // N x D double (centred)
  ffk::DBuf sqn;            // N double (|x_c|^2)
  ffk::DBuf Xp64, XpT64;    // X_c as FP64, padded: Nr x Dk and transposed Dr x Nr
  ffk::DBuf Xp32, XpT32;    // the same in FP32
  ffk::DBuf Xch, Xcl;       // N x D bf16 hi/lo
  ffk::DBuf XcTh, XcTl;     // D x N bf16 hi/lo
  ffk::CoeffSet coef[4];    // indexed by ffk_precision
  ffk::MvmWork work;
  double max_diag = -1.0;   // max diag(K), computed on demand
  // Symmetrized kernel (sum over a group of atom permutations p_q): the
  // systems of the permuted geometries P_q R, the permutations (S x M) and
  // their inverses on the device, and a work vector.  Empty: the plain kernel.
  std::vector<std::unique_ptr<ffk_system>> sym;
  std::vector<int32_t> sym_perm_host;
  ffk::DBuf sym_perm, sym_pinv;
  ffk::DBuf sym_work;
  int sym_identity = 0;     // index of the identity in the group
  ffk::RectCache rect;      // used when this system is a permuted copy
  // The symmetrized product as one rectangular product against the stacked
  // permuted copies: sources P_1 R, ..., P_S R (N S geometries, descriptors
  // centred with this system's mean), N x N S coefficient sets, the
  // product's workspace for that shape and the stacked permuted vector.
  std::unique_ptr<ffk_system> stack;
  ffk::CoeffSet stack_coef[4];
  ffk::MvmWork stack_work;
  ffk::DBuf stack_v;
};

struct ffk_precond {
  ffk_ctx* ctx = nullptr;
  int64_t n = 0, k = 0, k_eff = 0;
  int64_t ld = 0, ldf = 0;  // leading dimensions of L and Finv (multiples of 64)
  double lambda = 0.0;
  int32_t store = FFK_FP64;
  ffk::DBuf L;              // n x k column-major (double or float)
  ffk::DBuf Finv;           // k x k column-major lower-triangular inverse of F = chol(core)
  ffk::DBuf FinvT;          // its transpose (upper triangle), same layout
  ffk::DBuf y, t1, t;       // k-vectors
  ffk::DBuf work;           // partial sums of the split GEMVs
  int64_t bytes = 0;
  // Matrix-free form (L not stored): L = K[:, S] T^T with T = L_SS^-1, the
  // inverse of the factor's rows at the kept pivots S; the apply runs two
  // FP64 kernel products on `sys` instead of the two passes over L.
  bool matrix_free = false;
  ffk_system* sys = nullptr;  // not owned; must outlive the preconditioner
  ffk::DBuf sel;            // k_eff int64: the kept pivots, in factor order
  ffk::DBuf Tinv, TinvT;    // T (k x k lower, column-major, ldf) and its transpose
  ffk::DBuf q, u;           // n-vectors: K r, then the scattered T^T t and K of it
};

struct ffk_mlp {
  ffk_ctx* ctx = nullptr;
  int32_t D = 0, H = 0;
  int64_t nparam = 0;
  ffk::DBuf theta;          // params, then mean (D), inv_std (D), out offset/scale (2)
  ffk::DBuf m, v;           // Adam moments
  int64_t t = 0;            // Adam step count
  ffk::DBuf work;           // activations and temporaries
  ffk::DBuf wbf;            // bf16 copies of W1, W2 for inference
  bool wbf_valid = false;
};

namespace ffk {

// ---------------------------------------------------- internal interfaces ----
// descriptor.hip
void descriptor_build(ffk_system* sys, const double* R, hipStream_t st, bool coefficients = true);
// symmetry.hip -- the kernel symmetrized over a group of atom permutations
void set_symmetries(ffk_system* sys, const int32_t* perms_host, int S, hipStream_t st);
void sym_columns(const ffk_system* s, const int64_t* cols, int64_t k, double* out, int64_t ldo, double shift,
                 hipStream_t st);
void sym_diag(const ffk_system* s, double* d, hipStream_t st);
// columns.hip -- columns of K(s, src) in the numbering of src (targets from s)
void kernel_columns_src(const ffk_system* s, const ffk_system* src, const int64_t* cols, int64_t k, double* out,
                        int64_t ldo, double shift, bool accumulate, hipStream_t st);
// mvm.hip -- y (+)= K(tgt, src) alpha on the FP64 engine; with shift_v, the
// first (non-accumulating) pass also adds shift * shift_v
void rect_mvm(const ffk_system* src, const ffk_system* tgt, const double* alpha, double* y, bool accumulate,
              const double* shift_v, double shift, RectCache* cache, hipStream_t st);
void permute_atoms(const double* a, const int32_t* p, int64_t N, int M, double* out, hipStream_t st);
void ensure_coeffs(ffk_system* sys, int prec, hipStream_t st);
// Coefficient sets of K(t, src) (rows t->N, columns src->N, padded); both
// descriptors must be centred with one mean.  The pair (i, i + diag_off) is
// at distance zero (the source is the target itself).
void ensure_coeffs_pair(const ffk_system* t, const ffk_system* src, CoeffSet* sets, int prec, int64_t diag_off,
                        hipStream_t st);
void ensure_lowp_descriptor(ffk_system* sys, int prec, hipStream_t st);
// Re-centre a system's descriptor with another mean (X_c = X - mean, |x_c|^2).
void center_with(ffk_system* sys, const double* mean, hipStream_t st);

// fused.hip -- the product's two dense steps in one kernel (BF16, D <= 128)
// Operands of the fused product (layouts as in the two-GEMM form).
struct FusedArgs {
  const bf16_t *Uh, *Ul;     // U = J v: fragment-major, rows = sources (Nsr), K = d (KTd tiles)
  const bf16_t *Xh, *Xl;     // X_c of the targets: fragment-major, rows = targets (Ntr), K = d
  // [U^T | X_c^T] interleaved: fragment-major, rows = d, K = 2 Nsr (2 KTs
  // tiles); source j at K index 8 (j / 4) + j % 4 (U) and that + 4 (X_c)
  const bf16_t *Vh, *Vl;
  const void* CF;            // coefficient blocks (fused_coef_build): 2 KB per 16 targets x 16 sources
  const double* pd;          // pd_j = x_c,j . u_j, Nsr entries (zero past the sources)
  float* part;               // splits x Nt x D partial G rows
  double* wpart;             // Nt x splits partial row sums of W
  int64_t KTd, KTs, Nsr;
  int Nt, D, nchunks, splits;
};
constexpr int64_t kFusedMaxD = 128;
// Where the fused form was measured faster than the two GEMMs (MI355X, split
// BF16): D <= 96 at every size, and 96 < D <= 128 up to Nt Ns = 4096^2 (at
// D = 120, N = 10000: 733 us fused against 676).  One rule for BF16 and split
// BF16, which share the J v workspace and so its layout.
inline bool use_fused(int prec, int64_t D, int64_t Nt, int64_t Ns) {
  if (prec != FFK_BF16 && prec != FFK_BF16X3) return false;
  return D <= 96 || (D <= kFusedMaxD && Nt * Ns <= (int64_t)4096 * 4096);
}
int fused_splits(int64_t Nt, int64_t Ns, int64_t D, int max_splits);
void fused_mvm_launch(const FusedArgs& a, bool x3, hipStream_t st);
// The X_c^T slots of the interleaved operand (split BF16) from the sources'
// centred descriptor; zero past Ns and D.
// The coefficient blocks of the fused product (Ntr x Nsr x 8 bytes) from the
// FP64 dA and B (rows Nt, columns Ns, leading dimension ld).
void fused_coef_build(const double* dA, const double* B, int64_t Nt, int64_t Ns, int64_t ld, int64_t Ntr,
                      int64_t Nsr, void* out, hipStream_t st);
void fused_fill_x(const double* Xc, int64_t Ns, int64_t D, int64_t Dr, int64_t Nsr, bf16_t* Vh, bf16_t* Vl,
                  hipStream_t st);

// mvm.hip
void kernel_mvm(ffk_system* sys, const double* v, double* y, double shift, int prec, hipStream_t st);
int kernel_mvm_vy(ffk_system* sys, const double* v, double* y, double shift, int prec, hipStream_t st,
                  double* vy_part);
void kernel_mvm_phases(ffk_system* sys, const double* v, double* y, double shift, int prec, int iters,
                       double* ms, hipStream_t st);
void kernel_predict(const ffk_system* train, const ffk_system* test, const double* alpha,
                    double* F, hipStream_t st);
// The product with its workspace carved from the device memory [base, base +
// cap) instead of the system's own: allocates nothing.  The system's
// coefficients and descriptor copies for prec must already exist.
void kernel_mvm_scratch(ffk_system* sys, const double* v, double* y, double shift, int prec, hipStream_t st,
                        void* base, size_t cap);
// noalloc.hip -- the library's fixed scratch array on each device
constexpr size_t kScratchBytes = (size_t)128 << 20;
void scratch_init(int device);        // once per device, with that device current
void* scratch_ptr(int device);        // nullptr before scratch_init

// columns.hip
// out[:, c] = K[:, cols[c]] + shift * e_{cols[c]}, column-major with leading dimension ldo.
void kernel_columns(const ffk_system* sys, const int64_t* cols, int64_t k, double* out,
                    int64_t ldo, double shift, hipStream_t st);
void kernel_diag(const ffk_system* sys, double* d, hipStream_t st);
double max_diag(ffk_system* sys, hipStream_t st);

// dense.hip : FP64 GEMM (C = alpha A B^T + beta C on strided views) and factorizations
struct View64 {
  const double* p;
  int64_t s0, s1;   // element (i, j) at p[i * s0 + j * s1]
};
void gemm64(int M, int N, int K, double alpha, View64 A, View64 B, double beta, double* C,
            int64_t scm, int64_t scn, bool lower_only, hipStream_t st);
// The same product with FP32 operands, FP64 arithmetic and output.
struct View32 {
  const float* p;
  int64_t s0, s1;
};
void gemm64_in32(int M, int N, int K, double alpha, View32 A, View32 B, double beta, double* C, int64_t scm,
                 int64_t scn, hipStream_t st);
// Lower Cholesky in place of the n x n column-major matrix A (lda). Returns the
// index of the first failing pivot or -1.
int64_t potrf_lower(double* A, int64_t n, int64_t lda, hipStream_t st);
// In-place inverse of the lower-triangular n x n column-major matrix A.
void trtri_lower(double* A, int64_t n, int64_t lda, hipStream_t st);

// reduce.hip -- deterministic two-stage reductions; `part` holds >= kRedParts doubles.
constexpr int kRedParts = 1024;
void dot64(const double* a, const double* b, int64_t n, double* part, double* out_dev, hipStream_t st);
// The first stage of dot64 alone: block partials into part; returns their count.
int dot64_parts(const double* a, const double* b, int64_t n, double* part, hipStream_t st);
void reduce_max64(const double* a, int64_t n, double* part, double* out_dev, hipStream_t st);
// Kernels that fuse a dot product into an elementwise pass run fused_parts(n)
// blocks of 256 lanes over a grid-stride loop, reduce each block with
// block_sum256 into part[block], and finish with sum_parts64 (fixed order).
int fused_parts(int64_t n);
void sum_parts64(const double* part, int np, double* out_dev, hipStream_t st);
__device__ inline double block_sum256(double v, double* sh /* 256 doubles of LDS */) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  return sh[0];
}
// Fixed-order total of part[0..np) by one block of 256 lanes, returned to
// every lane: the order of the second stage of dot64, so a kernel that needs
// the total can form it itself instead of waiting for a separate launch.
__device__ inline double sum_parts_block(const double* part, int np, double* sh) {
  double acc = 0.0;
  for (int e = threadIdx.x; e < np; e += 256) acc += part[e];
  return block_sum256(acc, sh);
}

// select.hip
void select_uniform(const ffk_system* sys, int64_t k, uint64_t seed, int64_t* idx, hipStream_t st);
void select_weighted(int64_t n, const double* w, int64_t k, uint64_t seed, int stream_id,
                     int64_t* idx, hipStream_t st);
int64_t select_pivchol(ffk_system* sys, int64_t k, int64_t* idx, hipStream_t st);
void leverage_estimate(ffk_system* sys, const int64_t* pilot, int64_t s, double lambda,
                       double* tau, hipStream_t st);

// precond.hip
// Incomplete Cholesky with pivots forced to idx (order kept) of K + shift I.
// L: n x k column-major double with leading dimension ld (>= n, zero padded).
// kept (host, k) receives which columns survived.
int64_t icd_forced(ffk_system* sys, const int64_t* idx, int64_t k, double shift, double* L, int64_t ld,
                   std::vector<char>* kept, hipStream_t st);
// lowmem: build L straight into FP32 storage (one FP64 panel at a time) instead
// of an FP64 factor that is rounded afterwards; chosen automatically when the
// FP64 factor would not fit next to its FP32 copy.
ffk_precond* precond_build(ffk_system* sys, const int64_t* idx, int64_t k, double lambda,
                           int store, bool lowmem, bool* dropped, hipStream_t st, bool matrix_free = false);
void precond_apply(const ffk_precond* P, const double* r, double* z, hipStream_t st);
// z = M^-1 r and the block partials of r^T z in part (kRedParts doubles);
// returns the number of partials (fixed order; sum them with sum_parts64 or
// sum_parts_block)
int precond_apply_parts(const ffk_precond* P, const double* r, double* z, double* part, hipStream_t st);

// pcg.hip
ffk_status pcg_solve(ffk_system* sys, const ffk_precond* P, const double* F, double* alpha,
                     const ffk_pcg_opts* o, ffk_pcg_report* rep, hipStream_t st);

// rls.hip
void exact_rls(ffk_system* sys, double lambda, double* tau, hipStream_t st);

// mlp.hip
ffk_mlp* mlp_create(int32_t D, int32_t H, uint64_t seed);
void mlp_forward(const ffk_mlp* net, const float* X, int64_t B, float* out, int prec, hipStream_t st);
void mlp_grad(ffk_mlp* net, const float* X, const float* y, int64_t B, float* loss, float* grad,
              hipStream_t st);
void mlp_adam(ffk_mlp* net, const float* grad, float lr, hipStream_t st);
void mlp_scores(const ffk_mlp* net, const ffk_system* sys, double* scores, hipStream_t st);
void mlp_prepare_inputs(const ffk_mlp* net, const ffk_system* s, float* out, int standardize, hipStream_t st);
void mlp_fit_norm(ffk_mlp* net, const float* X, int64_t B, hipStream_t st);
void block_log_scores(const double* tau, int64_t N, int M, float* y, hipStream_t st);

// Row padding of the product's N- and D-sized operands: a multiple of every
// GEMM tile edge, so tiles never read past an array.
constexpr int64_t kRowPad = 256;
inline int64_t pad_rows(int64_t n) { return (n + kRowPad - 1) / kRowPad * kRowPad; }

// Fragment-major layout of the BF16 GEMM operands.  An operand with rows
// padded to 16 and K padded to 32 is stored as 1 KB blocks, one per (16-row
// group, 32-wide K tile), blocks of a row group consecutive in K; inside a
// block, the 16 bytes at offset 16 L hold row L % 16, K elements
// 8 (L / 16) .. +7 -- exactly what lane L of a 16x16x32 MFMA reads.  One
// contiguous 1 KB load per block then fills LDS in fragment order.
__host__ __device__ inline int64_t frag_off(int64_t row, int64_t k, int64_t KT) {
  return ((((row >> 4) * KT + (k >> 5)) << 9) | ((((k & 31) >> 3) << 4 | (row & 15)) << 3) | (k & 7));
}

// clock.cpp -- per-kernel event clocks (ids match ffk_clock in ffkrr.h)
enum ClockId {
  CLK_JV = 0, CLK_COLSUM, CLK_GEMM1, CLK_GEMM2, CLK_GEMM2_REDUCE, CLK_JTG,
  CLK_GEMV_T, CLK_GEMV_N, CLK_CORE, CLK_FUSED, CLK_COUNT
};
void clk_begin(int id, hipStream_t st);
void clk_end(int id, hipStream_t st);
// While one exists on a thread, the clocks record nothing there.
struct ClockPause {
  ClockPause();
  ~ClockPause();
};
void clock_enable(int stride);
void clock_read(int id, double* total_ms, int64_t* launches);

// rng shared by host and device code of the library
__host__ __device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline double uniform01_at(uint64_t seed, uint64_t stream, uint64_t i) {
  uint64_t z = splitmix64_at(seed, (stream << 40) + i);
  return static_cast<double>((z >> 11) + 1ull) * 0x1.0p-53;
}

}  // namespace ffk
