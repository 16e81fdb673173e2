// The force-field kernel symmetrized over a group S of atom permutations, the
// sGDML form behind the paper's kernels (section 2.1):
//   k_S(R, R') = sum_q k(x(R), x(P_q R')),   (P_q R)_a = R_{p_q(a)},
// whose force-kernel block is the mixed second derivative
//   K_S,ij = sum_q J(R_i)^T H(x(R_i), x(P_q R_j)) J(P_q R_j) Pi_q,
// with Pi_q the coordinate permutation (Pi_q v)_(a,t) = v_(p_q(a),t).
// Every part is a sum over q of the plain kernel against the system of the
// permuted geometries P_q R (kept in sys->sym):
//   product   K_S v      = sum_q K(R, P_q R) (Pi_q v)                (FP64)
//   column    K_S[:, c]  = sum_q K(R, P_q R)[:, (g, p_q^-1(a), t)]   for c = (g, a, t)
//   diagonal  K_S[c, c]  = sum_q K(R, P_q R)[c, (g, p_q^-1(a), t)]
// so selection, the preconditioner and PCG, which go through these, use the
// symmetrized kernel.  Cost: |S| plain evaluations each.
#include <algorithm>
#include <set>

#include "common.hpp"

namespace ffk {

// out[g][a][t] = a_in[g][p[a]][t] for N geometries of M atoms: P R for
// coordinates, Pi v for coordinate vectors
__global__ void k_permute_atoms(const double* __restrict__ a, const int32_t* __restrict__ p, int64_t N, int M,
                                double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * M * 3) return;
  const int64_t g = e / (3 * M);
  const int loc = (int)(e % (3 * M));
  out[e] = a[g * 3 * M + 3 * p[loc / 3] + loc % 3];
}

void permute_atoms(const double* a, const int32_t* p, int64_t N, int M, double* out, hipStream_t st) {
  k_permute_atoms<<<cdiv(N * M * 3, 256), 256, 0, st>>>(a, p, N, M, out);
  LAUNCHCHK();
}

// column c = (g, a, t) -> (g, pinv[a], t)
__global__ void k_map_cols(const int64_t* __restrict__ cols, int64_t k, const int32_t* __restrict__ pinv, int M,
                           int64_t* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k) return;
  const int64_t c = cols[e], m3 = 3 * M;
  const int loc = (int)(c % m3);
  out[e] = (c / m3) * m3 + 3 * pinv[loc / 3] + loc % 3;
}

__device__ inline int sym_pair(int a, int b) { return a > b ? a * (a - 1) / 2 + b : b * (b - 1) / 2 + a; }

// d[c] (+)= K(R, P R)[c, (g, pinv[a], t)] for every c = (g, a, t): one block
// per geometry g, with Rt/Xt its target geometry and descriptor, Rs/Xs those
// of the permuted copy (uncentred descriptors)
__global__ __launch_bounds__(128) void k_sym_diag(const double* __restrict__ Rt, const double* __restrict__ Xt,
                                                  const double* __restrict__ Rs, const double* __restrict__ Xs,
                                                  const int32_t* __restrict__ pinv, int M, int64_t D,
                                                  double inv_len, double a0, double bcoef, int accumulate,
                                                  double* __restrict__ d) {
  extern __shared__ double sm[];
  double* sd = sm;                // D: x_t - x_s
  double* srt = sd + D;           // 3M target coordinates
  double* srs = srt + 3 * M;      // 3M source coordinates
  __shared__ double red[2];
  const int64_t g = blockIdx.x;
  const int m3 = 3 * M;
  double r2 = 0.0;
  for (int64_t e = threadIdx.x; e < D; e += blockDim.x) {
    const double v = Xt[g * D + e] - Xs[g * D + e];
    sd[e] = v;
    r2 += v * v;
  }
  for (int e = threadIdx.x; e < m3; e += blockDim.x) {
    srt[e] = Rt[g * m3 + e];
    srs[e] = Rs[g * m3 + e];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) r2 += __shfl_xor(r2, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r2;
  __syncthreads();
  r2 = red[0] + (blockDim.x > 64 ? red[1] : 0.0);
  const double z = sqrt(r2) * inv_len;
  const double ez = exp(-z);
  const double A = a0 * (1.0 + z) * ez;
  for (int e = threadIdx.x; e < m3; e += blockDim.x) {
    const int a = e / 3, t = e % 3, ap = pinv[a];
    // u = J(P R) e_(ap, t): on the pairs {ap, b}, u_b = -(Rs_ap - Rs_b)_t / r^3
    auto u_of = [&](int b) {
      const double dx = srs[3 * ap] - srs[3 * b], dy = srs[3 * ap + 1] - srs[3 * b + 1],
                   dz = srs[3 * ap + 2] - srs[3 * b + 2];
      const double ir = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
      return -(t == 0 ? dx : (t == 1 ? dy : dz)) * ir * ir * ir;
    };
    double du = 0.0;
    for (int b = 0; b < M; ++b)
      if (b != ap) du += sd[sym_pair(ap, b)] * u_of(b);
    const double bdu = -bcoef * ez * du;
    const double ua = (a != ap) ? u_of(a) : 0.0;   // u on the pair {ap, a}
    // (J(R)^T h)_(a,t) = -sum_{b != a} h_{ab} (Rt_a - Rt_b)_t / r^3 with h = A u + bdu d
    double v = 0.0;
    for (int b = 0; b < M; ++b) {
      if (b == a) continue;
      const double ue = (a == ap) ? u_of(b) : (b == ap ? ua : 0.0);
      const double h = A * ue + bdu * sd[sym_pair(a, b)];
      const double dx = srt[3 * a] - srt[3 * b], dy = srt[3 * a + 1] - srt[3 * b + 1],
                   dz = srt[3 * a + 2] - srt[3 * b + 2];
      const double ir = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
      v -= h * (t == 0 ? dx : (t == 1 ? dy : dz)) * ir * ir * ir;
    }
    double* o = d + g * m3 + e;
    if (accumulate) *o += v;
    else *o = v;
  }
}

void set_symmetries(ffk_system* s, const int32_t* perms, int S, hipStream_t st) {
  const int M = s->M;
  require(perms != nullptr && S >= 1, "set_symmetries: need at least one permutation");
  std::set<std::vector<int32_t>> rows;
  std::vector<int32_t> ident(M);
  for (int a = 0; a < M; ++a) ident[a] = a;
  int identity = -1;
  for (int q = 0; q < S; ++q) {
    std::vector<int32_t> p(perms + (int64_t)q * M, perms + (int64_t)(q + 1) * M);
    std::vector<int32_t> sorted = p;
    std::sort(sorted.begin(), sorted.end());
    require(sorted == ident, "set_symmetries: a row is not a permutation of 0 .. M-1");
    require(rows.insert(p).second, "set_symmetries: a permutation is repeated");
    if (p == ident) identity = q;
  }
  require(identity >= 0, "set_symmetries: the identity is missing (the rows must form a group)");
  for (const auto& p : rows)
    for (const auto& q : rows) {
      std::vector<int32_t> c(M);
      for (int a = 0; a < M; ++a) c[a] = p[q[a]];
      require(rows.count(c) == 1, "set_symmetries: the rows are not closed under composition (not a group)");
    }
  s->sym.clear();
  s->sym_perm_host.clear();
  s->max_diag = -1.0;
  s->stack.reset();
  for (auto& c : s->stack_coef) c = CoeffSet();
  s->stack_work = MvmWork();
  s->stack_v.release();
  if (S == 1) return;   // the trivial group: the plain kernel
  std::vector<int32_t> pinv((size_t)S * M);
  for (int q = 0; q < S; ++q)
    for (int a = 0; a < M; ++a) pinv[(size_t)q * M + perms[(int64_t)q * M + a]] = a;
  s->sym_perm.alloc((size_t)S * M * sizeof(int32_t));
  s->sym_pinv.alloc((size_t)S * M * sizeof(int32_t));
  HIPCHK(hipMemcpyAsync(s->sym_perm.get(), perms, (size_t)S * M * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s->sym_pinv.get(), pinv.data(), (size_t)S * M * sizeof(int32_t), hipMemcpyHostToDevice, st));
  DBuf Rq(s->N * M * 3 * 8);
  for (int q = 0; q < S; ++q) {
    std::unique_ptr<ffk_system> c(new ffk_system());
    c->ctx = s->ctx;
    c->N = s->N;
    c->M = M;
    c->D = s->D;
    c->n = s->n;
    c->sigma = s->sigma;
    c->a0 = s->a0;
    c->bcoef = s->bcoef;
    permute_atoms(s->R.as<double>(), s->sym_perm.as<int32_t>() + (size_t)q * M, s->N, M, Rq.as<double>(), st);
    descriptor_build(c.get(), Rq.as<double>(), st, false);
    s->sym.push_back(std::move(c));
  }
  s->sym_perm_host.assign(perms, perms + (size_t)S * M);
  s->sym_identity = identity;
  s->sym_work.alloc(s->n * 8);
  // the product's sources: the S permuted copies stacked, their descriptors
  // centred with this system's mean (the kernel sees only differences)
  std::unique_ptr<ffk_system> stk(new ffk_system());
  stk->ctx = s->ctx;
  stk->N = s->N * S;
  stk->M = M;
  stk->D = s->D;
  stk->n = s->n * S;
  stk->sigma = s->sigma;
  stk->a0 = s->a0;
  stk->bcoef = s->bcoef;
  DBuf Rs((size_t)S * s->N * M * 3 * 8);
  for (int q = 0; q < S; ++q)
    HIPCHK(hipMemcpyAsync(Rs.as<double>() + (size_t)q * s->N * M * 3, s->sym[q]->R.get(), (size_t)s->N * M * 3 * 8,
                          hipMemcpyDeviceToDevice, st));
  descriptor_build(stk.get(), Rs.as<double>(), st, false);
  center_with(stk.get(), s->xmean.as<double>(), st);
  s->stack = std::move(stk);
  HIPCHK(hipStreamSynchronize(st));
}

void sym_columns(const ffk_system* s, const int64_t* cols, int64_t k, double* out, int64_t ldo, double shift,
                 hipStream_t st) {
  if (k <= 0) return;
  const int M = s->M;
  // the mapped column indices go to the system's work vector (k <= n), in
  // chunks so that a chunk's passes finish before the next chunk is mapped
  int64_t* cq = s->sym_work.as<int64_t>();
  for (int64_t c0 = 0; c0 < k; c0 += s->n) {
    const int64_t kc = std::min<int64_t>(s->n, k - c0);
    for (size_t q = 0; q < s->sym.size(); ++q) {
      k_map_cols<<<cdiv(kc, 256), 256, 0, st>>>(cols + c0, kc, s->sym_pinv.as<int32_t>() + q * M, M, cq);
      LAUNCHCHK();
      // the shift sits on the diagonal, which the identity's pass reaches with unmapped columns
      kernel_columns_src(s, s->sym[q].get(), cq, kc, out + c0 * ldo, ldo, (int)q == s->sym_identity ? shift : 0.0,
                         q > 0, st);
    }
  }
}

void sym_diag(const ffk_system* s, double* d, hipStream_t st) {
  const int M = s->M;
  const int64_t D = s->D;
  const size_t shm = (size_t)(D + 6 * M) * sizeof(double);
  for (size_t q = 0; q < s->sym.size(); ++q) {
    const ffk_system* c = s->sym[q].get();
    k_sym_diag<<<(unsigned)s->N, 128, shm, st>>>(s->R.as<double>(), s->X.as<double>(), c->R.as<double>(),
                                                 c->X.as<double>(), s->sym_pinv.as<int32_t>() + q * M, M, D,
                                                 sqrt(5.0) / s->sigma, s->a0, s->bcoef, q > 0 ? 1 : 0, d);
    LAUNCHCHK();
  }
}

}  // namespace ffk
