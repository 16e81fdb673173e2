// Single kernel columns K[:, c] and the diagonal diag(K) -- the get_col(i) and
// d := diag(K) inputs of the incomplete Cholesky (appendix, Algorithm 1).
//
// Column c = 3 M g + 3 p + t belongs to source geometry g, atom p, coordinate t.
// Its descriptor image u = J_g e_c is non-zero only on the M-1 pairs {p, b}:
//   u_{pb} = -(R_gp - R_gb)_t / r_gpb^3.
// For each target geometry i, with d = x_i - x_g and (a, b) the Matern-5/2
// Hessian coefficients at r = |d|,
//   K[i-block, c] = J_i^T (a u + b (d . u) d) = a J_i^T u + b (d . u) J_i^T d,
// where (J_i^T h)_q = -sum_{b != q} h_{qb} (R_iq - R_ib) / r_iqb^3.
// One wave handles one (target, column) pair; a block of 4 waves shares the
// target's geometry factors in LDS and walks a chunk of columns.
#include "common.hpp"

namespace ffk {

#define COLS_PER_BLOCK 64

__device__ inline int pair_of(int a, int b) { return a > b ? a * (a - 1) / 2 + b : b * (b - 1) / 2 + a; }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Targets (rows) come from R, X; the source geometry of each column from
// Rs, Xs (the same arrays for a plain kernel, a permuted copy for a
// symmetrized one).  With accumulate the values are added to out.
__global__ __launch_bounds__(256) void k_columns(const double* __restrict__ R, const double* __restrict__ X,
                                                 const double* __restrict__ Rs, const double* __restrict__ Xs,
                                                 const int* __restrict__ pairs, int M, int64_t D,
                                                 const int64_t* __restrict__ cols, int64_t k,
                                                 double* __restrict__ out, int64_t ldo, double shift,
                                                 double inv_len, double a0, double bcoef, int accumulate) {
  extern __shared__ double sm[];
  const int nw = blockDim.x >> 6;   // waves per block (1, 2 or 4)
  double* sRi = sm;                 // 3M
  double* sWi = sRi + 3 * M;        // 3D: (R_ia - R_ib)/r^3 for pair (a > b)
  double* sD = sWi + 3 * D;         // nw waves x D
  double* sU = sD + nw * D;         // nw waves x M
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m3 = 3 * M;
  const double* Xi = X + i * D;
  for (int e = threadIdx.x; e < m3; e += blockDim.x) sRi[e] = R[i * m3 + e];
  __syncthreads();
  for (int64_t e = threadIdx.x; e < D; e += blockDim.x) {
    const int pq = pairs[e];
    const int a = pq >> 16, b = pq & 0xFFFF;
    const double dx = sRi[3 * a] - sRi[3 * b], dy = sRi[3 * a + 1] - sRi[3 * b + 1], dz = sRi[3 * a + 2] - sRi[3 * b + 2];
    const double ir = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    const double ir3 = ir * ir * ir;
    sWi[3 * e] = dx * ir3;
    sWi[3 * e + 1] = dy * ir3;
    sWi[3 * e + 2] = dz * ir3;
  }
  __syncthreads();
  double* dW = sD + wave * D;
  double* uW = sU + wave * M;
  const int64_t c0 = (int64_t)blockIdx.y * COLS_PER_BLOCK;
  // uniform trip count so that the block barriers below are reached by all waves
  for (int it = 0; it < COLS_PER_BLOCK / nw; ++it) {
    const int64_t cidx = c0 + it * nw + wave;
    const bool active = cidx < k;
    int64_t col = 0, g = 0;
    int p = 0, t = 0;
    double r2 = 0.0;
    if (active) {
      col = cols[cidx];
      g = col / m3;
      const int loc = (int)(col % m3);
      p = loc / 3;
      t = loc % 3;
      for (int64_t e = lane; e < D; e += 64) {      // d = x_i - x_g and |d|^2
        const double dd = Xi[e] - Xs[g * D + e];
        dW[e] = dd;
        r2 += dd * dd;
      }
      r2 = wave_sum(r2);
      const double* Rg = Rs + g * m3;
      for (int b = lane; b < M; b += 64) {          // u on the pairs {p, b}
        double u = 0.0;
        if (b != p) {
          const double dx = Rg[3 * p] - Rg[3 * b], dy = Rg[3 * p + 1] - Rg[3 * b + 1],
                       dz = Rg[3 * p + 2] - Rg[3 * b + 2];
          const double ir = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
          const double comp = t == 0 ? dx : (t == 1 ? dy : dz);
          u = -comp * ir * ir * ir;
        }
        uW[b] = u;
      }
    }
    __syncthreads();
    if (active) {
      double du = 0.0;
      for (int b = lane; b < M; b += 64)
        if (b != p) du += dW[pair_of(p, b)] * uW[b];
      du = wave_sum(du);
      const double z = sqrt(r2) * inv_len;
      const double ez = exp(-z);
      const double a = a0 * (1.0 + z) * ez;
      const double bdu = -bcoef * ez * du;
      for (int q = lane; q < M; q += 64) {
        double jx = 0.0, jy = 0.0, jz = 0.0;   // (J_i^T d)_q
        double ux = 0.0, uy = 0.0, uz = 0.0;   // (J_i^T u)_q
        for (int b = 0; b < M; ++b) {
          if (b == q) continue;
          const int e = pair_of(q, b);
          const double sgn = q > b ? 1.0 : -1.0;   // sWi holds (R_larger - R_smaller)/r^3
          const double wx = sgn * sWi[3 * e], wy = sgn * sWi[3 * e + 1], wz = sgn * sWi[3 * e + 2];
          const double de = dW[e];
          jx -= de * wx;
          jy -= de * wy;
          jz -= de * wz;
          const double ue = (q == p) ? uW[b] : (b == p ? uW[q] : 0.0);
          ux -= ue * wx;
          uy -= ue * wy;
          uz -= ue * wz;
        }
        const int64_t row = i * m3 + 3 * q;
        double* o = out + cidx * ldo + row;
        const double v0 = a * ux + bdu * jx + (row == col ? shift : 0.0);
        const double v1 = a * uy + bdu * jy + (row + 1 == col ? shift : 0.0);
        const double v2 = a * uz + bdu * jz + (row + 2 == col ? shift : 0.0);
        if (accumulate) {
          o[0] += v0;
          o[1] += v1;
          o[2] += v2;
        } else {
          o[0] = v0;
          o[1] = v1;
          o[2] = v2;
        }
      }
    }
    __syncthreads();
  }
}

// Columns of K(s, src) in the source numbering (src = s for the plain kernel).
void kernel_columns_src(const ffk_system* s, const ffk_system* src, const int64_t* cols, int64_t k, double* out,
                        int64_t ldo, double shift, bool accumulate, hipStream_t st) {
  if (k <= 0) return;
  const int M = s->M;
  const int64_t D = s->D;
  static int max_lds = 0;
  if (max_lds == 0) {
    int dv = 0;
    HIPCHK(hipGetDevice(&dv));
    HIPCHK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dv));
  }
  int nw = 4;
  auto bytes = [&](int w) { return (size_t)(3 * M + 3 * D + w * (D + M)) * sizeof(double); };
  while (nw > 1 && bytes(nw) > (size_t)max_lds) nw >>= 1;
  if (bytes(nw) > (size_t)max_lds) fail(FFK_ERR_ARG, "kernel_columns: descriptor too large for the LDS staging");
  const int64_t per_launch = (int64_t)65535 * COLS_PER_BLOCK;
  for (int64_t c0 = 0; c0 < k; c0 += per_launch) {
    const int64_t kc = std::min(per_launch, k - c0);
    dim3 grid((unsigned)s->N, (unsigned)cdiv(kc, COLS_PER_BLOCK));
    k_columns<<<grid, 64 * nw, bytes(nw), st>>>(s->R.as<double>(), s->X.as<double>(), src->R.as<double>(),
                                                src->X.as<double>(), s->pairs.as<int>(), M, D, cols + c0, kc,
                                                out + c0 * ldo, ldo, shift, sqrt(5.0) / s->sigma, s->a0, s->bcoef,
                                                accumulate ? 1 : 0);
    LAUNCHCHK();
  }
}

void kernel_columns(const ffk_system* s, const int64_t* cols, int64_t k, double* out, int64_t ldo, double shift,
                    hipStream_t st) {
  if (!s->sym.empty()) sym_columns(s, cols, k, out, ldo, shift, st);
  else kernel_columns_src(s, s, cols, k, out, ldo, shift, false, st);
}

// diag(K)_{3Mg + 3p + t} = a(0) sum_{b != p} ((R_gp - R_gb)_t / r^3)^2
__global__ void k_diag(const double* __restrict__ R, int64_t N, int M, double a0, double* __restrict__ d) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * M) return;
  const int64_t g = e / M;
  const int p = (int)(e % M);
  const double* Rg = R + g * 3 * M;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int b = 0; b < M; ++b) {
    if (b == p) continue;
    const double dx = Rg[3 * p] - Rg[3 * b], dy = Rg[3 * p + 1] - Rg[3 * b + 1], dz = Rg[3 * p + 2] - Rg[3 * b + 2];
    const double ir = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    const double ir3 = ir * ir * ir;
    sx += dx * dx * ir3 * ir3;
    sy += dy * dy * ir3 * ir3;
    sz += dz * dz * ir3 * ir3;
  }
  d[3 * e] = a0 * sx;
  d[3 * e + 1] = a0 * sy;
  d[3 * e + 2] = a0 * sz;
}

void kernel_diag(const ffk_system* s, double* d, hipStream_t st) {
  if (!s->sym.empty()) {
    sym_diag(s, d, st);
    return;
  }
  k_diag<<<cdiv(s->N * s->M, 256), 256, 0, st>>>(s->R.as<double>(), s->N, s->M, s->a0, d);
  LAUNCHCHK();
}

double max_diag(ffk_system* s, hipStream_t st) {
  if (s->max_diag > 0) return s->max_diag;
  DBuf d(s->n * 8), m(8), part(kRedParts * 8);
  kernel_diag(s, d.as<double>(), st);
  reduce_max64(d.as<double>(), s->n, part.as<double>(), m.as<double>(), st);
  double h = 0;
  HIPCHK(hipMemcpyAsync(&h, m.get(), 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  s->max_diag = h;
  return h;
}

}  // namespace ffk
