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
#include <type_traits>

#include "gemm.hpp"

namespace ffk {

static int64_t rup(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// u_g = J_g v_g for a group of GT geometries per block (threads run over the
// descriptor pairs, so every global access is coalesced); also
// pd_g = x_c,g . u_g, the per-block column partial sums of U, and the copies of
// U the chosen precision needs (FP64, FP32, or split BF16 in both layouts).
// Small systems take 4 geometries per block so that the grid still covers the
// GPU; large ones take 16, which keeps the column partials few.
static int jv_group(int64_t N) { return N < 8192 ? 4 : 16; }

// MODE: 0 = FP64, 1 = FP32, 2 = split BF16 (hi in U/UT, lo in Ul/UTl),
// 3 = split BF16 with the transposed copy in the interleaved operand of the
// fused product (geometry g at K index 8 (g / 4) + g % 4; the slots
// 8 (g / 4) + 4 + g % 4 hold X_c^T and are not touched here).
// U is written row-major with leading dimension ldu (BF16: fragment-major
// with K = ldu); UT (if not null) is the transposed copy with leading
// dimension ldut (BF16: fragment-major, K = ldut).  Padding is left untouched.
template <int MODE, int GT>
__global__ __launch_bounds__(256) void k_jv_tile(const double* __restrict__ R, const int* __restrict__ pairs,
                                                 const double* __restrict__ v, const double* __restrict__ Xc,
                                                 int64_t N, int M, int64_t D, void* __restrict__ U,
                                                 void* __restrict__ Ul, int64_t ldu, void* __restrict__ UT,
                                                 void* __restrict__ UTl, int64_t ldut, double* __restrict__ pd,
                                                 double* __restrict__ cpart) {
  extern __shared__ double sm[];
  const int m3 = 3 * M;
  double* sR = sm;              // GT x 3M
  double* sv = sm + GT * m3;    // GT x 3M
  __shared__ double red[GT][4];
  const int64_t g0 = (int64_t)blockIdx.x * GT;
  const int ng = (int)(N - g0 < GT ? N - g0 : GT);
  for (int e = threadIdx.x; e < ng * m3; e += blockDim.x) {
    sR[e] = R[g0 * m3 + e];
    sv[e] = v[g0 * m3 + e];
  }
  __syncthreads();
  double pdp[GT];
#pragma unroll
  for (int gl = 0; gl < GT; ++gl) pdp[gl] = 0.0;
  for (int64_t d = threadIdx.x; d < D; d += blockDim.x) {
    const int pq = pairs[d];
    const int p = 3 * (pq >> 16), q = 3 * (pq & 0xFFFF);
    double cs = 0.0;
    double ug[GT], xg[GT];
    // the group's descriptor entries first: all GT loads in flight before
    // the first use (loaded inside the per-geometry branch below, each was
    // waited on in turn)
#pragma unroll
    for (int gl = 0; gl < GT; ++gl) xg[gl] = gl < ng ? Xc[(g0 + gl) * D + d] : 0.0;
#pragma unroll
    for (int gl = 0; gl < GT; ++gl) {
      double u = 0.0;
      if (gl < ng) {
        const double* Rg = sR + gl * m3;
        const double* vg = sv + gl * m3;
        const double dx = Rg[p] - Rg[q], dy = Rg[p + 1] - Rg[q + 1], dz = Rg[p + 2] - Rg[q + 2];
        const double ir = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
        u = -(dx * (vg[p] - vg[q]) + dy * (vg[p + 1] - vg[q + 1]) + dz * (vg[p + 2] - vg[q + 2])) * (ir * ir * ir);
        pdp[gl] += u * xg[gl];
        const int64_t o = (g0 + gl) * ldu + d;
        if (MODE == 0) static_cast<double*>(U)[o] = u;
        if (MODE == 1) static_cast<float*>(U)[o] = (float)u;
        if (MODE >= 2) {   // fragment-major, K = ldu
          const float f = (float)u;
          const bf16_t h = f2bf(f);
          const int64_t of = frag_off(g0 + gl, d, ldu / 32);
          static_cast<bf16_t*>(U)[of] = h;
          static_cast<bf16_t*>(Ul)[of] = f2bf(f - bf2f(h));
        }
      }
      cs += u;
      ug[gl] = u;
    }
    cpart[(int64_t)blockIdx.x * D + d] = cs;
    if (UT && MODE >= 2 && ng == GT) {
      // transposed split-BF16 copy of a full group: the GT geometries of row
      // d are consecutive K indices (four at a time in the interleaved
      // layout), written as 8-byte vectors instead of 2-byte stores
#pragma unroll
      for (int q4 = 0; q4 < GT; q4 += 4) {
        uint32_t h[2], l[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float f0 = (float)ug[q4 + 2 * e], f1 = (float)ug[q4 + 2 * e + 1];
          const bf16_t h0 = f2bf(f0), h1 = f2bf(f1);
          h[e] = (uint32_t)h0 | ((uint32_t)h1 << 16);
          l[e] = (uint32_t)f2bf(f0 - bf2f(h0)) | ((uint32_t)f2bf(f1 - bf2f(h1)) << 16);
        }
        const int64_t g = g0 + q4;   // a multiple of 4
        const int64_t of = frag_off(d, MODE == 3 ? 8 * (g >> 2) : g, ldut / 32);
        *reinterpret_cast<uint2*>(static_cast<bf16_t*>(UT) + of) = make_uint2(h[0], h[1]);
        *reinterpret_cast<uint2*>(static_cast<bf16_t*>(UTl) + of) = make_uint2(l[0], l[1]);
      }
    } else if (UT) {   // transposed copy: ng consecutive geometries of row d
#pragma unroll
      for (int gl = 0; gl < GT; ++gl)
        if (gl < ng) {
          const int64_t o = d * ldut + g0 + gl;
          if (MODE == 0) static_cast<double*>(UT)[o] = ug[gl];
          if (MODE == 1) static_cast<float*>(UT)[o] = (float)ug[gl];
          if (MODE >= 2) {   // fragment-major, K = ldut
            const float f = (float)ug[gl];
            const bf16_t h = f2bf(f);
            const int64_t g = g0 + gl;
            const int64_t of = frag_off(d, MODE == 3 ? 8 * (g >> 2) + (g & 3) : g, ldut / 32);
            static_cast<bf16_t*>(UT)[of] = h;
            static_cast<bf16_t*>(UTl)[of] = f2bf(f - bf2f(h));
          }
        }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int gl = 0; gl < GT; ++gl) {
    double x = pdp[gl];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0) red[gl][wave] = x;
  }
  __syncthreads();
  if (threadIdx.x < ng) {
    const int gl = threadIdx.x;
    pd[g0 + gl] = (red[gl][0] + red[gl][1]) + (red[gl][2] + red[gl][3]);
  }
}


template <int MODE, typename... A>
static void launch_jv(int64_t N, int M, hipStream_t st, A... args) {
  const int gt = jv_group(N);
  const size_t shm = (size_t)2 * gt * 3 * M * sizeof(double);
  if (gt == 4)
    k_jv_tile<MODE, 4><<<cdiv(N, 4), 256, shm, st>>>(args...);
  else
    k_jv_tile<MODE, 16><<<cdiv(N, 16), 256, shm, st>>>(args...);
}

// s = sum of the per-block column partials (nblk x D): one wave per column,
// four columns per block; lane l takes partials l, l + 64, ... and a fixed
// butterfly combines the lanes.  (Eight loads per lane in flight, with the
// ones past the end clamped and masked, made it slower at M = 60, N = 20000:
// 16.5 -> 19.9 us; at N = 2000 it sits at a 6 us floor either way.)
__global__ __launch_bounds__(256) void k_colsum_final(const double* __restrict__ part, int nblk, int64_t D,
                                                      double* __restrict__ s) {
  const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int q = threadIdx.x & 63;
  double a0 = 0.0, a1 = 0.0;
  if (col < D) {
    int i = q;
    for (; i + 64 < nblk; i += 128) {
      a0 += part[(int64_t)i * D + col];
      a1 += part[(int64_t)(i + 64) * D + col];
    }
    if (i < nblk) a0 += part[(int64_t)i * D + col];
  }
  double t = a0 + a1;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off);
  if (q == 0 && col < D) s[col] = t;
}

// Sum of x over a block of 64, 128 or 256 lanes: wave butterflies, then the
// wave totals in order; every lane gets the sum.
__device__ inline double block_sum_waves(double x) {
  __shared__ double wsum[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = x;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += wsum[w];
  return t;
}

// y_g = J_g^T G_g + shift v_g, one geometry per block.
// y = J^T G + shift v for geometry g from its coordinates sR (3M) and its
// row sG (D) of G, both in LDS.  With vy_part (and v), also v_g . y_g into
// vy_part[g]: the block partials of v^T y, which CG needs as p^T q.  Pair
// (a, b) adds -G_ab x_ab^3 (r_a - r_b) to atom a, x_ab = 1 / |r_a - r_b| its
// descriptor entry; the row sG arrives already scaled, G_ab x_ab^3 (the
// callers form it from the descriptor row as they fill sG), so the loop over
// partners needs no square root or divide.
// Each atom takes a group of L lanes (a power of two, within a wave, as many
// as the block holds for all M atoms): lane `part` sums the partners b =
// part, part + L, ..., and the group's sums meet in a fixed butterfly, so
// the result does not depend on timing.  (One lane per atom left most of the
// block idle behind a serial loop over M - 1 partners.)
__device__ inline void jtg_atoms(const double* sR, const double* sG, int64_t g, int M,
                                 const double* v, double shift, double* y, bool accumulate = false,
                                 double* vy_part = nullptr) {
  int L = 1;
  while (L < 64 && 2 * L * M <= (int)blockDim.x) L *= 2;
  const int part = (int)threadIdx.x & (L - 1);
  const int per = (int)blockDim.x / L;   // atoms per pass
  double vy = 0.0;
  for (int a0 = 0; a0 < M; a0 += per) {   // uniform across the block
    const int a = a0 + (int)threadIdx.x / L;
    double ax = 0.0, ay = 0.0, az = 0.0;
    if (a < M) {
      const double xa = sR[3 * a], ya = sR[3 * a + 1], za = sR[3 * a + 2];
      for (int b = part; b < M; b += L) {
        if (b == a) continue;
        const int idx = a > b ? a * (a - 1) / 2 + b : b * (b - 1) / 2 + a;
        const double dx = xa - sR[3 * b], dy = ya - sR[3 * b + 1], dz = za - sR[3 * b + 2];
        const double c = sG[idx];
        ax -= c * dx;
        ay -= c * dy;
        az -= c * dz;
      }
    }
    for (int o = L / 2; o >= 1; o >>= 1) {
      ax += __shfl_xor(ax, o);
      ay += __shfl_xor(ay, o);
      az += __shfl_xor(az, o);
    }
    if (a < M && part == 0) {
      const int64_t o = g * 3 * M + 3 * a;
      if (v) {
        ax += shift * v[o];
        ay += shift * v[o + 1];
        az += shift * v[o + 2];
      }
      if (accumulate) {
        y[o] += ax;
        y[o + 1] += ay;
        y[o + 2] += az;
      } else {
        y[o] = ax;
        y[o + 1] = ay;
        y[o + 2] = az;
      }
      if (vy_part) vy += (ax * v[o] + ay * v[o + 1]) + az * v[o + 2];
    }
  }
  if (vy_part) {   // uniform across the block
    const double t = block_sum_waves(vy);
    if (threadIdx.x == 0) vy_part[g] = t;
  }
}

// y = J^T G + shift v, or y += J^T G with accumulate (then v is unused).
// X: the uncentred descriptor rows, which scale G as it is staged.
__global__ void k_jtg(const double* __restrict__ R, const double* __restrict__ G, const double* __restrict__ X,
                      const double* __restrict__ v, double shift, int M, int64_t D,
                      double* __restrict__ y, int accumulate = 0, double* __restrict__ vy_part = nullptr) {
  extern __shared__ double sm[];
  double* sR = sm;
  double* sG = sm + 3 * M;
  const int64_t g = blockIdx.x;
  for (int i = threadIdx.x; i < 3 * M; i += blockDim.x) sR[i] = R[g * 3 * M + i];
  for (int64_t i = threadIdx.x; i < D; i += blockDim.x) {
    const double x = X[g * D + i];
    sG[i] = G[g * D + i] * (x * x * x);
  }
  __syncthreads();
  jtg_atoms(sR, sG, g, M, accumulate ? nullptr : v, shift, y, accumulate != 0,
            accumulate ? nullptr : vy_part);
}

// Sum of the n partials p[0..n) by the calling wave: lane l adds l, l + 64,
// ..., and a fixed butterfly combines the lanes; every lane gets the sum.
__device__ inline double wave_sum_parts(const double* __restrict__ p, int n) {
  double a = 0.0;
  for (int q = threadIdx.x & 63; q < n; q += 64) a += p[q];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  return a;
}

// The split-K reduction of GEMM 2 fused with J^T G: one block per geometry
// forms its row of G = sum_z part_z + a0 s + w Xt in LDS (the arithmetic and
// order of k_g_reduce) and applies J^T to it; G never goes to HBM.  The
// row is staged already scaled by x^3, with the descriptor x = x_c + mean
// recovered from the centred row the reduction reads anyway.
// SPL: the number of splits when fixed at compile time (1 to 8, 16), else 0.  A
// thread takes CC columns at a time (1 while a block's lanes cover the row,
// else 2) and, with SPL fixed, issues every load of them before the first
// wait (with the count known only at run time the loads of each split were
// waited on in turn).  LDS: 3M + D + 1 doubles.
template <typename PT, int SPL, int CC>
__global__ void k_jtg_reduce(const PT* __restrict__ part, int splits, int64_t rows, const double* __restrict__ s,
                             const double* __restrict__ Xt, const double* __restrict__ xmean,
                             const double* __restrict__ wpart, int ntn, double a0,
                             const double* __restrict__ R, const double* __restrict__ v, double shift, int M,
                             int64_t D, double* __restrict__ y, double* __restrict__ vy_part) {
  extern __shared__ double sm[];
  double* sR = sm;
  double* sG = sm + 3 * M;
  __shared__ double wsh;
  const int64_t g = blockIdx.x;
  if (threadIdx.x < 64) {
    const double w = wave_sum_parts(wpart + g * ntn, ntn);
    if (threadIdx.x == 0) wsh = w;
  }
  for (int i = threadIdx.x; i < 3 * M; i += blockDim.x) sR[i] = R[g * 3 * M + i];
  __syncthreads();
  const double w = wsh;
  const int64_t bd = blockDim.x, zs = rows * D;
  for (int64_t cb = threadIdx.x; cb < D; cb += CC * bd) {
    double xc[CC], sc[CC], xm[CC], acc[CC];
#pragma unroll
    for (int j = 0; j < CC; ++j) {
      const int64_t c = min(cb + j * bd, D - 1);   // a column past the end reads D - 1
      xc[j] = Xt[g * D + c];
      sc[j] = s[c];
      xm[j] = xmean[c];
    }
    if constexpr (SPL > 0) {
      // at most eight splits' loads in flight: sixteen 64-bit addresses
      // and values per column do not fit the 64 VGPRs of full occupancy
      constexpr int ZB = SPL < 8 ? SPL : 8;
      static_assert(SPL % ZB == 0, "split batches");
#pragma unroll
      for (int j = 0; j < CC; ++j) acc[j] = 0.0;
#pragma unroll 1
      for (int z0 = 0; z0 < SPL; z0 += ZB) {
        PT pz[CC][ZB];
#pragma unroll
        for (int j = 0; j < CC; ++j)
#pragma unroll
          for (int z = 0; z < ZB; ++z) pz[j][z] = part[g * D + min(cb + j * bd, D - 1) + (z0 + z) * zs];
#pragma unroll
        for (int j = 0; j < CC; ++j)
#pragma unroll
          for (int z = 0; z < ZB; ++z) acc[j] += (double)pz[j][z];
      }
    } else {
#pragma unroll
      for (int j = 0; j < CC; ++j) {
        const int64_t c = min(cb + j * bd, D - 1);
        acc[j] = 0.0;
#pragma unroll 4
        for (int z = 0; z < splits; ++z) acc[j] += (double)part[g * D + c + z * zs];
      }
    }
    // no branch here (the loads would sink into it): a column of the thread
    // past the end goes to the spare slot sG[D]
#pragma unroll
    for (int j = 0; j < CC; ++j) {
      const double x = xc[j] + xm[j];
      sG[min(cb + j * bd, D)] = (acc[j] + a0 * sc[j] + w * xc[j]) * (x * x * x);
    }
  }
  __syncthreads();
  jtg_atoms(sR, sG, g, M, v, shift, y, false, vy_part);
}

template <typename PT, int CC, typename... A>
static void launch_jtg_reduce_cc(int64_t N, size_t shm, hipStream_t st, const PT* part, int splits, A... args) {
  switch (splits) {
    case 1: k_jtg_reduce<PT, 1, CC><<<N, 256, shm, st>>>(part, splits, args...); break;
    case 2: k_jtg_reduce<PT, 2, CC><<<N, 256, shm, st>>>(part, splits, args...); break;
    case 3: k_jtg_reduce<PT, 3, CC><<<N, 256, shm, st>>>(part, splits, args...); break;
    case 4: k_jtg_reduce<PT, 4, CC><<<N, 256, shm, st>>>(part, splits, args...); break;
    case 5: k_jtg_reduce<PT, 5, CC><<<N, 256, shm, st>>>(part, splits, args...); break;
    case 6: k_jtg_reduce<PT, 6, CC><<<N, 256, shm, st>>>(part, splits, args...); break;
    case 7: k_jtg_reduce<PT, 7, CC><<<N, 256, shm, st>>>(part, splits, args...); break;
    case 8: k_jtg_reduce<PT, 8, CC><<<N, 256, shm, st>>>(part, splits, args...); break;
    case 16: k_jtg_reduce<PT, 16, CC><<<N, 256, shm, st>>>(part, splits, args...); break;
    default: k_jtg_reduce<PT, 0, CC><<<N, 256, shm, st>>>(part, splits, args...); break;
  }
}

template <typename PT, typename... A>
static void launch_jtg_reduce(int64_t N, int64_t D, size_t shm, hipStream_t st, const PT* part, int splits,
                              A... args) {
  if (D <= 256)
    launch_jtg_reduce_cc<PT, 1>(N, shm, st, part, splits, args...);
  else
    launch_jtg_reduce_cc<PT, 2>(N, shm, st, part, splits, args...);
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
    double* red = reinterpret_cast<double*>(smem);   // [wave columns][BM]
    // Loads go out in batches ahead of the stores (a load of B may not move
    // above a store of -W, which it could alias): pd for all columns, then B
    // for one block row at a time.  Indices are clamped to valid entries, so
    // every load is in bounds; only valid entries are used and stored.
    double pdv[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) pdv[j] = pd[min(f.col(j), Nc - 1)];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      double bv[4][TN];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          bv[v][j] = (double)Bc[(int64_t)min(f.row(i, v), Nr - 1) * ldb + min(f.col(j), Nc - 1)];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = f.row(i, v);
        double rs = 0.0;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int c = f.col(j);
          if (r < Nr && c < Nc) {
            const double w = bv[v][j] * ((double)acc[i][j][v] - pdv[j]);
            Wn[(int64_t)r * ldw + c] = (CT)(-w);
            rs += w;
          }
        }
        rs += __shfl_xor(rs, 1);
        rs += __shfl_xor(rs, 2);
        rs += __shfl_xor(rs, 4);
        rs += __shfl_xor(rs, 8);
        if ((f.lane & 15) == 0) red[f.wcol * BM + (r - f.m0)] = rs;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < BM; t += blockDim.x) {
      const int r = f.m0 + t;
      if (r < Nr) {
        double a = 0.0;
        for (int q = 0; q < f.nwcol; ++q) a += red[q * BM + t];
        wpart[(int64_t)r * ntn + f.tn] = a;
      }
    }
  }
};

// FP32 and BF16 products: GEMM 1 runs transposed, P^T = U X_c^T (A = U,
// B = X_c).  In their MFMA output layout lane l holds rows 4(l/16)+v of a
// 16x16 block, which are then four consecutive columns c0..c0+3 of one row r
// of W: B is read as one 16-byte vector, -W is written as one vector (FP32
// row-major; BF16 hi and lo in fragment order, 8 bytes each) and the row sum
// of W is mostly lane-local.  The coefficient B is FP32; FP32 products form W
// in FP64 arithmetic, BF16 products in FP32.  All padded entries are written
// (zero, as B is zero there).  Row-sum partials: one per row of W and tile of
// its columns (GEMM 1 tile row).
template <typename CT, bool X3>
struct EpiWT {
  const float* Bc; int64_t ld;   // B and -W share the padded leading dimension
  const double* pd;
  CT* Wh; CT* Wl;
  double* wpart; int nparts;
  int Nt, Ns;   // valid targets (rows of W) and sources (columns)
  template <typename T, int TM, int TN, class Acc>
  __device__ void run(const Acc (&acc)[TM][TN], const FragCoord& f, char* smem) const {
    static_assert(sizeof(CT) == 4 || sizeof(CT) == 2, "FP32 or BF16 storage");
    typedef typename std::conditional<sizeof(CT) == 4, double, float>::type MT;
    double* red = reinterpret_cast<double*>(smem);   // [wave rows][BN]
    const int WM = (blockDim.x >> 6) / f.nwcol, BN = f.nwcol * 16 * TN;
    const int wm = (f.wm0 - f.m0) / (16 * TM);
    double rs[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) rs[j] = 0.0;
    // BATCH: loads are issued in batches ahead of the stores they would
    // otherwise follow.  The compiler may not move a load of B above a store
    // of -W (they could alias), so loads written inside the loop each waited
    // a full memory round trip (48 per tile of the split 256 x 256 tile).
    // pd for all rows at once (pd has the padded length and is zero past the
    // sources, so every load is in bounds), then the B vectors of one row at
    // a time.  Not on the 4 x 4-block wave tiles of single BF16 and FP32:
    // there the batch's registers would cost single BF16 its second
    // workgroup per CU (115 -> 144 VGPRs; GEMM 1 at M = 60, N = 20000 1.66 ->
    // 2.01 ms), whose main loop hides this epilogue, and FP32 gained nothing.
    constexpr bool BATCH = X3 || TM * TN <= 4;
    MT p[TM][4];
    if constexpr (BATCH) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = f.row(i, 0) + v;
          const double pv = pd[c];
          p[i][v] = c < Ns ? (MT)pv : (MT)0;
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int c0 = f.row(i, 0);
      f4 bq[TN];
      if constexpr (BATCH) {
#pragma unroll
        for (int j = 0; j < TN; ++j) bq[j] = *reinterpret_cast<const f4*>(Bc + (int64_t)f.col(j) * ld + c0);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) p[i][v] = c0 + v < Ns ? (MT)pd[c0 + v] : (MT)0;
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int r = f.col(j);
        const f4 b = BATCH ? bq[j] : *reinterpret_cast<const f4*>(Bc + (int64_t)r * ld + c0);
        MT w[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          w[v] = (MT)b[v] * ((MT)acc[i][j][v] - p[i][v]);
          rs[j] += (double)w[v];
        }
        if constexpr (sizeof(CT) == 4) {
          *reinterpret_cast<f4*>(Wh + (int64_t)r * ld + c0) = f4{(float)-w[0], (float)-w[1], (float)-w[2], (float)-w[3]};
        } else {
          uint32_t h[4], l[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const bf16_t hv = f2bf((float)-w[v]);
            h[v] = hv;
            l[v] = X3 ? f2bf((float)-w[v] - bf2f(hv)) : 0u;
          }
          const int64_t o = frag_off(r, c0, ld / 32);   // c0 % 4 == 0: 8-byte aligned
          *reinterpret_cast<uint2*>(Wh + o) = make_uint2(h[0] | h[1] << 16, h[2] | h[3] << 16);
          if (X3) *reinterpret_cast<uint2*>(Wl + o) = make_uint2(l[0] | l[1] << 16, l[2] | l[3] << 16);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      double s = rs[j];
      s += __shfl_xor(s, 16);
      s += __shfl_xor(s, 32);
      if (f.lane < 16) red[wm * BN + (f.col(j) - f.n0)] = s;
    }
    __syncthreads();
    const int tm = f.m0 / (16 * TM * WM);
    for (int t = threadIdx.x; t < BN; t += blockDim.x) {
      const int r = f.n0 + t;
      if (r < Nt) {
        double a = 0.0;
        for (int q = 0; q < WM; ++q) a += red[q * BN + t];
        wpart[(int64_t)r * nparts + tm] = a;
      }
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

// Split-K reduction for GEMM 2: G = sum_z part_z + a0 s_c + w_r Xt_r,c (one block per row).
template <typename PT>
__global__ __launch_bounds__(256) void k_g_reduce(const PT* __restrict__ part, int splits, int64_t rows, int64_t cols,
                                                  const double* __restrict__ s, const double* __restrict__ Xt,
                                                  const double* __restrict__ wpart, int ntn, double a0,
                                                  double* __restrict__ G) {
  __shared__ double wsh;
  const int64_t r = blockIdx.x;
  if (threadIdx.x < 64) {
    const double w = wave_sum_parts(wpart + r * ntn, ntn);
    if (threadIdx.x == 0) wsh = w;
  }
  __syncthreads();
  const double w = wsh;
  for (int64_t c = threadIdx.x; c < cols; c += blockDim.x) {
    double acc = 0.0;
#pragma unroll 4
    for (int z = 0; z < splits; ++z) acc += (double)part[((int64_t)z * rows + r) * cols + c];
    G[r * cols + c] = acc + a0 * s[c] + w * Xt[r * cols + c];
  }
}

static inline void mark(hipEvent_t* ev, int i, hipStream_t st) {
  if (ev) HIPCHK(hipEventRecord(ev[i], st));
}

// Shared operands of one product: target descriptor (rows of GEMM 1/2) and
// source quantities.
struct MvmArgs {
  int64_t Nt, Ns, D;
  double a0;
  const double* Xt64;    // target X_c (FP64, Nt x D), for the diag(w) X term
  const double* pd;      // Ns
  const double* s;       // D
  double* wpart;         // Nt x ntn
  double* G;             // Nt x D
  void* part;            // split-K partials
  size_t part_bytes;
};

template <typename T>
static void mvm_gemms_scalar(const MvmArgs& a, const T* Xt, const T* Xs, const T* U, const T* dA, const T* Bc, T* Wn,
                             hipStream_t st, hipEvent_t* ev) {
  const int Nt = (int)a.Nt, Ns = (int)a.Ns;
  const int64_t D = a.D;
  const int ntn = cdiv(Ns, 128);
  {
    ScalarArgs<T> g{};
    g.M = Nt;
    g.N = Ns;
    g.nseg = 1;
    g.seg[0] = SegS<T>{Xt, D, 1, U, D, 1, (int)D};
    EpiW<T, 128> e{Bc, Ns, a.pd, Wn, Ns, a.wpart, ntn, Nt, Ns};
    clk_begin(CLK_GEMM1, st);
    gemm_scalar_kernel<T, 128, 128, 16, true, true, EpiW<T, 128>><<<dim3(ntn, cdiv(Nt, 128)), 256, 0, st>>>(g, e);
    LAUNCHCHK();
    clk_end(CLK_GEMM1, st);
  }
  mark(ev, 3, st);
  ScalarArgs<T> g{};
  g.M = Nt;
  g.N = (int)D;
  g.nseg = 2;
  g.seg[0] = SegS<T>{dA, Ns, 1, U, 1, D, Ns};
  g.seg[1] = SegS<T>{Wn, Ns, 1, Xs, 1, D, Ns};
  const int64_t tiles = (int64_t)cdiv(D, 128) * cdiv(Nt, 128);
  int splits = pick_splits(tiles, 2 * (int64_t)cdiv(Ns, 16));
  while (splits > 1 && (size_t)splits * Nt * D * sizeof(T) > a.part_bytes) splits >>= 1;
  if (splits == 1) {
    EpiG<128> e{a.s, a.Xt64, D, a.wpart, ntn, a.a0, a.G, D, Nt, (int)D};
    clk_begin(CLK_GEMM2, st);
    gemm_scalar_kernel<T, 128, 128, 16, true, false, EpiG<128>><<<dim3(cdiv(D, 128), cdiv(Nt, 128)), 256, 0, st>>>(g, e);
    LAUNCHCHK();
    clk_end(CLK_GEMM2, st);
  } else {
    EpiPart<T> e{static_cast<T*>(a.part), D, Nt, (int)D};
    clk_begin(CLK_GEMM2, st);
    gemm_scalar_kernel<T, 128, 128, 16, true, false, EpiPart<T>><<<dim3(cdiv(D, 128), cdiv(Nt, 128), splits), 256, 0, st>>>(g, e);
    LAUNCHCHK();
    clk_end(CLK_GEMM2, st);
    clk_begin(CLK_GEMM2_REDUCE, st);
    k_g_reduce<T><<<Nt, 256, 0, st>>>(static_cast<const T*>(a.part), splits, Nt, D, a.s, a.Xt64, a.wpart, ntn, a.a0, a.G);
    LAUNCHCHK();
    clk_end(CLK_GEMM2_REDUCE, st);
  }
}

// Both GEMMs of the product on the pipelined MFMA engine, for element type T
// (double, float or bf16; X3 = split BF16) and tile shapes TL1 (GEMM 1) and
// TL2 (GEMM 2).  Operands are the padded arrays: X_c (Nr x Dk) and its
// transpose (Dr x Nr), U likewise, dA, B and -W (Nr x Nr).
struct DmaOps {
  const void *Xh, *Xl, *XTh, *XTl;   // X_c
  const void *Uh, *Ul, *UTh, *UTl;   // U = J v
  const void *dAh, *dAl;             // dA
  const void* Bc;                    // B (FP64 for FP64, FP32 otherwise)
  void *Wh, *Wl;                     // -W
};

// K splits for GEMM 2.  A grid smaller than the workgroup slots of the GPU
// takes the fixed rule of pick_splits: at least 512 workgroups, or 256 for
// BF16 and FP32 operands below N = 4096, where the products are latency-bound
// and half the partials cost more than half the parallelism.  (At M = 21,
// N = 2000, 8 splits instead of 16: split BF16 61.6 -> 56.2 us, BF16 44.8 ->
// 41.5, FP32 98.5 -> 95.7; FP64 went 169.5 -> 187.0 and keeps 16.  At
// N = 5000 and 10000 the lower target was up to 22% slower.)  A larger grid
// takes the split count
// that minimises the estimated time: ceil(tiles s / slots) rounds of 1/s of
// the K loop each, plus the split-K partials written and read back once.
// Without it, 553 tiles of 256 x 256 on 256 slots run 3 rounds for 2.16
// rounds of work.  Rates per CU are the engine's measured main-loop rates
// (BF16 ~1.2 PFLOP/s, FP32 ~115 TFLOP/s, FP64 ~50 TFLOP/s over 256 CUs), and
// HBM ~5 TB/s for the partials; only their ratio matters.
template <typename T, bool X3, class TL, typename CT>
static int gemm2_splits(int64_t tiles, int64_t ktiles, int64_t N, int64_t D) {
  static int per_cu = 0, cus = 0;
  if (per_cu == 0) {
    int nb = 0, dev = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_dma_kernel<T, TL, X3, EpiPart<CT>>, TL::NT, 0));
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    per_cu = nb > 0 ? nb : 1;
  }
  const int64_t slots = (int64_t)cus * per_cu;
  if (tiles < slots) return pick_splits(tiles, ktiles, sizeof(T) <= 4 && N < 4096 ? 256 : 512);
  const double rate_cu = (sizeof(T) == 2 ? 1.2e15 : sizeof(T) == 4 ? 1.15e14 : 5.0e13) / 256.0;
  const double t_tile = 2.0 * TL::BM * TL::BN * (double)ktiles * (64 / sizeof(T)) * (X3 ? 3 : 1) / rate_cu;
  const double t_part = 2.0 * (double)N * D * sizeof(CT) / 5.0e12;
  int best = 1;
  double bt = 0.0;
  for (int s = 1; s <= 16 && (int64_t)s * 4 <= ktiles; ++s) {
    const double t = (double)((tiles * s + slots - 1) / slots) * per_cu * t_tile / s + (s > 1 ? s * t_part : 0.0);
    if (s == 1 || t < 0.98 * bt) {
      bt = t;
      best = s;
    }
  }
  return best;
}

// K split count of GEMM 2 (1: G is written; above 1: the split partials are
// left in a.part for k_jtg_reduce) and the row-sum partials per row of W.
struct GemmOut {
  int splits, ntn;
};

template <typename T, bool X3, typename CT, class TL1, class TL2>
static GemmOut mvm_gemms_dma(const MvmArgs& a, int64_t Ntr, int64_t Nsr, int64_t Dk, int64_t Dr, const DmaOps& o,
                             hipStream_t st, hipEvent_t* ev) {
  const int64_t N = a.Nt, Ns = a.Ns, D = a.D;
  // FP32 and BF16: GEMM 1 computes P^T (EpiWT), so the row-sum partials of W
  // are per GEMM 1 tile row; FP64 keeps P = X_c U^T and per tile column.
  constexpr bool kTrans = sizeof(T) != 8;
  const int ntn = (int)(Nsr / (kTrans ? TL1::BM : TL1::BN));   // row-sum partials per row of W (source tiles)
  {
    DmaArgs g{};
    g.nseg = 1;
    g.seg[0] = kTrans ? SegD{o.Uh, o.Ul, o.Xh, o.Xl, Dk, Dk, (int)Dk} : SegD{o.Xh, o.Xl, o.Uh, o.Ul, Dk, Dk, (int)Dk};
    // FP32 / BF16: rows of the product are sources, columns targets; FP64 the reverse
    const dim3 grid(kTrans ? (unsigned)(Ntr / TL1::BN) : (unsigned)(Nsr / TL1::BN),
                    kTrans ? (unsigned)(Nsr / TL1::BM) : (unsigned)(Ntr / TL1::BM));
    clk_begin(CLK_GEMM1, st);
    if constexpr (kTrans) {
      EpiWT<T, X3> e{static_cast<const float*>(o.Bc), Nsr, a.pd, static_cast<T*>(o.Wh), static_cast<T*>(o.Wl),
                     a.wpart, ntn, (int)N, (int)Ns};
      gemm_dma_kernel<T, TL1, X3, decltype(e)><<<grid, TL1::NT, 0, st>>>(g, e);
    } else {
      EpiW<T, TL1::BM> e{static_cast<const T*>(o.Bc), Nsr, a.pd, static_cast<T*>(o.Wh), Nsr, a.wpart, ntn, (int)N,
                         (int)Ns};
      gemm_dma_kernel<T, TL1, X3, decltype(e)><<<grid, TL1::NT, 0, st>>>(g, e);
    }
    LAUNCHCHK();
    clk_end(CLK_GEMM1, st);
  }
  mark(ev, 3, st);
  DmaArgs g{};
  g.nseg = 2;
  g.seg[0] = SegD{o.dAh, o.dAl, o.UTh, o.UTl, Nsr, Nsr, (int)Nsr};
  g.seg[1] = SegD{o.Wh, o.Wl, o.XTh, o.XTl, Nsr, Nsr, (int)Nsr};
  const int64_t tiles = (Dr / TL2::BN) * (Ntr / TL2::BM);
  int splits = gemm2_splits<T, X3, TL2, CT>(tiles, 2 * Nsr / (64 / (int64_t)sizeof(T)), N, D);
  while (splits > 1 && (size_t)splits * N * D * sizeof(CT) > a.part_bytes) splits >>= 1;
  const dim3 grid((unsigned)(Dr / TL2::BN), (unsigned)(Ntr / TL2::BM), (unsigned)splits);
  if (splits == 1) {
    EpiG<TL2::BM> e{a.s, a.Xt64, D, a.wpart, ntn, a.a0, a.G, D, (int)N, (int)D};
    clk_begin(CLK_GEMM2, st);
    gemm_dma_kernel<T, TL2, X3, EpiG<TL2::BM>><<<grid, TL2::NT, 0, st>>>(g, e);
    LAUNCHCHK();
    clk_end(CLK_GEMM2, st);
  } else {
    EpiPart<CT> e{static_cast<CT*>(a.part), D, (int)N, (int)D};
    clk_begin(CLK_GEMM2, st);
    gemm_dma_kernel<T, TL2, X3, EpiPart<CT>><<<grid, TL2::NT, 0, st>>>(g, e);
    LAUNCHCHK();
    clk_end(CLK_GEMM2, st);
  }
  return GemmOut{splits, ntn};
}

// Tile shapes.  Small N: 64 x 64 (GEMM 1) and 128 x 128 (GEMM 2; BF16: 64 x
// 256) by 4 waves, where the grid would otherwise leave CUs idle.  Large N:
// single BF16 uses 256 x 128 by 8 waves of 64 x 64 with three stages; that
// is 72 KB of LDS, so two workgroups share a CU and one's epilogue overlaps
// the other's main loop (at N = 20000: GEMM 1 2.02 -> 1.66 ms, GEMM 2 2.89 ->
// 2.46 ms against 256 x 256 by 8 waves, which fills a CU alone).  Split BF16
// (hi and lo operands) fills a CU either way and takes the larger tile
// below.  FP32 and FP64 stay at 128 x 128, which measured faster.
typedef DmaTile<64, 64, 2, 2, 4> TileM;        // GEMM 1 of small N: 4x more workgroups
// The same tile in split BF16 with two stages: its hi and lo operands take 16
// KB a stage, so four stages held a CU to two workgroups, and at N = 2000
// (seven K steps) the 1024 tiles ran in two rounds.  GEMM 1 19.9 -> 17.6 us
// at M = 21, N = 2000; single BF16 (14.4 against 13.4 us), FP32 and FP64
// keep four stages.
typedef DmaTile<64, 64, 2, 2, 2> TileMX3;
typedef DmaTile<128, 128, 2, 2, 4> TileS;
typedef DmaTile<256, 128, 4, 2, 3> TileL;      // BF16 and split BF16, large N
typedef DmaTile<64, 256, 1, 4, 3> TileW2;      // GEMM 2 of small N: one tile spans D <= 256 columns
// Split BF16 at large N: 256 x 256 by 8 waves of 64 x 128, two stages (128
// KB of LDS, one workgroup per CU).  Against 256 x 128 (three stages) at M =
// 60, N = 20000: GEMM 1 4.53 -> 3.98 ms, GEMM 2 7.25 -> 6.49 ms; 5% and 4%
// faster products at M = 42, N = 5000 and M = 21, N = 10000.  The two GEMMs'
// tiles can be set at build time (FFK_TILE_X3_G1, FFK_TILE_X3_G2).
#ifndef FFK_TILE_X3_G1
#define FFK_TILE_X3_G1 DmaTile<256, 256, 4, 2, 2>
#endif
#ifndef FFK_TILE_X3_G2
#define FFK_TILE_X3_G2 DmaTile<256, 256, 4, 2, 2>
#endif
typedef FFK_TILE_X3_G1 TileX3G1;
typedef FFK_TILE_X3_G2 TileX3G2;
constexpr int64_t kLargeN = 4096;

template <typename T, bool X3, typename CT>
static GemmOut mvm_gemms_for(const MvmArgs& a, int64_t Ntr, int64_t Nsr, int64_t Dk, int64_t Dr, const DmaOps& o,
                             hipStream_t st, hipEvent_t* ev) {
  if (a.Nt < kLargeN) {
    // BF16: one 256-wide GEMM 2 tile reads [dA | -W] once instead of once per
    // 128 columns (split BF16 at N = 2000, D = 210: 30 -> 27 us); FP32 and
    // FP64 measured 2% slower with it
    if constexpr (sizeof(T) == 2 && X3)
      return mvm_gemms_dma<T, X3, CT, TileMX3, TileW2>(a, Ntr, Nsr, Dk, Dr, o, st, ev);
    if constexpr (sizeof(T) == 2) return mvm_gemms_dma<T, X3, CT, TileM, TileW2>(a, Ntr, Nsr, Dk, Dr, o, st, ev);
    return mvm_gemms_dma<T, X3, CT, TileM, TileS>(a, Ntr, Nsr, Dk, Dr, o, st, ev);
  } else if constexpr (sizeof(T) == 2 && X3) {
    return mvm_gemms_dma<T, X3, CT, TileX3G1, TileX3G2>(a, Ntr, Nsr, Dk, Dr, o, st, ev);
  } else if constexpr (sizeof(T) == 2) {
    return mvm_gemms_dma<T, X3, CT, TileL, TileL>(a, Ntr, Nsr, Dk, Dr, o, st, ev);
  } else {
    // FP32 / FP64: MFMA-bound already at 128 x 128 (measured faster than the large tiles)
    return mvm_gemms_dma<T, X3, CT, TileS, TileS>(a, Ntr, Nsr, Dk, Dr, o, st, ev);
  }
}

static size_t part_budget(int64_t N, int64_t D) { return (size_t)16 * N * D * sizeof(double); }

// Device buffers of one product (all sized for the system's N and D):
// pd (N), s (D), spart (column partials of U), G (N x D), wpart (row-sum
// partials of W), part (split-K partials of GEMM 2, part_bytes), and the
// product-precision operands U / UT (hi and lo for split BF16) and -W.  The
// padding of U, UT and (FP64) -W must be zero; everything else is written
// before it is read.
struct MvmBufs {
  double *pd, *s, *spart, *G, *wpart;
  void* part;
  size_t part_bytes;
  void *U, *Ul, *UT, *UTl, *Wh, *Wl;
};

// Workspace of a product with Nt targets and Ns sources (the square product:
// Nt = Ns = N), allocated on first use and kept.
static void ensure_work(MvmWork& w, const ffk_system* src, int64_t Nt, int64_t D, int prec, hipStream_t st) {
  const int64_t Ns = src->N;
  if (!w.pd) {
    w.pd.alloc(pad_rows(Ns) * 8);   // zero past the sources (the fused product reads whole chunks)
    HIPCHK(hipMemsetAsync(w.pd.get(), 0, pad_rows(Ns) * 8, st));
    w.s.alloc(D * 8);
    w.spart.alloc((int64_t)cdiv(Ns, jv_group(Ns)) * D * 8);
    w.G.alloc(Nt * D * 8);
    w.wpart.alloc(Nt * (pad_rows(Ns) / 64) * 8);   // one partial per GEMM 1 tile of sources (tiles >= 64 wide)
    w.part.alloc(part_budget(Nt, D));
  }
  const int64_t Ntr = pad_rows(Nt), Nsr = pad_rows(Ns), Dk = rup(D, 64), Dr = pad_rows(D);
  // padding rows/columns stay zero: the kernels write only the valid part
  auto zeroed = [&](DBuf& b, int64_t bytes) {
    b.alloc(bytes);
    HIPCHK(hipMemsetAsync(b.get(), 0, bytes, st));
  };
  if (prec == FFK_FP64 && !w.U64) {
    zeroed(w.U64, Nsr * Dk * 8);
    zeroed(w.UT64, Dr * Nsr * 8);
    zeroed(w.Wn64, Ntr * Nsr * 8);
  }
  if (prec == FFK_FP32 && !w.U32) {
    zeroed(w.U32, Nsr * Dk * 4);
    zeroed(w.UT32, Dr * Nsr * 4);
    zeroed(w.Wn32, Ntr * Nsr * 4);
  }
  if ((prec == FFK_BF16 || prec == FFK_BF16X3) && !w.Uh) {
    zeroed(w.Uh, Nsr * Dk * 2);
    zeroed(w.Ul, Nsr * Dk * 2);
    if (use_fused(prec, D, Nt, Ns)) {
      // the interleaved [U^T | X_c^T] operand of the fused product
      zeroed(w.UTh, Dr * 2 * Nsr * 2);
      zeroed(w.UTl, Dr * 2 * Nsr * 2);
      fused_fill_x(src->Xc.as<double>(), Ns, D, Dr, Nsr, w.UTh.as<bf16_t>(), w.UTl.as<bf16_t>(), st);
    } else {
      zeroed(w.UTh, Dr * Nsr * 2);
      zeroed(w.UTl, Dr * Nsr * 2);
      w.Wnh.alloc(Ntr * Nsr * 2);   // every entry is written by the GEMM 1 epilogue
      w.Wnl.alloc(Ntr * Nsr * 2);
    }
  }
}

static MvmBufs handle_bufs(MvmWork& w, int prec) {
  MvmBufs b{w.pd.as<double>(), w.s.as<double>(), w.spart.as<double>(), w.G.as<double>(), w.wpart.as<double>(),
            w.part.get(), w.part.bytes(), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  if (prec == FFK_FP64) {
    b.U = w.U64.get(); b.UT = w.UT64.get(); b.Wh = w.Wn64.get();
  } else if (prec == FFK_FP32) {
    b.U = w.U32.get(); b.UT = w.UT32.get(); b.Wh = w.Wn32.get();
  } else {
    b.U = w.Uh.get(); b.Ul = w.Ul.get(); b.UT = w.UTh.get(); b.UTl = w.UTl.get();
    b.Wh = w.Wnh.get(); b.Wl = w.Wnl.get();
  }
  return b;
}

// y = K(t, src) vs + shift v on prepared coefficients (coef: t->N x src->N
// sets) and descriptor copies, with the workspace b: J v and the GEMM
// operands over the sources, G and J^T G over the targets.  The square
// product is t = src, vs = v.
static void kernel_mvm_core(ffk_system* t, ffk_system* src, CoeffSet* coef, const double* vs, const double* v,
                            double* y, double shift, int prec, hipStream_t st, hipEvent_t* ev, double* vy_part,
                            const MvmBufs& b) {
  mark(ev, 0, st);
  const int64_t N = t->N, Ns = src->N, D = t->D;
  const int M = t->M;
  const int64_t Ntr = pad_rows(N), Nsr = pad_rows(Ns), ldu = rup(D, 64);
  const int nblk = cdiv(Ns, jv_group(Ns));
  double* pd = b.pd;
  double* cp = b.spart;
  clk_begin(CLK_JV, st);
  if (prec == FFK_FP64)
    launch_jv<0>(Ns, M, st, src->R.as<double>(), src->pairs.as<int>(), vs, src->Xc.as<double>(), Ns, M, D,
                 b.U, nullptr, ldu, b.UT, nullptr, Nsr, pd, cp);
  else if (prec == FFK_FP32)
    launch_jv<1>(Ns, M, st, src->R.as<double>(), src->pairs.as<int>(), vs, src->Xc.as<double>(), Ns, M, D,
                 b.U, nullptr, ldu, b.UT, nullptr, Nsr, pd, cp);
  else if (use_fused(prec, D, N, Ns))
    launch_jv<3>(Ns, M, st, src->R.as<double>(), src->pairs.as<int>(), vs, src->Xc.as<double>(), Ns, M, D,
                 b.U, b.Ul, ldu, b.UT, b.UTl, 2 * Nsr, pd, cp);
  else
    launch_jv<2>(Ns, M, st, src->R.as<double>(), src->pairs.as<int>(), vs, src->Xc.as<double>(), Ns, M, D,
                 b.U, b.Ul, ldu, b.UT, b.UTl, Nsr, pd, cp);
  LAUNCHCHK();
  clk_end(CLK_JV, st);
  mark(ev, 1, st);
  clk_begin(CLK_COLSUM, st);
  k_colsum_final<<<cdiv(D, 4), 256, 0, st>>>(cp, nblk, D, b.s);
  LAUNCHCHK();
  clk_end(CLK_COLSUM, st);
  mark(ev, 2, st);
  MvmArgs a{N, Ns, D, t->a0, t->Xc.as<double>(), pd, b.s, b.wpart, b.G, b.part, b.part_bytes};
  GemmOut go{1, 0};
  CoeffSet& cs = coef[prec];
  const int64_t Dk = rup(D, 64), Dr = pad_rows(D);
  DmaOps o{};
  o.dAh = cs.dA_hi.get();
  o.Bc = cs.B.get();
  o.Uh = b.U; o.UTh = b.UT; o.Wh = b.Wh;
  // GEMM 1 takes the targets' descriptor, GEMM 2 the sources' (transposed)
  if (prec == FFK_FP64) {
    o.Xh = t->Xp64.get(); o.XTh = src->XpT64.get();
    go = mvm_gemms_for<double, false, double>(a, Ntr, Nsr, Dk, Dr, o, st, ev);
  } else if (prec == FFK_FP32) {
    o.Xh = t->Xp32.get(); o.XTh = src->XpT32.get();
    go = mvm_gemms_for<float, false, float>(a, Ntr, Nsr, Dk, Dr, o, st, ev);
  } else if (use_fused(prec, D, N, Ns)) {
    // both dense steps in one kernel: W stays on chip
    const bool x3 = prec == FFK_BF16X3;
    FusedArgs f{};
    f.Uh = static_cast<const bf16_t*>(b.U); f.Ul = static_cast<const bf16_t*>(b.Ul);
    f.Xh = t->Xch.as<bf16_t>(); f.Xl = t->Xcl.as<bf16_t>();
    f.Vh = static_cast<const bf16_t*>(b.UT); f.Vl = static_cast<const bf16_t*>(b.UTl);
    f.CF = cs.dA_hi.get();   // the fused layout of dA and B
    f.pd = pd;
    f.part = static_cast<float*>(b.part);
    f.wpart = b.wpart;
    f.KTd = Dk / 32; f.KTs = Nsr / 32; f.Nsr = Nsr;
    f.Nt = (int)N; f.D = (int)D; f.nchunks = (int)cdiv(Ns, 16);
    const int max_splits = (int)std::min<int64_t>({32, Nsr / 64, (int64_t)(b.part_bytes / ((size_t)N * D * 4))});
    f.splits = fused_splits(N, Ns, D, max_splits);
    clk_begin(CLK_FUSED, st);
    fused_mvm_launch(f, x3, st);
    clk_end(CLK_FUSED, st);
    mark(ev, 3, st);
    go = GemmOut{-f.splits, f.splits};   // negative: partials without a GEMM 2 epilogue, even for one split
  } else {
    const bool x3 = prec == FFK_BF16X3;
    o.Xh = t->Xch.get(); o.XTh = src->XcTh.get();
    if (x3) {
      o.Xl = t->Xcl.get(); o.XTl = src->XcTl.get();
      o.Ul = b.Ul; o.UTl = b.UTl;
      o.dAl = cs.dA_lo.get();
      o.Wl = b.Wl;
      go = mvm_gemms_for<bf16_t, true, float>(a, Ntr, Nsr, Dk, Dr, o, st, ev);
    } else {
      go = mvm_gemms_for<bf16_t, false, float>(a, Ntr, Nsr, Dk, Dr, o, st, ev);
    }
  }
  mark(ev, 4, st);
  const int tb = M <= 64 ? 64 : 128;
  const size_t shj = (3 * M + D + 1) * sizeof(double);
  const double* xm = t->xmean.as<double>();
  clk_begin(CLK_JTG, st);
  if (go.splits < 0)
    launch_jtg_reduce(N, D, shj, st, static_cast<const float*>(b.part), -go.splits, N, b.s, t->Xc.as<double>(), xm,
                      b.wpart, go.ntn, t->a0, t->R.as<double>(), v, shift, M, D, y, vy_part);
  else if (go.splits == 1)
    k_jtg<<<N, tb, shj, st>>>(t->R.as<double>(), b.G, t->X.as<double>(), v, shift, M, D, y, 0, vy_part);
  else if (prec == FFK_FP64)
    launch_jtg_reduce(N, D, shj, st, static_cast<const double*>(b.part), go.splits, N, b.s, t->Xc.as<double>(), xm,
                      b.wpart, go.ntn, t->a0, t->R.as<double>(), v, shift, M, D, y, vy_part);
  else
    launch_jtg_reduce(N, D, shj, st, static_cast<const float*>(b.part), go.splits, N, b.s, t->Xc.as<double>(), xm,
                      b.wpart, go.ntn, t->a0, t->R.as<double>(), v, shift, M, D, y, vy_part);
  LAUNCHCHK();
  clk_end(CLK_JTG, st);
  mark(ev, 5, st);
}

// The symmetrized product, sum_q K(R, P_q R) (Pi_q v), as one product against
// the stacked permuted copies: v is permuted into the stacked vector, the
// sources are the N S stacked geometries.
__global__ void k_permute_stack(const double* __restrict__ v, const int32_t* __restrict__ perms, int S, int64_t N,
                                int M, double* __restrict__ out) {
  const int64_t n = N * 3 * M;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * S) return;
  const int64_t q = e / n, r = e % n;
  const int64_t g = r / (3 * M);
  const int loc = (int)(r % (3 * M));
  out[e] = v[g * 3 * M + 3 * perms[q * M + loc / 3] + loc % 3];
}

static void stack_mvm(ffk_system* s, const double* v, double* y, double shift, int prec, hipStream_t st,
                      hipEvent_t* ev, double* vy_part) {
  ffk_system* src = s->stack.get();
  const int S = (int)s->sym.size();
  ensure_coeffs_pair(s, src, s->stack_coef, prec, (int64_t)s->sym_identity * s->N, st);
  ensure_lowp_descriptor(s, prec, st);
  ensure_lowp_descriptor(src, prec, st);
  ensure_work(s->stack_work, src, s->N, s->D, prec, st);
  if (!s->stack_v) s->stack_v.alloc(src->n * 8);
  k_permute_stack<<<cdiv(src->n, 256), 256, 0, st>>>(v, s->sym_perm.as<int32_t>(), S, s->N, s->M,
                                                      s->stack_v.as<double>());
  LAUNCHCHK();
  kernel_mvm_core(s, src, s->stack_coef, s->stack_v.as<double>(), v, y, shift, prec, st, ev, vy_part,
                  handle_bufs(s->stack_work, prec));
}

void kernel_mvm_ev(ffk_system* s, const double* v, double* y, double shift, int prec, hipStream_t st,
                   hipEvent_t* ev, double* vy_part = nullptr) {
  require(prec >= FFK_FP64 && prec <= FFK_BF16X3, "kernel_mvm: unknown precision");
  if (!s->sym.empty()) {
    stack_mvm(s, v, y, shift, prec, st, ev, vy_part);
    return;
  }
  ensure_coeffs(s, prec, st);
  ensure_lowp_descriptor(s, prec, st);
  ensure_work(s->work, s, s->N, s->D, prec, st);
  kernel_mvm_core(s, s, s->coef, v, v, y, shift, prec, st, ev, vy_part, handle_bufs(s->work, prec));
}

// ------------------------------------------------- caller-free workspace ----
// Zero fill of n bytes (n a multiple of 16) with 16-byte stores: a kernel
// rather than a memset node, so that the whole product stays kernels.
__global__ void k_zero16(uint4* __restrict__ p, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

static void zero_fill(void* p, size_t bytes, hipStream_t st) {
  const int64_t n16 = (int64_t)(bytes / 16);
  const int blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n16 + 255) / 256));
  k_zero16<<<blocks, 256, 0, st>>>(static_cast<uint4*>(p), n16);
  LAUNCHCHK();
}

// Carve the workspace of one product out of [base, base + cap): the fixed
// buffers first (256-byte aligned), then the split-K partials with what is
// left, capped at the budget the handle path uses.  Returns the bytes the
// fixed buffers and one split need (the smallest workable cap); *b is set
// only when that fits.
static size_t carve_bufs(const ffk_system* s, int prec, char* base, size_t cap, MvmBufs* b) {
  const int64_t N = s->N, D = s->D;
  const int64_t Nr = pad_rows(N), Dk = rup(D, 64), Dr = pad_rows(D);
  const size_t es = prec == FFK_FP64 ? 8 : prec == FFK_FP32 ? 4 : 2;   // operand element size
  const size_t ps = prec == FFK_FP64 ? 8 : 4;                            // split-K partial element size
  const bool two = prec == FFK_BF16 || prec == FFK_BF16X3;               // hi and lo arrays
  size_t off = 0;
  auto take = [&](size_t bytes) -> size_t {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  const bool fused = use_fused(prec, D, N, N);   // no -W buffers
  const size_t o_pd = take(Nr * 8), o_s = take(D * 8), o_sp = take((size_t)cdiv(N, jv_group(N)) * D * 8);
  const size_t o_G = take(N * D * 8), o_wp = take(N * (Nr / 64) * 8);
  const size_t o_U = take(Nr * Dk * es), o_Ul = two ? take(Nr * Dk * es) : 0;
  const int64_t KV = fused ? 2 * Nr : Nr;   // K of the transposed operand (interleaved when fused)
  const size_t o_UT = take(Dr * KV * es), o_UTl = two ? take(Dr * KV * es) : 0;
  const size_t o_W = fused ? 0 : take(Nr * Nr * es), o_Wl = two && !fused ? take(Nr * Nr * es) : 0;
  const size_t o_part = off;
  const size_t need = o_part + N * D * ps;
  if (need > cap || !b) return need;
  *b = MvmBufs{reinterpret_cast<double*>(base + o_pd), reinterpret_cast<double*>(base + o_s),
               reinterpret_cast<double*>(base + o_sp), reinterpret_cast<double*>(base + o_G),
               reinterpret_cast<double*>(base + o_wp), base + o_part,
               std::min(cap - o_part, part_budget(N, D)),
               base + o_U, two ? base + o_Ul : nullptr, base + o_UT, two ? base + o_UTl : nullptr,
               fused ? nullptr : base + o_W, two && !fused ? base + o_Wl : nullptr};
  return need;
}

void kernel_mvm_scratch(ffk_system* s, const double* v, double* y, double shift, int prec, hipStream_t st,
                        void* base, size_t cap) {
  require(prec >= FFK_FP64 && prec <= FFK_BF16X3, "kernel_mvm_noalloc: unknown precision");
  require(s->sym.empty(), "kernel_mvm_noalloc: a symmetrized kernel is not supported");
  const bool prepared = s->coef[prec].ready && s->coef[FFK_FP64].ready &&
                        (prec == FFK_FP64   ? (bool)s->Xp64
                         : prec == FFK_FP32 ? (bool)s->Xp32
                                            : (bool)s->Xch && (prec == FFK_BF16 || use_fused(prec, s->D, s->N, s->N) ||
                                                               (bool)s->coef[prec].dA_lo));
  require(prepared, "kernel_mvm_noalloc: the system's coefficients for this precision are not built yet "
                    "(one ffk_kernel_mvm in this precision builds them)");
  MvmBufs b{};
  const size_t need = carve_bufs(s, prec, static_cast<char*>(base), cap, &b);
  if (need > cap) {
    char msg[192];
    snprintf(msg, sizeof(msg), "kernel_mvm_noalloc: the product at N = %lld, D = %lld needs %zu bytes of scratch, "
             "more than the %zu available", (long long)s->N, (long long)s->D, need, cap);
    fail(FFK_ERR_ARG, msg);
  }
  // every call shares the scratch: clear the operand padding that the
  // GEMMs read (U and its transpose; -W in FP64, whose epilogue writes only
  // the valid part; pd past the sources, which the fused product reads)
  const int64_t Nr = pad_rows(s->N), Dk = rup(s->D, 64), Dr = pad_rows(s->D);
  const size_t es = prec == FFK_FP64 ? 8 : prec == FFK_FP32 ? 4 : 2;
  const bool fused = use_fused(prec, s->D, s->N, s->N);
  const int64_t KV = fused ? 2 * Nr : Nr;
  zero_fill(b.pd, Nr * 8, st);
  zero_fill(b.U, Nr * Dk * es, st);
  zero_fill(b.UT, Dr * KV * es, st);
  if (b.Ul) zero_fill(b.Ul, Nr * Dk * es, st);
  if (b.UTl) zero_fill(b.UTl, Dr * KV * es, st);
  if (fused)
    fused_fill_x(s->Xc.as<double>(), s->N, s->D, Dr, Nr, static_cast<bf16_t*>(b.UT), static_cast<bf16_t*>(b.UTl),
                 st);
  if (prec == FFK_FP64) zero_fill(b.Wh, Nr * Nr * es, st);
  ClockPause pause;   // the library's clocks would create events
  kernel_mvm_core(s, s, s->coef, v, v, y, shift, prec, st, nullptr, nullptr, b);
}

void kernel_mvm(ffk_system* s, const double* v, double* y, double shift, int prec, hipStream_t st) {
  kernel_mvm_ev(s, v, y, shift, prec, st, nullptr);
}

// The product, plus the per-geometry partials of v^T y in vy_part (N doubles),
// summed in a fixed order by the caller.  Returns the number of partials
// written (N).
int kernel_mvm_vy(ffk_system* s, const double* v, double* y, double shift, int prec, hipStream_t st,
                  double* vy_part) {
  kernel_mvm_ev(s, v, y, shift, prec, st, nullptr, vy_part);
  return (int)s->N;
}

// Average time of each phase over `iters` products: [J v (+ copies, column
// partials), column-sum reduction, GEMM 1 + W epilogue, GEMM 2 + G epilogue
// (+ split-K reduction), J^T G].
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

void center_with(ffk_system* sys, const double* mean, hipStream_t st) {
  k_center_with<<<(unsigned)sys->N, 256, 0, st>>>(sys->X.as<double>(), mean, sys->D, sys->Xc.as<double>(),
                                                  sys->sqn.as<double>());
  LAUNCHCHK();
}

// y (+)= K(tgt, src) alpha on the scalar FP64 engine (rectangular: targets
// and sources are different systems of the same molecule).  The target
// descriptors are centred with the source mean (the kernel depends on
// differences only).  With a cache, the coefficients of the pair and the
// workspaces are kept for the next call with the same target.
void rect_mvm(const ffk_system* tr, const ffk_system* te, const double* alpha, double* F, bool accumulate,
              const double* shift_v, double shift, RectCache* cache, hipStream_t st) {
  require(tr->M == te->M, "kernel product: the two systems differ in molecule size");
  require(tr->sigma == te->sigma, "kernel product: sigma differs");
  const int64_t Ns = tr->N, Nt = te->N, D = tr->D;
  const int M = tr->M;
  const int nblk = cdiv(Ns, jv_group(Ns));
  const int ntn = cdiv(Ns, 128);
  RectCache local;
  RectCache& c = cache ? *cache : local;
  if (!cache || c.tgt != te) {
    c.tgt = nullptr;
    c.U.alloc(Ns * D * 8);
    c.pd.alloc(Ns * 8);
    c.sv.alloc(D * 8);
    c.cpart.alloc((int64_t)nblk * D * 8);
    c.Xt.alloc(Nt * D * 8);
    c.sqt.alloc(Nt * 8);
    c.dA.alloc(Nt * Ns * 8);
    c.B.alloc(Nt * Ns * 8);
    c.Wn.alloc(Nt * Ns * 8);
    c.wpart.alloc(Nt * ntn * 8);
    c.G.alloc(Nt * D * 8);
    c.part.alloc(part_budget(Nt, D));
    k_center_with<<<Nt, 256, 0, st>>>(te->X.as<double>(), tr->xmean.as<double>(), D, c.Xt.as<double>(),
                                      c.sqt.as<double>());
    LAUNCHCHK();
    ScalarArgs<double> g{};
    g.M = (int)Nt;
    g.N = (int)Ns;
    g.nseg = 1;
    g.seg[0] = SegS<double>{c.Xt.as<double>(), D, 1, tr->Xc.as<double>(), D, 1, (int)D};
    EpiCoeffRect e{c.sqt.as<double>(), tr->sqn.as<double>(), c.dA.as<double>(), c.B.as<double>(), (int)Nt,
                   (int)Ns, sqrt(5.0) / tr->sigma, tr->a0, tr->bcoef};
    gemm_scalar_kernel<double, 128, 128, 16, true, true, EpiCoeffRect><<<dim3(ntn, cdiv(Nt, 128)), 256, 0, st>>>(g, e);
    LAUNCHCHK();
    if (cache) c.tgt = te;
  }
  launch_jv<0>(Ns, M, st, tr->R.as<double>(), tr->pairs.as<int>(), alpha, tr->Xc.as<double>(), Ns, M, D, c.U.get(),
               nullptr, D, nullptr, nullptr, (int64_t)0, c.pd.as<double>(), c.cpart.as<double>());
  LAUNCHCHK();
  k_colsum_final<<<cdiv(D, 4), 256, 0, st>>>(c.cpart.as<double>(), nblk, D, c.sv.as<double>());
  LAUNCHCHK();
  MvmArgs a{Nt, Ns, D, tr->a0, c.Xt.as<double>(), c.pd.as<double>(), c.sv.as<double>(), c.wpart.as<double>(),
            c.G.as<double>(), c.part.get(), c.part.bytes()};
  mvm_gemms_scalar<double>(a, c.Xt.as<double>(), tr->Xc.as<double>(), c.U.as<double>(), c.dA.as<double>(),
                           c.B.as<double>(), c.Wn.as<double>(), st, nullptr);
  const int tb = M <= 64 ? 64 : 128;
  k_jtg<<<Nt, tb, (3 * M + D) * sizeof(double), st>>>(te->R.as<double>(), c.G.as<double>(), te->X.as<double>(),
                                                      shift_v, shift, M, D, F, accumulate ? 1 : 0);
  LAUNCHCHK();
  if (!cache) HIPCHK(hipStreamSynchronize(st));   // the temporaries are freed on return
}

// F = K(test, train) alpha; a symmetrized training system predicts with
// sum_q K(test, train_q) (Pi_q alpha), train_q its permuted copies
void kernel_predict(const ffk_system* tr, const ffk_system* te, const double* alpha, double* F, hipStream_t st) {
  if (tr->sym.empty()) {
    rect_mvm(tr, te, alpha, F, false, nullptr, 0.0, nullptr, st);
    return;
  }
  DBuf aq(tr->n * 8);
  const int M = tr->M;
  for (size_t q = 0; q < tr->sym.size(); ++q) {
    permute_atoms(alpha, tr->sym_perm.as<int32_t>() + q * M, tr->N, M, aq.as<double>(), st);
    rect_mvm(tr->sym[q].get(), te, aq.as<double>(), F, q > 0, nullptr, 0.0, nullptr, st);
  }
  HIPCHK(hipStreamSynchronize(st));
}

}  // namespace ffk
