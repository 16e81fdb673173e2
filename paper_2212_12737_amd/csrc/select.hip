// Inducing-column selection (section 3, "Column selection strategies").
//
//  * uniform: the k columns with the largest SplitMix64 draws u_i (stream 0);
//  * weighted (leverage / scores): Efraimidis-Spirakis keys log(u_i)/w_i, k largest;
//    the ordering is (key descending, index ascending), done by a bitonic sort;
//  * pivoted (incomplete) Cholesky, Algorithm 1: greedy pivot on the largest
//    remaining diagonal of the Schur complement; each step evaluates one kernel
//    column, subtracts the Schur correction L[:, :m] L[pivot, :m]^T (a GEMV
//    over the column-major factor, coalesced thread-per-row), scales by the
//    pivot and updates the diagonal; the argmax for the next step is fused
//    into the same pass;
//  * leverage: ridge-leverage estimates from a uniform pilot set S0,
//    tau_i = (K_ii - K_iS0 (K_S0S0 + lambda I)^-1 K_S0i) / lambda, obtained as
//    (K_ii - |row i of L0|^2)/lambda with L0 the incomplete Cholesky factor of
//    K + lambda I in the pilot order; clipped to [1e-12, 1], pilot columns 1.
#include "common.hpp"

namespace ffk {

constexpr double kWeightFloor = 1e-12;

__device__ inline bool before(double ka, int ia, double kb, int ib) {
  return ka > kb || (ka == kb && ia < ib);
}

__global__ void k_keys_uniform(int64_t n, int64_t P, uint64_t seed, int stream, double* key, int* idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  key[i] = i < n ? uniform01_at(seed, (uint64_t)stream, (uint64_t)i) : -INFINITY;
  idx[i] = i < n ? (int)i : 0x7FFFFFFF;
}

__global__ void k_keys_weighted(int64_t n, int64_t P, const double* w, uint64_t seed, int stream, double* key,
                                int* idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  if (i < n) {
    const double u = uniform01_at(seed, (uint64_t)stream, (uint64_t)i);
    key[i] = log(u) / fmax(w[i], kWeightFloor);
    idx[i] = (int)i;
  } else {
    key[i] = -INFINITY;
    idx[i] = 0x7FFFFFFF;
  }
}

// One global bitonic compare-exchange step (size kk, distance j).
__global__ void k_bitonic_global(double* key, int* idx, int64_t P, int64_t kk, int64_t j) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const int64_t l = i ^ j;
  if (l <= i) return;
  const bool up = (i & kk) == 0;
  const double ki = key[i], kl = key[l];
  const int ii = idx[i], il = idx[l];
  const bool swap = up ? before(kl, il, ki, ii) : before(ki, ii, kl, il);
  if (swap) {
    key[i] = kl; key[l] = ki;
    idx[i] = il; idx[l] = ii;
  }
}

// All steps with distance <= 256 of stage kk, inside 512-element blocks.
__global__ __launch_bounds__(256) void k_bitonic_shared(double* key, int* idx, int64_t kk, int64_t jmax) {
  __shared__ double sk[512];
  __shared__ int si[512];
  const int64_t base = (int64_t)blockIdx.x * 512;
  const int t = threadIdx.x;
  sk[t] = key[base + t];
  si[t] = idx[base + t];
  sk[t + 256] = key[base + t + 256];
  si[t + 256] = idx[base + t + 256];
  __syncthreads();
  for (int64_t j = jmax; j > 0; j >>= 1) {
    const int a = (int)((t / j) * 2 * j + (t % j));   // lower element of the pair
    const int b = a + (int)j;
    const bool up = ((base + a) & kk) == 0;
    const double ka = sk[a], kb = sk[b];
    const int ia = si[a], ib = si[b];
    const bool swap = up ? before(kb, ib, ka, ia) : before(ka, ia, kb, ib);
    if (swap) {
      sk[a] = kb; sk[b] = ka;
      si[a] = ib; si[b] = ia;
    }
    __syncthreads();
  }
  key[base + t] = sk[t];
  idx[base + t] = si[t];
  key[base + t + 256] = sk[t + 256];
  idx[base + t + 256] = si[t + 256];
}

__global__ void k_take(const int* idx, int64_t k, int64_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) out[i] = idx[i];
}

static int64_t pow2_at_least(int64_t n) {
  int64_t p = 512;
  while (p < n) p <<= 1;
  return p;
}

static void bitonic_sort(double* key, int* idx, int64_t P, hipStream_t st) {
  for (int64_t kk = 2; kk <= P; kk <<= 1) {
    int64_t j = kk >> 1;
    for (; j > 256; j >>= 1) {
      k_bitonic_global<<<cdiv(P, 256), 256, 0, st>>>(key, idx, P, kk, j);
      LAUNCHCHK();
    }
    k_bitonic_shared<<<(unsigned)(P / 512), 256, 0, st>>>(key, idx, kk, j);
    LAUNCHCHK();
  }
}

static void topk_from_keys(int64_t n, int64_t k, DBuf& key, DBuf& idx, int64_t P, int64_t* out, hipStream_t st) {
  bitonic_sort(key.as<double>(), idx.as<int>(), P, st);
  k_take<<<cdiv(k, 256), 256, 0, st>>>(idx.as<int>(), k, out);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));
}

void select_uniform_n(int64_t n, int64_t k, uint64_t seed, int stream, int64_t* out, hipStream_t st) {
  const int64_t P = pow2_at_least(n);
  DBuf key(P * 8), idx(P * 4);
  k_keys_uniform<<<cdiv(P, 256), 256, 0, st>>>(n, P, seed, stream, key.as<double>(), idx.as<int>());
  LAUNCHCHK();
  topk_from_keys(n, k, key, idx, P, out, st);
}

void select_uniform(const ffk_system* s, int64_t k, uint64_t seed, int64_t* out, hipStream_t st) {
  select_uniform_n(s->n, k, seed, 0, out, st);
}

void select_weighted(int64_t n, const double* w, int64_t k, uint64_t seed, int stream, int64_t* out,
                     hipStream_t st) {
  const int64_t P = pow2_at_least(n);
  DBuf key(P * 8), idx(P * 4);
  k_keys_weighted<<<cdiv(P, 256), 256, 0, st>>>(n, P, w, seed, stream, key.as<double>(), idx.as<int>());
  LAUNCHCHK();
  topk_from_keys(n, k, key, idx, P, out, st);
}

// ---------------------------------------------------------- pivoted ICD ----
struct Cand {
  double v;
  int i;
};
__device__ inline Cand better(Cand a, Cand b) { return before(a.v, a.i, b.v, b.i) ? a : b; }

__device__ inline Cand block_best(Cand c, Cand* sh) {
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = better(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  return sh[0];
}

// First argmax partials over the initial diagonal.
__global__ __launch_bounds__(256) void k_argmax_part(const double* d, int64_t n, Cand* part) {
  __shared__ Cand sh[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  Cand c{-INFINITY, 0x7FFFFFFF};
  if (i < n) c = Cand{d[i], (int)i};
  c = block_best(c, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = c;
}

// Combine partials; choose pivot m or stop; gather row pivot of L[:, :m].
__global__ __launch_bounds__(256) void k_pivot(const Cand* part, int np, int64_t m, double thr, int64_t* piv,
                                               double* pivval, int* stop, int* keff, const double* L, int64_t n,
                                               double* vbuf) {
  __shared__ Cand sh[256];
  __shared__ int go;
  Cand c{-INFINITY, 0x7FFFFFFF};
  for (int e = threadIdx.x; e < np; e += 256) c = better(c, part[e]);
  c = block_best(c, sh);
  if (threadIdx.x == 0) {
    go = 0;
    if (*stop == 0) {
      if (c.i == 0x7FFFFFFF || !(c.v > thr)) {
        *stop = 1;
      } else {
        piv[m] = c.i;
        *pivval = sqrt(c.v);
        *keff = (int)(m + 1);
        go = 1;
      }
    }
  }
  __syncthreads();
  if (!go) return;
  const int64_t p = c.i;
  for (int64_t j = threadIdx.x; j < m; j += 256) vbuf[j] = L[p + j * n];
}

// Column m of L from the raw kernel column stored there; diagonal update and
// argmax partials for the next step.
__global__ __launch_bounds__(256) void k_pivchol_update(double* L, int64_t n, int64_t m, const double* vbuf,
                                                        const double* pivval, const int64_t* piv,
                                                        unsigned char* sel, double* d, const int* stop,
                                                        Cand* part) {
  constexpr int CH = 2048;
  __shared__ double sv[CH];
  __shared__ Cand sh[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool halted = *stop != 0;   // same value for the whole grid
  Cand c{-INFINITY, 0x7FFFFFFF};
  if (halted) {
    if (i < n) L[i + m * n] = 0.0;
  } else {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int64_t j0 = 0; j0 < m; j0 += CH) {   // Schur correction L[i, :m] . L[pivot, :m]
      const int64_t jn = m - j0 < CH ? m - j0 : CH;
      __syncthreads();
      for (int64_t j = threadIdx.x; j < jn; j += 256) sv[j] = vbuf[j0 + j];
      __syncthreads();
      if (i < n) {
        const double* Li = L + i + j0 * n;
        int64_t j = 0;
        for (; j + 4 <= jn; j += 4) {
          s0 += Li[j * n] * sv[j];
          s1 += Li[(j + 1) * n] * sv[j + 1];
          s2 += Li[(j + 2) * n] * sv[j + 2];
          s3 += Li[(j + 3) * n] * sv[j + 3];
        }
        for (; j < jn; ++j) s0 += Li[j * n] * sv[j];
      }
    }
    if (i < n) {
      const int64_t p = piv[m];
      const double pv = *pivval;
      const double schur = (s0 + s1) + (s2 + s3);
      double l;
      if (i == p) {
        l = pv;
        sel[i] = 1;
      } else if (sel[i]) {
        l = 0.0;
      } else {
        l = (L[i + m * n] - schur) / pv;
        const double dn = d[i] - l * l;
        d[i] = dn;
        c = Cand{dn, (int)i};
      }
      L[i + m * n] = l;
    }
  }
  c = block_best(c, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = c;
}

int64_t select_pivchol(ffk_system* s, int64_t k, int64_t* idx_out, hipStream_t st) {
  const int64_t n = s->n;
  const double thr = 1e-12 * max_diag(s, st);
  DBuf L(n * k * 8), d(n * 8), sel(n), piv(k * 8), vbuf(std::max<int64_t>(k, 1) * 8), scal(64);
  const int np = cdiv(n, 256);
  DBuf part(np * sizeof(Cand));
  HIPCHK(hipMemsetAsync(sel.get(), 0, n, st));
  HIPCHK(hipMemsetAsync(piv.get(), 0, k * 8, st));
  HIPCHK(hipMemsetAsync(scal.get(), 0, 64, st));
  double* pivval = scal.as<double>();
  int* stop = reinterpret_cast<int*>(scal.as<char>() + 8);
  int* keff = reinterpret_cast<int*>(scal.as<char>() + 12);
  kernel_diag(s, d.as<double>(), st);
  k_argmax_part<<<np, 256, 0, st>>>(d.as<double>(), n, part.as<Cand>());
  LAUNCHCHK();
  int hstop = 0;
  for (int64_t m = 0; m < k; ++m) {
    k_pivot<<<1, 256, 0, st>>>(part.as<Cand>(), np, m, thr, piv.as<int64_t>(), pivval, stop, keff,
                               L.as<double>(), n, vbuf.as<double>());
    LAUNCHCHK();
    kernel_columns(s, piv.as<int64_t>() + m, 1, L.as<double>() + m * n, n, 0.0, st);
    k_pivchol_update<<<np, 256, 0, st>>>(L.as<double>(), n, m, vbuf.as<double>(), pivval,
                                                          piv.as<int64_t>(), sel.as<unsigned char>(),
                                                          d.as<double>(), stop, part.as<Cand>());
    LAUNCHCHK();
    if ((m & 31) == 31) {
      HIPCHK(hipMemcpyAsync(&hstop, stop, 4, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (hstop) break;
    }
  }
  int hk = 0;
  HIPCHK(hipMemcpyAsync(&hk, keff, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hk > 0) HIPCHK(hipMemcpyAsync(idx_out, piv.get(), hk * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return hk;
}

// ------------------------------------------------------------- leverage ----
__global__ void k_leverage(const double* L0, int64_t n, int64_t s, const double* diag, double lambda,
                           const unsigned char* pilot, double* tau) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a0 = 0.0, a1 = 0.0;
  int64_t j = 0;
  for (; j + 2 <= s; j += 2) {
    const double x0 = L0[i + j * n], x1 = L0[i + (j + 1) * n];
    a0 += x0 * x0;
    a1 += x1 * x1;
  }
  for (; j < s; ++j) a0 += L0[i + j * n] * L0[i + j * n];
  double t = (diag[i] - (a0 + a1)) / lambda;
  if (pilot[i]) t = 1.0;
  tau[i] = fmin(fmax(t, kWeightFloor), 1.0);
}

__global__ void k_expand_scores(const double* geom, int64_t n, int m3, double* w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = fmax(geom[i / m3], kWeightFloor);
}

void expand_scores(const double* geom, int64_t N, int M, double* w, hipStream_t st) {
  const int64_t n = N * 3 * M;
  k_expand_scores<<<cdiv(n, 256), 256, 0, st>>>(geom, n, 3 * M, w);
  LAUNCHCHK();
}

__global__ void k_mark(const int64_t* idx, int64_t k, unsigned char* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) flag[idx[i]] = 1;
}

void leverage_estimate(ffk_system* s, const int64_t* pilot, int64_t ns, double lambda, double* tau,
                       hipStream_t st) {
  const int64_t n = s->n;
  DBuf L0(n * ns * 8), diag(n * 8), flag(n);
  HIPCHK(hipMemsetAsync(L0.get(), 0, n * ns * 8, st));
  std::vector<char> kept;
  icd_forced(s, pilot, ns, lambda, L0.as<double>(), n, &kept, st);
  kernel_diag(s, diag.as<double>(), st);
  HIPCHK(hipMemsetAsync(flag.get(), 0, n, st));
  k_mark<<<cdiv(ns, 256), 256, 0, st>>>(pilot, ns, flag.as<unsigned char>());
  LAUNCHCHK();
  k_leverage<<<cdiv(n, 256), 256, 0, st>>>(L0.as<double>(), n, ns, diag.as<double>(), lambda,
                                           flag.as<unsigned char>(), tau);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));
}

}  // namespace ffk
