// MFMA GEMM engines for gfx950.
//
// Both engines compute a BM x BN tile of  acc = sum_k A(m, k) B(n, k)  (an
// "A B^T" product) with 256 threads = 4 wave64s in a 2 x 2 arrangement; each
// wave owns a (BM/2) x (BN/2) sub-tile made of 16 x 16 MFMA blocks.  Operand
// lane layout (all three instructions): lane l supplies row l%16 and the
// K-slice l/16.  Output lane layout: lane l, register v holds column l%16 and
// row 4*(l/16) + v for the FP32-output instructions, but row 4*v + l/16 for
// v_mfma_f64_16x16x4_f64.
// After the K loop the engine hands the accumulators to an epilogue functor,
// which does all stores (and any fused elementwise work and row reductions).
//
// ScalarEngine<T>: T = double (v_mfma_f64_16x16x4_f64) or float
//   (v_mfma_f32_16x16x4_f32).  One operand element per lane per instruction, so
//   operands may be K-contiguous or M-contiguous strided views; LDS tiles are
//   stored [k][m] with 16 elements of padding per row.  Bounds are checked.
//
// Bf16Engine: v_mfma_f32_16x16x32_bf16, FP32 accumulation, optional split
//   mode (X3) that adds hi*hi + hi*lo + lo*hi.  Operands are K-contiguous bf16
//   arrays whose row count is padded to a multiple of BM (or BN) and whose
//   leading dimension is padded to a multiple of BK with zeros, so tiles are
//   loaded with unpredicated 16-byte vectors.  LDS tiles are [m][k] with 8
//   elements of row padding, which makes the 16-byte operand reads of one
//   16-lane group hit distinct banks.
#pragma once

#include "common.hpp"

namespace ffk {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma16;
template <> struct Mfma16<double> {
  typedef d4 acc_t;
  __device__ static inline acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma16<float> {
  typedef f4 acc_t;
  __device__ static inline acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

__device__ inline f4 mfma_bf16(u4 a, u4 b, f4 c) {
  bf8 av = __builtin_bit_cast(bf8, a);
  bf8 bv = __builtin_bit_cast(bf8, b);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
}

// Coordinates of accumulator element (tm, tn, v) for this lane, relative to the tile.
struct FragCoord {
  int wm0, wn0, lane;   // absolute origin of this wave's sub-tile
  int m0, n0;           // absolute origin of the block tile
  bool f64;             // FP64 MFMA output layout
  int tn;               // tile column index (n0 / BN)
  int wcol, nwcol;      // this wave's column index among the block's wave columns
  int split;            // K-split index of the block (which partial it writes)
  __device__ inline int row(int tm, int v) const {
    return wm0 + tm * 16 + (f64 ? 4 * v + (lane >> 4) : 4 * (lane >> 4) + v);
  }
  __device__ inline int col(int tn) const { return wn0 + tn * 16 + (lane & 15); }
};

// Operand segment of a scalar GEMM: element (m, k) at p[m*s0 + k*s1].  The
// stored type TI may be narrower than the compute type (float -> double is exact).
template <typename TI> struct SegS {
  const TI* A; int64_t sa0, sa1;
  const TI* B; int64_t sb0, sb1;
  int K;
};

template <typename TI> struct ScalarArgs {
  int M, N;
  int nseg;
  SegS<TI> seg[2];
  bool lower_only;   // skip tiles whose columns all exceed their rows
  bool a_lower;      // A(m, k) = 0 for k > m (restricts the K range per tile)
};

// ---------------------------------------------------------------------------
// Scalar-operand MFMA engine (FP64 / FP32)
// ---------------------------------------------------------------------------
// Conversion of a stored operand element to the compute type; bf16_t is the
// raw 16-bit pattern of a bfloat16, not an integer.
template <typename T, typename TI> __device__ inline T to_compute(TI x) { return (T)x; }
template <> __device__ inline double to_compute<double, bf16_t>(bf16_t x) { return (double)bf2f(x); }
template <> __device__ inline float to_compute<float, bf16_t>(bf16_t x) { return bf2f(x); }

template <typename T, int BM, int BN, int BK, bool AKC, bool BKC, class Epi, typename TI = T>
__global__ __launch_bounds__(256) void gemm_scalar_kernel(ScalarArgs<TI> g, Epi epi) {
  constexpr int PAD = 16;
  constexpr int EA = BM * BK / 256;
  constexpr int EB = BN * BK / 256;
  constexpr int TM = BM / 32;   // 16x16 blocks per wave along M
  constexpr int TN = BN / 32;
  typedef typename Mfma16<T>::acc_t acc_t;
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  if (g.lower_only && n0 > m0 + BM - 1) return;
  const int wm0 = (wave >> 1) * (BM / 2), wn0 = (wave & 1) * (BN / 2);

  // tiles of every segment, walked as one sequence
  int kend0 = g.seg[0].K;
  if (g.a_lower) kend0 = min(kend0, m0 + BM);
  const int t0 = (kend0 + BK - 1) / BK;
  const int t1 = g.nseg > 1 ? (g.seg[1].K + BK - 1) / BK : 0;
  const int T_ = t0 + t1;

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  T ra[EA], rb[EB];
  auto load = [&](int t) {
    const SegS<TI>& s = (t < t0) ? g.seg[0] : g.seg[1];
    const bool tri = g.a_lower && t < t0;
    const int k0 = (t < t0 ? t : t - t0) * BK;
    const int Kl = (t < t0) ? kend0 : s.K;
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      const int e = tid + 256 * i;
      const int mm = AKC ? e / BK : e % BM;
      const int kk = AKC ? e % BK : e / BM;
      const int m = m0 + mm, k = k0 + kk;
      ra[i] = (m < g.M && k < Kl && !(tri && k > m)) ? to_compute<T>(s.A[(int64_t)m * s.sa0 + (int64_t)k * s.sa1]) : T(0);
    }
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int e = tid + 256 * i;
      const int nn = BKC ? e / BK : e % BN;
      const int kk = BKC ? e % BK : e / BN;
      const int n = n0 + nn, k = k0 + kk;
      rb[i] = (n < g.N && k < Kl) ? to_compute<T>(s.B[(int64_t)n * s.sb0 + (int64_t)k * s.sb1]) : T(0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      const int e = tid + 256 * i;
      const int mm = AKC ? e / BK : e % BM;
      const int kk = AKC ? e % BK : e / BM;
      As[buf][kk][mm] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      const int e = tid + 256 * i;
      const int nn = BKC ? e / BK : e % BN;
      const int kk = BKC ? e % BK : e / BN;
      Bs[buf][kk][nn] = rb[i];
    }
  };

  // split-K: block z of gridDim.z takes a contiguous range of the tiles
  const int tb = (int)((int64_t)T_ * blockIdx.z / gridDim.z);
  const int te = (int)((int64_t)T_ * (blockIdx.z + 1) / gridDim.z);
  if (te > tb) {
    load(tb);
    store(0);
  }
  __syncthreads();
  for (int t = tb; t < te; ++t) {
    const int buf = (t - tb) & 1;
    if (t + 1 < te) load(t + 1);
#pragma unroll
    for (int k4 = 0; k4 < BK / 4; ++k4) {
      T a[TM], b[TN];
      const int kr = k4 * 4 + (lane >> 4);
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[buf][kr][wm0 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[buf][kr][wn0 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = Mfma16<T>::run(a[i], b[j], acc[i][j]);
    }
    if (t + 1 < te) store(buf ^ 1);
    __syncthreads();
  }
  FragCoord fc{m0 + wm0, n0 + wn0, lane, m0, n0, sizeof(T) == 8, (int)blockIdx.x, wave & 1, 2, (int)blockIdx.z};
  epi.template run<T, TM, TN>(acc, fc, reinterpret_cast<char*>(&As[0][0][0]));
}

// ---------------------------------------------------------------------------
// BF16 MFMA engine (optionally 3-product split)
// ---------------------------------------------------------------------------
struct SegB {
  const bf16_t *Ah, *Al;   // rows padded to BM multiple, ld multiple of BK
  const bf16_t *Bh, *Bl;
  int64_t lda, ldb;
  int K;                   // multiple of BK (padded)
};
struct Bf16Args {
  int nseg;
  SegB seg[2];
};

template <int BM, int BN, int BK, bool X3, class Epi>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(Bf16Args g, Epi epi) {
  constexpr int PAD = 8;
  constexpr int LDS_ROW = BK + PAD;
  constexpr int VA = BM * BK / 8 / 256;   // 16-byte vectors per thread
  constexpr int VB = BN * BK / 8 / 256;
  constexpr int TM = BM / 32, TN = BN / 32;
  constexpr int NARR = X3 ? 2 : 1;
  __shared__ bf16_t As[NARR][BM * LDS_ROW];
  __shared__ bf16_t Bs[NARR][BN * LDS_ROW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm0 = (wave >> 1) * (BM / 2), wn0 = (wave & 1) * (BN / 2);
  const int t0 = g.seg[0].K / BK;
  const int T_ = t0 + (g.nseg > 1 ? g.seg[1].K / BK : 0);

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0, 0, 0, 0};

  u4 ra[NARR][VA], rb[NARR][VB];
  auto load = [&](int t) {
    const SegB& s = (t < t0) ? g.seg[0] : g.seg[1];
    const int k0 = (t < t0 ? t : t - t0) * BK;
#pragma unroll
    for (int i = 0; i < VA; ++i) {
      const int e = tid + 256 * i;
      const int mm = e / (BK / 8), kv = e % (BK / 8);
      const int64_t off = (int64_t)(m0 + mm) * s.lda + k0 + kv * 8;
      ra[0][i] = *reinterpret_cast<const u4*>(s.Ah + off);
      if (X3) ra[NARR - 1][i] = *reinterpret_cast<const u4*>(s.Al + off);
    }
#pragma unroll
    for (int i = 0; i < VB; ++i) {
      const int e = tid + 256 * i;
      const int nn = e / (BK / 8), kv = e % (BK / 8);
      const int64_t off = (int64_t)(n0 + nn) * s.ldb + k0 + kv * 8;
      rb[0][i] = *reinterpret_cast<const u4*>(s.Bh + off);
      if (X3) rb[NARR - 1][i] = *reinterpret_cast<const u4*>(s.Bl + off);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int h = 0; h < NARR; ++h) {
#pragma unroll
      for (int i = 0; i < VA; ++i) {
        const int e = tid + 256 * i;
        const int mm = e / (BK / 8), kv = e % (BK / 8);
        *reinterpret_cast<u4*>(&As[h][mm * LDS_ROW + kv * 8]) = ra[h][i];
      }
#pragma unroll
      for (int i = 0; i < VB; ++i) {
        const int e = tid + 256 * i;
        const int nn = e / (BK / 8), kv = e % (BK / 8);
        *reinterpret_cast<u4*>(&Bs[h][nn * LDS_ROW + kv * 8]) = rb[h][i];
      }
    }
  };

  const int tb = (int)((int64_t)T_ * blockIdx.z / gridDim.z);
  const int te = (int)((int64_t)T_ * (blockIdx.z + 1) / gridDim.z);
  if (te > tb) {
    load(tb);
    store();
  }
  __syncthreads();
  for (int t = tb; t < te; ++t) {
    if (t + 1 < te) load(t + 1);
#pragma unroll
    for (int kk = 0; kk < BK / 32; ++kk) {
      const int ko = kk * 32 + 8 * (lane >> 4);
      u4 ah[TM], bh[TN];
      u4 al[X3 ? TM : 1], bl[X3 ? TN : 1];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = wm0 + i * 16 + (lane & 15);
        ah[i] = *reinterpret_cast<const u4*>(&As[0][r * LDS_ROW + ko]);
        if (X3) al[i] = *reinterpret_cast<const u4*>(&As[NARR - 1][r * LDS_ROW + ko]);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int r = wn0 + j * 16 + (lane & 15);
        bh[j] = *reinterpret_cast<const u4*>(&Bs[0][r * LDS_ROW + ko]);
        if (X3) bl[j] = *reinterpret_cast<const u4*>(&Bs[NARR - 1][r * LDS_ROW + ko]);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          if (X3) {
            acc[i][j] = mfma_bf16(al[i], bh[j], acc[i][j]);
            acc[i][j] = mfma_bf16(ah[i], bl[X3 ? j : 0], acc[i][j]);
          }
          acc[i][j] = mfma_bf16(ah[i], bh[j], acc[i][j]);
        }
    }
    __syncthreads();
    if (t + 1 < te) {
      store();
      __syncthreads();
    }
  }
  FragCoord fc{m0 + wm0, n0 + wn0, lane, m0, n0, false, (int)blockIdx.x, wave & 1, 2, (int)blockIdx.z};
  epi.template run<float, TM, TN>(acc, fc, reinterpret_cast<char*>(&As[0][0]));
}

// ---------------------------------------------------------------------------
// BF16 MFMA engine, pipelined through direct global->LDS loads (gfx950
// global_load_lds_dwordx4).  Each wave-wide load moves 64 x 16 bytes into 1 KB
// of LDS at base + lane*16, so a 16-row x 32-k operand block is fetched with
// lane L taking row L%16 and 16-byte chunk L/16: exactly the lane layout the
// 16x16x32 MFMA reads, hence every ds_read_b128 of an operand fragment is a
// contiguous, conflict-free 1 KB read and no staging registers are needed.
// S stages of BK = 32 keep S-1 tiles in flight behind the MFMAs.
// ---------------------------------------------------------------------------
// gfx9 s_waitcnt immediate for vmcnt(N): low bits [3:0], high bits [15:14];
// expcnt and lgkmcnt left at "no wait".
template <int N> struct VmCnt {
  static constexpr unsigned v = (unsigned)((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
};

__device__ inline void dma16(const void* g, void* lds_base) {
  __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)g,
                                   (void __attribute__((address_space(3)))*)lds_base, 16, 0, 0);
}

// XCD-aware tile order.  Workgroup w of the grid (x fastest, then y, then z)
// runs on XCD w % 8 as that XCD's (w / 8)-th.  ALL: each XCD gets a
// contiguous range of all (K split, tile) items, whatever their count (the
// tiles of one row of a 79 x 7 grid had gone to seven L2s: split BF16 at M =
// 60, N = 20000, GEMM 1 3.78 -> 3.66 ms and GEMM 2 6.09 -> 5.94 ms; 6% at M =
// 42, N = 5000).  Otherwise the split is blockIdx.z and the tiles of a split
// are remapped only when their count is a multiple of 8 (the FP32 GEMM 2 on
// 128 x 128 tiles, 14 x 158 x splits, measured 17% slower with the general
// remap).  Within a split, tiles are grouped by 8 tile rows, so tiles that
// run together on an XCD share operand rows in its L2.
template <bool ALL>
__device__ inline void tile_coords(int& tm, int& tn, int& tz) {
  const int nt_n = gridDim.x, nt_m = gridDim.y;
  const int T = nt_m * nt_n;
  int lin;
  if constexpr (ALL) {
    const int W = T * (int)gridDim.z;
    const int w = ((int)blockIdx.z * nt_m + (int)blockIdx.y) * nt_n + (int)blockIdx.x;
    const int xcd = w % 8, idx = w / 8, q = W / 8, r = W % 8;
    const int L = (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + idx;
    tz = L / T;
    lin = L % T;
  } else {
    tz = (int)blockIdx.z;
    lin = (int)blockIdx.y * nt_n + (int)blockIdx.x;
    if (T % 8 == 0) lin = (lin % 8) * (T / 8) + lin / 8;
  }
  const int G = 8;
  const int per_group = G * nt_n;
  const int grp = lin / per_group;
  const int first = grp * G;
  const int gsz = min(nt_m - first, G);
  const int in = lin % per_group;
  tm = first + in % gsz;
  tn = in / gsz;
}

// Per element type: what one pair of 16-byte operand fragments (one 64-byte
// K chunk of a 16-row group per lane group) feeds to the matrix cores.
//   bf16:   8 elements, one v_mfma_f32_16x16x32_bf16
//   float:  4 elements, four v_mfma_f32_16x16x4_f32 (instruction j takes
//           element j of every lane: K slot l/16 of instruction j is k = 4(l/16)+j)
//   double: 2 elements, two v_mfma_f64_16x16x4_f64 (k = 2(l/16)+j)
// Every K index is consumed exactly once by A and B alike, so the sum is the
// full dot product whatever the order.
template <typename T> struct DmaMfma;
template <> struct DmaMfma<bf16_t> {
  typedef f4 acc_t;
  typedef float scalar_t;
  static constexpr int SLICES = 1;
  __device__ static inline acc_t slice(const u4& a, const u4& b, acc_t c, int) { return mfma_bf16(a, b, c); }
};
template <> struct DmaMfma<float> {
  typedef f4 acc_t;
  typedef float scalar_t;
  static constexpr int SLICES = 4;
  __device__ static inline acc_t slice(const u4& a, const u4& b, acc_t c, int j) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[j]), __uint_as_float(b[j]), c, 0, 0, 0);
  }
};
template <> struct DmaMfma<double> {
  typedef d4 acc_t;
  typedef double scalar_t;
  static constexpr int SLICES = 2;
  __device__ static inline acc_t slice(const u4& a, const u4& b, acc_t c, int j) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(__hiloint2double((int)a[2 * j + 1], (int)a[2 * j]),
                                                 __hiloint2double((int)b[2 * j + 1], (int)b[2 * j]), c, 0, 0, 0);
  }
};

// Operand segment of the pipelined engine: K-contiguous arrays of T whose row
// count is padded to the tile and whose leading dimension (in elements) and K
// are multiples of 64 bytes; padding is zero.  BF16 operands are in the
// fragment-major layout (frag_off, with K tiles of 32) and ignore lda/ldb.
// The lo arrays are used only in the split-BF16 mode.
struct SegD {
  const void *Ah, *Al;
  const void *Bh, *Bl;
  int64_t lda, ldb;   // elements
  int K;              // elements, multiple of 64 bytes
};
struct DmaArgs {
  int nseg;
  SegD seg[2];
  int lower_only;   // square tiles strictly above the diagonal do nothing (symmetric products)
};

// Tile shape of the pipelined engine: BM x BN block tile computed by WM x WN
// waves (each (BM/WM) x (BN/WN)), S pipeline stages.
template <int BM_, int BN_, int WM_, int WN_, int S_>
struct DmaTile {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, S = S_;
  static constexpr int NT = 64 * WM * WN;
};

template <typename T, class TL, bool X3, class Epi>
__global__ __launch_bounds__(TL::NT) void gemm_dma_kernel(DmaArgs g, Epi epi) {
  static_assert(!X3 || sizeof(T) == 2, "the split mode is for bf16 operands");
  constexpr int BM = TL::BM, BN = TL::BN, WM = TL::WM, WN = TL::WN, S = TL::S, NW = WM * WN;
  constexpr int BK = 64 / (int)sizeof(T);               // one 64-byte chunk of each row per K tile
  constexpr int NARR = X3 ? 2 : 1;
  constexpr int GROUP_BYTES = 1024;                     // 16 rows x 64 bytes
  constexpr int GA = BM / 16, GB = BN / 16;             // row groups per operand tile
  static_assert(GA % NW == 0 && GB % NW == 0, "row groups must split evenly over the waves");
  constexpr int A_BYTES = GA * GROUP_BYTES;
  constexpr int B_BYTES = GB * GROUP_BYTES;
  constexpr int STAGE_BYTES = NARR * (A_BYTES + B_BYTES);
  constexpr int QA = GA / NW, QB = GB / NW;             // groups loaded per wave
  constexpr int LPT = NARR * (QA + QB);                 // wave-wide loads per tile per wave
  static_assert(LPT * (S > 2 ? S - 2 : 0) < 64, "vmcnt holds at most 63 loads in flight");
  constexpr int TM = BM / WM / 16, TN = BN / WN / 16;   // 16x16 blocks per wave
  typedef typename DmaMfma<T>::acc_t acc_t;
  __shared__ __attribute__((aligned(1024))) char smem[S * STAGE_BYTES];

  // BF16 operands: the wave index in a scalar register, so every operand
  // address is a scalar base plus the lane's offset (228 rather than 252
  // VGPRs on the split 256 x 256 tile).  The FP32 and FP64 loops are left as
  // they were measured.
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = sizeof(T) == 2 ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid >> 6;
  int tmi, tni, tzi;
  tile_coords<X3 && TM * TN >= 32>(tmi, tni, tzi);
  if (g.lower_only && tni > tmi) return;
  const int m0 = tmi * BM, n0 = tni * BN;
  const int wm = wave / WN, wn = wave % WN;
  const int t0 = g.seg[0].K / BK;
  const int T_ = t0 + (g.nseg > 1 ? g.seg[1].K / BK : 0);
  const int tb = (int)((int64_t)T_ * tzi / gridDim.z);
  const int te = (int)((int64_t)T_ * (tzi + 1) / gridDim.z);

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  // Row-major operands (FP32, FP64): lane L of a group load takes row L%16,
  // 16-byte chunk L/16.  BF16 operands are fragment-major (frag_off): the
  // 1 KB block of a (row group, K tile) is contiguous, lane L takes bytes
  // 16 L .. 16 L + 15, and whole cache lines move per load.
  constexpr bool FRAG = sizeof(T) == 2;
  const int lrow = lane & 15, lchunk = lane >> 4;
  auto issue = [&](int t) {
    const SegD& sg = (t < t0) ? g.seg[0] : g.seg[1];
    const int64_t tk = (t < t0 ? t : t - t0);
    const int64_t k0 = tk * BK + lchunk * (16 / (int)sizeof(T));
    const int64_t KT = sg.K / BK;
    char* st = smem + (t % S) * STAGE_BYTES;
#pragma unroll
    for (int h = 0; h < NARR; ++h) {
      const T* A = static_cast<const T*>(h ? sg.Al : sg.Ah);
      const T* B = static_cast<const T*>(h ? sg.Bl : sg.Bh);
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        const int grp = wave * QA + q;
        const T* src = FRAG ? A + (((int64_t)(m0 / 16 + grp) * KT + tk) * 512 + lane * 8)
                            : A + (int64_t)(m0 + grp * 16 + lrow) * sg.lda + k0;
        dma16(src, st + h * A_BYTES + grp * GROUP_BYTES);
      }
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int grp = wave * QB + q;
        const T* src = FRAG ? B + (((int64_t)(n0 / 16 + grp) * KT + tk) * 512 + lane * 8)
                            : B + (int64_t)(n0 + grp * 16 + lrow) * sg.ldb + k0;
        dma16(src, st + NARR * A_BYTES + h * B_BYTES + grp * GROUP_BYTES);
      }
    }
  };

#pragma unroll
  for (int s = 0; s < S - 1; ++s)
    if (tb + s < te) issue(tb + s);
  for (int t = tb; t < te; ++t) {
    // this wave's loads of tile t have landed; the barrier (without the
    // memory fence of __syncthreads, which would drain every load in flight)
    // makes that true for all waves and frees the stage written next
    if (S > 2 && t + S - 2 < te) __builtin_amdgcn_s_waitcnt(VmCnt<LPT * (S > 2 ? S - 2 : 0)>::v);
    else __builtin_amdgcn_s_waitcnt(VmCnt<0>::v);
    asm volatile("s_barrier" ::: "memory");
    if (t + S - 1 < te) issue(t + S - 1);
    const char* st = smem + (t % S) * STAGE_BYTES;
    u4 ah[TM], bh[TN], al[X3 ? TM : 1], bl[X3 ? TN : 1];
    if constexpr (X3 && TM * TN >= 32) {
      // split BF16 on large wave tiles: the hi fragments, then the hi*hi
      // products with the lo fragment reads slotted between them (two MFMAs,
      // one LDS read), so the lo reads run while the matrix cores work.  At
      // M = 60, N = 20000 on 256 x 256 tiles: GEMM 2 6.45 -> 6.22 ms, GEMM 1
      // 4.01 -> 3.89 ms; issuing the lo reads right after the hi ones (one
      // wait for all) gained nothing.
#pragma unroll
      for (int j = 0; j < TN; ++j)
        bh[j] = *reinterpret_cast<const u4*>(st + NARR * A_BYTES + (wn * TN + j) * GROUP_BYTES + lane * 16);
#pragma unroll
      for (int i = 0; i < TM; ++i) ah[i] = *reinterpret_cast<const u4*>(st + (wm * TM + i) * GROUP_BYTES + lane * 16);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = DmaMfma<T>::slice(ah[i], bh[j], acc[i][j], 0);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        bl[j] = *reinterpret_cast<const u4*>(st + NARR * A_BYTES + B_BYTES + (wn * TN + j) * GROUP_BYTES + lane * 16);
#pragma unroll
      for (int i = 0; i < TM; ++i)
        al[i] = *reinterpret_cast<const u4*>(st + A_BYTES + (wm * TM + i) * GROUP_BYTES + lane * 16);
#pragma unroll
      for (int g = 0; g < TM + TN; ++g) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);   // two MFMAs
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
      }
      __builtin_amdgcn_sched_group_barrier(0x008, TM * TN - 2 * (TM + TN), 0);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = DmaMfma<T>::slice(ah[i], bl[j], acc[i][j], 0);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = DmaMfma<T>::slice(al[i], bh[j], acc[i][j], 0);
      continue;
    }

#pragma unroll
    for (int i = 0; i < TM; ++i) {
      ah[i] = *reinterpret_cast<const u4*>(st + (wm * TM + i) * GROUP_BYTES + lane * 16);
      if (X3) al[X3 ? i : 0] = *reinterpret_cast<const u4*>(st + A_BYTES + (wm * TM + i) * GROUP_BYTES + lane * 16);
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      bh[j] = *reinterpret_cast<const u4*>(st + NARR * A_BYTES + (wn * TN + j) * GROUP_BYTES + lane * 16);
      if (X3) bl[X3 ? j : 0] = *reinterpret_cast<const u4*>(st + NARR * A_BYTES + B_BYTES + (wn * TN + j) * GROUP_BYTES + lane * 16);
    }
    // all fragment reads are issued before the first MFMA: left to itself the
    // scheduler interleaves them in pairs, each behind a full LDS-latency wait
    __builtin_amdgcn_sched_barrier(0);
    // FP64: slice-outer order, so consecutive instructions update different
    // accumulators (measured faster); FP32 and BF16: block-outer order
    if (sizeof(T) != 8) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int sl = 0; sl < DmaMfma<T>::SLICES; ++sl) {
            if (X3) {
              acc[i][j] = DmaMfma<T>::slice(al[X3 ? i : 0], bh[j], acc[i][j], sl);
              acc[i][j] = DmaMfma<T>::slice(ah[i], bl[X3 ? j : 0], acc[i][j], sl);
            }
            acc[i][j] = DmaMfma<T>::slice(ah[i], bh[j], acc[i][j], sl);
          }
    } else
#pragma unroll
    for (int sl = 0; sl < DmaMfma<T>::SLICES; ++sl) {
      if (X3) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = DmaMfma<T>::slice(al[X3 ? i : 0], bh[j], acc[i][j], sl);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = DmaMfma<T>::slice(ah[i], bl[X3 ? j : 0], acc[i][j], sl);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = DmaMfma<T>::slice(ah[i], bh[j], acc[i][j], sl);
    }
  }
  __syncthreads();
  FragCoord fc{m0 + wm * (BM / WM), n0 + wn * (BN / WN), lane, m0, n0, sizeof(T) == 8, tni, wn, WN, tzi};
  epi.template run<typename DmaMfma<T>::scalar_t, TM, TN>(acc, fc, smem);
}

// Shared LDS for epilogues that need it: the engines pass their operand LDS
// after the final barrier of the K loop.

// ---------------------------------------------------------------------------
// Generic epilogue: C(m, n) = alpha * acc + beta * C(m, n) on a strided view.
// ---------------------------------------------------------------------------
template <typename CT> struct EpiAxpby {
  CT* C;
  int64_t scm, scn;
  int M, N;
  double alpha, beta;
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
            CT* p = C + (int64_t)r * scm + (int64_t)c * scn;
            const double val = alpha * (double)acc[i][j][v];
            *p = (CT)(beta == 0.0 ? val : val + beta * (double)*p);
          }
        }
  }
};

// Split-K partial store: part[(z * rows + r) * ldp + c] = acc for r < rows, c < cols.
template <typename PT> struct EpiPart {
  PT* part;
  int64_t ldp;
  int rows, cols;
  template <typename T, int TM, int TN, class Acc>
  __device__ void run(const Acc (&acc)[TM][TN], const FragCoord& f, char*) const {
    PT* base = part + (int64_t)f.split * rows * ldp;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = f.row(i, v), c = f.col(j);
          if (r < rows && c < cols) base[(int64_t)r * ldp + c] = (PT)acc[i][j][v];
        }
  }
};

// Number of K splits that brings a GEMM with `tiles` output tiles to >=
// `target` workgroups while keeping at least two K tiles per split.
inline int pick_splits(int64_t tiles, int64_t ktiles, int64_t target = 512) {
  int s = 1;
  while (tiles * s < target && (int64_t)s * 4 <= ktiles) s *= 2;
  return s;
}

}  // namespace ffk
