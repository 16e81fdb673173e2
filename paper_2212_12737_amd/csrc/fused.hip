// Fused kernel product for short descriptors in BF16 and split BF16 (where it
// was measured faster: D <= 96, and D <= 128 up to N_t N_s = 4096^2).
//
// The product's two dense steps (the block structure of Sec. 2.1 rewritten
// over geometry pairs, see mvm.hip):
//   P  = X_c U^T,   W = B o (P - 1 pd^T)              (step A, K = D)
//   G  = dA U - W X_c  (+ a(0) 1 s^T + diag(w) X_c)   (step C, K = sources)
// run here in one kernel, so the N x N matrix W never reaches HBM.  For
// short descriptors the two-GEMM form is bound by HBM: it writes -W (hi and lo) and
// reads it back, 8 bytes per geometry pair on top of the 8 of the
// coefficients B and dA; fused, only the coefficients stream.
//
// A workgroup takes 64 target geometries (16 per wave) and a range of
// sources, in chunks of 16 sources:
//  * step A: the transposed tile P^T (16 sources x 16 targets per group) on
//    v_mfma_f32_16x16x32_bf16, with U (the chunk's rows) from LDS and the
//    wave's target descriptors held in registers for the whole range;
//  * the W epilogue in registers: lane l holds sources 4(l/16) .. +3 of
//    target l%16, which is the operand layout of step C if each lane's eight
//    K slots carry four sources of dA followed by the same four sources of
//    -W.  The B operand then carries U^T and X_c^T of those four sources: an
//    interleaved copy [U^T | X_c^T] (U^T written there by J v, X_c^T once per
//    workspace) makes that one 16-byte fragment, as in the GEMM engine;
//  * step C: the wave's G rows (16 targets x D per group) accumulate in
//    registers over the whole source range.
// Every operand of a chunk goes global -> LDS by DMA (three stages): U,
// [U^T | X_c^T], the coefficients in blocks laid out for this kernel (dA hi
// and lo, B: each lane's 16 bytes where its MFMA operands want them) and pd;
// every LDS read is a 16-byte vector at 16 x lane (read as double2, pd made
// the compiler wait for all DMA in flight before it).  Three stages; a stage
// is 34 KB at D = 128.
//
// Where it pays: the two-GEMM form moves about 16 bytes per geometry pair
// (B, dA, -W written and read) plus its operand panels; the fused form moves
// the 8 bytes of B and dA plus the chunk operands once per 64 targets, which
// grows with D (about 41 bytes per pair at D = 210).  Measured on MI355X,
// split BF16 product, fused against two GEMMs: N = 2000, D = 36, 66, 120:
// 37, 45, 54 us against 54, 58, 61; N = 10000: D = 36 331 against 611 us,
// D = 120 733 against 676, D = 210 1159 against 790.
// Each workgroup writes its partial G rows and row sums of W; the
// split-K reduction and J^T G follow in k_jtg_reduce, as after GEMM 2.
#include "gemm.hpp"

namespace ffk {

template <int N> __device__ inline void wait_vm() { __builtin_amdgcn_s_waitcnt(VmCnt<N>::v); }

__device__ inline uint32_t pack_bf16(bf16_t a, bf16_t b) { return (uint32_t)a | ((uint32_t)b << 16); }

// c ? x : y on values (a conditional between two lvalues would select their
// addresses and keep the variables in memory)
template <typename T> __device__ inline T pick(bool c, T x, T y) { return c ? x : y; }

template <int KD, bool X3>
__global__ __launch_bounds__(256) void k_fused_mvm(FusedArgs a) {
  constexpr int NARR = X3 ? 2 : 1;
  constexpr int DB = 2 * KD;               // 16-wide column groups of G
  constexpr int NU = NARR * KD;            // loads of the chunk's U rows (K tiles of d; hi, lo)
  constexpr int NV = NARR * DB;            // loads of the chunk's K tile of V (per column group; hi, lo)
  constexpr int NC = 8;                    // coefficient blocks: [dA] and [B] of the 4 target groups
  constexpr int NLD = NU + NV + NC + 2;    // + pd of the chunk's sources (two slots)
  constexpr int STAGE = NLD * 1024;        // one 1 KB slot per load
  constexpr int LW = (NLD + 3) / 4;        // loads per wave per chunk
  // three stages (deeper pipelines, four to six stages at these widths,
  // measured slower: 498 against 346 us at D = 36, N = 10000)
  constexpr int S = 3;
  static_assert((S - 2) * LW <= 63, "pipeline depth");
  __shared__ __attribute__((aligned(1024))) char smem[S * STAGE];

  const int lane = threadIdx.x & 63;
  // the wave index as a scalar: the load schedule below depends on it
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int q = lane >> 4, r = lane & 15;
  // consecutive workgroups go to different XCDs: with the split index
  // fastest, the workgroups of one source range share an XCD when the split
  // count is a multiple of 8
  const int z = blockIdx.x % a.splits;
  const int rb = blockIdx.x / a.splits;
  const int cb = (int)((int64_t)a.nchunks * z / a.splits);
  const int ce = (int)((int64_t)a.nchunks * (z + 1) / a.splits);
  const int tg = rb * 4 + wave;             // this wave's group of 16 targets
  const int tw = 16 * tg;

  // DMA of a chunk's operands into a stage, load i into slot i: U blocks
  // (K tile of d; hi, then lo), V blocks (column group; hi, then lo), the
  // coefficient blocks ([dA hi | lo] and [B] of target groups 4 rb .. +3),
  // pd.  Every wave issues LW loads per chunk (a wave whose share is one
  // short repeats its previous load: same data, same place), so the number
  // of loads behind any point of the loop is fixed.  Addresses are picked
  // without branches.
  const char* const pUh = reinterpret_cast<const char*>(a.Uh);
  const char* const pUl = reinterpret_cast<const char*>(X3 ? a.Ul : a.Uh);
  const char* const pVh = reinterpret_cast<const char*>(a.Vh);
  const char* const pVl = reinterpret_cast<const char*>(X3 ? a.Vl : a.Vh);
  const char* const pCF = reinterpret_cast<const char*>(a.CF);
  const char* const pPD = reinterpret_cast<const char*>(a.pd);
  const int64_t KTd = a.KTd, KTv = 2 * a.KTs, NCH = a.Nsr / 16;
  auto issue = [&](int c, int stage) {
    char* st = smem + stage * STAGE;
#pragma unroll
    for (int j = 0; j < LW; ++j) {
      int i = 4 * j + wave;
      if (i >= NLD) i -= 4;
      const bool isU = i < NU, isV = !isU && i < NU + NV, isC = !isU && !isV && i < NU + NV + NC;
      const int iu = i, iv = i - NU, ic = i - NU - NV, ip = i - NU - NV - NC;
      const bool lu = X3 && iu >= KD, lv = X3 && iv >= DB;
      const char* u = pick(lu, pUl, pUh) + (((int64_t)c * KTd + (lu ? iu - KD : iu)) * 512) * 2;
      const char* v = pick(lv, pVl, pVh) + (((int64_t)(lv ? iv - DB : iv) * KTv + c) * 512) * 2;
      const char* cf = pCF + ((int64_t)(rb * 4 + (ic >> 1)) * NCH + c) * 2048 + (ic & 1) * 1024;
      // pd: slot 0 holds sources 16 c + 4 (l / 16) + 0, 1 at lane l, slot 1 the + 2, 3
      const char* pdp = pPD + (int64_t)c * 128 + (lane >> 4) * 32 + ip * 16 - lane * 16;
      const char* src = pick(isU, u, pick(isV, v, pick(isC, cf, pdp)));
      dma16(src + lane * 16, st + i * 1024);
    }
  };

  // the wave's target descriptors: the B operand of step A for every chunk
  u4 xh[KD], xl[X3 ? KD : 1];
#pragma unroll
  for (int kt = 0; kt < KD; ++kt) {
    const int64_t o = ((int64_t)tg * KTd + kt) * 512 + lane * 8;
    xh[kt] = *reinterpret_cast<const u4*>(a.Xh + o);
    if (X3) xl[kt] = *reinterpret_cast<const u4*>(a.Xl + o);
  }
  // landed before any DMA is issued: the compiler does not count the DMA
  // loads, so a later wait of its own for these registers would drain them all
  wait_vm<0>();

  f4 acc[DB];
#pragma unroll
  for (int j = 0; j < DB; ++j) acc[j] = f4{0, 0, 0, 0};
  double rs = 0.0;

  // Loads in flight at the top of iteration c, oldest first: DMA(c) ..
  // DMA(c + S - 2); DMA(c) goes to stage c % S.  Past the last chunk the
  // loads fetch the last chunk again (into a stage nobody reads any more),
  // so every iteration issues the same loads and (S - 2) LW of them may stay
  // in flight.
  const int last = ce - 1;
  if (cb < ce) {
#pragma unroll
    for (int k = 0; k < S - 1; ++k) issue(min(cb + k, last), (cb + k) % S);
    wait_vm<(S - 2) * LW>();   // DMA(cb)
    for (int c = cb; c < ce; ++c) {
      if (c > cb) wait_vm<(S - 2) * LW>();
      // every wave's DMA of chunk c has landed, and every wave is done with
      // chunk c - 1, whose stage DMA(c + S - 1) overwrites
      asm volatile("s_barrier" ::: "memory");
      issue(min(c + S - 1, last), (c + S - 1) % S);
      const char* st = smem + (c % S) * STAGE;

      // step A: P^T (sources x targets) over the K tiles of d.  All operand
      // reads go out before the first MFMA (one LDS wait, not one per
      // tile); two accumulators keep consecutive MFMAs independent.
      u4 uh[KD], ul[X3 ? KD : 1];
#pragma unroll
      for (int kt = 0; kt < KD; ++kt) {
        uh[kt] = *reinterpret_cast<const u4*>(st + kt * 1024 + lane * 16);
        if (X3) ul[kt] = *reinterpret_cast<const u4*>(st + (KD + kt) * 1024 + lane * 16);
      }
      const char* cst = st + (NU + NV) * 1024;
      const u4 dA = *reinterpret_cast<const u4*>(cst + (2 * wave) * 1024 + lane * 16);
      const f4 bco = *reinterpret_cast<const f4*>(cst + (2 * wave + 1) * 1024 + lane * 16);
      const u4 pda = *reinterpret_cast<const u4*>(cst + NC * 1024 + lane * 16);
      const u4 pdb = *reinterpret_cast<const u4*>(cst + (NC + 1) * 1024 + lane * 16);
      __builtin_amdgcn_sched_barrier(0);
      f4 p0 = f4{0, 0, 0, 0}, p1 = f4{0, 0, 0, 0};
#pragma unroll
      for (int kt = 0; kt < KD; ++kt) {
        f4& pp = (kt & 1) ? p1 : p0;
        pp = mfma_bf16(uh[kt], xh[kt], pp);
        if (X3) {
          pp = mfma_bf16(uh[kt], xl[kt], pp);
          pp = mfma_bf16(ul[kt], xh[kt], pp);
        }
      }
      // W = B o (P - pd) in FP32 (the two-GEMM form's arithmetic), its row
      // sums in FP64, and the A operand of step C: [dA (4 sources) | -W (the
      // same 4)], split into hi and lo
      const float pf[4] = {(float)__hiloint2double((int)pda.y, (int)pda.x), (float)__hiloint2double((int)pda.w, (int)pda.z),
                           (float)__hiloint2double((int)pdb.y, (int)pdb.x), (float)__hiloint2double((int)pdb.w, (int)pdb.z)};
      bf16_t h[4], l[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float w = bco[v] * ((p0[v] + p1[v]) - pf[v]);
        rs += (double)w;
        h[v] = f2bf(-w);
        l[v] = X3 ? f2bf(-w - bf2f(h[v])) : (bf16_t)0;
      }
      const u4 ah = u4{dA.x, dA.y, pack_bf16(h[0], h[1]), pack_bf16(h[2], h[3])};
      const u4 al = u4{dA.z, dA.w, pack_bf16(l[0], l[1]), pack_bf16(l[2], l[3])};
      // step C: G += [dA | -W] [U ; X_c] over the chunk's sources
      const char* vb = st + NU * 1024 + lane * 16;
#pragma unroll
      for (int dg = 0; dg < DB; ++dg) {
        const u4 bh = *reinterpret_cast<const u4*>(vb + dg * 1024);
        acc[dg] = mfma_bf16(ah, bh, acc[dg]);
        if (X3) {
          const u4 bl = *reinterpret_cast<const u4*>(vb + (DB + dg) * 1024);
          acc[dg] = mfma_bf16(ah, bl, acc[dg]);
          acc[dg] = mfma_bf16(al, bh, acc[dg]);
        }
      }
    }
  }
  wait_vm<0>();   // no DMA may still be writing the LDS when the workgroup ends

  // partial G rows (lane: targets 4q + v of the group, column 16 dg + r) and
  // the partial row sums of W (summed over the lane's four source slots)
  float* part = a.part + (int64_t)z * a.Nt * a.D;
#pragma unroll
  for (int dg = 0; dg < DB; ++dg) {
    const int d = 16 * dg + r;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int t = tw + 4 * q + v;
      if (t < a.Nt && d < a.D) part[(int64_t)t * a.D + d] = acc[dg][v];
    }
  }
  double x = rs;
  x += __shfl_xor(x, 16);
  x += __shfl_xor(x, 32);
  const int t = tw + r;
  if (q == 0 && t < a.Nt) a.wpart[(int64_t)t * a.splits + z] = x;
}

// The coefficient blocks of the fused product from the FP64 coefficients
// (rows Nt, columns Ns, leading dimension ld): for target group tg and chunk
// c (16 sources), 2 KB at ((tg Nsr / 16) + c) 2 KB: lane l = 16 q + r (target
// 16 tg + r, sources 16 c + 4 q .. +3) holds dA as four BF16 hi then four lo
// at 16 l, and B as four FP32 at 1024 + 16 l.  Zero outside Nt x Ns.
__global__ void k_fused_coef(const double* __restrict__ dA, const double* __restrict__ B, int64_t Nt, int64_t Ns,
                             int64_t ld, int64_t Ntr, int64_t Nsr, char* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (target, quad of sources)
  if (e >= Ntr * (Nsr / 4)) return;
  const int64_t t = e / (Nsr / 4), s0 = (e % (Nsr / 4)) * 4;
  const int64_t tg = t >> 4, c = s0 >> 4;
  const int l = (int)(((s0 & 15) >> 2) * 16 + (t & 15));
  char* blk = out + (tg * (Nsr / 16) + c) * 2048;
  uint32_t hp[2] = {0, 0}, lp[2] = {0, 0};
  float b[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t s = s0 + v;
    const bool in = t < Nt && s < Ns;
    const float x = in ? (float)dA[t * ld + s] : 0.f;
    const bf16_t h = f2bf(x), lo = f2bf(x - bf2f(h));
    hp[v >> 1] |= (uint32_t)h << (16 * (v & 1));
    lp[v >> 1] |= (uint32_t)lo << (16 * (v & 1));
    b[v] = in ? (float)B[t * ld + s] : 0.f;
  }
  *reinterpret_cast<uint4*>(blk + l * 16) = make_uint4(hp[0], hp[1], lp[0], lp[1]);
  *reinterpret_cast<float4*>(blk + 1024 + l * 16) = make_float4(b[0], b[1], b[2], b[3]);
}

void fused_coef_build(const double* dA, const double* B, int64_t Nt, int64_t Ns, int64_t ld, int64_t Ntr,
                      int64_t Nsr, void* out, hipStream_t st) {
  const int64_t n = Ntr * (Nsr / 4);
  k_fused_coef<<<(unsigned)cdiv(n, 256), 256, 0, st>>>(dA, B, Nt, Ns, ld, Ntr, Nsr, static_cast<char*>(out));
  LAUNCHCHK();
}

// X_c^T slots of the interleaved operand: element (d, 8 (j / 4) + 4 + j % 4)
// = split(X_c[j][d]) for d < Dr, j < Nsr (zero outside Ns x D); 64 x 64 tiles
// through LDS so that both the reads and the writes are coalesced.
__global__ void k_fill_vx(const double* __restrict__ Xc, int64_t Ns, int64_t D, int64_t Dr, int64_t Nsr,
                          bf16_t* __restrict__ Vh, bf16_t* __restrict__ Vl) {
  __shared__ float tile[64][65];
  const int64_t j0 = (int64_t)blockIdx.x * 64, d0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t j = j0 + i, d = d0 + tx;
    tile[i][tx] = (j < Ns && d < D) ? (float)Xc[j * D + d] : 0.f;
  }
  __syncthreads();
  const int64_t KT = 2 * Nsr / 32;
  for (int i = ty; i < 64; i += 4) {
    const int64_t d = d0 + i, j = j0 + tx;
    if (d < Dr && j < Nsr) {
      const float x = tile[tx][i];
      const bf16_t h = f2bf(x);
      const int64_t o = frag_off(d, 8 * (j >> 2) + 4 + (j & 3), KT);
      Vh[o] = h;
      Vl[o] = f2bf(x - bf2f(h));
    }
  }
}

void fused_fill_x(const double* Xc, int64_t Ns, int64_t D, int64_t Dr, int64_t Nsr, bf16_t* Vh, bf16_t* Vl,
                  hipStream_t st) {
  k_fill_vx<<<dim3((unsigned)cdiv(Nsr, 64), (unsigned)cdiv(Dr, 64)), 256, 0, st>>>(Xc, Ns, D, Dr, Nsr, Vh, Vl);
  LAUNCHCHK();
}

// Split count of the fused product from a cost model: rounds of
// workgroups (64 targets each, one per CU) over the CUs times the chunks per
// split, plus the partials each split adds (written and read back).
int fused_splits(int64_t Nt, int64_t Ns, int64_t D, int max_splits) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  const int64_t rows = cdiv(Nt, 64);
  const int64_t chunks = cdiv(Ns, 16);
  const int64_t KD = cdiv(D, 32);
  // one chunk: 3 KD split-BF16 MFMA triples per wave, ~50% busy
  const double t_chunk = 3.0 * KD * 3.0 * 16.0 / 2.1e9 / 0.5;
  const double t_part = 2.0 * Nt * D * 4.0 / 4.0e12;
  int best = 1;
  double bt = 0.0;
  for (int s = 1; s <= max_splits && s <= chunks; ++s) {
    const double rounds = (double)((rows * s + cus - 1) / cus);
    const double t = rounds * (double)((chunks + s - 1) / s) * t_chunk + (s > 1 ? s * t_part : 0.0);
    if (s == 1 || t < 0.98 * bt) {
      bt = t;
      best = s;
    }
  }
  return best;
}

template <int KD, bool X3>
static void launch_kd(const FusedArgs& a, int rows, hipStream_t st) {
  k_fused_mvm<KD, X3><<<rows * a.splits, 256, 0, st>>>(a);
}

template <bool X3>
static void launch_x3(const FusedArgs& a, int KD, int rows, hipStream_t st) {
  switch (KD) {
    case 1: launch_kd<1, X3>(a, rows, st); break;
    case 2: launch_kd<2, X3>(a, rows, st); break;
    case 3: launch_kd<3, X3>(a, rows, st); break;
    default: launch_kd<4, X3>(a, rows, st); break;
  }
}

void fused_mvm_launch(const FusedArgs& a, bool x3, hipStream_t st) {
  const int KD = (int)cdiv(a.D, 32);
  require(KD >= 1 && 32 * KD <= kFusedMaxD, "fused product: D out of range");
  require(a.KTd * 32 >= 32 * KD && a.splits >= 1 && a.nchunks * 16 <= a.Nsr, "fused product: operand shapes");
  const int rows = (int)cdiv(a.Nt, 64);
  if (x3) launch_x3<true>(a, KD, rows, st);
  else launch_x3<false>(a, KD, rows, st);
  LAUNCHCHK();
}

}  // namespace ffk
