// Complex64 matrix products: FP32 MFMA tiles and a SIMT kernel for thin shapes.
#include "kernel_util.h"

namespace qflex {
namespace dev {

// =============================================================================================
// Complex64 matrix product (paper, Methods B.2: each pairwise contraction is one matrix
// multiplication after the permutation).
//
// MFMA kernel: WM x WN wavefronts (2x2 for the 64x64 and 128x128 tiles, 4x2 for 256x128), each
// owning a (BM/WM)x(BN/WN) complex block made of 32x32 sub-tiles of v_mfma_f32_32x32x2f32.
// The complex product runs in 4M form on the real instruction: Cr += ar*br + (-ai)*bi,
// Ci += ar*bi + ai*br.  Operand tiles of BK = 16 complex k-values are staged in LDS with k
// contiguous for both operands (rows padded to 144 bytes), double buffered with one barrier
// per k-tile; the global loads of tile t+1 are issued before the MFMAs of tile t and stored to
// LDS before its last k step.  Within a k-tile, lanes 0-31 take k = 0..7 and lanes 32-63 take
// k = 8..15 (the two halves of the instruction's K=2), so each lane reads its operands as
// 16-byte vectors.  The 256x128 tile (one workgroup of 8 wavefronts per compute unit, two per
// SIMD) loads 25% fewer operand bytes per MFMA than 128x128 and runs large products at about
// 0.91 of the FP32 peak, against 0.89.
//
// G3: the same tiles in the 3-multiplication (Gauss) form: P1 += ar*br, P2 += ai*bi,
// P3 += (ar + ai)*(br + bi), then Cr = P1 - P2 and Ci = P3 - P1 - P2.  Three MFMAs per pair of
// complex k instead of four (the sums are two vector adds per operand value), for a third more
// accumulator registers.  Ci loses the accuracy that the cancellation in P3 - P1 - P2 costs:
// its FP32 rounding error is about 1.7 times that of the 4-multiplication form on random data.
// =============================================================================================

// SC: C written through g.om (a separate instantiation, so that the plain epilogue compiles as
// it would alone)
template <bool TA, bool TB, int BM, int BN, int WM = 2, int WN = 2, bool G3 = false,
          bool SC = false>
__global__ void __launch_bounds__(64 * WM * WN) gemm_mfma_kernel(const Gemm g) {
  constexpr int NT = 64 * WM * WN;
  constexpr int BK = 16, LDK = BK + 2;
  constexpr int WTM = BM / WM, WTN = BN / WN;  // wavefront block (complex)
  constexpr int TMI = WTM / 32, TNI = WTN / 32;
  constexpr int AV = BM * BK / 2 / NT, BV = BN * BK / 2 / NT;  // float4 (2 complex) loads per thread
  static_assert(AV * NT == BM * BK / 2 && BV * NT == BN * BK / 2, "tile does not split evenly");
  __shared__ __attribute__((aligned(16))) float2 As[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) float2 Bs[2][BN * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int h = lane >> 5, r = lane & 31;
  const int64_t tiles_n = g.N / BN;
  int64_t tm, tn;
  grouped_tile(blockIdx.x, g.M / BM, tiles_n, tm, tn);
  const int b = blockIdx.y, z = blockIdx.z;
  const float2* __restrict__ A = g.A + g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs) + z * g.a_ks;
  const float2* __restrict__ B = g.B + g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs) + z * g.b_ks;
  // split K: chunk z's partial product goes to the workspace, densely packed
  float2* __restrict__ C = g.split > 1 ? g.ws + ((int64_t)z * g.batch + b) * g.M * g.N
                                       : g.C + b * g.c_bs;
  const int64_t ldc = g.split > 1 ? g.N : g.ldc;
  const int64_t m0 = tm * BM, n0 = tn * BN;

  // An operand stored k-major (B [K][N], or A [K][M]) is transposed while staging: pair e of a
  // tile (2 consecutive columns of one k row) goes to LDS rows 2np and 2np + 1 at column kr.
  // With A stored k-major too, groups of 8 lanes take 8 consecutive pairs of one k row (128
  // contiguous bytes) and the wave's 8 groups 8 consecutive k, for both operands: the 8-byte
  // writes of a wave then spread over the banks (rows of 144 bytes), where a whole wave on one k
  // row put its 64 writes 288 bytes apart, on 8 banks; on (32768^2, 4096) this took the
  // transposed-A product from 162 to 184 TFLOP/s.  With A stored row-major, B keeps whole k
  // rows per wave: the same mapping of B alone cost that product 5% (179 -> 169 TFLOP/s).
  auto t_slot = [](int e, int pairs, int& kr, int& np) {
    static_assert(BK == 16, "16 k rows per tile");
    if (pairs >= 8) {
      kr = (e >> 3) & 15;
      np = (e & 7) + 8 * (e >> 7);
    } else {  // whole k rows per wave: pairs = 0 stands for BN / 2
      const int w = pairs > 0 ? pairs : BN / 2;
      kr = e / w;
      np = e % w;
    }
  };
  auto b_slot = [&](int e, int& kr, int& np) { t_slot(e, TA ? BN / 2 : 0, kr, np); };
  auto a_slot = [&](int e, int& kr, int& mp) { t_slot(e, BM / 2, kr, mp); };
  f32x4 ra[AV], rb[BV];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int e = tid + v * NT;
      if (!TA) {
        const int row = e >> 3, kp = e & 7;
        ra[v] = *reinterpret_cast<const f32x4*>(A + (m0 + row) * g.lda + k0 + 2 * kp);
      } else {
        int kr, mp;
        a_slot(e, kr, mp);
        ra[v] = *reinterpret_cast<const f32x4*>(A + (k0 + kr) * g.lda + m0 + 2 * mp);
      }
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int e = tid + v * NT;
      if (!TB) {
        int kr, np;
        b_slot(e, kr, np);
        rb[v] = *reinterpret_cast<const f32x4*>(B + (k0 + kr) * g.ldb + n0 + 2 * np);
      } else {
        const int row = e >> 3, kp = e & 7;
        rb[v] = *reinterpret_cast<const f32x4*>(B + (n0 + row) * g.ldb + k0 + 2 * kp);
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int e = tid + v * NT;
      if (!TA) {
        const int row = e >> 3, kp = e & 7;
        *reinterpret_cast<f32x4*>(&As[buf][row * LDK + 2 * kp]) = ra[v];
      } else {
        int kr, mp;
        a_slot(e, kr, mp);
        As[buf][(2 * mp) * LDK + kr] = make_float2(ra[v].x, ra[v].y);
        As[buf][(2 * mp + 1) * LDK + kr] = make_float2(ra[v].z, ra[v].w);
      }
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int e = tid + v * NT;
      if (!TB) {
        int kr, np;
        b_slot(e, kr, np);
        Bs[buf][(2 * np) * LDK + kr] = make_float2(rb[v].x, rb[v].y);
        Bs[buf][(2 * np + 1) * LDK + kr] = make_float2(rb[v].z, rb[v].w);
      } else {
        const int row = e >> 3, kp = e & 7;
        *reinterpret_cast<f32x4*>(&Bs[buf][row * LDK + 2 * kp]) = rb[v];
      }
    }
  };

  // 4M: cr, ci are the real and imaginary parts; 3M: cr, ci, c3 hold P1, P2, P3
  floatx16 cr[TMI][TNI], ci[TMI][TNI], c3[G3 ? TMI : 1][G3 ? TNI : 1];
#pragma unroll
  for (int i = 0; i < TMI; ++i)
#pragma unroll
    for (int j = 0; j < TNI; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) cr[i][j][v] = ci[i][j][v] = 0.f;
  if constexpr (G3) {
#pragma unroll
    for (int i = 0; i < TMI; ++i)
#pragma unroll
      for (int j = 0; j < TNI; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) c3[i][j][v] = 0.f;
  }

  const int nk = (int)(g.K / BK);
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((int64_t)(kt + 1) * BK);
    const float2* as = As[buf];
    const float2* bs = Bs[buf];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      f32x4 af[TMI], bf[TNI];
#pragma unroll
      for (int i = 0; i < TMI; ++i)
        af[i] = *reinterpret_cast<const f32x4*>(
            &as[(wm * WTM + i * 32 + r) * LDK + h * 8 + 2 * s2]);
#pragma unroll
      for (int j = 0; j < TNI; ++j)
        bf[j] = *reinterpret_cast<const f32x4*>(
            &bs[(wn * WTN + j * 32 + r) * LDK + h * 8 + 2 * s2]);
      if constexpr (G3) {
        // one pass over the sub-tiles per product, so that consecutive MFMAs never feed the
        // same accumulator
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          float ar[TMI], ai[TMI], sa[TMI], br[TNI], bi[TNI], sb[TNI];
#pragma unroll
          for (int i = 0; i < TMI; ++i) {
            ar[i] = u ? af[i].z : af[i].x;
            ai[i] = u ? af[i].w : af[i].y;
            sa[i] = ar[i] + ai[i];
          }
#pragma unroll
          for (int j = 0; j < TNI; ++j) {
            br[j] = u ? bf[j].z : bf[j].x;
            bi[j] = u ? bf[j].w : bf[j].y;
            sb[j] = br[j] + bi[j];
          }
#pragma unroll
          for (int i = 0; i < TMI; ++i)
#pragma unroll
            for (int j = 0; j < TNI; ++j)
              cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[i], br[j], cr[i][j], 0, 0, 0);
#pragma unroll
          for (int i = 0; i < TMI; ++i)
#pragma unroll
            for (int j = 0; j < TNI; ++j)
              ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[i], bi[j], ci[i][j], 0, 0, 0);
#pragma unroll
          for (int i = 0; i < TMI; ++i)
#pragma unroll
            for (int j = 0; j < TNI; ++j)
              c3[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[i], sb[j], c3[i][j], 0, 0, 0);
        }
      } else {
        // the two terms of each part are issued in separate passes over the sub-tiles, so that
        // consecutive MFMAs never feed the same accumulator
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#pragma unroll
          for (int pass = 0; pass < 2; ++pass)
#pragma unroll
            for (int i = 0; i < TMI; ++i) {
              const float ar = u ? af[i].z : af[i].x;
              const float ai = u ? af[i].w : af[i].y;
#pragma unroll
              for (int j = 0; j < TNI; ++j) {
                const float br = u ? bf[j].z : bf[j].x;
                const float bi = u ? bf[j].w : bf[j].y;
                if (pass == 0) {
                  cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, cr[i][j], 0, 0, 0);
                  ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi, ci[i][j], 0, 0, 0);
                } else {
                  cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai, bi, cr[i][j], 0, 0, 0);
                  ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, br, ci[i][j], 0, 0, 0);
                }
              }
            }
        }
      }
      // the next tile goes to the other buffer while this one still has a k step to go, so
      // its LDS writes overlap MFMAs instead of sitting between the last MFMA and the barrier
      if (s2 == 2 && kt + 1 < nk) sstore(buf ^ 1);
    }
    __syncthreads();
  }
  // D layout of the 32x32 instruction: lane -> column r, register v -> row 8*(v/4)+4*h+(v%4)
  if constexpr (SC) {
    // C through its bit-deposit maps: the tile's row and column offsets, computed once into
    // the LDS that the k loop no longer reads (its last barrier has passed)
    int32_t* roff = reinterpret_cast<int32_t*>(&As[0][0]);
    int32_t* coff = roff + BM;
    for (int t = tid; t < BM + BN; t += NT) {
      const bool row = t < BM;
      const int64_t v = row ? m0 + t : n0 + (t - BM);
      const int8_t* pos = row ? g.om.mpos : g.om.npos;
      const int nb = row ? g.om.nm : g.om.nn;
      int32_t o = 0;
      for (int i = 0; i < nb; ++i) o |= (int32_t)((v >> i) & 1) << pos[i];
      if (row) roff[t] = o;
      else coff[t - BM] = o;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TMI; ++i)
#pragma unroll
      for (int j = 0; j < TNI; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = wm * WTM + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
          const int col = wn * WTN + j * 32 + r;
          float re = cr[i][j][v], im = ci[i][j][v];
          if constexpr (G3) re = cr[i][j][v] - ci[i][j][v], im = c3[i][j][v] - cr[i][j][v] - ci[i][j][v];
          C[roff[row] + coff[col]] = make_float2(re, im);
        }
    return;
  }
#pragma unroll
  for (int i = 0; i < TMI; ++i)
#pragma unroll
    for (int j = 0; j < TNI; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wm * WTM + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        const int col = wn * WTN + j * 32 + r;
        float re = cr[i][j][v], im = ci[i][j][v];
        if constexpr (G3) re = cr[i][j][v] - ci[i][j][v], im = c3[i][j][v] - cr[i][j][v] - ci[i][j][v];
        C[(m0 + row) * ldc + n0 + col] = make_float2(re, im);
      }
}

// SIMT fallback for shapes too small or thin for MFMA tiles: BM x BN outputs per workgroup,
// one per thread, k-tiles of 16 staged through LDS with bounds checks on every dimension.
template <int BM, int BN, bool TA, bool TB>
__global__ void __launch_bounds__(256) gemm_simt_kernel(const Gemm g) {
  static_assert(BM * BN == 256, "one output per thread");
  constexpr int BK = 16;
  __shared__ float2 As[BM][BK + 1];
  __shared__ float2 Bs[BK][BN + 1];
  const int tid = threadIdx.x;
  const int64_t tiles_n = (g.N + BN - 1) / BN;
  const int64_t m0 = (int64_t)(blockIdx.x / tiles_n) * BM, n0 = (int64_t)(blockIdx.x % tiles_n) * BN;
  const int b = blockIdx.y, z = blockIdx.z;
  const float2* A = g.A + g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs) + z * g.a_ks;
  const float2* B = g.B + g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs) + z * g.b_ks;
  float2* C = g.split > 1 ? g.ws + ((int64_t)z * g.batch + b) * g.M * g.N : g.C + b * g.c_bs;
  const int64_t ldc = g.split > 1 ? g.N : g.ldc;
  const int tm = tid / BN, tn = tid % BN;
  float accr = 0.f, acci = 0.f;
  for (int64_t k0 = 0; k0 < g.K; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      int mm, kk;
      if (!TA) mm = e / BK, kk = e % BK;
      else kk = e / BM, mm = e % BM;
      const int64_t m = m0 + mm, k = k0 + kk;
      float2 v = make_float2(0.f, 0.f);
      if (m < g.M && k < g.K) v = TA ? A[k * g.lda + m] : A[m * g.lda + k];
      As[mm][kk] = v;
    }
    for (int e = tid; e < BN * BK; e += 256) {
      int nn, kk;
      if (!TB) kk = e / BN, nn = e % BN;
      else nn = e / BK, kk = e % BK;
      const int64_t n = n0 + nn, k = k0 + kk;
      float2 v = make_float2(0.f, 0.f);
      if (n < g.N && k < g.K) v = TB ? B[n * g.ldb + k] : B[k * g.ldb + n];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      const float2 a = As[tm][kk], bb = Bs[kk][tn];
      accr = fmaf(a.x, bb.x, accr);
      accr = fmaf(-a.y, bb.y, accr);
      acci = fmaf(a.x, bb.y, acci);
      acci = fmaf(a.y, bb.x, acci);
    }
    __syncthreads();
  }
  const int64_t m = m0 + tm, n = n0 + tn;
  if (m < g.M && n < g.N) C[m * ldc + n] = make_float2(accr, acci);
}

// Tall-skinny products (M >= 256 rows, N <= 32 columns): one output row per thread, its
// N <= NB complex accumulators in registers.  A k-tile of BK values of 256 rows is staged in
// LDS as [k][row] (so each thread reads its own row without bank conflicts) and B's k-tile
// as [k][NB] (every lane reads the same B values: LDS broadcast).  Such products move far more
// bytes than they compute (HBM-bound), so the loads are 16-byte vectors along the
// contiguous dimension of A, and the next tile's loads are issued before this tile's math.
// BK = 16, or 8 for products whose K is 8.
template <int NB, bool TA, bool TB, int BK = 16>
__global__ void __launch_bounds__(256) gemm_rows_kernel(const Gemm g) {
  constexpr int BM = 256;
  constexpr int KP = BK / 2;             // 16-byte vectors (2 complex) per row of a k-tile
  constexpr int AV = BM * BK / 2 / 256;  // 16-byte (2 complex) loads of A per thread per tile
  static_assert(2 * BK * (BM + 2) >= BM * NB, "the output staging fits the A buffers");
  __shared__ __attribute__((aligned(16))) float2 As[2][BK][BM + 2];
  __shared__ __attribute__((aligned(16))) float2 Bs[2][BK][NB];
  const int tid = threadIdx.x;
  const int b = blockIdx.y, z = blockIdx.z;
  const int64_t m0 = (int64_t)blockIdx.x * BM;
  const float2* __restrict__ A = g.A + g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs) + z * g.a_ks;
  const float2* __restrict__ B = g.B + g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs) + z * g.b_ks;
  float2* __restrict__ C = g.split > 1 ? g.ws + ((int64_t)z * g.batch + b) * g.M * g.N
                                       : g.C + b * g.c_bs;
  const int64_t ldc = g.split > 1 ? g.N : g.ldc;
  const int N = (int)g.N;
  f32x4 ra[AV];
  float2 rb[(BK * NB + 255) / 256];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int e = tid + v * 256;
      if (!TA) {  // [M][K]: KP vectors of 2 k per row
        const int row = e / KP, kp = e % KP;
        ra[v] = *reinterpret_cast<const f32x4*>(A + (m0 + row) * g.lda + k0 + 2 * kp);
      } else {    // [K][M]: 128 vectors of 2 rows per k
        const int kr = e >> 7, mp = e & 127;
        ra[v] = *reinterpret_cast<const f32x4*>(A + (k0 + kr) * g.lda + m0 + 2 * mp);
      }
    }
#pragma unroll
    for (int v = 0; v < (BK * NB + 255) / 256; ++v) {
      const int e = tid + v * 256;
      const int kr = e / NB, n = e % NB;
      float2 x = make_float2(0.f, 0.f);
      if (e < BK * NB && n < N) x = TB ? B[(int64_t)n * g.ldb + k0 + kr] : B[(k0 + kr) * g.ldb + n];
      rb[v] = x;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int e = tid + v * 256;
      if (!TA) {
        const int row = e / KP, kp = e % KP;
        As[buf][2 * kp][row] = make_float2(ra[v].x, ra[v].y);
        As[buf][2 * kp + 1][row] = make_float2(ra[v].z, ra[v].w);
      } else {
        const int kr = e >> 7, mp = e & 127;
        *reinterpret_cast<f32x4*>(&As[buf][kr][2 * mp]) = ra[v];
      }
    }
#pragma unroll
    for (int v = 0; v < (BK * NB + 255) / 256; ++v) {
      const int e = tid + v * 256;
      if (e < BK * NB) Bs[buf][e / NB][e % NB] = rb[v];
    }
  };
  float accr[NB], acci[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) accr[n] = acci[n] = 0.f;
  const int nk = (int)(g.K / BK);
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((int64_t)(kt + 1) * BK);
    // partial unrolling: a full one would hoist all BK x NB values of B into registers
#pragma unroll 2
    for (int kk = 0; kk < BK; ++kk) {
      const float2 a = As[buf][kk][tid];
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        const float2 w = Bs[buf][kk][n];
        accr[n] = fmaf(a.x, w.x, accr[n]);
        accr[n] = fmaf(-a.y, w.y, accr[n]);
        acci[n] = fmaf(a.x, w.y, acci[n]);
        acci[n] = fmaf(a.y, w.x, acci[n]);
      }
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }
  if (ldc == N && N == NB && NB >= 2) {
    // the workgroup's 256 output rows are one contiguous block of 256*NB values: stage it in
    // LDS (the A buffers are free after the last barrier) and write it with 16-byte stores
    float2* stage = &As[0][0][0];  // 256*NB <= 2*BK*258 values
#pragma unroll
    for (int n = 0; n < NB; ++n) stage[tid * NB + ((n + tid) % NB)] = make_float2(accr[n], acci[n]);
    __syncthreads();
    f32x4* out = reinterpret_cast<f32x4*>(C + m0 * ldc);
#pragma unroll
    for (int v = 0; v < NB / 2; ++v) {
      const int e = tid + v * 256;          // pair of values 2e, 2e+1
      const int r0 = (2 * e) / NB, c0 = (2 * e) % NB;  // c0 even, c0 + 1 < NB
      const float2 p0 = stage[r0 * NB + ((c0 + r0) % NB)];
      const float2 p1 = stage[r0 * NB + ((c0 + 1 + r0) % NB)];
      f32x4 w;
      w.x = p0.x;
      w.y = p0.y;
      w.z = p1.x;
      w.w = p1.y;
      out[e] = w;
    }
  } else {
    float2* c = C + (m0 + tid) * ldc;
#pragma unroll
    for (int n = 0; n < NB; ++n)
      if (n < N) c[n] = make_float2(accr[n], acci[n]);
  }
}

// Reduction-shaped products (M <= 32 rows, 4 <= N columns, a long K): C = op(A) B with B
// stored [K][N], as in the cotangent of a product's right operand.  Each thread owns one
// column n of a 256-column tile (NT = min(N, 256) columns, 256 / NT k-subgroups), streams
// B[k][n] from HBM (coalesced along n) and keeps the column's M complex sums in registers;
// A's k-tile ([BK][M], BK = 64 k) is broadcast from LDS.  Subgroups are summed through LDS
// at the end.
template <int MB, bool TA>
__global__ void __launch_bounds__(256) gemm_reduce_kernel(const Gemm g) {
  constexpr int BKMAX = 64;
  __shared__ float2 As[BKMAX][MB];
  __shared__ float2 red[256];
  const int tid = threadIdx.x;
  const int b = blockIdx.y, z = blockIdx.z;
  const int NT = g.N < 256 ? (int)g.N : 256;
  const int nsub = 256 / NT;
  const int BK = BKMAX;  // K is a multiple of 64: 64 / nsub k per thread per tile
  const int col_in = tid % NT, sub = tid / NT;
  const int64_t n0 = (int64_t)blockIdx.x * NT;
  const int M = (int)g.M;
  const float2* __restrict__ A = g.A + g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs) + z * g.a_ks;
  const float2* __restrict__ B = g.B + g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs) + z * g.b_ks;
  float2* __restrict__ C = g.split > 1 ? g.ws + ((int64_t)z * g.batch + b) * g.M * g.N
                                       : g.C + b * g.c_bs;
  const int64_t ldc = g.split > 1 ? g.N : g.ldc;
  float accr[MB], acci[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) accr[m] = acci[m] = 0.f;
  for (int64_t k0 = 0; k0 < g.K; k0 += BK) {
    for (int e = tid; e < BK * MB; e += 256) {
      const int kk = e / MB, m = e % MB;
      float2 v = make_float2(0.f, 0.f);
      if (m < M) v = TA ? A[(k0 + kk) * g.lda + m] : A[(int64_t)m * g.lda + k0 + kk];
      As[kk][m] = v;
    }
    __syncthreads();
    for (int kk = sub; kk < BK; kk += nsub) {
      const float2 w = B[(k0 + kk) * g.ldb + n0 + col_in];
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        const float2 a = As[kk][m];
        accr[m] = fmaf(a.x, w.x, accr[m]);
        accr[m] = fmaf(-a.y, w.y, accr[m]);
        acci[m] = fmaf(a.x, w.y, acci[m]);
        acci[m] = fmaf(a.y, w.x, acci[m]);
      }
    }
    __syncthreads();
  }
  // sum the subgroups' partial columns, one row at a time
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    if (m >= M) break;
    if (nsub == 1) {
      C[m * ldc + n0 + col_in] = make_float2(accr[m], acci[m]);
      continue;
    }
    red[tid] = make_float2(accr[m], acci[m]);
    __syncthreads();
    if (sub == 0) {
      float2 t = red[col_in];
      for (int j = 1; j < nsub; ++j) {
        const float2 u = red[j * NT + col_in];
        t.x += u.x;
        t.y += u.y;
      }
      C[m * ldc + n0 + col_in] = t;
    }
    __syncthreads();
  }
}

// Products with a short K (K < 16) and N >= 32 columns, which write far more than they read:
// each thread owns one output column of a 256-column tile and a set of rows, keeps its
// column of B (K values) in registers, and reads each row of A from LDS (broadcast); the
// stores are coalesced along the row.  SC: C written through g.om (see gemm_mfma_kernel).
template <int KB, bool TA, bool TB, bool SC = false>
__global__ void __launch_bounds__(256) gemm_smallk_kernel(const Gemm g) {
  constexpr int BM = 64;
  __shared__ float2 As[BM][KB];
  const int tid = threadIdx.x;
  const int b = blockIdx.y;
  const int NT = g.N < 256 ? (int)g.N : 256;
  const int64_t tiles_n = g.N / NT;
  const int64_t m0 = (int64_t)(blockIdx.x / tiles_n) * BM;
  const int64_t n0 = (int64_t)(blockIdx.x % tiles_n) * NT;
  const int col_in = tid % NT, rsub = tid / NT, nrs = 256 / NT;
  const int K = (int)g.K;
  const float2* __restrict__ A = g.A + g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs);
  const float2* __restrict__ B = g.B + g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs);
  float2* __restrict__ C = g.C + b * g.c_bs;
  float2 w[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k)
    w[k] = k < K ? (TB ? B[(n0 + col_in) * g.ldb + k] : B[(int64_t)k * g.ldb + n0 + col_in])
                 : make_float2(0.f, 0.f);
  for (int e = tid; e < BM * KB; e += 256) {
    const int r = e / KB, k = e % KB;
    float2 v = make_float2(0.f, 0.f);
    if (m0 + r < g.M && k < K) v = TA ? A[(int64_t)k * g.lda + m0 + r] : A[(m0 + r) * g.lda + k];
    As[r][k] = v;
  }
  // output through the bit-deposit maps: the tile's row offsets in LDS, this thread's column
  // offset in a register
  __shared__ int32_t roff[SC ? BM : 1];
  int32_t coff = 0;
  if constexpr (SC) {
    auto dep = [](int64_t v, const int8_t* pos, int nb) {
      int32_t o = 0;
      for (int i = 0; i < nb; ++i) o |= (int32_t)((v >> i) & 1) << pos[i];
      return o;
    };
    if (tid < BM) roff[tid] = dep(m0 + tid, g.om.mpos, g.om.nm);
    coff = dep(n0 + col_in, g.om.npos, g.om.nn);
  }
  __syncthreads();
  for (int r = rsub; r < BM; r += nrs) {
    if (m0 + r >= g.M) break;
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const float2 a = As[r][k];
      re = fmaf(a.x, w[k].x, re);
      re = fmaf(-a.y, w[k].y, re);
      im = fmaf(a.x, w[k].y, im);
      im = fmaf(a.y, w[k].x, im);
    }
    if constexpr (SC) C[roff[r] + coff] = make_float2(re, im);
    else C[(m0 + r) * g.ldc + n0 + col_in] = make_float2(re, im);
  }
}

static bool pow2_or_256(int64_t n) { return n <= 256 ? (n & (n - 1)) == 0 : n % 256 == 0; }

bool gemm_variant_fits(const Gemm& g, int v) {
  switch (v) {
    case 0: return true;
    case 1: return g.K % 16 == 0 && g.M % 64 == 0 && g.N % 64 == 0;
    case 2: return g.K % 16 == 0 && g.M % 128 == 0 && g.N % 128 == 0;
    case 3: return (g.K % 16 == 0 || (g.K == 8 && g.N <= 16)) && g.M % 256 == 0 && g.N <= 32;
    case 4: return !g.tb && g.M <= 32 && g.N >= 4 && pow2_or_256(g.N) && g.K >= 256 && g.K % 64 == 0;
    case 5: return g.K < 16 && (g.K & (g.K - 1)) == 0 && g.N >= 32 && pow2_or_256(g.N);
    case 6: return g.K % 16 == 0 && g.M % 256 == 0 && g.N % 128 == 0;
    case 7: return !g.tb && g.M <= 16 && g.N % 64 == 0 && g.K >= 256 && g.K % 64 == 0;
    case 8: return g.K % 16 == 0 && g.M % 256 == 0 && g.N <= 16;
    case 9: return gemm_variant_fits(g, 6);
    case 10: return gemm_variant_fits(g, 2);
    default: return false;
  }
}

int gemm_variant(const Gemm& g) {
  if (g.force_variant >= 0 && gemm_variant_fits(g, g.force_variant)) return g.force_variant;
  // the 256x128 tile once its workgroups cover every compute unit (one each: the tile's LDS
  // leaves room for no second); below that, 128x128 tiles give twice as many workgroups
  // (in the 3-multiplication form: three MFMAs per complex multiply-add pair instead of four)
  if (gemm_variant_fits(g, 9) && (g.M / 256) * (g.N / 128) * g.batch >= 256) return 9;
  if (gemm_variant_fits(g, 10)) return 10;
  if (gemm_variant_fits(g, 1)) return 1;
  // rows kernels: one workgroup per 256 rows, so only when that fills half the chip or more;
  // on MFMA for 8 < N <= 16 (at N = 16 the vector kernel is ALU-bound, at N <= 8 it is not)
  if (gemm_variant_fits(g, 8) && g.N > 8 && (g.M / 256) * g.batch >= 128) return 8;
  if (gemm_variant_fits(g, 3) && (g.M / 256) * g.batch >= 128) return 3;
  if (gemm_variant_fits(g, 7)) return 7;  // reduction-shaped, on MFMA
  if (gemm_variant_fits(g, 4)) return 4;  // reduction-shaped
  if (gemm_variant_fits(g, 5)) return 5;  // short K
  return 0;
}

const char* gemm_name(const Gemm& g) {
  if (g.gather) {
    static const char* gnames[4] = {"gemm_rows_mfma_gather_nn", "gemm_rows_mfma_gather_nt",
                                    "gemm_rows_mfma_gather_tn", "gemm_rows_mfma_gather_tt"};
    return gnames[(g.ta ? 2 : 0) + (g.tb ? 1 : 0)];
  }
  static const char* names[kGemmVariants][4] = {
      {"gemm_simt_nn", "gemm_simt_nt", "gemm_simt_tn", "gemm_simt_tt"},
      {"gemm_mfma_64x64_nn", "gemm_mfma_64x64_nt", "gemm_mfma_64x64_tn", "gemm_mfma_64x64_tt"},
      {"gemm_mfma_128x128_nn", "gemm_mfma_128x128_nt", "gemm_mfma_128x128_tn",
       "gemm_mfma_128x128_tt"},
      {"gemm_rows_nn", "gemm_rows_nt", "gemm_rows_tn", "gemm_rows_tt"},
      {"gemm_reduce_nn", "gemm_reduce_nt", "gemm_reduce_tn", "gemm_reduce_tt"},
      {"gemm_smallk_nn", "gemm_smallk_nt", "gemm_smallk_tn", "gemm_smallk_tt"},
      {"gemm_mfma_256x128_nn", "gemm_mfma_256x128_nt", "gemm_mfma_256x128_tn",
       "gemm_mfma_256x128_tt"},
      {"gemm_reduce_mfma_nn", "gemm_reduce_mfma_nt", "gemm_reduce_mfma_tn",
       "gemm_reduce_mfma_tt"},
      {"gemm_rows_mfma_nn", "gemm_rows_mfma_nt", "gemm_rows_mfma_tn", "gemm_rows_mfma_tt"},
      {"gemm_mfma3m_256x128_nn", "gemm_mfma3m_256x128_nt", "gemm_mfma3m_256x128_tn",
       "gemm_mfma3m_256x128_tt"},
      {"gemm_mfma3m_128x128_nn", "gemm_mfma3m_128x128_nt", "gemm_mfma3m_128x128_tn",
       "gemm_mfma3m_128x128_tt"}};
  return names[gemm_variant(g)][(g.ta ? 2 : 0) + (g.tb ? 1 : 0)];
}

// Output tiles of the kernel gemm() picks (one workgroup each, per batch element).
static int64_t gemm_tiles(const Gemm& g) {
  switch (gemm_variant(g)) {
    case 6:
    case 9: return (g.M / 256) * (g.N / 128);
    case 7: return g.N / 64;
    case 8: return g.M / 256;
    case 2:
    case 10: return (g.M / 128) * (g.N / 128);
    case 1: return (g.M / 64) * (g.N / 64);
    case 3: return g.M / 256;
    case 4: return g.N / std::min<int64_t>(g.N, 256);
    case 5: return ((g.M + 63) / 64) * (g.N / std::min<int64_t>(g.N, 256));
    default: {
      const int bn = g.N >= 16 && g.M >= 16 ? 16 : g.N >= 8 ? 8 : g.N >= 4 ? 4 : g.N >= 2 ? 2 : 1;
      const int bm = 256 / bn;
      return ((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
    }
  }
}

// Split K when fewer than ~2048 workgroups would run and every chunk keeps >= 256 k values
// (chunks are a power of two dividing K, so every K tile of 16 stays whole).
int gemm_splitk(const Gemm& g) {
  constexpr int64_t kTarget = 2048, kMinChunk = 256, kMaxSplit = 64;
  // the 256x128 tile is only picked by shape once it fills the chip, one workgroup per unit
  if (gemm_variant(g) == 6 || gemm_variant(g) == 9) return 1;
  const int64_t wgs = gemm_tiles(g) * g.batch;
  if (wgs >= kTarget / 2 || g.K < 2 * kMinChunk || (g.K & (g.K - 1))) return 1;
  int split = 1;
  while (split < kMaxSplit && wgs * split < kTarget && g.K / (2 * split) >= kMinChunk) split *= 2;
  return split;
}

int64_t gemm_splitk_elems(const Gemm& g) {
  const int split = gemm_splitk(g);
  return split > 1 ? (int64_t)split * g.batch * g.M * g.N : 0;
}

// Reduction-shaped products on MFMA (M <= 16 rows, N a multiple of 64, a long K, B stored
// [K][N]): the same products as gemm_reduce_kernel, whose 4 M vector FMAs per element of B
// make it as much an ALU kernel as an HBM one.  Here v_mfma_f32_16x16x4f32 does the
// arithmetic, with A's rows padded to 16 by zeros.  A workgroup owns 64 columns (4 blocks of 16)
// and its 4 wavefronts split K: blocks of 16 k go round robin to the wavefronts.  Per block,
// each lane loads its 4 values of A (row i = lane % 16, k = 4 s + lane / 16) and 16 of B
// (k likewise, column 16 c + lane % 16) straight from HBM; every load instruction of the
// wavefront reads whole 128-byte lines.  The wavefronts' sums meet in LDS and are added in a
// fixed order.
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <bool TA>
__global__ void __launch_bounds__(256) gemm_reduce_mfma_kernel(const Gemm g) {
  __shared__ float red[4][32][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int b = blockIdx.y, z = blockIdx.z;
  const int64_t n0 = (int64_t)blockIdx.x * 64;
  const int M = (int)g.M;
  const float2* __restrict__ A = g.A + g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs) + z * g.a_ks;
  const float2* __restrict__ B =
      g.B + g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs) + z * g.b_ks + n0 + i;
  float2* __restrict__ C = g.split > 1 ? g.ws + ((int64_t)z * g.batch + b) * g.M * g.N
                                       : g.C + b * g.c_bs;
  const int64_t ldc = g.split > 1 ? g.N : g.ldc;
  floatx4 cr[4], ci[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) cr[c] = ci[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int64_t nblk = g.K / 16;
  for (int64_t blk = wave; blk < nblk; blk += 4) {
    const int64_t k0 = blk * 16 + kq;
    float2 a[4], w[4][4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int64_t k = k0 + 4 * st;
      a[st] = make_float2(0.f, 0.f);
      if (i < M) a[st] = TA ? A[k * g.lda + i] : A[(int64_t)i * g.lda + k];
#pragma unroll
      for (int c = 0; c < 4; ++c) w[st][c] = B[k * g.ldb + 16 * c];
    }
#pragma unroll
    for (int st = 0; st < 4; ++st) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        cr[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[st].x, w[st][c].x, cr[c], 0, 0, 0);
        ci[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[st].x, w[st][c].y, ci[c], 0, 0, 0);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        cr[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[st].y, w[st][c].y, cr[c], 0, 0, 0);
        ci[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[st].y, w[st][c].x, ci[c], 0, 0, 0);
      }
    }
  }
  // D layout of the 16x16 instruction: lane -> column lane % 16, register v -> row
  // 4 (lane / 16) + v
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      red[wave][8 * c + v][lane] = cr[c][v];
      red[wave][8 * c + 4 + v][lane] = ci[c][v];
    }
  __syncthreads();
  for (int e = tid; e < 16 * 64; e += 256) {
    const int c = e >> 8, v = (e >> 6) & 3, l = e & 63;
    const int row = 4 * (l >> 4) + v;
    if (row >= M) continue;
    float re = red[0][8 * c + v][l], im = red[0][8 * c + 4 + v][l];
#pragma unroll
    for (int u = 1; u < 4; ++u) {
      re += red[u][8 * c + v][l];
      im += red[u][8 * c + 4 + v][l];
    }
    C[row * ldc + n0 + 16 * c + (l & 15)] = make_float2(re, im);
  }
}

// Tall-skinny products on MFMA (M a multiple of 256, N <= 16, K a multiple of 16): the products
// of gemm_rows_kernel, whose 4 N vector FMAs per element of A cap it below the copy rate at
// N = 16.  Here v_mfma_f32_16x16x4f32 does the arithmetic with B's columns padded to 16 by
// zeros.  Each wavefront owns 64 rows as 4 blocks of 16; per 16 k, lane (q = lane / 16,
// i = lane % 16) holds k = 4 q + s of its rows for instruction s (the order of k within a
// block is free, as long as A and B agree).  A is read straight from HBM in 16-byte vectors:
// [M][K] as 4 consecutive k of one row, [K][M] as 2 consecutive rows of one k (the two rows
// then belong to an even and an odd row block).  B is staged in LDS 64 k at a time.
// GA: A is an intermediate read in its own storage order through g.ga (element (m, k) at
// f(m) + (k & 3) + g(k >> 2)), as [M][K]: the 4 consecutive k a lane loads are 32 contiguous
// bytes, and no permutation pass over A is needed.  GA with TA: A is the transpose of such an
// operand (element (m, k) at f(k) + (m & 3) + g(m >> 2)), as in the cotangent X^T Zbar of a
// product that read X so; the 2 consecutive rows a lane loads are 16 contiguous bytes.  With
// split-K chunks the k index runs on from z times the chunk length.
template <bool TA, bool TB, bool GA = false>
__global__ void __launch_bounds__(256) gemm_rows_mfma_kernel(const Gemm g) {
  constexpr int KC = 64;
  __shared__ float2 Bs[KC][16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 15, q = lane >> 4;
  const int b = blockIdx.y, z = blockIdx.z;
  const int64_t mw = (int64_t)blockIdx.x * 256 + wave * 64;
  const float2* __restrict__ A = g.A + g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs) + z * g.a_ks;
  const float2* __restrict__ B = g.B + g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs) + z * g.b_ks;
  float2* __restrict__ C = g.split > 1 ? g.ws + ((int64_t)z * g.batch + b) * g.M * g.N
                                       : g.C + b * g.c_bs;
  const int64_t ldc = g.split > 1 ? g.N : g.ldc;
  const int N = (int)g.N;
  floatx4 cr[4], ci[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) cr[r] = ci[r] = floatx4{0.f, 0.f, 0.f, 0.f};
  int64_t frow[GA ? 4 : 1];  // gathered A: row offsets plus this lane's k group within 16 k
  const int64_t kz = (int64_t)z * g.K;  // gathered A: first k of this split-K chunk
  if constexpr (GA && TA) {  // offsets of this lane's row pairs, one per h
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t v = (mw + 32 * h + 2 * i) >> 2;
      int64_t f = (v & 1) << g.ga.kpos[0] | ((v >> 1) & 1) << g.ga.kpos[1];
      if (g.ga.nkr <= kGatherRuns) {
        f |= deposit_runs(v >> 2, g.ga.krun, g.ga.nkr);
      } else {
        for (int j = 2; j < g.ga.nk; ++j) f |= ((v >> j) & 1) << g.ga.kpos[j];
      }
      frow[h] = f + 2 * (i & 1);
    }
  } else if constexpr (GA) {
    const int64_t fq = (int64_t)(q & 1) << g.ga.kpos[0] | (int64_t)(q >> 1) << g.ga.kpos[1];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = mw + 16 * r + i;
      int64_t f = fq;
      if (g.ga.nmr <= kGatherRuns) {
        f |= deposit_runs(m, g.ga.mrun, g.ga.nmr);
      } else {
        for (int j = 0; j < g.ga.nm; ++j) f |= ((m >> j) & 1) << g.ga.mpos[j];
      }
      frow[r] = f;
    }
  }
  for (int64_t kc = 0; kc < g.K; kc += KC) {
    const int kn = g.K - kc < KC ? (int)(g.K - kc) : KC;
    __syncthreads();  // the previous chunk's reads of Bs are done
    for (int e = tid; e < kn * 16; e += 256) {
      const int kr = e >> 4, n = e & 15;
      float2 x = make_float2(0.f, 0.f);
      if (n < N) x = TB ? B[(int64_t)n * g.ldb + kc + kr] : B[(kc + kr) * g.ldb + n];
      Bs[kr][n] = x;
    }
    __syncthreads();
    for (int kb = 0; kb < kn; kb += 16) {
      const int64_t k0 = kc + kb;
      float2 a[4][4];  // [row block][instruction]
      if constexpr (GA && TA) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int64_t kk = kz + k0 + 4 * q + st;
          int64_t fm = 0;
          if (g.ga.nmr <= kGatherRuns) {
            fm = deposit_runs(kk, g.ga.mrun, g.ga.nmr);
          } else {
            for (int j = 0; j < g.ga.nm; ++j) fm |= ((kk >> j) & 1) << g.ga.mpos[j];
          }
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const f32x4 v = *reinterpret_cast<const f32x4*>(A + fm + frow[h]);
            a[2 * h][st] = make_float2(v.x, v.y);
            a[2 * h + 1][st] = make_float2(v.z, v.w);
          }
        }
      } else if constexpr (GA) {
        const int64_t kt = (kz + k0) >> 4;  // index of this tile of 16 k
        int64_t gk = 0;
        if (g.ga.nkr <= kGatherRuns) {
          gk = deposit_runs(kt, g.ga.krun, g.ga.nkr);
        } else {
          for (int j = 2; j < g.ga.nk; ++j) gk |= ((kt >> (j - 2)) & 1) << g.ga.kpos[j];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float2* p = A + frow[r] + gk;
          const f32x4 v0 = *reinterpret_cast<const f32x4*>(p);
          const f32x4 v1 = *reinterpret_cast<const f32x4*>(p + 2);
          a[r][0] = make_float2(v0.x, v0.y);
          a[r][1] = make_float2(v0.z, v0.w);
          a[r][2] = make_float2(v1.x, v1.y);
          a[r][3] = make_float2(v1.z, v1.w);
        }
      } else if (!TA) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float2* p = A + (mw + 16 * r + i) * g.lda + k0 + 4 * q;
          const f32x4 v0 = *reinterpret_cast<const f32x4*>(p);
          const f32x4 v1 = *reinterpret_cast<const f32x4*>(p + 2);
          a[r][0] = make_float2(v0.x, v0.y);
          a[r][1] = make_float2(v0.z, v0.w);
          a[r][2] = make_float2(v1.x, v1.y);
          a[r][3] = make_float2(v1.z, v1.w);
        }
      } else {
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const f32x4 v = *reinterpret_cast<const f32x4*>(A + (k0 + 4 * q + st) * g.lda + mw +
                                                            32 * h + 2 * i);
            a[2 * h][st] = make_float2(v.x, v.y);
            a[2 * h + 1][st] = make_float2(v.z, v.w);
          }
      }
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const float2 w = Bs[kb + 4 * q + st][i];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          cr[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][st].x, w.x, cr[r], 0, 0, 0);
          ci[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][st].x, w.y, ci[r], 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          cr[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[r][st].y, w.y, cr[r], 0, 0, 0);
          ci[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][st].y, w.x, ci[r], 0, 0, 0);
        }
      }
    }
  }
  // D layout of the 16x16 instruction: lane -> column i, register v -> row 4 q + v of the block
  if (i < N) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = 4 * q + v;
        const int64_t m = TA ? mw + 32 * (r >> 1) + 2 * rr + (r & 1) : mw + 16 * r + rr;
        C[m * ldc + i] = make_float2(cr[r][v], ci[r][v]);
      }
  }
}

// C[b] = sum over chunks z of ws[z][b] (in chunk order), written with C's row stride
__global__ void splitk_reduce_kernel(const float2* __restrict__ ws, int split, int batch,
                                     int64_t M, int64_t N, float2* __restrict__ C, int64_t ldc,
                                     int64_t c_bs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t mn = M * N;
  if (e >= mn) return;
  const int b = blockIdx.y;
  float re = 0.f, im = 0.f;
  for (int z = 0; z < split; ++z) {
    const float2 v = ws[((int64_t)z * batch + b) * mn + e];
    re += v.x;
    im += v.y;
  }
  C[b * c_bs + (e / N) * ldc + e % N] = make_float2(re, im);
}

template <bool TA, bool TB>
static void gemm_t(const Gemm& g, hipStream_t s) {
  const int v = gemm_variant(g);
  const unsigned z = (unsigned)g.split;
  if (v == 8) {
    dim3 grid((unsigned)(g.M / 256), (unsigned)g.batch, z);
    if (g.gather)
      hipLaunchKernelGGL((gemm_rows_mfma_kernel<TA, TB, true>), grid, dim3(256), 0, s, g);
    else
      hipLaunchKernelGGL((gemm_rows_mfma_kernel<TA, TB>), grid, dim3(256), 0, s, g);
  } else if (v == 7) {
    dim3 grid((unsigned)(g.N / 64), (unsigned)g.batch, z);
    hipLaunchKernelGGL((gemm_reduce_mfma_kernel<TA>), grid, dim3(256), 0, s, g);
  } else if (gemm_scatter_variant(v) && g.scatter) {
    // the output-mapped tiles, instantiated for A stored [M][K] only (an operand cotangent
    // Xbar = Zbar Y^T)
    if constexpr (TA) {
      throw std::runtime_error("gemm: an output map needs A stored [M][K]");
    } else if (v == 5) {
      dim3 grid((unsigned)(((g.M + 63) / 64) * (g.N / std::min<int64_t>(g.N, 256))),
                (unsigned)g.batch);
      auto sk = [&](auto kern) { hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, g); };
      if (g.K > 4) sk(gemm_smallk_kernel<8, false, TB, true>);
      else if (g.K > 2) sk(gemm_smallk_kernel<4, false, TB, true>);
      else if (g.K > 1) sk(gemm_smallk_kernel<2, false, TB, true>);
      else sk(gemm_smallk_kernel<1, false, TB, true>);
    } else {
      const int bm = v == 6 || v == 9 ? 256 : v == 1 ? 64 : 128, bn = v == 1 ? 64 : 128;
      dim3 grid((unsigned)((g.M / bm) * (g.N / bn)), (unsigned)g.batch, z);
      if (v == 6)
        hipLaunchKernelGGL((gemm_mfma_kernel<false, TB, 256, 128, 4, 2, false, true>), grid,
                           dim3(512), 0, s, g);
      else if (v == 9)
        hipLaunchKernelGGL((gemm_mfma_kernel<false, TB, 256, 128, 4, 2, true, true>), grid,
                           dim3(512), 0, s, g);
      else if (v == 10)
        hipLaunchKernelGGL((gemm_mfma_kernel<false, TB, 128, 128, 2, 2, true, true>), grid,
                           dim3(256), 0, s, g);
      else if (v == 2)
        hipLaunchKernelGGL((gemm_mfma_kernel<false, TB, 128, 128, 2, 2, false, true>), grid,
                           dim3(256), 0, s, g);
      else
        hipLaunchKernelGGL((gemm_mfma_kernel<false, TB, 64, 64, 2, 2, false, true>), grid,
                           dim3(256), 0, s, g);
    }
  } else if (v == 6) {
    dim3 grid((unsigned)((g.M / 256) * (g.N / 128)), (unsigned)g.batch, z);
    hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB, 256, 128, 4, 2>), grid, dim3(512), 0, s, g);
  } else if (v == 9) {
    dim3 grid((unsigned)((g.M / 256) * (g.N / 128)), (unsigned)g.batch, z);
    hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB, 256, 128, 4, 2, true>), grid, dim3(512), 0, s,
                       g);
  } else if (v == 10) {
    dim3 grid((unsigned)((g.M / 128) * (g.N / 128)), (unsigned)g.batch, z);
    hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB, 128, 128, 2, 2, true>), grid, dim3(256), 0, s,
                       g);
  } else if (v == 2) {
    dim3 grid((unsigned)((g.M / 128) * (g.N / 128)), (unsigned)g.batch, z);
    hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB, 128, 128>), grid, dim3(256), 0, s, g);
  } else if (v == 1) {
    dim3 grid((unsigned)((g.M / 64) * (g.N / 64)), (unsigned)g.batch, z);
    hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB, 64, 64>), grid, dim3(256), 0, s, g);
  } else if (v == 3) {
    dim3 grid((unsigned)(g.M / 256), (unsigned)g.batch, z);
    if (g.K == 8) {  // N <= 16
      auto rows8 = [&](auto kern) { hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, g); };
      if (g.N > 8) rows8(gemm_rows_kernel<16, TA, TB, 8>);
      else if (g.N > 4) rows8(gemm_rows_kernel<8, TA, TB, 8>);
      else if (g.N > 2) rows8(gemm_rows_kernel<4, TA, TB, 8>);
      else if (g.N > 1) rows8(gemm_rows_kernel<2, TA, TB, 8>);
      else rows8(gemm_rows_kernel<1, TA, TB, 8>);
    } else if (g.N > 16) {
      hipLaunchKernelGGL((gemm_rows_kernel<32, TA, TB>), grid, dim3(256), 0, s, g);
    } else if (g.N > 8) {
      hipLaunchKernelGGL((gemm_rows_kernel<16, TA, TB>), grid, dim3(256), 0, s, g);
    } else if (g.N > 4) {
      hipLaunchKernelGGL((gemm_rows_kernel<8, TA, TB>), grid, dim3(256), 0, s, g);
    } else if (g.N > 2) {
      hipLaunchKernelGGL((gemm_rows_kernel<4, TA, TB>), grid, dim3(256), 0, s, g);
    } else if (g.N > 1) {
      hipLaunchKernelGGL((gemm_rows_kernel<2, TA, TB>), grid, dim3(256), 0, s, g);
    } else {
      hipLaunchKernelGGL((gemm_rows_kernel<1, TA, TB>), grid, dim3(256), 0, s, g);
    }
  } else if (v == 4) {
    dim3 grid((unsigned)(g.N / std::min<int64_t>(g.N, 256)), (unsigned)g.batch, z);
    if (g.M > 16) hipLaunchKernelGGL((gemm_reduce_kernel<32, TA>), grid, dim3(256), 0, s, g);
    else if (g.M > 8) hipLaunchKernelGGL((gemm_reduce_kernel<16, TA>), grid, dim3(256), 0, s, g);
    else if (g.M > 4) hipLaunchKernelGGL((gemm_reduce_kernel<8, TA>), grid, dim3(256), 0, s, g);
    else if (g.M > 2) hipLaunchKernelGGL((gemm_reduce_kernel<4, TA>), grid, dim3(256), 0, s, g);
    else if (g.M > 1) hipLaunchKernelGGL((gemm_reduce_kernel<2, TA>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((gemm_reduce_kernel<1, TA>), grid, dim3(256), 0, s, g);
  } else if (v == 5) {
    dim3 grid((unsigned)(((g.M + 63) / 64) * (g.N / std::min<int64_t>(g.N, 256))),
              (unsigned)g.batch);
    if (g.K > 4) hipLaunchKernelGGL((gemm_smallk_kernel<8, TA, TB>), grid, dim3(256), 0, s, g);
    else if (g.K > 2) hipLaunchKernelGGL((gemm_smallk_kernel<4, TA, TB>), grid, dim3(256), 0, s, g);
    else if (g.K > 1) hipLaunchKernelGGL((gemm_smallk_kernel<2, TA, TB>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((gemm_smallk_kernel<1, TA, TB>), grid, dim3(256), 0, s, g);
  } else {
    auto launch = [&](auto kern, int bm, int bn) {
      const int64_t tiles = ((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
      hipLaunchKernelGGL(kern, dim3((unsigned)tiles, (unsigned)g.batch, z), dim3(256), 0, s, g);
    };
    if (g.N >= 16 && g.M >= 16) launch(gemm_simt_kernel<16, 16, TA, TB>, 16, 16);
    else if (g.N >= 8) launch(gemm_simt_kernel<32, 8, TA, TB>, 32, 8);
    else if (g.N >= 4) launch(gemm_simt_kernel<64, 4, TA, TB>, 64, 4);
    else if (g.N >= 2) launch(gemm_simt_kernel<128, 2, TA, TB>, 128, 2);
    else launch(gemm_simt_kernel<256, 1, TA, TB>, 256, 1);
  }
  check_launch("gemm");
}

bool gemm_scatter_variant(int v) {
  return v == 1 || v == 2 || v == 5 || v == 6 || v == 9 || v == 10;
}

void gemm(const Gemm& g0, hipStream_t s) {
  if (g0.batch < 1 || g0.batch > 65535) throw std::runtime_error("gemm: bad batch");
  if (g0.scatter) {  // C through its bit-deposit maps, on the MFMA tiles only
    if (g0.gather || g0.ta || !gemm_scatter_variant(gemm_variant(g0)))
      throw std::runtime_error("gemm: an output map needs an MFMA tile and A stored [M][K]");
    const int nb = g0.om.nm + g0.om.nn;
    if (g0.om.nm < 0 || g0.om.nn < 0 || nb > 31 || (int64_t(1) << g0.om.nm) != g0.M ||
        (int64_t(1) << g0.om.nn) != g0.N || int64_t(1) << nb > g0.c_bs)
      throw std::runtime_error("gemm: output map does not match the shape");
    // every offset below 2^nb <= c_bs: the positions are a permutation of 0 .. nb - 1
    uint32_t seen = 0;
    for (int i = 0; i < nb; ++i) {
      const int p = i < g0.om.nm ? g0.om.mpos[i] : g0.om.npos[i - g0.om.nm];
      if (p < 0 || p >= nb || (seen >> p) & 1)
        throw std::runtime_error("gemm: output map positions are not a permutation");
      seen |= 1u << p;
    }
  }
  if (g0.gather) {  // A read through its gather descriptor, on the MFMA rows kernel only
    if (g0.force_variant != 8 || !gemm_variant_fits(g0, 8))
      throw std::runtime_error("gemm: a gathered A needs the MFMA rows kernel");
    // the descriptor's row bits index A's rows (ta = 0) or its k (ta = 1, A = X^T)
    const int64_t rows = g0.ta ? g0.K : g0.M, cols = g0.ta ? g0.M : g0.K;
    if (g0.ga.nm + g0.ga.nk + 2 > kGatherMaxBits || g0.ga.nk < 2 ||
        (int64_t(1) << g0.ga.nm) != rows || (int64_t(4) << g0.ga.nk) != cols)
      throw std::runtime_error("gemm: gather descriptor does not match the shape");
  }
  Gemm g = g0;
  if (g.gather) {
    g.ga.nmr = gather_runs(g.ga.mpos, 0, g.ga.nm, g.ga.mrun);
    g.ga.nkr = gather_runs(g.ga.kpos, 2, g.ga.nk, g.ga.krun);
  }
  g.split = 1;
  g.a_ks = g.b_ks = 0;
  if (g0.ws && !g0.scatter) {
    const int split = gemm_splitk(g0);
    if (split > 1 && (int64_t)split * g0.batch * g0.M * g0.N <= g0.ws_elems) {
      const int64_t chunk = g0.K / split;
      g.split = split;
      g.K = chunk;
      // a gathered A has no pointer offset per chunk: the kernel runs its k index on instead
      g.a_ks = g0.gather ? 0 : g0.ta ? chunk * g0.lda : chunk;
      g.b_ks = g0.tb ? chunk : chunk * g0.ldb;
    }
  }
  if (g.ta) {
    if (g.tb) gemm_t<true, true>(g, s);
    else gemm_t<true, false>(g, s);
  } else {
    if (g.tb) gemm_t<false, true>(g, s);
    else gemm_t<false, false>(g, s);
  }
  if (g.split > 1) {
    dim3 grid((unsigned)((g.M * g.N + 255) / 256), (unsigned)g.batch);
    hipLaunchKernelGGL(splitk_reduce_kernel, grid, dim3(256), 0, s, g.ws, g.split, g.batch, g.M,
                       g.N, g0.C, g0.ldc, g0.c_bs);
    check_launch("splitk_reduce");
  }
}
}  // namespace dev
}  // namespace qflex
