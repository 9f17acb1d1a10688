// Split-precision complex products on 16-bit MFMA.
#include "kernel_util.h"

#include <string>
#include <type_traits>
#include <vector>

namespace qflex {
namespace dev {

// Complex product on 16-bit MFMA from the compact split layout.  WM x WN wavefronts per
// workgroup (8 for the 256x128 and 128x256 complex tiles: two per SIMD hide each other's
// barrier and LDS latency, and the larger tile halves the bytes loaded per MFMA; 128x256 reads
// a 256-column product's row operand once), each owning a 64x64 complex
// block = 2x2 sub-tiles of v_mfma_f32_32x32x16_{bf16,f16} with separate real and imaginary
// accumulators.  One instruction step covers 8 complex k: lanes 0-31 hold
// k-group g, lanes 32-63 group g+1, each lane's 8 values being [re(4 k), im(4 k)] of one part:
//   Cr += Ah.Brh + Ah.Brl + Al.Brh,  Brh = [Br_h, -Bi_h]
//   Ci += Ah.Bih + Ah.Bil + Al.Bih,  Bih = [Bi_h,  Br_h]
// (Brh / Bih are built from one 16-byte LDS read by a sign flip / a half swap; both formats
// keep the sign in bit 15).  k-tiles of 16 complex are staged in LDS (rows of 128 bytes padded
// to 144), double buffered; the next tile's global loads are issued before the current tile's
// MFMAs.  fp16 operands carry power-of-two scales, undone on the FP32 results.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <typename V>
__device__ inline V as_vec(u32x4 v) {
  return __builtin_bit_cast(V, v);
}
__device__ inline floatx16 mfma16(bf16x8 a, bf16x8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ inline floatx16 mfma16(f16x8 a, f16x8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// Gathered operands (complex64 storage read through a SplitGather): offset of the 4-k group
// `grp` (k bits 2 and 3 within a tile of 16 k) of row or column `idx`, fixed for the whole k
// loop, and offset of tile `kt` of 16 k (k bits 4..).  The 4 consecutive k of a group are the
// 2 lowest storage bits: 32 contiguous bytes.
__device__ inline int64_t gather_fixed(const SplitGather& d, int64_t idx, int grp) {
  int64_t f = (int64_t)(grp & 1) << d.kpos[0] | (int64_t)(grp >> 1) << d.kpos[1];
  if (d.nmr <= kGatherRuns) {
    f |= deposit_runs(idx, d.mrun, d.nmr);
  } else {
    for (int i = 0; i < d.nm; ++i) f |= ((idx >> i) & 1) << d.mpos[i];
  }
  return f;
}
__device__ inline int64_t gather_ktile(const SplitGather& d, int64_t kt) {
  if (d.nkr <= kGatherRuns) return deposit_runs(kt, d.krun, d.nkr);
  int64_t gk = 0;
  for (int j = 2; j < d.nk; ++j) gk |= ((kt >> (j - 2)) & 1) << d.kpos[j];
  return gk;
}

// GA: A comes from complex64 storage through the gather descriptor (one permutation and one
// split pass over A fewer): each thread loads whole groups of 4 consecutive k (32 contiguous
// bytes) of its rows, and splits them into the compact layout while storing the tile to LDS.
//
// At least two wavefronts per SIMD: left to itself the compiler gives the fp16 128x128 tile
// 300 registers, which leaves one.
// GB: the same for B (the column operand), through g.gb, when A is not gathered.
template <int BM, int BN, int WM, int WN, bool F16, bool GA, bool GB = false>
__global__ void __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(2)))
gemm_split_kernel(const GemmSplit g) {
  static_assert(!(GA && GB), "one gathered operand per product");
  using V = typename std::conditional<F16, f16x8, bf16x8>::type;
  constexpr int NT = 64 * WM * WN;       // threads: WM x WN wavefronts
  constexpr int BK = 16;                 // complex k per tile
  constexpr int ROW = BK * 4;            // 16-bit values per row per tile (128 bytes)
  constexpr int LDR = ROW + 8;           // padded row (144 bytes)
  constexpr int WTM = BM / WM, WTN = BN / WN;  // wavefront tile (complex)
  constexpr int TMI = WTM / 32, TNI = WTN / 32;
  constexpr int AV = BM * ROW / 8 / NT, BV = BN * ROW / 8 / NT;  // 16-byte loads per thread
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * LDR];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * LDR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int h = lane >> 5, r = lane & 31;
  const int64_t tiles_n = g.N / BN;
  int64_t tm, tn;
  grouped_tile(blockIdx.x, g.M / BM, tiles_n, tm, tn);
  const int b = blockIdx.y;
  const uint16_t* __restrict__ A =
      g.A + kSplitValues * (g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs));
  const uint16_t* __restrict__ B =
      GB ? nullptr : g.B + kSplitValues * (g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs));
  float2* __restrict__ C = g.C + b * g.c_bs;
  const int64_t lda = kSplitValues * g.K, ldb = kSplitValues * g.K;
  auto chunk = [](int64_t kt, int ch) { return kt * ROW + 8 * ch; };
  const int64_t m0 = tm * BM, n0 = tn * BN;

  u32x4 ra[AV], rb[BV];
  // gathered A: AG groups of 4 k per thread per tile, rows fixed for the whole k loop
  constexpr int AG = BM * (BK / 4) / NT;
  f32x4 rc[GA ? AG : 1][2];
  int64_t frow[GA ? AG : 1];  // row offset plus the offset of the thread's k group
  const float2* __restrict__ Ac =
      GA ? g.Ac + g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs) : nullptr;
  float ascale = 1.f;
  if constexpr (GA) {
#pragma unroll
    for (int u = 0; u < AG; ++u) {
      frow[u] = gather_fixed(g.ga, m0 + ((tid + u * NT) >> 2), (tid + u * NT) & 3);
    }
    if constexpr (F16) ascale = fp16_scale(*g.a_amax);
  }
  // gathered B: BG groups of 4 k per thread per tile, columns fixed for the whole k loop
  constexpr int BG = BN * (BK / 4) / NT;
  f32x4 rd[GB ? BG : 1][2];
  int64_t fcol[GB ? BG : 1];
  const float2* __restrict__ Bc =
      GB ? g.Bc + g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs) : nullptr;
  float bscale = 1.f;
  if constexpr (GB) {
#pragma unroll
    for (int u = 0; u < BG; ++u) {
      fcol[u] = gather_fixed(g.gb, n0 + ((tid + u * NT) >> 2), (tid + u * NT) & 3);
    }
    if constexpr (F16) bscale = fp16_scale(*g.b_amax);
  }
  auto gload = [&](int64_t kt) {  // tile kt of 16 k
    if constexpr (GA) {
      const int64_t gk = gather_ktile(g.ga, kt);
#pragma unroll
      for (int u = 0; u < AG; ++u) {
        const float2* p = Ac + frow[u] + gk;
        rc[u][0] = *reinterpret_cast<const f32x4*>(p);
        rc[u][1] = *reinterpret_cast<const f32x4*>(p + 2);
      }
    } else {
#pragma unroll
      for (int v = 0; v < AV; ++v) {
        const int e = tid + v * NT, row = e >> 3, ch = e & 7;
        ra[v] = *reinterpret_cast<const u32x4*>(A + (m0 + row) * lda + chunk(kt, ch));
      }
    }
    if constexpr (GB) {
      const int64_t gk = gather_ktile(g.gb, kt);
#pragma unroll
      for (int u = 0; u < BG; ++u) {
        const float2* p = Bc + fcol[u] + gk;
        rd[u][0] = *reinterpret_cast<const f32x4*>(p);
        rd[u][1] = *reinterpret_cast<const f32x4*>(p + 2);
      }
    } else {
#pragma unroll
      for (int v = 0; v < BV; ++v) {
        const int e = tid + v * NT, row = e >> 3, ch = e & 7;
        rb[v] = *reinterpret_cast<const u32x4*>(B + (n0 + row) * ldb + chunk(kt, ch));
      }
    }
  };
  auto sstore = [&](int buf) {
    if constexpr (GA) {
#pragma unroll
      for (int u = 0; u < AG; ++u) {
        const int e = tid + u * NT, row = e >> 2, grp = e & 3;
        // 4 complex (re, im pairs) -> [rh(4) ih(4)] and [rl(4) il(4)]
        const f32x4 p0 = rc[u][0] * ascale, p1 = rc[u][1] * ascale;
        uint32_t h0, h1, h2, h3, l0, l1, l2, l3;
        split16x2<F16>(p0.x, p0.z, h0, l0);
        split16x2<F16>(p1.x, p1.z, h1, l1);
        split16x2<F16>(p0.y, p0.w, h2, l2);
        split16x2<F16>(p1.y, p1.w, h3, l3);
        const u32x4 hi = {h0, h1, h2, h3}, lo = {l0, l1, l2, l3};
        *reinterpret_cast<u32x4*>(&As[buf][row * LDR + 16 * grp]) = hi;
        *reinterpret_cast<u32x4*>(&As[buf][row * LDR + 16 * grp + 8]) = lo;
      }
    } else {
#pragma unroll
      for (int v = 0; v < AV; ++v) {
        const int e = tid + v * NT, row = e >> 3, ch = e & 7;
        *reinterpret_cast<u32x4*>(&As[buf][row * LDR + 8 * ch]) = ra[v];
      }
    }
    if constexpr (GB) {
#pragma unroll
      for (int u = 0; u < BG; ++u) {
        const int e = tid + u * NT, row = e >> 2, grp = e & 3;
        const f32x4 p0 = rd[u][0] * bscale, p1 = rd[u][1] * bscale;
        uint32_t h0, h1, h2, h3, l0, l1, l2, l3;
        split16x2<F16>(p0.x, p0.z, h0, l0);
        split16x2<F16>(p1.x, p1.z, h1, l1);
        split16x2<F16>(p0.y, p0.w, h2, l2);
        split16x2<F16>(p1.y, p1.w, h3, l3);
        const u32x4 hi = {h0, h1, h2, h3}, lo = {l0, l1, l2, l3};
        *reinterpret_cast<u32x4*>(&Bs[buf][row * LDR + 16 * grp]) = hi;
        *reinterpret_cast<u32x4*>(&Bs[buf][row * LDR + 16 * grp + 8]) = lo;
      }
    } else {
#pragma unroll
      for (int v = 0; v < BV; ++v) {
        const int e = tid + v * NT, row = e >> 3, ch = e & 7;
        *reinterpret_cast<u32x4*>(&Bs[buf][row * LDR + 8 * ch]) = rb[v];
      }
    }
  };
  floatx16 cr[TMI][TNI], ci[TMI][TNI];
#pragma unroll
  for (int i = 0; i < TMI; ++i)
#pragma unroll
    for (int j = 0; j < TNI; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) cr[i][j][v] = ci[i][j][v] = 0.f;
  const int nk = (int)(g.K / BK);
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload(kt + 1);
    const uint16_t* as = As[buf];
    const uint16_t* bs = Bs[buf];
#pragma unroll
    for (int s2 = 0; s2 < BK / 8; ++s2) {
      const int col = 16 * (2 * s2 + h);  // this lane's 4-k group, in 16-bit units
      V ah[TMI], al[TMI], brh[TNI], brl[TNI], bih[TNI], bil[TNI];
#pragma unroll
      for (int i = 0; i < TMI; ++i) {
        const uint16_t* p = &as[(wm * WTM + i * 32 + r) * LDR + col];
        ah[i] = as_vec<V>(*reinterpret_cast<const u32x4*>(p));
        al[i] = as_vec<V>(*reinterpret_cast<const u32x4*>(p + 8));
      }
#pragma unroll
      for (int j = 0; j < TNI; ++j) {
        const uint16_t* p = &bs[(wn * WTN + j * 32 + r) * LDR + col];
        const u32x4 vh = *reinterpret_cast<const u32x4*>(p);
        const u32x4 vl = *reinterpret_cast<const u32x4*>(p + 8);
        const u32x4 sgn = {0u, 0u, 0x80008000u, 0x80008000u};
        brh[j] = as_vec<V>(vh ^ sgn);
        brl[j] = as_vec<V>(vl ^ sgn);
        bih[j] = as_vec<V>(vh.zwxy);
        bil[j] = as_vec<V>(vl.zwxy);
      }
      // term by term over all sub-tiles, so that consecutive MFMAs never feed the same
      // accumulator (each chain has 2*TMI*TNI-1 independent instructions between its links)
#pragma unroll
      for (int i = 0; i < TMI; ++i)
#pragma unroll
        for (int j = 0; j < TNI; ++j) {
          cr[i][j] = mfma16(ah[i], brh[j], cr[i][j]);
          ci[i][j] = mfma16(ah[i], bih[j], ci[i][j]);
        }
#pragma unroll
      for (int i = 0; i < TMI; ++i)
#pragma unroll
        for (int j = 0; j < TNI; ++j) {
          cr[i][j] = mfma16(ah[i], brl[j], cr[i][j]);
          ci[i][j] = mfma16(ah[i], bil[j], ci[i][j]);
        }
#pragma unroll
      for (int i = 0; i < TMI; ++i)
#pragma unroll
        for (int j = 0; j < TNI; ++j) {
          cr[i][j] = mfma16(al[i], brh[j], cr[i][j]);
          ci[i][j] = mfma16(al[i], bih[j], ci[i][j]);
        }
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }
  float ua = 1.f, ub = 1.f, cmax = 0.f;
  if constexpr (F16) ua = fp16_unscale(*g.a_amax), ub = fp16_unscale(*g.b_amax);
#pragma unroll
  for (int i = 0; i < TMI; ++i)
#pragma unroll
    for (int j = 0; j < TNI; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wm * WTM + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        const int col = wn * WTN + j * 32 + r;
        float re = cr[i][j][v], im = ci[i][j][v];
        if constexpr (F16) re = re * ua * ub, im = im * ua * ub;
        C[(m0 + row) * g.N + n0 + col] = make_float2(re, im);
        if constexpr (F16) cmax = fmaxf(cmax, fmaxf(fabsf(re), fabsf(im)));
      }
  if constexpr (F16) {
    // the product's largest magnitude, for the fp16 scale of whoever consumes it next
    if (g.c_amax) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) cmax = fmaxf(cmax, __shfl_xor(cmax, o, 64));
      if (lane == 0)
        atomicMax(reinterpret_cast<unsigned long long*>(g.c_amax),
                  (unsigned long long)(g.c_tag << 32 | __float_as_uint(cmax)));
    }
  }
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Two 16-bit values of a packed word as FP32.
template <bool F16>
__device__ inline f32x2 unpack16x2(uint32_t w) {
  if constexpr (F16) return __builtin_convertvector(__builtin_bit_cast(f16x2, w), f32x2);
  else return __builtin_convertvector(__builtin_bit_cast(bf16x2, w), f32x2);
}

// Complex product on 16-bit MFMA in the 3-multiplication (Gauss) form: with P1 = Ar.Br,
// P2 = Ai.Bi and P3 = (Ar + Ai).(Br + Bi), Re C = P1 - P2 and Im C = P3 - P1 - P2.  Each of the
// three real products takes one v_mfma_f32_32x32x16 per 16 complex k and hi/lo term, 9 per
// 32x32 block instead of the packed form's 12, at the price of a third accumulator set and of
// three operand planes per part (re, im and the sum s = re + im; halved for fp16, which keeps
// its values under the format's maximum, P3 then multiplied back by 4).  A k-tile of 16 complex k
// is staged in LDS as six planes of 16 values per row (re, im, s; hi and lo each), 208-byte
// rows (192 bytes and 16 of padding: the 16-byte reads of 16 consecutive rows hit distinct
// banks).  Staging forms the sums: from hi + lo for pre-split operands (whose hi and lo parts
// are copied), from the complex64 values for gathered ones.
//
// The three accumulator sets take 192 of the 256 registers two wavefronts per SIMD leave, so
// the registers that carry the next tile must stay few: the split layout's 8 bytes per
// complex, not 12 with the sums stored (then the loop spills, and a spill reload waits for the
// prefetch loads issued before it).  They are loaded a tile ahead and converted into the
// other LDS buffer after the first product's MFMAs, whose execution hides the conversion;
// every global address is a wave-uniform base plus one 32-bit lane offset.  WM x WN
// wavefronts of 64x64 blocks.
template <int BM, int BN, int WM, int WN, bool F16, bool GA, bool GB>
__global__ void __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(2)))
gemm_split3m_kernel(const GemmSplit g) {
  static_assert(!(GA && GB), "one gathered operand per product");
  using V = typename std::conditional<F16, f16x8, bf16x8>::type;
  constexpr int NT = 64 * WM * WN;
  constexpr int BK = 16;                       // complex k per tile
  constexpr int LDR = 6 * BK + 8;              // six planes of 16 values + 16 bytes
  constexpr int WTM = BM / WM, WTN = BN / WN;  // wavefront tile (complex)
  constexpr int TMI = WTM / 32, TNI = WTN / 32;
  constexpr int AG = BM * (BK / 4) / NT, BG = BN * (BK / 4) / NT;  // 4-k groups per thread
  static_assert(AG >= 1 && BG >= 1 && AG * NT == BM * (BK / 4) && BG * NT == BN * (BK / 4),
                "tile and thread count");
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * LDR];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * LDR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int h = lane >> 5, r = lane & 31;
  const int grp = tid & 3;  // the 4-k group this thread stages (NT is a multiple of 4)
  int64_t tm, tn;
  grouped_tile(blockIdx.x, g.M / BM, g.N / BN, tm, tn);
  const int b = blockIdx.y;
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int64_t a_base = g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs);
  const int64_t b_base = g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs);
  const int64_t ld = kSplitValues * g.K;  // row stride of the split layout, 16-bit values
  // pre-split operands: the tile's first row; lane offsets in bytes (row * 2 ld, which the
  // tile fit bounds to 31 bits, plus the group's chunk)
  const char* __restrict__ A =
      GA ? nullptr : reinterpret_cast<const char*>(g.A + kSplitValues * a_base + m0 * ld);
  const char* __restrict__ B =
      GB ? nullptr : reinterpret_cast<const char*>(g.B + kSplitValues * b_base + n0 * ld);
  const float2* __restrict__ Ac = GA ? g.Ac + a_base : nullptr;
  const float2* __restrict__ Bc = GB ? g.Bc + b_base : nullptr;
  float2* __restrict__ C = g.C + b * g.c_bs;

  // per thread, per tile: AG groups of A rows and BG of B rows
  uint32_t fa[GA ? 1 : AG], fb[GB ? 1 : BG];     // pre-split: row offset, bytes
  int64_t ga_off[GA ? AG : 1], gb_off[GB ? BG : 1];  // gathered: complex64 offsets
  u32x4 ra[GA ? 1 : AG][2], rb[GB ? 1 : BG][2];  // pre-split: hi and lo chunks
  f32x4 rc[GA ? AG : 1][2], rd[GB ? BG : 1][2];  // gathered: 4 complex64
#pragma unroll
  for (int u = 0; u < AG; ++u) {
    const int row = (tid + u * NT) >> 2;
    if constexpr (GA) ga_off[u] = gather_fixed(g.ga, m0 + row, grp);
    else fa[u] = (uint32_t)(2 * row * ld);
  }
#pragma unroll
  for (int u = 0; u < BG; ++u) {
    const int row = (tid + u * NT) >> 2;
    if constexpr (GB) gb_off[u] = gather_fixed(g.gb, n0 + row, grp);
    else fb[u] = (uint32_t)(2 * row * ld);
  }
  float ascale = 1.f, bscale = 1.f;
  if constexpr (F16 && GA) ascale = fp16_scale(*g.a_amax);
  if constexpr (F16 && GB) bscale = fp16_scale(*g.b_amax);

  auto gload = [&](int kt) {
    // pre-split: byte offset of the group's hi and lo chunks in tile kt
    const uint32_t main_k = (uint32_t)kt * (8 * BK) + 32 * grp;
    if constexpr (GA) {
      const int64_t gk = gather_ktile(g.ga, kt);
#pragma unroll
      for (int u = 0; u < AG; ++u) {
        const float2* p = Ac + ga_off[u] + gk;
        rc[u][0] = *reinterpret_cast<const f32x4*>(p);
        rc[u][1] = *reinterpret_cast<const f32x4*>(p + 2);
      }
    } else {
#pragma unroll
      for (int u = 0; u < AG; ++u) {
        ra[u][0] = *reinterpret_cast<const u32x4*>(A + (fa[u] + main_k));
        ra[u][1] = *reinterpret_cast<const u32x4*>(A + (fa[u] + main_k + 16));
      }
    }
    if constexpr (GB) {
      const int64_t gk = gather_ktile(g.gb, kt);
#pragma unroll
      for (int u = 0; u < BG; ++u) {
        const float2* p = Bc + gb_off[u] + gk;
        rd[u][0] = *reinterpret_cast<const f32x4*>(p);
        rd[u][1] = *reinterpret_cast<const f32x4*>(p + 2);
      }
    } else {
#pragma unroll
      for (int u = 0; u < BG; ++u) {
        rb[u][0] = *reinterpret_cast<const u32x4*>(B + (fb[u] + main_k));
        rb[u][1] = *reinterpret_cast<const u32x4*>(B + (fb[u] + main_k + 16));
      }
    }
  };
  // one group of 4 k of one row into the six planes at `dst` (the row's start + 4 grp)
  auto put_planes = [&](uint16_t* dst, u32x2 reh, u32x2 rel, u32x2 imh, u32x2 iml, u32x2 sh,
                        u32x2 sl) {
    *reinterpret_cast<u32x2*>(dst + 0 * BK) = reh;
    *reinterpret_cast<u32x2*>(dst + 1 * BK) = rel;
    *reinterpret_cast<u32x2*>(dst + 2 * BK) = imh;
    *reinterpret_cast<u32x2*>(dst + 3 * BK) = iml;
    *reinterpret_cast<u32x2*>(dst + 4 * BK) = sh;
    *reinterpret_cast<u32x2*>(dst + 5 * BK) = sl;
  };
  auto stage_split = [&](uint16_t* dst, const u32x4 (&v)[2]) {
    // v[0] = hi parts [re(k0 k1), re(k2 k3), im(k0 k1), im(k2 k3)], v[1] the lo parts
    constexpr float f = F16 ? 0.5f : 1.f;
    const f32x2 re01 = unpack16x2<F16>(v[0].x) + unpack16x2<F16>(v[1].x);
    const f32x2 re23 = unpack16x2<F16>(v[0].y) + unpack16x2<F16>(v[1].y);
    const f32x2 im01 = unpack16x2<F16>(v[0].z) + unpack16x2<F16>(v[1].z);
    const f32x2 im23 = unpack16x2<F16>(v[0].w) + unpack16x2<F16>(v[1].w);
    const f32x2 s01 = f * (re01 + im01), s23 = f * (re23 + im23);
    uint32_t sh0, sl0, sh1, sl1;
    split16x2<F16>(s01.x, s01.y, sh0, sl0);
    split16x2<F16>(s23.x, s23.y, sh1, sl1);
    put_planes(dst, v[0].xy, v[1].xy, v[0].zw, v[1].zw, u32x2{sh0, sh1}, u32x2{sl0, sl1});
  };
  auto stage_complex = [&](uint16_t* dst, f32x4 p0, f32x4 p1) {
    // p0 = (re0, im0, re1, im1), p1 = (re2, im2, re3, im3)
    uint32_t rh0, rl0, rh1, rl1, ih0, il0, ih1, il1, sh0, sl0, sh1, sl1;
    split16x2<F16>(p0.x, p0.z, rh0, rl0);
    split16x2<F16>(p1.x, p1.z, rh1, rl1);
    split16x2<F16>(p0.y, p0.w, ih0, il0);
    split16x2<F16>(p1.y, p1.w, ih1, il1);
    constexpr float f = F16 ? 0.5f : 1.f;
    split16x2<F16>(f * (p0.x + p0.y), f * (p0.z + p0.w), sh0, sl0);
    split16x2<F16>(f * (p1.x + p1.y), f * (p1.z + p1.w), sh1, sl1);
    put_planes(dst, u32x2{rh0, rh1}, u32x2{rl0, rl1}, u32x2{ih0, ih1}, u32x2{il0, il1},
               u32x2{sh0, sh1}, u32x2{sl0, sl1});
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < AG; ++u) {
      uint16_t* dst = &As[buf][((tid + u * NT) >> 2) * LDR + 4 * grp];
      if constexpr (GA) stage_complex(dst, rc[u][0] * ascale, rc[u][1] * ascale);
      else stage_split(dst, ra[u]);
    }
#pragma unroll
    for (int u = 0; u < BG; ++u) {
      uint16_t* dst = &Bs[buf][((tid + u * NT) >> 2) * LDR + 4 * grp];
      if constexpr (GB) stage_complex(dst, rd[u][0] * bscale, rd[u][1] * bscale);
      else stage_split(dst, rb[u]);
    }
  };

  floatx16 acc[3][TMI][TNI];  // P1, P2 and P3 (fp16: P3 / 4)
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int i = 0; i < TMI; ++i)
#pragma unroll
      for (int j = 0; j < TNI; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[p][i][j][v] = 0.f;
  // Registers carry tile kt + 1 while the MFMAs of tile kt run: it is staged into the other
  // LDS buffer after the first of the three products, and the loads of tile kt + 2 are issued
  // right after, a whole iteration ahead of their use.
  const int nk = (int)(g.K / BK);
  gload(0);
  sstore(0);
  if (nk > 1) gload(1);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    const uint16_t* as = As[buf] + (wm * WTM + r) * LDR + 8 * h;
    const uint16_t* bs = Bs[buf] + (wn * WTN + r) * LDR + 8 * h;
#pragma unroll
    for (int p = 0; p < 3; ++p) {  // planes 2p (hi) and 2p + 1 (lo)
      if (p == 1 && kt + 1 < nk) {
        sstore(buf ^ 1);
        if (kt + 2 < nk) gload(kt + 2);
      }
      // the column operands for the whole pass, the row operands one 32-row block at a time
      // (fewer live registers: the accumulators leave little room)
      V bh[TNI], bl[TNI];
#pragma unroll
      for (int j = 0; j < TNI; ++j) {
        bh[j] = as_vec<V>(*reinterpret_cast<const u32x4*>(bs + j * 32 * LDR + 2 * p * BK));
        bl[j] = as_vec<V>(*reinterpret_cast<const u32x4*>(bs + j * 32 * LDR + (2 * p + 1) * BK));
      }
#pragma unroll
      for (int i = 0; i < TMI; ++i) {
        const V ah = as_vec<V>(*reinterpret_cast<const u32x4*>(as + i * 32 * LDR + 2 * p * BK));
        const V al =
            as_vec<V>(*reinterpret_cast<const u32x4*>(as + i * 32 * LDR + (2 * p + 1) * BK));
#pragma unroll
        for (int j = 0; j < TNI; ++j) acc[p][i][j] = mfma16(ah, bh[j], acc[p][i][j]);
#pragma unroll
        for (int j = 0; j < TNI; ++j) acc[p][i][j] = mfma16(ah, bl[j], acc[p][i][j]);
#pragma unroll
        for (int j = 0; j < TNI; ++j) acc[p][i][j] = mfma16(al, bh[j], acc[p][i][j]);
      }
    }
    __syncthreads();
  }
  float uab = 1.f, cmax = 0.f;
  if constexpr (F16) uab = fp16_unscale(*g.a_amax) * fp16_unscale(*g.b_amax);
#pragma unroll
  for (int i = 0; i < TMI; ++i)
#pragma unroll
    for (int j = 0; j < TNI; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wm * WTM + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        const int col = wn * WTN + j * 32 + r;
        const float p1 = acc[0][i][j][v], p2 = acc[1][i][j][v], p3 = acc[2][i][j][v];
        float re = p1 - p2, im = (F16 ? 4.f : 1.f) * p3 - p1 - p2;
        if constexpr (F16) re *= uab, im *= uab;
        C[(m0 + row) * g.N + n0 + col] = make_float2(re, im);
        if constexpr (F16) cmax = fmaxf(cmax, fmaxf(fabsf(re), fabsf(im)));
      }
  if constexpr (F16) {
    if (g.c_amax) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) cmax = fmaxf(cmax, __shfl_xor(cmax, o, 64));
      if (lane == 0)
        atomicMax(reinterpret_cast<unsigned long long*>(g.c_amax),
                  (unsigned long long)(g.c_tag << 32 | __float_as_uint(cmax)));
    }
  }
}

bool gemm_split_ok(int64_t M, int64_t N, int64_t K) {
  return M > 0 && N > 0 && K > 0 && M % 64 == 0 && N % 64 == 0 && K % 16 == 0;
}

bool gemm_split_tile_fits(const GemmSplit& g, int tile) {
  switch (tile) {
    case 0: return g.M % 256 == 0 && g.N % 128 == 0;
    case 1: return g.M % 128 == 0 && g.N % 128 == 0;
    case 2: return g.M % 64 == 0 && g.N % 64 == 0;
    case 3: return g.M % 128 == 0 && g.N % 256 == 0;
    // the 3-multiplication tiles address a tile's rows with 31-bit byte offsets
    case 4: return g.M % 256 == 0 && g.N % 128 == 0 && 2 * 256 * kSplitValues * g.K < (1ll << 31);
    case 5: return g.M % 128 == 0 && g.N % 256 == 0 && 2 * 256 * kSplitValues * g.K < (1ll << 31);
    default: return false;
  }
}

static int split_tile(const GemmSplit& g) {
  if (g.tile >= 0 && gemm_split_tile_fits(g, g.tile)) return g.tile;
  // the 3-multiplication form where its tiles fit (12-15% faster than the packed form's on
  // large products); a gathered row operand is read from complex64 storage once per column
  // tile: 256 columns per tile where they fit
  if (g.Ac && gemm_split_tile_fits(g, 5)) return 5;
  if (gemm_split_tile_fits(g, 4)) return 4;
  if (g.Ac && gemm_split_tile_fits(g, 3)) return 3;
  return gemm_split_tile_fits(g, 0) ? 0 : gemm_split_tile_fits(g, 1) ? 1 : 2;
}

const char* gemm_split_name(const GemmSplit& g) {
  // [3-multiplication][fp16][operand gathered: none, A, B][tile]
  static const std::vector<std::string> names = [] {
    static const char* dims[kSplitTiles] = {"256x128", "128x128", "64x64",
                                            "128x256", "256x128", "128x256"};
    static const char* how[3] = {"", "_gather", "_gatherb"};
    std::vector<std::string> v;
    for (int f = 0; f < 2; ++f)
      for (int gth = 0; gth < 3; ++gth)
        for (int t = 0; t < kSplitTiles; ++t)
          v.push_back(std::string(t >= 4 ? "gemm_split3m_" : "gemm_split_") +
                      (f ? "fp16" : "bf16") + how[gth] + "_" + dims[t]);
    return v;
  }();
  const int gth = g.Ac ? 1 : g.Bc ? 2 : 0;
  return names[((g.a_amax != nullptr) * 3 + gth) * kSplitTiles + split_tile(g)].c_str();
}

template <bool F16, bool GA, bool GB = false>
static void gemm_split_t(const GemmSplit& g, hipStream_t s) {
  const int tile = split_tile(g);
  if (tile == 4) {
    dim3 grid((unsigned)((g.M / 256) * (g.N / 128)), (unsigned)g.batch);
    hipLaunchKernelGGL((gemm_split3m_kernel<256, 128, 4, 2, F16, GA, GB>), grid, dim3(512), 0, s,
                       g);
  } else if (tile == 5) {
    dim3 grid((unsigned)((g.M / 128) * (g.N / 256)), (unsigned)g.batch);
    hipLaunchKernelGGL((gemm_split3m_kernel<128, 256, 2, 4, F16, GA, GB>), grid, dim3(512), 0, s,
                       g);
  } else if (tile == 3) {
    dim3 grid((unsigned)((g.M / 128) * (g.N / 256)), (unsigned)g.batch);
    hipLaunchKernelGGL((gemm_split_kernel<128, 256, 2, 4, F16, GA, GB>), grid, dim3(512), 0, s, g);
  } else if (tile == 0) {
    dim3 grid((unsigned)((g.M / 256) * (g.N / 128)), (unsigned)g.batch);
    hipLaunchKernelGGL((gemm_split_kernel<256, 128, 4, 2, F16, GA, GB>), grid, dim3(512), 0, s, g);
  } else if (tile == 1) {
    dim3 grid((unsigned)((g.M / 128) * (g.N / 128)), (unsigned)g.batch);
    hipLaunchKernelGGL((gemm_split_kernel<128, 128, 2, 2, F16, GA, GB>), grid, dim3(256), 0, s, g);
  } else {
    dim3 grid((unsigned)((g.M / 64) * (g.N / 64)), (unsigned)g.batch);
    hipLaunchKernelGGL((gemm_split_kernel<64, 64, 2, 2, F16, GA, GB>), grid, dim3(256), 0, s, g);
  }
}

// Bits first .. n-1 of a map as runs of consecutive positions; bit i of the source is bit
// (i - first) of the index the kernel deposits.  Returns kGatherRuns + 1 if they do not fit.
int32_t gather_runs(const int8_t* pos, int first, int n, int32_t* runs) {
  int32_t nr = 0;
  for (int i = first; i < n;) {
    int len = 1;
    while (i + len < n && pos[i + len] == pos[i] + len) ++len;
    if (nr == kGatherRuns) return kGatherRuns + 1;
    runs[nr++] = (i - first) | len << 8 | (int32_t)pos[i] << 16;
    i += len;
  }
  return nr;
}

void gemm_split(const GemmSplit& g_in, hipStream_t s) {
  GemmSplit g = g_in;
  if (!gemm_split_ok(g.M, g.N, g.K)) throw std::runtime_error("gemm_split: unsupported shape");
  if (g.batch < 1 || g.batch > 65535) throw std::runtime_error("gemm_split: bad batch");
  if ((g.a_amax == nullptr) != (g.b_amax == nullptr))
    throw std::runtime_error("gemm_split: both operands must use the same format");
  if (g.Ac && g.Bc) throw std::runtime_error("gemm_split: one gathered operand per product");
  if (g.Ac) {
    // the gathered k groups need the 2 lowest k bits in the 2 lowest storage bits
    if (g.ga.nm + g.ga.nk + 2 > kGatherMaxBits || g.ga.nk < 2 || (int64_t(1) << g.ga.nm) != g.M ||
        (int64_t(4) << g.ga.nk) != g.K)
      throw std::runtime_error("gemm_split: gather descriptor does not match the shape");
    g.ga.nmr = gather_runs(g.ga.mpos, 0, g.ga.nm, g.ga.mrun);
    g.ga.nkr = gather_runs(g.ga.kpos, 2, g.ga.nk, g.ga.krun);
    if (g.a_amax) gemm_split_t<true, true>(g, s);
    else gemm_split_t<false, true>(g, s);
  } else if (g.Bc) {
    if (g.gb.nm + g.gb.nk + 2 > kGatherMaxBits || g.gb.nk < 2 || (int64_t(1) << g.gb.nm) != g.N ||
        (int64_t(4) << g.gb.nk) != g.K)
      throw std::runtime_error("gemm_split: gather descriptor does not match the shape");
    g.gb.nmr = gather_runs(g.gb.mpos, 0, g.gb.nm, g.gb.mrun);
    g.gb.nkr = gather_runs(g.gb.kpos, 2, g.gb.nk, g.gb.krun);
    if (g.a_amax) gemm_split_t<true, false, true>(g, s);
    else gemm_split_t<false, false, true>(g, s);
  } else {
    if (g.a_amax) gemm_split_t<true, false>(g, s);
    else gemm_split_t<false, false>(g, s);
  }
  check_launch("gemm_split");
}

}  // namespace dev
}  // namespace qflex
