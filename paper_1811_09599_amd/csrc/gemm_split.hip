// Split-precision complex products on 16-bit MFMA.
#include "kernel_util.h"

#include <type_traits>

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
  const uint16_t* __restrict__ A = g.A + 4 * (g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs));
  const uint16_t* __restrict__ B =
      GB ? nullptr : g.B + 4 * (g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs));
  float2* __restrict__ C = g.C + b * g.c_bs;
  const int64_t lda = 4 * g.K, ldb = 4 * g.K;
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
      const int64_t m = m0 + ((tid + u * NT) >> 2);
      const int grp = (tid + u * NT) & 3;  // k bits 2 and 3 within the tile
      int64_t f = (int64_t)(grp & 1) << g.ga.kpos[0] | (int64_t)(grp >> 1) << g.ga.kpos[1];
      if (g.ga.nmr <= kGatherRuns) {
        f |= deposit_runs(m, g.ga.mrun, g.ga.nmr);
      } else {
        for (int i = 0; i < g.ga.nm; ++i) f |= ((m >> i) & 1) << g.ga.mpos[i];
      }
      frow[u] = f;
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
      const int64_t n = n0 + ((tid + u * NT) >> 2);
      const int grp = (tid + u * NT) & 3;
      int64_t f = (int64_t)(grp & 1) << g.gb.kpos[0] | (int64_t)(grp >> 1) << g.gb.kpos[1];
      if (g.gb.nmr <= kGatherRuns) {
        f |= deposit_runs(n, g.gb.mrun, g.gb.nmr);
      } else {
        for (int i = 0; i < g.gb.nm; ++i) f |= ((n >> i) & 1) << g.gb.mpos[i];
      }
      fcol[u] = f;
    }
    if constexpr (F16) bscale = fp16_scale(*g.b_amax);
  }
  auto gload = [&](int64_t k0) {  // k0 in 16-bit units along the row
    if constexpr (GA) {
      const int64_t kt = k0 / ROW;
      int64_t gk = 0;  // k bits 4.. of the tile
      if (g.ga.nkr <= kGatherRuns) {
        gk = deposit_runs(kt, g.ga.krun, g.ga.nkr);
      } else {
        for (int j = 2; j < g.ga.nk; ++j) gk |= ((kt >> (j - 2)) & 1) << g.ga.kpos[j];
      }
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
        ra[v] = *reinterpret_cast<const u32x4*>(A + (m0 + row) * lda + k0 + 8 * ch);
      }
    }
    if constexpr (GB) {
      const int64_t kt = k0 / ROW;
      int64_t gk = 0;
      if (g.gb.nkr <= kGatherRuns) {
        gk = deposit_runs(kt, g.gb.krun, g.gb.nkr);
      } else {
        for (int j = 2; j < g.gb.nk; ++j) gk |= ((kt >> (j - 2)) & 1) << g.gb.kpos[j];
      }
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
        rb[v] = *reinterpret_cast<const u32x4*>(B + (n0 + row) * ldb + k0 + 8 * ch);
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
    if (kt + 1 < nk) gload((int64_t)(kt + 1) * ROW);
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

bool gemm_split_ok(int64_t M, int64_t N, int64_t K) {
  return M > 0 && N > 0 && K > 0 && M % 64 == 0 && N % 64 == 0 && K % 16 == 0;
}

bool gemm_split_tile_fits(const GemmSplit& g, int tile) {
  switch (tile) {
    case 0: return g.M % 256 == 0 && g.N % 128 == 0;
    case 1: return g.M % 128 == 0 && g.N % 128 == 0;
    case 2: return g.M % 64 == 0 && g.N % 64 == 0;
    case 3: return g.M % 128 == 0 && g.N % 256 == 0;
    default: return false;
  }
}

static int split_tile(const GemmSplit& g) {
  if (g.tile >= 0 && gemm_split_tile_fits(g, g.tile)) return g.tile;
  // a gathered row operand is read from complex64 storage once per column tile: 256 columns
  // per tile where they fit
  if (g.Ac && gemm_split_tile_fits(g, 3)) return 3;
  return gemm_split_tile_fits(g, 0) ? 0 : gemm_split_tile_fits(g, 1) ? 1 : 2;
}

const char* gemm_split_name(const GemmSplit& g) {
  static const char* names[2][2][kSplitTiles] = {
      {{"gemm_split_bf16_256x128", "gemm_split_bf16_128x128", "gemm_split_bf16_64x64",
        "gemm_split_bf16_128x256"},
       {"gemm_split_fp16_256x128", "gemm_split_fp16_128x128", "gemm_split_fp16_64x64",
        "gemm_split_fp16_128x256"}},
      {{"gemm_split_bf16_gather_256x128", "gemm_split_bf16_gather_128x128",
        "gemm_split_bf16_gather_64x64", "gemm_split_bf16_gather_128x256"},
       {"gemm_split_fp16_gather_256x128", "gemm_split_fp16_gather_128x128",
        "gemm_split_fp16_gather_64x64", "gemm_split_fp16_gather_128x256"}}};
  static const char* names_gb[2][kSplitTiles] = {
      {"gemm_split_bf16_gatherb_256x128", "gemm_split_bf16_gatherb_128x128",
       "gemm_split_bf16_gatherb_64x64", "gemm_split_bf16_gatherb_128x256"},
      {"gemm_split_fp16_gatherb_256x128", "gemm_split_fp16_gatherb_128x128",
       "gemm_split_fp16_gatherb_64x64", "gemm_split_fp16_gatherb_128x256"}};
  if (g.Bc && !g.Ac) return names_gb[g.a_amax != nullptr][split_tile(g)];
  return names[g.Ac != nullptr][g.a_amax != nullptr][split_tile(g)];
}

template <bool F16, bool GA, bool GB = false>
static void gemm_split_t(const GemmSplit& g, hipStream_t s) {
  const int tile = split_tile(g);
  if (tile == 3) {
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
