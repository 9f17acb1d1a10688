// Device kernels of the contraction path, written for gfx950 (CDNA4: 64-lane wavefronts,
// FP32 MFMA, 160 KB LDS per CU).
#include "kernels.h"

#include <algorithm>
#include <stdexcept>
#include <string>

namespace qflex {
namespace dev {

static void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

// =============================================================================================
// Grid build: time collapse of every qubit's gates (paper, Methods B.1).
// One thread per (qubit, value of the qubit's link bonds): it carries the 2-vector
// |v> = P_t(k_t) ... P_1(k_1) |0> in FP64 through the qubit's pieces, each piece's matrix picked
// by that piece's bond digits, and stores <0|v>, <1|v> as complex64 at the addresses the
// plan's layout assigns to (output bit, bond values).
// =============================================================================================
__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ void __launch_bounds__(256) grid_build_kernel(const GridQubit* __restrict__ qd,
                                                         const GridPiece* __restrict__ pieces,
                                                         const double2* __restrict__ mats,
                                                         const int32_t* __restrict__ pos,
                                                         float2* __restrict__ out) {
  const GridQubit d = qd[blockIdx.y];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t(1) << d.nlb)) return;
  double2 v0 = make_double2(1.0, 0.0), v1 = make_double2(0.0, 0.0);
  for (int p = d.piece_begin; p < d.piece_end; ++p) {
    const GridPiece pc = pieces[p];
    const int k = (int)((c >> pc.kshift) & pc.kmask);
    const double2* M = mats + 4 * (pc.mat + k);
    const double2 a = cmul(M[0], v0), b = cmul(M[1], v1);
    const double2 e = cmul(M[2], v0), f = cmul(M[3], v1);
    v0 = make_double2(a.x + b.x, a.y + b.y);
    v1 = make_double2(e.x + f.x, e.y + f.y);
  }
  int64_t addr = 0;
  for (int j = 0; j < d.nlb; ++j) addr |= ((c >> (d.nlb - 1 - j)) & 1) << pos[d.pos_base + j];
  out[d.offset + addr] = make_float2((float)v0.x, (float)v0.y);
  out[d.offset + (addr | (int64_t(1) << d.pos_out))] = make_float2((float)v1.x, (float)v1.y);
}

void grid_build(const GridQubit* q, int n_qubits, int max_nlb, const GridPiece* pieces,
                const double2* mats, const int32_t* pos, float2* out, hipStream_t s) {
  const int64_t combos = int64_t(1) << max_nlb;
  dim3 grid((unsigned)((combos + 255) / 256), (unsigned)n_qubits);
  hipLaunchKernelGGL(grid_build_kernel, grid, dim3(256), 0, s, q, pieces, mats, pos, out);
  check_launch("grid_build");
}

// =============================================================================================
// Binary index permutation (paper, Methods B.2: reordering so that contracted indexes are
// contiguous for the matrix product).  GPU form: each workgroup moves one tile of 2^tile_bits
// elements through LDS.  The tile holds the lowest input bits (so every read is a run of
// consecutive addresses) and the lowest output bits (so every write is too); the remaining
// bits enumerate tiles.  A permutation that keeps the low bits in place degenerates into a
// block copy.
// =============================================================================================
PermTile make_perm_tile(int nbits, const int* perm) {
  if (nbits > kPermMaxBits) throw std::runtime_error("permute: too many index bits");
  PermTile t{};
  t.nbits = nbits;
  int inv[kPermMaxBits];
  for (int j = 0; j < nbits; ++j) inv[perm[j]] = j;
  const int T = std::min(nbits, kPermMaxTile);
  bool in_tile[kPermMaxBits] = {false};
  int size = 0;
  for (int p = 0; p < std::min(nbits, 5); ++p) in_tile[p] = true, ++size;
  for (int j = 0; j < nbits && size < T; ++j)
    if (!in_tile[perm[j]]) in_tile[perm[j]] = true, ++size;
  for (int p = 0; p < nbits && size < T; ++p)
    if (!in_tile[p]) in_tile[p] = true, ++size;
  t.tile_bits = size;
  int ti = 0;
  int read_index_of[kPermMaxBits];
  for (int p = 0; p < nbits; ++p)
    if (in_tile[p]) read_index_of[p] = ti, t.tile_in[ti++] = (int8_t)p;
  // write order: tile bits by output position
  int to = 0;
  for (int j = 0; j < nbits; ++j)
    if (in_tile[perm[j]]) {
      t.tile_out[to] = (int8_t)j;
      t.j2i[to] = (int8_t)read_index_of[perm[j]];
      ++to;
    }
  int r = 0;
  for (int p = 0; p < nbits; ++p)
    if (!in_tile[p]) {
      t.rest_in[r] = (int8_t)p;
      t.rest_out[r] = (int8_t)inv[p];
      ++r;
    }
  t.nrest = r;
  return t;
}

__device__ inline int lds_pad(int i) { return i + (i >> 5); }

// Offsets of tile element i = t + 256*k are split into a per-thread part (bits 0..7 of i,
// computed once) and a per-k part (bits 8..9), so that each element costs one add instead of
// a loop over the tile bits.  Every loop over descriptor entries is fully unrolled with a
// static index, so the descriptor stays in scalar registers.
__device__ inline int64_t rest_offset(int64_t T, const int8_t* pos, int n) {
  int64_t o = 0;
#pragma unroll
  for (int r = 0; r < kPermMaxBits; ++r)
    if (r < n) o |= ((T >> r) & 1) << pos[r];
  return o;
}

// bits [from, to) of v (v's bit 0 is bit `from`) deposited at positions pos[from..to)
template <int FROM, int TO>
__device__ inline int64_t deposit(int v, const int8_t* pos, int limit) {
  int64_t o = 0;
#pragma unroll
  for (int b = FROM; b < TO; ++b)
    if (b < limit) o |= (int64_t)((v >> (b - FROM)) & 1) << pos[b];
  return o;
}

template <int FROM, int TO>
__device__ inline int deposit_i(int v, const int8_t* pos, int limit) {
  int o = 0;
#pragma unroll
  for (int b = FROM; b < TO; ++b)
    if (b < limit) o |= ((v >> (b - FROM)) & 1) << pos[b];
  return o;
}

__global__ void __launch_bounds__(256) permute_kernel(const float2* __restrict__ in,
                                                      float2* __restrict__ out,
                                                      const PermTile t) {
  __shared__ float2 tile[(1 << kPermMaxTile) + (1 << kPermMaxTile) / 32];
  const int64_t batch_stride = int64_t(1) << t.nbits;
  in += (int64_t)blockIdx.y * batch_stride;
  out += (int64_t)blockIdx.y * batch_stride;
  const int64_t T = blockIdx.x;
  const int64_t in_base = rest_offset(T, t.rest_in, t.nrest);
  const int64_t out_base = rest_offset(T, t.rest_out, t.nrest);
  const int tb = t.tile_bits;
  const int tsize = 1 << tb;
  const int tid = threadIdx.x;
  const int nk = tsize > 256 ? tsize >> 8 : 1;
  if (tid < tsize) {
    const int64_t in_lo = in_base + deposit<0, 8>(tid, t.tile_in, tb);
    for (int k = 0; k < nk; ++k)
      tile[lds_pad(tid + (k << 8))] = in[in_lo + deposit<8, kPermMaxTile>(k, t.tile_in, tb)];
  }
  __syncthreads();
  if (tid < tsize) {
    const int i_lo = deposit_i<0, 8>(tid, t.j2i, tb);
    const int64_t out_lo = out_base + deposit<0, 8>(tid, t.tile_out, tb);
    for (int k = 0; k < nk; ++k) {
      const int i = i_lo | deposit_i<8, kPermMaxTile>(k, t.j2i, tb);
      out[out_lo + deposit<8, kPermMaxTile>(k, t.tile_out, tb)] = tile[lds_pad(i)];
    }
  }
}

void permute(const float2* in, float2* out, int64_t batch, const PermTile& t, hipStream_t s) {
  const int64_t tiles = int64_t(1) << t.nrest;
  if (batch < 1 || batch > 65535) throw std::runtime_error("permute: bad batch");
  hipLaunchKernelGGL(permute_kernel, dim3((unsigned)tiles, (unsigned)batch), dim3(256), 0, s, in,
                     out, t);
  check_launch("permute");
}

// =============================================================================================
// Complex64 matrix product (paper, Methods B.2: each pairwise contraction is one matrix
// multiplication after the permutation).
//
// MFMA kernel: 256 threads = 4 wavefronts in 2x2, each owning a (BM/2)x(BN/2) complex block
// made of 32x32 sub-tiles of v_mfma_f32_32x32x2f32.  The complex product runs in 4M form on
// the real instruction: Cr += ar*br + (-ai)*bi, Ci += ar*bi + ai*br.  Operand tiles of
// BK = 16 complex k-values are staged in LDS with k contiguous for both operands (rows padded
// to 144 bytes), double buffered with one barrier per k-tile; the global loads of tile t+1
// are issued before the MFMAs of tile t.  Within a k-tile, lanes 0-31 take k = 0..7 and
// lanes 32-63 take k = 8..15 (the two halves of the instruction's K=2), so each lane reads its
// operands as 16-byte vectors.
// =============================================================================================
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <bool TA, bool TB, int BM, int BN>
__global__ void __launch_bounds__(256) gemm_mfma_kernel(const Gemm g) {
  constexpr int BK = 16, LDK = BK + 2;
  constexpr int TMI = BM / 64, TNI = BN / 64;
  constexpr int AV = BM / 32, BV = BN / 32;  // float4 (2 complex) loads per thread per tile
  __shared__ __attribute__((aligned(16))) float2 As[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) float2 Bs[2][BN * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int h = lane >> 5, r = lane & 31;
  const int64_t tiles_n = g.N / BN;
  const int64_t tm = (int64_t)blockIdx.x / tiles_n, tn = (int64_t)blockIdx.x % tiles_n;
  const int b = blockIdx.y;
  const float2* __restrict__ A = g.A + g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs);
  const float2* __restrict__ B = g.B + g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs);
  float2* __restrict__ C = g.C + b * g.c_bs;
  const int64_t m0 = tm * BM, n0 = tn * BN;

  float4 ra[AV], rb[BV];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int e = tid + v * 256;
      if (!TA) {
        const int row = e >> 3, kp = e & 7;
        ra[v] = *reinterpret_cast<const float4*>(A + (m0 + row) * g.lda + k0 + 2 * kp);
      } else {
        const int kr = e / (BM / 2), mp = e % (BM / 2);
        ra[v] = *reinterpret_cast<const float4*>(A + (k0 + kr) * g.lda + m0 + 2 * mp);
      }
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int e = tid + v * 256;
      if (!TB) {
        const int kr = e / (BN / 2), np = e % (BN / 2);
        rb[v] = *reinterpret_cast<const float4*>(B + (k0 + kr) * g.ldb + n0 + 2 * np);
      } else {
        const int row = e >> 3, kp = e & 7;
        rb[v] = *reinterpret_cast<const float4*>(B + (n0 + row) * g.ldb + k0 + 2 * kp);
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int e = tid + v * 256;
      if (!TA) {
        const int row = e >> 3, kp = e & 7;
        *reinterpret_cast<float4*>(&As[buf][row * LDK + 2 * kp]) = ra[v];
      } else {
        const int kr = e / (BM / 2), mp = e % (BM / 2);
        As[buf][(2 * mp) * LDK + kr] = make_float2(ra[v].x, ra[v].y);
        As[buf][(2 * mp + 1) * LDK + kr] = make_float2(ra[v].z, ra[v].w);
      }
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int e = tid + v * 256;
      if (!TB) {
        const int kr = e / (BN / 2), np = e % (BN / 2);
        Bs[buf][(2 * np) * LDK + kr] = make_float2(rb[v].x, rb[v].y);
        Bs[buf][(2 * np + 1) * LDK + kr] = make_float2(rb[v].z, rb[v].w);
      } else {
        const int row = e >> 3, kp = e & 7;
        *reinterpret_cast<float4*>(&Bs[buf][row * LDK + 2 * kp]) = rb[v];
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
    if (kt + 1 < nk) gload((int64_t)(kt + 1) * BK);
    const float2* as = As[buf];
    const float2* bs = Bs[buf];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      float4 af[TMI], bf[TNI];
#pragma unroll
      for (int i = 0; i < TMI; ++i)
        af[i] = *reinterpret_cast<const float4*>(
            &as[(wm * (BM / 2) + i * 32 + r) * LDK + h * 8 + 2 * s2]);
#pragma unroll
      for (int j = 0; j < TNI; ++j)
        bf[j] = *reinterpret_cast<const float4*>(
            &bs[(wn * (BN / 2) + j * 32 + r) * LDK + h * 8 + 2 * s2]);
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
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }
  // D layout of the 32x32 instruction: lane -> column r, register v -> row 8*(v/4)+4*h+(v%4)
#pragma unroll
  for (int i = 0; i < TMI; ++i)
#pragma unroll
    for (int j = 0; j < TNI; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wm * (BM / 2) + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        const int col = wn * (BN / 2) + j * 32 + r;
        C[(m0 + row) * g.ldc + n0 + col] = make_float2(cr[i][j][v], ci[i][j][v]);
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
  const int b = blockIdx.y;
  const float2* A = g.A + g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs);
  const float2* B = g.B + g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs);
  float2* C = g.C + b * g.c_bs;
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
  if (m < g.M && n < g.N) C[m * g.ldc + n] = make_float2(accr, acci);
}

int gemm_variant(const Gemm& g) {
  if (g.K % 16 == 0 && g.M % 128 == 0 && g.N % 128 == 0) return 2;
  if (g.K % 16 == 0 && g.M % 64 == 0 && g.N % 64 == 0) return 1;
  return 0;
}

const char* gemm_name(const Gemm& g) {
  static const char* names[3][4] = {
      {"gemm_simt_nn", "gemm_simt_nt", "gemm_simt_tn", "gemm_simt_tt"},
      {"gemm_mfma_64x64_nn", "gemm_mfma_64x64_nt", "gemm_mfma_64x64_tn", "gemm_mfma_64x64_tt"},
      {"gemm_mfma_128x128_nn", "gemm_mfma_128x128_nt", "gemm_mfma_128x128_tn",
       "gemm_mfma_128x128_tt"}};
  return names[gemm_variant(g)][(g.ta ? 2 : 0) + (g.tb ? 1 : 0)];
}

template <bool TA, bool TB>
static void gemm_t(const Gemm& g, hipStream_t s) {
  if (g.batch < 1 || g.batch > 65535) throw std::runtime_error("gemm: bad batch");
  const int v = gemm_variant(g);
  if (v == 2) {
    dim3 grid((unsigned)((g.M / 128) * (g.N / 128)), (unsigned)g.batch);
    hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB, 128, 128>), grid, dim3(256), 0, s, g);
  } else if (v == 1) {
    dim3 grid((unsigned)((g.M / 64) * (g.N / 64)), (unsigned)g.batch);
    hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB, 64, 64>), grid, dim3(256), 0, s, g);
  } else {
    auto launch = [&](auto kern, int bm, int bn) {
      const int64_t tiles = ((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
      hipLaunchKernelGGL(kern, dim3((unsigned)tiles, (unsigned)g.batch), dim3(256), 0, s, g);
    };
    if (g.N >= 16 && g.M >= 16) launch(gemm_simt_kernel<16, 16, TA, TB>, 16, 16);
    else if (g.N >= 8) launch(gemm_simt_kernel<32, 8, TA, TB>, 32, 8);
    else if (g.N >= 4) launch(gemm_simt_kernel<64, 4, TA, TB>, 64, 4);
    else if (g.N >= 2) launch(gemm_simt_kernel<128, 2, TA, TB>, 128, 2);
    else launch(gemm_simt_kernel<256, 1, TA, TB>, 256, 1);
  }
  check_launch("gemm");
}

void gemm(const Gemm& g, hipStream_t s) {
  if (g.ta) {
    if (g.tb) gemm_t<true, true>(g, s);
    else gemm_t<true, false>(g, s);
  } else {
    if (g.tb) gemm_t<false, true>(g, s);
    else gemm_t<false, false>(g, s);
  }
}

// =============================================================================================
// Split-precision complex products on bf16 MFMA (see kernels.h for the operand layouts).
// =============================================================================================
__device__ inline uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// One thread per group of 4 consecutive k of a row: the tile's write order starts with the
// lowest output bits, so a group is 4 consecutive write indices and is stored as two 16-byte
// vectors.
__global__ void __launch_bounds__(256) split_permute_kernel(const float2* __restrict__ in,
                                                            uint16_t* __restrict__ out,
                                                            const PermTile t) {
  __shared__ float2 tile[(1 << kPermMaxTile) + (1 << kPermMaxTile) / 32];
  const int64_t n_el = int64_t(1) << t.nbits;
  in += (int64_t)blockIdx.y * n_el;
  out += (int64_t)blockIdx.y * n_el * 4;
  const int64_t T = blockIdx.x;
  const int64_t in_base = rest_offset(T, t.rest_in, t.nrest);
  const int64_t out_base = rest_offset(T, t.rest_out, t.nrest);
  const int tb = t.tile_bits;
  const int tsize = 1 << tb;
  const int tid = threadIdx.x;
  const int nk = tsize > 256 ? tsize >> 8 : 1;
  if (tid < tsize) {
    const int64_t in_lo = in_base + deposit<0, 8>(tid, t.tile_in, tb);
    for (int k = 0; k < nk; ++k)
      tile[lds_pad(tid + (k << 8))] = in[in_lo + deposit<8, kPermMaxTile>(k, t.tile_in, tb)];
  }
  __syncthreads();
  // group q holds write indices 4q..4q+3 (write bits 0 and 1 are the two lowest k bits);
  // q = tid + 256*k2, k2 < 1 for tiles of up to 1024 elements
  const int ngroups = tsize >> 2;
  if (tid < ngroups) {
    const int q = tid;
    // write index bits 2.. come from q
    int ig = 0;
    int64_t e0 = out_base;
#pragma unroll
    for (int b = 2; b < kPermMaxTile; ++b)
      if (b < tb) {
        const int bit = (q >> (b - 2)) & 1;
        ig |= bit << t.j2i[b];
        e0 |= (int64_t)bit << t.tile_out[b];
      }
    uint16_t h[16];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = ig | ((u & 1) << t.j2i[0]) | (((u >> 1) & 1) << t.j2i[1]);
      const float2 v = tile[lds_pad(i)];
      const uint16_t rh = bf16_rne(v.x), ih = bf16_rne(v.y);
      h[u] = rh;
      h[4 + u] = ih;
      h[8 + u] = bf16_rne(v.x - bf16_to_f(rh));
      h[12 + u] = bf16_rne(v.y - bf16_to_f(ih));
    }
    uint4 lo, hi;
    lo.x = h[0] | ((uint32_t)h[1] << 16);
    lo.y = h[2] | ((uint32_t)h[3] << 16);
    lo.z = h[4] | ((uint32_t)h[5] << 16);
    lo.w = h[6] | ((uint32_t)h[7] << 16);
    hi.x = h[8] | ((uint32_t)h[9] << 16);
    hi.y = h[10] | ((uint32_t)h[11] << 16);
    hi.z = h[12] | ((uint32_t)h[13] << 16);
    hi.w = h[14] | ((uint32_t)h[15] << 16);
    uint4* o = reinterpret_cast<uint4*>(out + 4 * e0);  // e0 is a multiple of 4
    o[0] = lo;
    o[1] = hi;
  }
}

void split_permute(const float2* in, uint16_t* out, int64_t batch, const PermTile& t, int kbits,
                   hipStream_t s) {
  if (batch < 1 || batch > 65535) throw std::runtime_error("split_permute: bad batch");
  // a thread's 4 consecutive write indices must be the 4 lowest k of one row
  if (kbits < 2 || t.tile_bits < 2 || t.tile_out[0] != 0 || t.tile_out[1] != 1)
    throw std::runtime_error("split_permute: K must be >= 4 and the tile must hold the 2 lowest bits");
  const int64_t tiles = int64_t(1) << t.nrest;
  hipLaunchKernelGGL(split_permute_kernel, dim3((unsigned)tiles, (unsigned)batch), dim3(256), 0,
                     s, in, out, t);
  check_launch("split_permute");
}

// Complex product on bf16 MFMA from the compact split layout.  WM x WN wavefronts per
// workgroup (8 for the 256x128 complex tile: two per SIMD hide each other's barrier and LDS
// latency, and the larger tile halves the bytes loaded per MFMA), each owning a 64x64 complex
// block = 2x2 sub-tiles of v_mfma_f32_32x32x16_bf16 with separate real and imaginary
// accumulators.  One instruction step covers 8 complex k: lanes 0-31 hold
// k-group g, lanes 32-63 group g+1, each lane's 8 bf16 being [re(4 k), im(4 k)] of one part:
//   Cr += Ah.Brh + Ah.Brl + Al.Brh,  Brh = [Br_h, -Bi_h]
//   Ci += Ah.Bih + Ah.Bil + Al.Bih,  Bih = [Bi_h,  Br_h]
// (Brh / Bih are built from one 16-byte LDS read by a sign flip / a half swap).  k-tiles of
// 16 complex are staged in LDS (rows of 128 bytes padded to 144), double buffered; the next
// tile's global loads are issued before the current tile's MFMAs.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline bf16x8 as_bf16x8(uint4 v) {
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) gemm_split_kernel(const GemmSplit g) {
  constexpr int NT = 64 * WM * WN;       // threads: WM x WN wavefronts
  constexpr int BK = 16;                 // complex k per tile
  constexpr int ROW = BK * 4;            // bf16 per row per tile (128 bytes)
  constexpr int LDR = ROW + 8;           // padded row (144 bytes)
  constexpr int WTM = BM / WM, WTN = BN / WN;  // wavefront tile (complex)
  constexpr int TMI = WTM / 32, TNI = WTN / 32;
  constexpr int AV = BM * ROW / 8 / NT, BV = BN * ROW / 8 / NT;  // uint4 loads per thread
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * LDR];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * LDR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int h = lane >> 5, r = lane & 31;
  const int64_t tiles_n = g.N / BN;
  const int64_t tm = (int64_t)blockIdx.x / tiles_n, tn = (int64_t)blockIdx.x % tiles_n;
  const int b = blockIdx.y;
  const uint16_t* __restrict__ A = g.A + 4 * (g.a_add + (g.a_off ? g.a_off[b] : b * g.a_bs));
  const uint16_t* __restrict__ B = g.B + 4 * (g.b_add + (g.b_off ? g.b_off[b] : b * g.b_bs));
  float2* __restrict__ C = g.C + b * g.c_bs;
  const int64_t lda = 4 * g.K, ldb = 4 * g.K;
  const int64_t m0 = tm * BM, n0 = tn * BN;

  uint4 ra[AV], rb[BV];
  auto gload = [&](int64_t k0) {  // k0 in bf16 units along the row
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int e = tid + v * NT, row = e >> 3, ch = e & 7;
      ra[v] = *reinterpret_cast<const uint4*>(A + (m0 + row) * lda + k0 + 8 * ch);
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int e = tid + v * NT, row = e >> 3, ch = e & 7;
      rb[v] = *reinterpret_cast<const uint4*>(B + (n0 + row) * ldb + k0 + 8 * ch);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int e = tid + v * NT, row = e >> 3, ch = e & 7;
      *reinterpret_cast<uint4*>(&As[buf][row * LDR + 8 * ch]) = ra[v];
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int e = tid + v * NT, row = e >> 3, ch = e & 7;
      *reinterpret_cast<uint4*>(&Bs[buf][row * LDR + 8 * ch]) = rb[v];
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
      const int col = 16 * (2 * s2 + h);  // this lane's 4-k group, in bf16
      bf16x8 ah[TMI], al[TMI], brh[TNI], brl[TNI], bih[TNI], bil[TNI];
#pragma unroll
      for (int i = 0; i < TMI; ++i) {
        const uint16_t* p = &as[(wm * WTM + i * 32 + r) * LDR + col];
        ah[i] = as_bf16x8(*reinterpret_cast<const uint4*>(p));
        al[i] = as_bf16x8(*reinterpret_cast<const uint4*>(p + 8));
      }
#pragma unroll
      for (int j = 0; j < TNI; ++j) {
        const uint16_t* p = &bs[(wn * WTN + j * 32 + r) * LDR + col];
        const uint4 vh = *reinterpret_cast<const uint4*>(p);
        const uint4 vl = *reinterpret_cast<const uint4*>(p + 8);
        brh[j] = as_bf16x8(make_uint4(vh.x, vh.y, vh.z ^ 0x80008000u, vh.w ^ 0x80008000u));
        brl[j] = as_bf16x8(make_uint4(vl.x, vl.y, vl.z ^ 0x80008000u, vl.w ^ 0x80008000u));
        bih[j] = as_bf16x8(make_uint4(vh.z, vh.w, vh.x, vh.y));
        bil[j] = as_bf16x8(make_uint4(vl.z, vl.w, vl.x, vl.y));
      }
      // term by term over all sub-tiles, so that consecutive MFMAs never feed the same
      // accumulator (each chain has 2*TMI*TNI-1 independent instructions between its links)
#pragma unroll
      for (int i = 0; i < TMI; ++i)
#pragma unroll
        for (int j = 0; j < TNI; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], brh[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bih[j], ci[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < TMI; ++i)
#pragma unroll
        for (int j = 0; j < TNI; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], brl[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bil[j], ci[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < TMI; ++i)
#pragma unroll
        for (int j = 0; j < TNI; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], brh[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bih[j], ci[i][j], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < TMI; ++i)
#pragma unroll
    for (int j = 0; j < TNI; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wm * WTM + i * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
        const int col = wn * WTN + j * 32 + r;
        C[(m0 + row) * g.N + n0 + col] = make_float2(cr[i][j][v], ci[i][j][v]);
      }
}

bool gemm_split_ok(int64_t M, int64_t N, int64_t K) {
  return M > 0 && N > 0 && K > 0 && M % 64 == 0 && N % 64 == 0 && K % 16 == 0;
}

const char* gemm_split_name(const GemmSplit& g) {
  if (g.M % 256 == 0 && g.N % 128 == 0) return "gemm_split_bf16_256x128";
  if (g.M % 128 == 0 && g.N % 128 == 0) return "gemm_split_bf16_128x128";
  return "gemm_split_bf16_64x64";
}

void gemm_split(const GemmSplit& g, hipStream_t s) {
  if (!gemm_split_ok(g.M, g.N, g.K)) throw std::runtime_error("gemm_split: unsupported shape");
  if (g.batch < 1 || g.batch > 65535) throw std::runtime_error("gemm_split: bad batch");
  if (g.M % 256 == 0 && g.N % 128 == 0) {
    dim3 grid((unsigned)((g.M / 256) * (g.N / 128)), (unsigned)g.batch);
    hipLaunchKernelGGL((gemm_split_kernel<256, 128, 4, 2>), grid, dim3(512), 0, s, g);
  } else if (g.M % 128 == 0 && g.N % 128 == 0) {
    dim3 grid((unsigned)((g.M / 128) * (g.N / 128)), (unsigned)g.batch);
    hipLaunchKernelGGL((gemm_split_kernel<128, 128, 2, 2>), grid, dim3(256), 0, s, g);
  } else {
    dim3 grid((unsigned)((g.M / 64) * (g.N / 64)), (unsigned)g.batch);
    hipLaunchKernelGGL((gemm_split_kernel<64, 64, 2, 2>), grid, dim3(256), 0, s, g);
  }
  check_launch("gemm_split");
}

// =============================================================================================
// FP64 accumulation of a slice's result into the amplitude batch (paper, Methods B.1: the
// amplitude is the sum of the path contributions; Methods C.1: a fraction of them).
// =============================================================================================
__global__ void accumulate_kernel(const float2* __restrict__ res, const int64_t* __restrict__ r_off,
                                  int64_t r_bs, int64_t r_add, int64_t n,
                                  const uint32_t* __restrict__ bidx, double2* __restrict__ amps,
                                  int64_t amp_stride) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int b = blockIdx.y;
  const float2 v = res[r_add + (r_off ? r_off[b] : b * r_bs) + e];
  double2* a = amps + b * amp_stride + bidx[e];
  double2 t = *a;
  t.x += (double)v.x;
  t.y += (double)v.y;
  *a = t;
}

void accumulate(const float2* res, const int64_t* r_off, int64_t r_bs, int64_t r_add, int64_t n,
                const uint32_t* bidx, double2* amps, int64_t amp_stride, int batch,
                hipStream_t s) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)batch);
  hipLaunchKernelGGL(accumulate_kernel, grid, dim3(256), 0, s, res, r_off, r_bs, r_add, n, bidx,
                     amps, amp_stride);
  check_launch("accumulate");
}

__global__ void fill_zero_kernel(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

void fill_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  check_launch("fill_zero");
}

// =============================================================================================
// Adjoint of the contraction (gradients).
// =============================================================================================
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One thread per (qubit, bond values): recompute the kets v_t = P_t ... P_1 |0> of the qubit's
// time line (kept in private memory), then carry the cotangent row vector
// u_L = (tbar[o=0], tbar[o=1]) backwards: dP_t[a][b] += u_t[a] v_{t-1}[b], u_{t-1} = u_t P_t.
// Contributions to each piece matrix are summed over the wavefront, then added atomically.
__global__ void __launch_bounds__(256) grid_adjoint_kernel(const GridQubit* __restrict__ qd,
                                                           const GridPiece* __restrict__ pieces,
                                                           const double2* __restrict__ mats,
                                                           const int32_t* __restrict__ pos,
                                                           const double2* __restrict__ tbar,
                                                           double2* __restrict__ pbar) {
  const GridQubit d = qd[blockIdx.y];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = c < (int64_t(1) << d.nlb);
  if ((int64_t)blockIdx.x * blockDim.x >= (int64_t(1) << d.nlb)) return;  // whole block idle
  const int np = d.piece_end - d.piece_begin;
  double2 v0[kMaxPiecesGrad + 1], v1[kMaxPiecesGrad + 1];
  v0[0] = make_double2(1.0, 0.0);
  v1[0] = make_double2(0.0, 0.0);
  for (int t = 0; t < np; ++t) {
    const GridPiece pc = pieces[d.piece_begin + t];
    const int k = active ? (int)((c >> pc.kshift) & pc.kmask) : 0;
    const double2* M = mats + 4 * (pc.mat + k);
    v0[t + 1] = cadd(cmul(M[0], v0[t]), cmul(M[1], v1[t]));
    v1[t + 1] = cadd(cmul(M[2], v0[t]), cmul(M[3], v1[t]));
  }
  double2 u0 = make_double2(0, 0), u1 = make_double2(0, 0);
  if (active) {
    int64_t addr = 0;
    for (int j = 0; j < d.nlb; ++j) addr |= ((c >> (d.nlb - 1 - j)) & 1) << pos[d.pos_base + j];
    u0 = tbar[d.offset + addr];
    u1 = tbar[d.offset + (addr | (int64_t(1) << d.pos_out))];
  }
  const int lane = threadIdx.x & 63;
  for (int t = np - 1; t >= 0; --t) {
    const GridPiece pc = pieces[d.piece_begin + t];
    const int k = active ? (int)((c >> pc.kshift) & pc.kmask) : 0;
    const double2 a0 = v0[t], a1 = v1[t];
    // outer product u (row) x v_{t-1} (column)
    const double2 g[4] = {cmul(u0, a0), cmul(u0, a1), cmul(u1, a0), cmul(u1, a1)};
    for (int kk = 0; kk <= pc.kmask; ++kk) {
      const bool mine = active && k == kk;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double re = wave_sum(mine ? g[e].x : 0.0);
        const double im = wave_sum(mine ? g[e].y : 0.0);
        if (lane == 0 && (re != 0.0 || im != 0.0)) {
          atomicAdd(&pbar[4 * (pc.mat + kk) + e].x, re);
          atomicAdd(&pbar[4 * (pc.mat + kk) + e].y, im);
        }
      }
    }
    const double2* M = mats + 4 * (pc.mat + k);
    const double2 n0 = cadd(cmul(u0, M[0]), cmul(u1, M[2]));
    const double2 n1 = cadd(cmul(u0, M[1]), cmul(u1, M[3]));
    u0 = n0;
    u1 = n1;
  }
}

void grid_adjoint(const GridQubit* q, int n_qubits, int max_nlb, const GridPiece* pieces,
                  const double2* mats, const int32_t* pos, const double2* tbar, double2* pbar,
                  hipStream_t s) {
  const int64_t combos = int64_t(1) << max_nlb;
  dim3 grid((unsigned)((combos + 255) / 256), (unsigned)n_qubits);
  hipLaunchKernelGGL(grid_adjoint_kernel, grid, dim3(256), 0, s, q, pieces, mats, pos, tbar, pbar);
  check_launch("grid_adjoint");
}

struct PermBits {
  int8_t p[kPermMaxBits];
};

__global__ void scatter_add_perm_kernel(const float2* __restrict__ in, int nbits, PermBits pb,
                                        double2* __restrict__ out, const int64_t* __restrict__ off,
                                        int64_t add) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = int64_t(1) << nbits;
  if (e >= n) return;
  const int b = blockIdx.y;
  int64_t o = 0;
  for (int j = 0; j < nbits; ++j) o |= ((e >> pb.p[j]) & 1) << j;
  const float2 v = in[(int64_t)b * n + e];
  double2* dst = out + add + (off ? off[b] : 0) + o;
  atomicAdd(&dst->x, (double)v.x);
  atomicAdd(&dst->y, (double)v.y);
}

void scatter_add_perm(const float2* in, int nbits, const int8_t* perm, int batch, double2* out,
                      const int64_t* off, int64_t add, hipStream_t s) {
  if (nbits > kPermMaxBits) throw std::runtime_error("scatter_add_perm: too many bits");
  PermBits pb{};
  for (int j = 0; j < nbits; ++j) pb.p[j] = perm[j];
  const int64_t n = int64_t(1) << nbits;
  hipLaunchKernelGGL(scatter_add_perm_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)batch),
                     dim3(256), 0, s, in, nbits, pb, out, off, add);
  check_launch("scatter_add_perm");
}

__global__ void seed_cotangent_kernel(const double2* __restrict__ gbar,
                                      const uint32_t* __restrict__ bidx, int64_t n, int64_t namp,
                                      float2* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int b = blockIdx.y;
  const double2 v = gbar[(int64_t)b * namp + bidx[e]];
  dst[(int64_t)b * n + e] = make_float2((float)v.x, (float)-v.y);
}

void seed_cotangent(const double2* gbar, const uint32_t* bidx, int64_t n, int64_t namp,
                    int batch, float2* dst, hipStream_t s) {
  hipLaunchKernelGGL(seed_cotangent_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)batch),
                     dim3(256), 0, s, gbar, bidx, n, namp, dst);
  check_launch("seed_cotangent");
}

__global__ void xeb_cotangent_kernel(const double2* __restrict__ amps, int64_t n, double scale,
                                     double2* __restrict__ gbar, double* __restrict__ sum_sq) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const double2 a = amps[i];
    gbar[i] = make_double2(scale * a.x, scale * a.y);
    v = a.x * a.x + a.y * a.y;
  }
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0 && v != 0.0) atomicAdd(sum_sq, v);
}

void xeb_cotangent(const double2* amps, int64_t n, double scale, double2* gbar, double* sum_sq,
                   hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(xeb_cotangent_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     amps, n, scale, gbar, sum_sq);
  check_launch("xeb_cotangent");
}

}  // namespace dev
}  // namespace qflex
