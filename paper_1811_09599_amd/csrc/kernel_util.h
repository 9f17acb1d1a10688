// Device helpers shared by the kernel sources of the contraction path (gfx950).
#pragma once

#include <stdexcept>
#include <string>

#include "kernels.h"

namespace qflex {
namespace dev {

inline void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

typedef float floatx16 __attribute__((ext_vector_type(16)));
// Register staging uses native vector types: HIP's float4 / uint4 are structs whose copies
// lower to memcpy calls, which keep staging arrays in memory (scratch or LDS) instead of
// registers and expose every global load's latency.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---- fp16 split operands: power-of-two scale from the largest magnitude (low 32 bits of the
// slot absmax() fills).  The scaled maximum lies in [2^14, 2^15): hi parts stay below the
// fp16 maximum (65504) and lo parts stay normal down to 2^-17 of it.
__device__ inline float pow2f(int k) {  // 2^k for -126 <= k <= 127
  return __uint_as_float((uint32_t)(127 + k) << 23);
}
__device__ inline int fp16_scale_exp(uint64_t slot) {
  const uint32_t bits = (uint32_t)slot;
  const int e = (int)((bits >> 23) & 0xff);  // biased exponent: max in [2^(e-127), 2^(e-126))
  if (e == 0 || e == 0xff) return 0;  // zero or subnormal maximum, inf or NaN: no scaling
  const int k = 14 - (e - 127);
  return k < -100 ? -100 : (k > 100 ? 100 : k);
}
__device__ inline float fp16_scale(uint64_t slot) { return pow2f(fp16_scale_exp(slot)); }
__device__ inline float fp16_unscale(uint64_t slot) { return pow2f(-fp16_scale_exp(slot)); }

// ---- hi + lo split of FP32 values into 16-bit parts (bf16 or fp16)
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// (a, b) = hi + lo per value, both rounded to nearest even, packed two per 32-bit word (a in
// the low half); the differences are exact in FP32.  gfx950 converts a pair in one
// instruction (v_cvt_pk_bf16_f32 / v_cvt_pk_f16_f32).
template <bool F16>
__device__ inline void split16x2(float a, float b, uint32_t& hi, uint32_t& lo) {
  const f32x2 x = {a, b};
  if constexpr (F16) {
    const f16x2 h = __builtin_convertvector(x, f16x2);
    const f16x2 l = __builtin_convertvector(x - __builtin_convertvector(h, f32x2), f16x2);
    hi = __builtin_bit_cast(uint32_t, h);
    lo = __builtin_bit_cast(uint32_t, l);
  } else {
    const bf16x2 h = __builtin_convertvector(x, bf16x2);
    const bf16x2 l = __builtin_convertvector(x - __builtin_convertvector(h, f32x2), bf16x2);
    hi = __builtin_bit_cast(uint32_t, h);
    lo = __builtin_bit_cast(uint32_t, l);
  }
}

// ---- binary index tiles (see permute.hip)
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

// f(v) of a bit map given as runs (see SplitGather); the n <= kGatherRuns run words sit in
// the kernel arguments at fixed offsets, so they are read once, by scalar loads
// Output tile (tm, tn) of workgroup `bid` of a tiled product, in grouped order: groups of up to
// 16 row tiles sweep the column tiles together.  The 256 workgroups resident at once (one per
// compute unit) then cover a 16 x 16 block of tiles, whose 16 row and 16 column panels are
// shared through the caches, instead of one row panel against 256 column panels that stream
// from HBM for every row panel.  Workgroups go to the 8 XCDs round robin, so each XCD gets 2 of
// the block's row tiles against all 16 column tiles.
__device__ inline void grouped_tile(int64_t bid, int64_t tiles_m, int64_t tiles_n, int64_t& tm,
                                    int64_t& tn) {
  constexpr int64_t GM = 16;
  const int64_t per_group = GM * tiles_n;
  const int64_t group = bid / per_group;
  const int64_t first = group * GM;
  const int64_t gsz = tiles_m - first < GM ? tiles_m - first : GM;
  const int64_t r = bid - group * per_group;
  tm = first + r % gsz;
  tn = r / gsz;
}

__device__ inline int64_t deposit_runs(int64_t v, const int32_t (&runs)[kGatherRuns], int n) {
  int64_t f = 0;
#pragma unroll
  for (int r = 0; r < kGatherRuns; ++r) {
    if (r < n) {
      const int32_t w = runs[r];
      const int s = w & 0xff, len = (w >> 8) & 0xff, d = (w >> 16) & 0xff;
      f |= ((v >> s) & ((int64_t(1) << len) - 1)) << d;
    }
  }
  return f;
}
}  // namespace dev
}  // namespace qflex
